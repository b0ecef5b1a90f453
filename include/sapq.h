/*
 * sapq.h -- C ABI of libsapq, an MI355X (gfx950) solver for the clover-Wilson
 * system D x = b with the SAP preconditioner, SSOR block inverses in
 * locally-lexicographic order, and a nested FP64/low-precision BiCGStab, after
 * Boku et al., "Multi-block/multi-core SSOR preconditioner for the QCD quark
 * solver for K computer" (Lattice 2012, arXiv:1210.7398).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers (e.g. a torch tensor's data_ptr())
 *    unless marked "host".  The library never allocates device memory: the
 *    caller passes one arena of sapq_arena_bytes() bytes to sapq_create() and
 *    keeps it alive until sapq_destroy().  The caller owns every buffer.
 *  - Interchange layout, complex128 as interleaved (re, im) doubles, site index
 *    n = x + Lx*(y + Ly*(z + Lz*t)):
 *        spinor  [V][4][3]        spin alpha, colour a
 *        links   [V][4][3][3]     U_mu(n)[a][b], the link from n to n+mu, mu = x,y,z,t
 *        clover  [V][2][6][6]     inverse clover F(n): two chiral 6x6 blocks acting on
 *                                 spins {0,1} and {2,3}; row/column 3*(alpha-2k)+a
 *    Gamma matrices are the chiral hermitian Euclidean basis with
 *    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0, 1], [1, 0]],
 *    gamma5 = g1 g2 g3 g4 = diag(1, 1, -1, -1).
 *  - Work is enqueued on the HIP stream given to sapq_create().  sapq_dslash,
 *    sapq_ssor, sapq_dk and sapq_sap_precondition are asynchronous; the solvers
 *    synchronise the stream for their convergence tests and return when done.
 *  - Every call returns a sapq_status.  On SAPQ_EINVAL / SAPQ_ESHAPE outputs are
 *    untouched; sapq_last_error() gives a message (thread-local, host string).
 *  - A context is not thread-safe; separate contexts are independent.
 */
#ifndef SAPQ_H
#define SAPQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sapq_ctx sapq_ctx;

typedef enum {
    SAPQ_OK = 0,
    SAPQ_EINVAL = -1,     /* bad argument (null pointer, bad enum, bad parameter) */
    SAPQ_ESHAPE = -2,     /* geometry not allowed, see sapq_geom */
    SAPQ_ENOTSU3 = -3,    /* links are not SU(3) to 1e-10 (2-row storage needs det U = 1) */
    SAPQ_ENOTCONV = -4,   /* solver stopped at maxit; best iterate and stats returned */
    SAPQ_EBREAKDOWN = -5, /* BiCGStab breakdown that restarts could not cure */
    SAPQ_EHIP = -6,       /* a HIP runtime call failed */
    SAPQ_ENOMEM = -7,     /* the arena is smaller than sapq_arena_bytes() */
    SAPQ_ESTATE = -8      /* fields not loaded yet */
} sapq_status;

/* storage precision of the SAP preconditioner and inner solver vectors/fields;
 * arithmetic is FP32 for FP32/FP16/BF16 storage and FP64 for FP64. */
typedef enum { SAPQ_FP64 = 0, SAPQ_FP32 = 1, SAPQ_FP16 = 2, SAPQ_BF16 = 3 } sapq_prec;

/* outer iteration (section 2 of the paper: flexible outer BiCGStab around the inner solver) */
typedef enum { SAPQ_OUTER_FBICGSTAB = 0, SAPQ_OUTER_DEFECT = 1 } sapq_outer;

/*
 * Geometry.  L: lattice extents (x,y,z,t).  block: SAP block extents; the blocks
 * are coloured like a checkerboard, E = colour 0 holds the origin (eq. 2.3).
 * subblock: sub-block extents of the locally-lexicographic ordering (section 3), or
 * {0, 0, 0, 0} for the even-odd site ordering that section 3 compares it against: the
 * sites of a block with an even sum of block-local coordinates first, then the odd ones
 * (the SSOR then has two hyperplanes, the two parities).
 * bc_sign: +1 periodic, -1 antiperiodic fermion boundary per direction; the sign
 * multiplies the hops that cross the lattice boundary.
 * Constraints (else SAPQ_ESHAPE): block[mu] divides L[mu] and L[mu]/block[mu] is
 * even and >= 2 (so neighbouring blocks always have opposite colours);
 * unless all are 0, subblock[mu] divides block[mu] and is >= 2 (so sites at the same sub-block-local
 * position never couple); at most 1024 sites in one hyperplane of a block.
 */
typedef struct {
    int L[4];
    int block[4];
    int subblock[4];
    int bc_sign[4];
} sapq_geom;

/*
 * Parameters (else SAPQ_EINVAL).  kappa: hopping parameter of D (eq. 2.2), > 0.  omega:
 * SSOR relaxation, 0 < omega < 2;
 * n_ssor: symmetric (forward + backward) SSOR sweeps from x = 0 per block inverse;
 * n_sap: N_SAP of eq. (2.4).  tol_inner / maxit_inner: relative residual target and
 * iteration cap of the inner BiCGStab.  maxit_outer: outer iteration cap.
 * prec_inner: storage precision of SAP + inner solver (SAPQ_FP32, _FP16, _BF16).
 * outer: sapq_outer.  flags: SAPQ_FLAG_* below.
 */
typedef struct {
    double kappa, omega, tol_inner;
    int n_ssor, n_sap, maxit_inner, maxit_outer;
    int prec_inner;
    int outer;
    int flags;
} sapq_params;

#define SAPQ_FLAG_GUESS 1   /* sapq_solve starts from the x passed in */
#define SAPQ_FLAG_PROFILE 2 /* sapq_solve times its kernels with HIP events (see sapq_stats) */
#define SAPQ_FLAG_NN 4      /* reserve the learned stage (at sapq_create) and use it in the inner
                               solver once weights are set (see sapq_nn_*) */
#define SAPQ_FLAG_NN_FP32 8 /* learned-stage layers in FP32 FMAs instead of BF16 MFMA */
/* Block inverses A_EE, A_OO by the even-odd site-preconditioned block solve that section 3
 * measures the SSOR against, instead of the SSOR: inside a block, the system reduced to the
 * even sites, (1 - K_eo K_oe) x_e = v_e + K_eo v_o with K = kappa F H in the block, gets
 * 2 n_ssor minimal-residual steps from 0 (the cost of n_ssor symmetric SSOR sweeps), then
 * x_o = v_o + K_oe x_e.  Needs the even-odd site order (subblock {0, 0, 0, 0}), an even
 * number of sites per block and a block whose vector fits one workgroup's LDS (96 bytes per
 * site: at most 1700 sites in gfx950's 160 KiB) (sapq_create: SAPQ_ESHAPE; sapq_set_params:
 * SAPQ_EINVAL).  omega is unused.  sapq_autotune and sapq_solve_batch refuse such a context
 * (SAPQ_EINVAL). */
#define SAPQ_FLAG_EOMR 16
/* Reserve FP32 copies of the fields (at sapq_create; an FP16/BF16 context only, else ignored)
 * so that sapq_solve can fall back to FP32 storage when an inner solve in FP16/BF16 storage
 * breaks down (see sapq_solve).  Costs 480 bytes per site of fields and widens the inner work
 * vectors to FP32. */
#define SAPQ_FLAG_FALLBACK_FP32 32

/* Per-solve statistics (host struct). */
typedef struct {
    int outer_its;       /* outer iterations (each applies the inner solver once or twice) */
    int inner_its;       /* inner BiCGStab iterations summed over the solve */
    int n_msap;          /* M_SAP applications */
    int n_dslash64;      /* FP64 operator applications */
    int restarts;        /* true-residual restarts of the outer iteration */
    int n_hist;          /* entries in relres_hist */
    double true_relres;  /* |b - D x| / |b| in FP64 at exit */
    double time_s;       /* wall time of the solve on the host clock */
    /* with params.flags & SAPQ_FLAG_PROFILE: HIP-event time (ms) summed per kernel kind
     * and launches per kind, measured on the context's stream during the solve.
     * kinds: SAPQ_K_PHASE_E, SAPQ_K_PHASE_O, SAPQ_K_FACE, SAPQ_K_DSLASH64, SAPQ_K_BLAS */
    double kern_ms[8];
    int kern_n[8];
    double relres_hist[256];
    int breakdowns;      /* inner solves that broke down (a non-finite scalar) and were redone */
    int fallback;        /* SAPQ_FALLBACK_* taken during the solve (bit mask) */
} sapq_stats;

/* sapq_stats.fallback bits */
#define SAPQ_FALLBACK_NN 1   /* the learned stage was dropped: plain M_SAP for the rest of the solve */
#define SAPQ_FALLBACK_FP32 2 /* FP16/BF16 storage was replaced by FP32 for the rest of the solve */

enum { SAPQ_K_PHASE_E = 0, SAPQ_K_PHASE_O = 1, SAPQ_K_FACE = 2, SAPQ_K_DSLASH64 = 3, SAPQ_K_BLAS = 4 };

/* Bytes of device arena a context needs (host call; 0 on a bad geometry). */
size_t sapq_arena_bytes(const sapq_geom *geom, const sapq_params *params);

/*
 * Create a context.  arena: device memory of >= sapq_arena_bytes() bytes, 256-byte
 * aligned, owned by the caller.  stream: hipStream_t (NULL = default stream).
 * Builds the block/sub-block/hyperplane tables on the device.
 * Environment switches read here (all optional; for study and testing only):
 *   SAPQ_PARTS=0|1|2        0: four-lane SAP kernels; 1 / 2: one / two workgroups per block
 *                           for the two-lane phase kernel wherever they fit (default: choose).
 *   SAPQ_SSOR_THREADS=n     cap on the four-lane kernels' workgroup size (64..1024; default 512).
 *   SAPQ_NO_STAGING=1       four-lane kernels keep the block's links in HBM instead of LDS.
 *   SAPQ_HALO_TIMEOUT_TEST=1  every halo wait of a split block times out after 64 polls,
 *                           so that the SAPQ_EHIP path can be tested.
 *   SAPQ_TEST_LOWPREC_NAN=1 every inner solve in FP16/BF16 storage gets a NaN scale for its
 *                           right-hand side, so that the breakdown and FP32 fallback paths of
 *                           sapq_solve can be tested (FP32 storage is left alone).
 * sapq_solve_batch reads SAPQ_BATCH_NR=1..4 (sources per workgroup; default 1).
 */
int sapq_create(const sapq_geom *geom, const sapq_params *params, void *arena, size_t arena_bytes,
                void *stream, sapq_ctx **out);

/* Change kappa, omega, n_ssor, n_sap, tolerances or outer kind (not prec_inner). */
int sapq_set_params(sapq_ctx *ctx, const sapq_params *params);

/*
 * Load the gauge field U (links layout above).  Stores rows 0 and 1 of every link
 * (row 2 is rebuilt as conj(row0 x row1), section 3 "SIMDzation") in FP64 and in the
 * inner storage precision.  Returns SAPQ_ENOTSU3 if max |U^+ U - 1| or |det U - 1|
 * exceeds 1e-10; *max_dev (host, nullable) receives that maximum.
 */
int sapq_load_gauge(sapq_ctx *ctx, const double *U, double *max_dev);

/* Load the inverse clover field F of eq. (2.2) (clover layout above; hermitian blocks). */
int sapq_load_clover_inv(sapq_ctx *ctx, const double *F);

/*
 * out = D in, eq. (2.2): D = 1 - kappa F(n) sum_mu [(1-gamma_mu) U_mu(n) delta(n+mu,m)
 * + (1+gamma_mu) U_mu(n-mu)^+ delta(n-mu,m)].  prec: SAPQ_FP64 computes in FP64, otherwise
 * the fields and vectors are held in that storage precision with FP32 arithmetic.
 * in, out: spinor layout; may not alias.
 */
int sapq_dslash(sapq_ctx *ctx, double *out, const double *in, int prec);

/*
 * Measurement: the operator kernel of sapq_dslash alone (without the layout conversions),
 * applied reps >= 1 times to in (packed once into the context's internal work vectors) between
 * two HIP events on the context's stream, after one untimed application; *avg_us (host)
 * receives the mean time per application in microseconds.  prec as for sapq_dslash.  Synchronises.
 */
int sapq_time_dslash(sapq_ctx *ctx, const double *in, int prec, int reps, double *avg_us);

/*
 * For callers that cannot allocate device memory at call time (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): out = D in exactly as sapq_dslash
 * computes it, but its two staging vectors (the operand and the result in the internal layout)
 * live in a static device array of the library, 256 MiB per GPU, held until the process ends,
 * instead of the context's arena.  Needs 2 x 12 V x (16 bytes for SAPQ_FP64, 8 for FP32, 4 for
 * FP16/BF16) rounded up to 256-byte vectors, at most 256 MiB (FP64: V <= 699,050 sites, e.g.
 * 24^3x48); a larger lattice is refused with SAPQ_ENOMEM before any work.  Allocates nothing
 * (no hipMalloc, hipFree or allocating library call).  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (several streams or threads) race.  in, out, prec and
 * errors as for sapq_dslash; asynchronous on the context's stream.
 */
int sapq_dslash_noalloc(sapq_ctx *ctx, double *out, const double *in, int prec);

/*
 * x = A_cc v: the SSOR approximate inverse of the block operator on every block of
 * colour `colour` (0 = E, 1 = O), section 3 "Inverse of block operator": from x = 0,
 * n_ssor forward+backward substitution sweeps in locally-lexicographic order (with
 * SAPQ_FLAG_EOMR: the even-odd minimal-residual block solve instead).  Runs in the inner
 * precision.  Sites of the other colour get x = 0.
 */
int sapq_ssor(sapq_ctx *ctx, double *x, const double *v, int colour);

/* (x, w) = (K v, D K v) by Algorithm 1 (K of eq. 2.4), in the inner precision. */
int sapq_dk(sapq_ctx *ctx, double *x, double *w, const double *v);

/*
 * out = M_SAP in, eq. (2.4): N_SAP cycles of r <- r - D K r, out = sum of the K r;
 * d_out (nullable) = D M_SAP in, which the recurrence yields as in - r_N.  Inner precision.
 */
int sapq_sap_precondition(sapq_ctx *ctx, double *out, double *d_out, const double *in);

/*
 * out = P in for the inner solver's preconditioner P: M_SAP, or, with the learned stage on
 * (SAPQ_FLAG_NN and weights set), P = N + M_SAP (1 - D N); d_out (nullable) = D P in, which
 * the SAP recurrence yields without another operator application.  Inner precision.
 */
int sapq_precondition(sapq_ctx *ctx, double *out, double *d_out, const double *in);

/*
 * e ~ D^-1 r by the inner BiCGStab right-preconditioned with M_SAP (section 2), from
 * e = 0, to |r - D e| <= tol_inner |r| (recursive residual) or maxit_inner iterations.
 * *iters (host, nullable) receives the iteration count.  Inner precision.
 */
int sapq_inner_solve(sapq_ctx *ctx, double *e, const double *r, int *iters);

/*
 * Solve D x = b to |b - D x|_2 / |b|_2 <= tol (true residual in FP64), section 2: the
 * outer FP64 flexible BiCGStab (or defect correction) whose preconditioner is the inner
 * low-precision BiCGStab with M_SAP.  x: initial guess if params.flags & SAPQ_FLAG_GUESS,
 * solution on return.  stats (host, nullable).  SAPQ_ENOTCONV leaves the best iterate.
 * b = 0 gives x = 0 at once.
 * Failure handling: every scalar the iterations read back is checked.  An inner solve that
 * meets a non-finite scalar is redone on the same input with a more robust preconditioner,
 * which the flexible outer iteration allows (its preconditioner may change from one call to
 * the next): first without the learned stage (plain M_SAP), then, for a context created with
 * SAPQ_FLAG_FALLBACK_FP32, with FP32 storage; the change holds until the solve returns
 * (stats->fallback, stats->breakdowns).  With nothing left to fall back to, or a source or an
 * outer scalar that is not finite, the solve returns SAPQ_EBREAKDOWN with the last finite
 * iterate in x.
 */
int sapq_solve(sapq_ctx *ctx, double *x, const double *b, double tol, sapq_stats *stats);

/*
 * Batched solve: nctx contexts (one gauge field each; any lattice sizes, but one SAP block and
 * sub-block shape and one prec_inner), with nrhs[i] right-hand sides for context i.  b[i] and x[i]
 * are device arrays of nrhs[i] spinors in the spinor layout ([nrhs[i]][V_i][4][3]).  All fields and
 * right-hand sides advance together: the outer iteration is FP64 defect correction
 * (x += Inner(b - D x), true residual per right-hand side), and each SAP phase is one kernel
 * launch over all fields, blocks and groups of right-hand sides, the links and clover rows of a
 * site being loaded once per group.  The whole iteration runs on the device as two hipGraphs:
 * the outer step (apply the inner solve, true residual, per-source status and scale, a fresh
 * inner solve) and K inner iterations; the host reads one count of running sources per replay.
 * Krylov scalars and convergence flags are per right-hand side, on the device; finished ones are
 * masked.  The graphs, the batch's stream and a pinned host buffer are kept (per device) and a
 * later call on the same batch replays them.  A non-finite source, residual or inner scalar
 * stops that right-hand side at its last finite iterate (stats.breakdowns = 1) and the call
 * returns SAPQ_EBREAKDOWN.  When every context has the
 * learned stage on (weights set, params.flags & SAPQ_FLAG_NN), the inner preconditioner is
 * z = N r + M_SAP (r - D N r) for each right-hand side, the network applied per right-hand side
 * on its context and the SAP phases batched.  The arena size depends on that setting: size it
 * after setting the flags.  Parameters (kappa, n_ssor, n_sap,
 * tol_inner, maxit_*) are each context's; the stream is ctxs[0]'s.  arena: device memory of at
 * least sapq_batch_arena_bytes() bytes, 256-byte aligned.  stats (host, nullable): one entry per
 * right-hand side, contexts in order.  Returns SAPQ_ENOTCONV if any right-hand side missed tol.
 */
size_t sapq_batch_arena_bytes(sapq_ctx *const *ctxs, int nctx, const int *nrhs);
int sapq_solve_batch(sapq_ctx *const *ctxs, int nctx, const int *nrhs, double *const *x, const double *const *b,
                     double tol, void *arena, size_t arena_bytes, sapq_stats *stats);

/*
 * Autotune the batched solver's kernel choices for one batch (arguments as sapq_solve_batch):
 * right-hand sides per workgroup of the SAP phase kernel, NR in 1..4 (where the LDS and the
 * workgroup size allow), and inner BiCGStab iterations per graph replay between two host
 * checks, K in {1, 2, 4}.  Every candidate times three batched solves of the given sources to
 * tol and keeps the median; the fastest pair is stored in every context, where later
 * sapq_solve_batch calls use it, and returned in *nr_out, *k_out (host, nullable).  x holds
 * the last solve's solutions.  cache_json_path (host, nullable): JSON lines keyed by the
 * lattices, right-hand-side counts, block, sub-block, prec_inner and learned stage; a hit skips
 * the timing, a miss appends the result with every timed candidate's median
 * ("candidates": [[nr, k, seconds], ...]).  SAPQ_ENOTCONV if no candidate reaches tol.
 * The sub-block shape is sapq_autotune's (per context); the environment switch SAPQ_BATCH_NR,
 * when set, overrides NR.
 */
int sapq_autotune_batch(sapq_ctx *const *ctxs, int nctx, const int *nrhs, double *const *x, const double *const *b,
                        double tol, void *arena, size_t arena_bytes, const char *cache_json_path, int *nr_out,
                        int *k_out);

/*
 * Autotune the sub-block shape of a context: every sub-block shape whose extents are 2 or more
 * and divide the block, and the even-odd site order {0, 0, 0, 0} where the context's phase
 * kernel takes it, is timed on three solves of the point source at the origin (spin 0,
 * colour 0) to 1e-10, and the one with the fastest median is kept (the ordering, hence the
 * preconditioner, changes with it).  The phase kernel's workgroup size is not a free choice:
 * two lanes per site of the widest hyperplane.
 * cache_json_path (host, nullable): a JSON file of earlier choices, keyed by lattice, block,
 * kappa and prec_inner; a hit skips the timing, a miss appends the result.  *subblock_out
 * (host, nullable, 4 ints) receives the choice.
 */
int sapq_autotune(sapq_ctx *ctx, const char *cache_json_path, int *subblock_out);

/*
 * Learned gauge-covariant preconditioner stage (not in the paper; an extension of its
 * inner preconditioner).  N is three linear parallel-transport convolution layers with
 * channels 1 -> SAPQ_NN_CHANNELS -> SAPQ_NN_CHANNELS -> 1; a layer maps c_in spinor
 * channels to c_out as
 *     out[c'](n) = sum_{d=0..8} sum_c W[d][c'][c] (T_d in[c])(n)
 * with W[d][c'][c] a 4x4 complex spin matrix, T_0 = 1, T_{1+2mu} psi(n) = U_mu(n) psi(n+mu),
 * T_{2+2mu} psi(n) = U_mu(n-mu)^+ psi(n-mu) (boundary signs as in D).  With the stage on, the
 * inner solver's preconditioner becomes z = N r + M_SAP (r - D N r), which is linear in r,
 * so the inner BiCGStab still sees a fixed operator, and plain SAP is the fallback.
 * Weight blob: sapq_nn_param_count() floats, layer after layer, W[9][c_out][c_in][4][4]
 * complex as (re, im) pairs.  The weights are used rounded to BF16 (Adam keeps FP32 master
 * weights).  By default a layer's spin/channel mixing is a BF16 MFMA contraction with FP32
 * accumulation over BF16-rounded transported inputs; with SAPQ_FLAG_NN_FP32 the layers use
 * FP32 FMAs on FP32 inputs instead.  All sapq_nn_* calls need a context created with
 * params.flags & SAPQ_FLAG_NN (else SAPQ_ESTATE); training needs prec_inner = SAPQ_FP32.
 */
#define SAPQ_NN_CHANNELS 8
size_t sapq_nn_param_count(void);

/* Set the weights (device float array) and reset the Adam moments; enables the stage. */
int sapq_nn_set_weights(sapq_ctx *ctx, const float *w);

/* Copy the FP32 master weights out (device float array). */
int sapq_nn_get_weights(sapq_ctx *ctx, float *w);

/* Copy the training state of src (FP32 master weights and both Adam moments) into dst, so
 * that training can go on with dst's field without restarting Adam; enables the stage in dst.
 * Both contexts need SAPQ_FLAG_NN and set weights in src (else SAPQ_ESTATE) and must be on
 * one device.  src's stream is synchronized first; the copy runs on dst's stream. */
int sapq_nn_copy_state(sapq_ctx *dst, sapq_ctx *src);

/* out = N in (spinor layout, FP64 at the boundary, FP32 inside). */
int sapq_nn_forward(sapq_ctx *ctx, double *out, const double *in);

/*
 * Gradients of a real loss L(N in) given grad_out = dL/dRe z + i dL/dIm z at z = N in:
 * grad_w (device float, sapq_nn_param_count()) = dL/dRe W + i dL/dIm W in the blob layout,
 * grad_in (nullable) = N^+ grad_out.
 */
int sapq_nn_backward(sapq_ctx *ctx, float *grad_w, double *grad_in, const double *grad_out, const double *in);

/*
 * One Adam step (lr, step count t >= 1) on the mean over a batch of the loss
 * |N(D e) - e|^2 / |e|^2.  e: device float array of n_vec error vectors, each in the spinor
 * layout as (re, im) float pairs ([n_vec][V][4][3][2]); idx (host): the batch's batch indices
 * into it.  The residual r = D e is formed on the device in FP32.  *loss (host, nullable):
 * the batch mean before the step.
 */
int sapq_nn_train_step(sapq_ctx *ctx, const float *e, long n_vec, const int *idx, int batch, float lr, int t,
                       double *loss);

/*
 * One Adam step (Kingma and Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the FP32
 * master weights with the gradient grad_w that the caller supplies (device float,
 * sapq_nn_param_count() entries in the weight-blob layout, e.g. from sapq_nn_backward), learning
 * rate lr > 0 and step count t >= 1; the BF16-rounded weights the layers use are refreshed.
 * The moments live in the context (reset by sapq_nn_set_weights, carried by
 * sapq_nn_copy_state).  Needs set weights (else SAPQ_ESTATE).
 */
int sapq_nn_adam_step(sapq_ctx *ctx, const float *grad_w, float lr, int t);

/*
 * Residual -> error training pairs from the plain SAP solver (the learned stage's training
 * data).  From x_0 = 0, the defect-correction iterates x_{k+1} = x_k + Inner(b - D x_k) of
 * section 2's outer iteration (this context's inner solver, learned stage off) give
 * e_k = xstar - x_k for k = 0 .. n_iter - 1, written to e (device float, [n_iter][V][4][3]
 * as (re, im) pairs, the layout sapq_nn_train_step reads; when xstar solves D x = b, the
 * residual of the pair is r_k = b - D x_k = D e_k).  b, xstar: spinor layout, FP64.  Returns
 * SAPQ_EBREAKDOWN (the remaining e_k unwritten) if an inner solve breaks down.
 */
int sapq_defect_errors(sapq_ctx *ctx, float *e, const double *b, const double *xstar, int n_iter);

/*
 * The SAP phase kernel a context runs, chosen at creation from the block and the device's
 * LDS: 0 four lanes per site and one workgroup per block (the SSOR iterate in LDS, or in a
 * global scratch when it does not fit); 1 two lanes per site (forward / backward hops), one
 * workgroup per block, iterate in LDS; 2 two lanes per site with the block split along t into
 * two workgroups that exchange their boundary layers.  -1 for a null context.
 */
int sapq_phase_kernel(const sapq_ctx *ctx);

/* Release the context (host memory only; the arena stays the caller's). */
void sapq_destroy(sapq_ctx *ctx);

/* Message for the last non-OK return on this thread (host string, never NULL). */
const char *sapq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SAPQ_H */
