// Internal declarations of libsapq: context, device geometry tables, storage
// types and the per-site device building blocks shared by the kernels.
//
// Internal layouts (all structure-of-arrays so that a wavefront touches
// consecutive addresses):
//   site      (ib, s): block ib (E blocks first, then O blocks) and slot s inside
//             the block; slots are sorted by hyperplane h = sum_mu (x_mu mod S_mu),
//             so every hyperplane is a contiguous slot range.
//   spinor    [ib][12][Vb]       complex, component 3*alpha + a
//   links     [ib][4][6][Vb]     rows 0 and 1 of U_mu(n) (row 2 = conj(row0 x row1))
//   clover    [ib][2][18][Vb]    per chiral block: 3 complex slots holding the 6 real
//                                diagonal entries pairwise, then the 15 entries below
//                                the diagonal row by row; F is hermitian
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sapq.h"
#include "tables.h"

namespace sapq {


// ---------------------------------------------------------------- device geometry
struct GeomDev {
    int Vb;           // sites per block
    int NB;           // blocks
    int NBc;          // blocks per colour
    long V;           // sites
    int nplanes;      // hyperplanes per block
    float bc[4];      // boundary sign per direction
    const int *loc_nbr;     // [8][Vb]: >= 0 slot inside the block, else -1 - slot in the next block
    const unsigned *nbr16;  // [4][Vb]: forward | backward << 16 slots of direction mu, bit 15/31 = inside
    const int *blk_nbr;     // [8][NB]: neighbouring block id | WRAP_BIT
    const int *plane_start; // [nplanes + 1]
    const int *slot_lex;    // [Vb] block-local lexicographic index of each slot
    const int *blk_lex;     // [NB] lexicographic block index of each internal block id
    const int *lex_blk;     // [NB] internal block id of each lexicographic block index
    const int *zord_blk;    // [NB] internal block ids in Z (Morton) order of the block coordinates
    int B[4];
    int nbk[4];             // blocks per direction
};

// ---------------------------------------------------------------- storage precisions
template <int P> struct Prec;
template <> struct Prec<SAPQ_FP64> { using S2 = double2; using C = double; };
template <> struct Prec<SAPQ_FP32> { using S2 = float2; using C = float; };
template <> struct Prec<SAPQ_FP16> { using S2 = __half2; using C = float; };
template <> struct Prec<SAPQ_BF16> { using S2 = __hip_bfloat162; using C = float; };

template <typename T> struct cx { T r, i; };

template <typename T> __device__ __forceinline__ cx<T> cxz() { return {T(0), T(0)}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <typename T> __device__ __forceinline__ cx<T> conjx(cx<T> a) { return {a.r, -a.i}; }
template <typename T> __device__ __forceinline__ cx<T> itimes(cx<T> a) { return {-a.i, a.r}; }

// Fused forms for the site kernels: every product is added into its accumulator by a fused
// multiply-add (two per real component of a complex product, one of a real one), instead of
// being rounded and added separately.
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }

// complex products, with the fused multiply-add spelled out: left to contraction, which of
// the two products of a component gets fused would depend on the instruction order around
// it, and so would the rounding
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {fmx(a.r, b.r, -(a.i * b.i)), fmx(a.r, b.i, a.i * b.r)};
}
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // conj(a) * b
    return {fmx(a.r, b.r, a.i * b.i), fmx(a.r, b.i, -(a.i * b.r))};
}
template <typename T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {  // acc + a b
    return {fmx(-a.i, b.i, fmx(a.r, b.r, acc.r)), fmx(a.i, b.r, fmx(a.r, b.i, acc.i))};
}
template <typename T> __device__ __forceinline__ cx<T> cfmac(cx<T> a, cx<T> b, cx<T> acc) {  // acc + conj(a) b
    return {fmx(a.i, b.i, fmx(a.r, b.r, acc.r)), fmx(-a.i, b.r, fmx(a.r, b.i, acc.i))};
}
template <typename T> __device__ __forceinline__ cx<T> rfma(T s, cx<T> a, cx<T> acc) {  // acc + s a, s real
    return {fmx(s, a.r, acc.r), fmx(s, a.i, acc.i)};
}
// row 2 of an SU(3) link from rows 0 and 1: conj(row0 x row1)
template <typename T> __device__ __forceinline__ void su3_row2(cx<T> u[9]) {
    const cx<T> m1 = {-u[1].r, -u[1].i}, m2 = {-u[2].r, -u[2].i}, m0 = {-u[0].r, -u[0].i};
    u[6] = conjx(cfma(m2, u[4], cmul(u[1], u[5])));
    u[7] = conjx(cfma(m0, u[5], cmul(u[2], u[3])));
    u[8] = conjx(cfma(m1, u[3], cmul(u[0], u[4])));
}

// storage <-> compute
__device__ __forceinline__ cx<double> ld(const double2 *p) { double2 v = *p; return {v.x, v.y}; }
__device__ __forceinline__ cx<float> ld(const float2 *p) { float2 v = *p; return {v.x, v.y}; }
__device__ __forceinline__ cx<float> ld(const __half2 *p) { float2 v = __half22float2(*p); return {v.x, v.y}; }
__device__ __forceinline__ cx<float> ld(const __hip_bfloat162 *p) {
    __hip_bfloat162 h = *p;
    return {__bfloat162float(h.x), __bfloat162float(h.y)};
}
__device__ __forceinline__ void st(double2 *p, cx<double> v) { *p = make_double2(v.r, v.i); }
__device__ __forceinline__ void st(float2 *p, cx<float> v) { *p = make_float2(v.r, v.i); }
__device__ __forceinline__ void st(__half2 *p, cx<float> v) { *p = __floats2half2_rn(v.r, v.i); }
__device__ __forceinline__ void st(__hip_bfloat162 *p, cx<float> v) {
    __hip_bfloat162 h;
    h.x = __float2bfloat16(v.r);
    h.y = __float2bfloat16(v.i);
    *p = h;
}

// ---------------------------------------------------------------- spinor / link access
template <typename S2>
__device__ __forceinline__ const S2 *spin_at(const S2 *f, const GeomDev &g, int ib, int s) {
    return f + (size_t)ib * 12 * g.Vb + s;
}
template <typename S2, typename C>
__device__ __forceinline__ void load_spinor(cx<C> psi[12], const S2 *f, const GeomDev &g, int ib, int s) {
    const S2 *p = spin_at(f, g, ib, s);
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = ld(p + (size_t)c * g.Vb);
}
template <typename S2, typename C>
__device__ __forceinline__ void store_spinor(S2 *f, const GeomDev &g, int ib, int s, const cx<C> psi[12]) {
    S2 *p = f + (size_t)ib * 12 * g.Vb + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) st(p + (size_t)c * g.Vb, psi[c]);
}

// link U_mu at (ib, s) rebuilt to 3x3 (row-major u[3*a+b])
template <typename S2, typename C>
__device__ __forceinline__ void load_link(cx<C> u[9], const S2 *U, const GeomDev &g, int ib, int s, int mu) {
    const S2 *p = U + ((size_t)ib * 4 + mu) * 6 * g.Vb + s;
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = ld(p + (size_t)e * g.Vb);
    su3_row2(u);
}

// out = U h (dag = false) or U^+ h (dag = true) for a colour 3-vector
template <typename C>
__device__ __forceinline__ void su3_mul(cx<C> out[3], const cx<C> u[9], const cx<C> h[3], bool dag) {
    if (!dag) {
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = cfma(u[3 * a + 2], h[2], cfma(u[3 * a + 1], h[1], cmul(u[3 * a], h[0])));
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a] = cfmac(u[6 + a], h[2], cfmac(u[3 + a], h[1], cmulc(u[a], h[0])));
    }
}

// ---------------------------------------------------------------- host dispatch on the storage precision
#define PREC_SWITCH(prec, BODY)                                   \
    switch (prec) {                                               \
    case SAPQ_FP64: { constexpr int P_ = SAPQ_FP64; BODY; } break; \
    case SAPQ_FP32: { constexpr int P_ = SAPQ_FP32; BODY; } break; \
    case SAPQ_FP16: { constexpr int P_ = SAPQ_FP16; BODY; } break; \
    case SAPQ_BF16: { constexpr int P_ = SAPQ_BF16; BODY; } break; \
    default: break;                                               \
    }

#define INNER_SWITCH(prec, BODY)                                  \
    switch (prec) {                                               \
    case SAPQ_FP32: { constexpr int P_ = SAPQ_FP32; BODY; } break; \
    case SAPQ_FP16: { constexpr int P_ = SAPQ_FP16; BODY; } break; \
    case SAPQ_BF16: { constexpr int P_ = SAPQ_BF16; BODY; } break; \
    default: break;                                               \
    }

// ---------------------------------------------------------------- context
struct Ctx;

// kernel launchers (defined in the .hip files)
void launch_pack_spinor(Ctx *c, int prec, void *dst, const double *src, double scale);
void launch_unpack_spinor(Ctx *c, int prec, double *dst, const void *src, double scale);
int launch_pack_links(Ctx *c, const double *U, double *max_dev);
void launch_pack_clover(Ctx *c, const double *F);
bool launch_permute_fields(Ctx *c, const int *perm);
void launch_dslash(Ctx *c, int prec, void *out, const void *in);
void launch_sap_phase(Ctx *c, int colour, bool first, const void *rsrc, void *r, void *x, void *y);
void launch_sap_face(Ctx *c, int colour, void *r, const void *x);
void launch_sap_phase_parts(Ctx *c, int colour, int gather, int first, int ssor_only, const void *rsrc, void *r,
                            void *x, void *y);
int set_parts_lds_limit(Ctx *c);
// the even-odd minimal-residual block solve (SAPQ_FLAG_EOMR) in place of the SSOR
bool eomr_supported(const Ctx *c, std::string &why);
void launch_sap_phase_eomr(Ctx *c, int colour, int gather, int first, int ssor_only, const void *rsrc, void *r,
                           void *x, void *y);
int set_eomr_lds_limit(Ctx *c);
void launch_sap_face_2l(Ctx *c, int colour, void *r, const void *x);
void launch_ssor_only(Ctx *c, int colour, const void *v, void *x);

// BLAS-1 on internal vectors (n = 12 V complex entries)
void blas_dots(Ctx *c, int prec, int ndot, const void *const *a, const void *const *b, double2 *host_out);
void blas_copy(Ctx *c, int prec, void *dst, const void *src);
void blas_zero(Ctx *c, int prec, void *dst);
// z = x + a*y  (complex a)
void blas_xpay(Ctx *c, int prec, void *z, const void *x, double2 a, const void *y);
// z = x + a y and, in the same pass, out[0] = <w, z> (w not null), out[1] = <z, z> (zz),
// out[2] = <z, x> (zx), read back to the host (synchronizes the stream)
void blas_xpay_dots(Ctx *c, int prec, void *z, const void *x, double2 a, const void *y, const void *w, int zz, int zx,
                    double2 out[3]);
// p = r + beta*(p - om*v)
void blas_bicg_p(Ctx *c, int prec, void *p, const void *r, double2 beta, double2 om, const void *v);
// e += a*ph + b*sh
void blas_axpbypz(Ctx *c, int prec, void *e, double2 a, const void *ph, double2 b, const void *sh);
// dst (prec_d) = scale * src (prec_s)
void blas_convert(Ctx *c, int prec_d, void *dst, int prec_s, const void *src, double scale);

// HIP-event timing of kernel launches, harvested at the host synchronisation points
struct Prof {
    bool on = false;
    std::vector<hipEvent_t> ev;      // pairs
    std::vector<int> kind;           // kind of each recorded pair
    int used = 0;
    double ms[8] = {0};
    int n[8] = {0};
};

struct Ctx {
    sapq_geom geom;
    sapq_params prm;
    hipStream_t stream;
    int device = 0;  // the device current at creation (the arena's)
    // identity for the batched solver's graph cache: a number unique to the context and a
    // count of the changes that alter what a captured graph launches (sub-block shape,
    // parameters, learned stage)
    unsigned long long serial = 0, version = 0;
    // the batched solver's kernel choices from sapq_autotune_batch (0: default)
    int batch_nr = 0, batch_k = 0;
    GeomDev g;
    int max_plane;
    int ssor_threads;
    bool ssor_lds;
    size_t lds_bytes;   // SSOR iterate in LDS
    size_t lds_extra;   // neighbour words and plane starts in LDS
    bool ssor_staged;   // links and clover field of a block staged in LDS as well
    size_t staged_bytes;
    // two-lanes-per-site phase kernel, the block split along t into sap_np workgroups
    bool use_parts = false;
    int sap_np = 1, part_Vp = 0, part_Hp = 0, part_threads = 512;
    size_t parts_lds = 0;
    bool parts_staged = false;  // phase kernel in the staged load order (one workgroup per CU by LDS)
    int *part_gslot, *part_pstart, *part_exp, *part_imp, *part_imps;
    uint2 *part_nb, *part_gnb;
    unsigned long long *xch;  // tagged halo words exchanged between the two workgroups of a block
    unsigned *xsync;          // ticket, done, epoch, error
    long V;
    size_t nvec;  // 12 V complex entries
    // fields
    double2 *U64, *F64;
    int *slot_perm;   // [Vb] staging of a slot re-ordering (sub-block change)
    int halo_spin_limit = 1 << 20;  // polls of a split block's bounded wait on a halo word
    unsigned halo_wait_xor = 0;     // nonzero: every such wait times out (failure-path tests)
    void *Uin, *Fin;  // inner storage precision
    bool have_U, have_F;
    // failure handling (sapq_solve): FP32 copies of the fields that an FP16/BF16 context can
    // fall back to (SAPQ_FLAG_FALLBACK_FP32), the fields of the creation precision while it
    // has, and the state of the current solve
    int prec_created = SAPQ_FP32;
    bool fb_fp32 = false;
    void *Uin32 = nullptr, *Fin32 = nullptr, *Uin_lp = nullptr, *Fin_lp = nullptr;
    bool nn_suspended = false;   // learned stage dropped for the rest of the solve
    int fallback = 0, breakdowns = 0;
    bool poison_lowprec = false; // SAPQ_TEST_LOWPREC_NAN: NaN-scaled inner solves in FP16/BF16
    // FP64 work vectors (internal layout)
    double2 *d_b, *d_x, *d_r, *d_rt, *d_p, *d_v, *d_s, *d_t, *d_ph, *d_sh, *d_tmp;
    // inner-precision work vectors
    void *i_r, *i_rt, *i_p, *i_v, *i_s, *i_t, *i_e, *i_ph, *i_sh, *i_rin, *i_tmp;
    // SAP state
    void *sap_r, *sap_x;
    float2 *ssor_scratch;  // SSOR iterate when the block does not fit LDS
    // reductions
    double2 *partials, *dev_res;
    double2 *host_res;  // pinned host
    double *dev_dev;    // unitarity deviation partials
    int red_blocks;
    // counters
    long n_msap, n_d64;
    Prof prof;
    // learned stage (allocated when params.flags & SAPQ_FLAG_NN)
    bool nn_alloc = false, have_nn = false;
    float *nn_w, *nn_wq, *nn_G, *nn_m, *nn_v;
    float2 *nn_wt;                       // adjoint weights of one layer
    float2 *nn_a0, *nn_a1, *nn_a2, *nn_z; // layer inputs (1, 8, 8 channels) and output
    float2 *nn_gz, *nn_g2, *nn_g1, *nn_gin, *nn_e;
    void *i_z, *i_rp;                    // N r and r - D N r in inner storage
    void *nn_afrag[3];                   // BF16 MFMA fragments of the three layers' weights
    void *nn_afrag_t;                    // fragments of an adjoint layer
    float2 *nn_L;                        // transport links [V][8][9] of the layers (FP32)
};

constexpr int NN_C = SAPQ_NN_CHANNELS;
constexpr int NN_PARAMS = 2 * 16 * 9 * (NN_C + NN_C * NN_C + NN_C);
constexpr int NN_OFF[3] = {0, 2 * 16 * 9 * NN_C, 2 * 16 * 9 * (NN_C + NN_C * NN_C)};  // floats
constexpr int NN_CIN[3] = {1, NN_C, NN_C};
constexpr int NN_COUT[3] = {NN_C, NN_C, 1};

void launch_nn_layer(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const float2 *W);
void launch_nn_wgrad(Ctx *c, int cin, int cout, const float2 *gout, const float2 *in, float2 *G, bool bf16_records);
void launch_nn_adjoint_weights(Ctx *c, int cin, int cout, const float2 *W, float2 *Wt);
void launch_nn_adam(Ctx *c, int n, float *w, const float *grad, float gscale, float *m, float *v, float lr, int t, float *wq);
void launch_nn_round(Ctx *c, int n, const float *w, float *wq);
size_t nn_afrag_elems(int cin, int cout);
size_t nn_link_elems(const Ctx *c);
void launch_nn_links(Ctx *c);
void launch_nn_afrag(Ctx *c, int cin, int cout, const float2 *W, void *A);
// p_in / p_out: storage precision of a one-channel input / output (spinor layout); skip:
// nullable device flag, nonzero leaves the output untouched
void launch_nn_layer_mfma(Ctx *c, int cin, int cout, const void *in, void *out, const void *A, int p_in, int p_out,
                          const int *skip);
void launch_pack_spinor_f32(Ctx *c, void *dst, const float *src);
void launch_unpack_spinor_f32(Ctx *c, float *dst, const double2 *src);
// learned stage on inner-precision vectors: z = N p, rp = p - D z
void nn_apply(Ctx *c, const void *p, void *z, void *rp, const int *skip = nullptr);

// bracket a launch with HIP events when profiling is on
int prof_begin(Ctx *c, int kind);
void prof_end(Ctx *c, int slot);
void prof_harvest(Ctx *c);

size_t elem_bytes(int prec);  // bytes of one stored complex
// the static scratch of sapq_dslash_noalloc: its device address on device dev (the current
// device), looked up once per device
int noalloc_scratch_init(int dev);
size_t noalloc_scratch_bytes();
void set_error(const std::string &msg);

}  // namespace sapq

struct sapq_ctx {
    sapq::Ctx c;
};
