/*
 * sapq_oracle.c -- plain FP64 CPU oracle for the clover-Wilson SAP/SSOR solver
 * of Boku et al., "Multi-block/multi-core SSOR preconditioner for the QCD quark
 * solver for K computer" (Lattice 2012, arXiv:1210.7398).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the GPU library; it is written for a reader who
 * checks it against the paper by eye, not for speed.
 *
 * Conventions (one chiral spin basis everywhere; where the paper is silent or
 * garbled, the reading taken is stated at the routine that depends on it):
 *   site      n = x + Lx*(y + Ly*(z + Lz*t)); mu = 0..3 stands for x,y,z,t
 *   spinor    psi[n][alpha][a]  complex128, spin alpha = 0..3, colour a = 0..2
 *   links     U[n][mu][a][b]    U_mu(n), the link from n to n+mu
 *   clover    F[n][k][i][j]     two 6x6 chiral blocks, i = 3*(alpha-2k)+a
 *   gamma     chiral hermitian Euclidean basis, gamma5 = g1 g2 g3 g4 = diag(1,1,-1,-1)
 *   geometry  int g[16] = { L[4], B[4] (SAP block), S[4] (sub-block), bc[4] (+1/-1) }
 *
 * Functions and the passages they follow:
 *   orc_dslash          eq. (2.2): D = 1 - kappa F(n) sum_mu [(1-g_mu) U_mu(n) d(n+mu,m)
 *                                   + (1+g_mu) U_mu(n-mu)^dagger d(n-mu,m)]
 *   orc_clover_A/_inv   the inverse clover term named under eq. (2.2)
 *   orc_dslash_part     the 2x2 block form eq. (2.3): D_EE/D_OO (same-block pairs) and
 *                       D_EO/D_OE (pairs in different blocks)
 *   orc_ssor            section 3, "Inverse of block operator": SSOR forward and backward
 *                       substitution in locally-lexicographic (ll) order
 *   orc_eomr            section 3, the even-odd site-preconditioned block solve the SSOR is
 *                       measured against (minimal residual on the even-odd reduced block system)
 *   orc_dk              Algorithm 1 (w = D K v), with K of eq. (2.4)
 *   orc_msap            eq. (2.4): M_SAP = K sum_{j<N_SAP} (1 - D K)^j
 *   orc_inner_bicgstab  section 2: BiCGStab preconditioned by M_SAP (textbook van der Vorst)
 *   orc_solve           section 2: the flexible (nested) outer BiCGStab, or defect correction
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex dc;

typedef struct {
    double kappa, omega, tol_inner;
    int n_ssor, n_sap, maxit_inner, maxit_outer, outer_kind;
    int block_solver; /* 0: SSOR (orc_ssor); 1: even-odd minimal residual (orc_eomr) */
} orc_params;

typedef struct {
    int L[4], B[4], S[4], bc[4];
    long V;
} geom_t;

/* ------------------------------------------------------------------ gamma matrices */

static dc GAM[5][4][4];
static int gam_ready = 0;

static void init_gamma(void)
{
    if (gam_ready) return;
    /* Pauli matrices */
    dc s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(GAM, 0, sizeof(GAM));
    /* gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], k = 1..3 (index 0..2) */
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                GAM[k][i][2 + j] = -I * s[k][i][j];
                GAM[k][2 + i][j] = I * s[k][i][j];
            }
    /* gamma_4 = [[0, 1], [1, 0]] (index 3) */
    for (int i = 0; i < 2; ++i) {
        GAM[3][i][2 + i] = 1;
        GAM[3][2 + i][i] = 1;
    }
    /* gamma_5 = g1 g2 g3 g4 (index 4) */
    dc t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            dc a = 0;
            for (int k = 0; k < 4; ++k) a += GAM[0][i][k] * GAM[1][k][j];
            t1[i][j] = a;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            dc a = 0;
            for (int k = 0; k < 4; ++k) a += t1[i][k] * GAM[2][k][j];
            t2[i][j] = a;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            dc a = 0;
            for (int k = 0; k < 4; ++k) a += t2[i][k] * GAM[3][k][j];
            GAM[4][i][j] = a;
        }
    gam_ready = 1;
}

void orc_gamma(int mu, dc *out)
{
    init_gamma();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) out[4 * i + j] = GAM[mu][i][j];
}

/* ------------------------------------------------------------------ geometry */

static void geom_from(const int *g, geom_t *G)
{
    for (int m = 0; m < 4; ++m) {
        G->L[m] = g[m];
        G->B[m] = g[4 + m];
        G->S[m] = g[8 + m];
        G->bc[m] = g[12 + m];
    }
    G->V = (long)G->L[0] * G->L[1] * G->L[2] * G->L[3];
}

static void coords(const geom_t *G, long n, int c[4])
{
    for (int m = 0; m < 4; ++m) {
        c[m] = (int)(n % G->L[m]);
        n /= G->L[m];
    }
}

static long site_of(const geom_t *G, const int c[4])
{
    return c[0] + (long)G->L[0] * (c[1] + (long)G->L[1] * (c[2] + (long)G->L[2] * c[3]));
}

/* neighbour n + sgn*mu with periodic wrap; *phase is the boundary sign of the hop */
static long neighbour(const geom_t *G, long n, int mu, int sgn, double *phase)
{
    int c[4];
    coords(G, n, c);
    int v = c[mu] + sgn;
    *phase = 1.0;
    if (v >= G->L[mu]) {
        v -= G->L[mu];
        *phase = G->bc[mu];
    } else if (v < 0) {
        v += G->L[mu];
        *phase = G->bc[mu];
    }
    c[mu] = v;
    return site_of(G, c);
}

static long block_of(const geom_t *G, long n)
{
    int c[4];
    coords(G, n, c);
    long id = 0, mult = 1;
    for (int m = 0; m < 4; ++m) {
        id += (c[m] / G->B[m]) * mult;
        mult *= G->L[m] / G->B[m];
    }
    return id;
}

/* block colour: parity of the sum of block coordinates; E = 0 holds the origin */
static int colour_of(const geom_t *G, long n)
{
    int c[4], s = 0;
    coords(G, n, c);
    for (int m = 0; m < 4; ++m) s += c[m] / G->B[m];
    return s & 1;
}

int orc_site_colour(const int *g, long n)
{
    geom_t G;
    geom_from(g, &G);
    return colour_of(&G, n);
}

/* ------------------------------------------------------------------ small linear algebra */

static void cmat3_mul(const dc *a, const dc *b, dc *c) /* c = a b */
{
    dc t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dc s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(c, t, sizeof(t));
}

static void cmat3_dag(const dc *a, dc *c)
{
    dc t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = conj(a[3 * j + i]);
    memcpy(c, t, sizeof(t));
}

static const dc *link(const dc *U, long n, int mu) { return U + 9 * (4 * n + mu); }

/* ------------------------------------------------------------------ hopping term */

/*
 * out = sum over the selected neighbour pairs (n,m) of H_nm psi(m), where
 *   H_{n,n+mu} = (1 - gamma_mu) U_mu(n),  H_{n,n-mu} = (1 + gamma_mu) U_mu(n-mu)^dagger
 * mode 0: every pair; 1: pairs inside the same SAP block; 2: pairs in different blocks.
 */
static void hop_at(const geom_t *G, const dc *U, const dc *in, long n, int mode, dc out[12])
{
    long bn = block_of(G, n);
    for (int i = 0; i < 12; ++i) out[i] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        for (int sgn = 1; sgn >= -1; sgn -= 2) {
            double ph;
            long m = neighbour(G, n, mu, sgn, &ph);
            int same = (block_of(G, m) == bn);
            if (mode == 1 && !same) continue;
            if (mode == 2 && same) continue;
            const dc *psi = in + 12 * m;
            dc t[4][3];
            if (sgn > 0) {
                const dc *u = link(U, n, mu);
                for (int be = 0; be < 4; ++be)
                    for (int a = 0; a < 3; ++a) {
                        dc s = 0;
                        for (int b = 0; b < 3; ++b) s += u[3 * a + b] * psi[3 * be + b];
                        t[be][a] = s;
                    }
            } else {
                const dc *u = link(U, m, mu);
                for (int be = 0; be < 4; ++be)
                    for (int a = 0; a < 3; ++a) {
                        dc s = 0;
                        for (int b = 0; b < 3; ++b) s += conj(u[3 * b + a]) * psi[3 * be + b];
                        t[be][a] = s;
                    }
            }
            for (int al = 0; al < 4; ++al)
                for (int a = 0; a < 3; ++a) {
                    dc s = 0;
                    for (int be = 0; be < 4; ++be) {
                        dc P = (al == be ? 1.0 : 0.0) - sgn * GAM[mu][al][be];
                        if (P != 0) s += P * t[be][a];
                    }
                    out[3 * al + a] += ph * s;
                }
        }
    }
}

void orc_hop(const int *g, const dc *U, const dc *in, dc *out, int mode)
{
    geom_t G;
    geom_from(g, &G);
    init_gamma();
#pragma omp parallel for schedule(static)
    for (long n = 0; n < G.V; ++n) hop_at(&G, U, in, n, mode, out + 12 * n);
}

/* y = F(n) x for one site: the two 6x6 chiral blocks act on spins {0,1} and {2,3} */
static void clover_site(const dc *Fn, const dc *x, dc *y)
{
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 6; ++i) {
            dc s = 0;
            for (int j = 0; j < 6; ++j) s += Fn[36 * k + 6 * i + j] * x[6 * k + j];
            y[6 * k + i] = s;
        }
}

void orc_apply_clover(const int *g, const dc *F, const dc *in, dc *out)
{
    geom_t G;
    geom_from(g, &G);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < G.V; ++n) clover_site(F + 72 * n, in + 12 * n, out + 12 * n);
}

/*
 * Parts of D (eq. 2.2 in the block form of eq. 2.3):
 *   part 0: D                          out = in - kappa F H in
 *   part 1: block-diagonal D_EE+D_OO   out = in - kappa F H_same-block in
 *   part 2: off-block D_EO+D_OE        out =    - kappa F H_other-block in
 * target_colour >= 0 writes only sites of that block colour and zeroes the others.
 */
void orc_dslash_part(const int *g, const dc *U, const dc *F, double kappa, const dc *in, dc *out,
                     int part, int target_colour)
{
    geom_t G;
    geom_from(g, &G);
    init_gamma();
    int mode = (part == 0) ? 0 : (part == 1 ? 1 : 2);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < G.V; ++n) {
        dc *o = out + 12 * n;
        if (target_colour >= 0 && colour_of(&G, n) != target_colour) {
            for (int i = 0; i < 12; ++i) o[i] = 0;
            continue;
        }
        dc h[12], fh[12];
        hop_at(&G, U, in, n, mode, h);
        clover_site(F + 72 * n, h, fh);
        for (int i = 0; i < 12; ++i) o[i] = (part == 2 ? 0.0 : in[12 * n + i]) - kappa * fh[i];
    }
}

void orc_dslash(const int *g, const dc *U, const dc *F, double kappa, const dc *in, dc *out)
{
    orc_dslash_part(g, U, F, kappa, in, out, 0, -1);
}

/* ------------------------------------------------------------------ clover term */

/* sum of the four plaquette leaves Q_{mu nu}(n) in the mu-nu plane around n */
static void clover_leaves(const geom_t *G, const dc *U, long n, int mu, int nu, dc *Q)
{
    double ph;
    long n_pmu = neighbour(G, n, mu, 1, &ph);
    long n_pnu = neighbour(G, n, nu, 1, &ph);
    long n_mmu = neighbour(G, n, mu, -1, &ph);
    long n_mnu = neighbour(G, n, nu, -1, &ph);
    long n_mmu_pnu = neighbour(G, n_mmu, nu, 1, &ph);
    long n_mmu_mnu = neighbour(G, n_mmu, nu, -1, &ph);
    long n_pmu_mnu = neighbour(G, n_pmu, nu, -1, &ph);
    dc a[9], b[9], t[9];
    for (int i = 0; i < 9; ++i) Q[i] = 0;
    /* leaf 1: n -> n+mu -> n+mu+nu -> n+nu -> n */
    cmat3_mul(link(U, n, mu), link(U, n_pmu, nu), t);
    cmat3_dag(link(U, n_pnu, mu), a);
    cmat3_mul(t, a, t);
    cmat3_dag(link(U, n, nu), a);
    cmat3_mul(t, a, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    /* leaf 2: n -> n+nu -> n-mu+nu -> n-mu -> n */
    cmat3_dag(link(U, n_mmu_pnu, mu), a);
    cmat3_mul(link(U, n, nu), a, t);
    cmat3_dag(link(U, n_mmu, nu), b);
    cmat3_mul(t, b, t);
    cmat3_mul(t, link(U, n_mmu, mu), t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    /* leaf 3: n -> n-mu -> n-mu-nu -> n-nu -> n */
    cmat3_dag(link(U, n_mmu, mu), a);
    cmat3_dag(link(U, n_mmu_mnu, nu), b);
    cmat3_mul(a, b, t);
    cmat3_mul(t, link(U, n_mmu_mnu, mu), t);
    cmat3_mul(t, link(U, n_mnu, nu), t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
    /* leaf 4: n -> n-nu -> n+mu-nu -> n+mu -> n */
    cmat3_dag(link(U, n_mnu, nu), a);
    cmat3_mul(a, link(U, n_mnu, mu), t);
    cmat3_mul(t, link(U, n_pmu_mnu, nu), t);
    cmat3_dag(link(U, n, mu), b);
    cmat3_mul(t, b, t);
    for (int i = 0; i < 9; ++i) Q[i] += t[i];
}

/*
 * A(n) = 1 - c_SW kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(n)  as a full 12x12 matrix,
 * row/column index 3*alpha + a, with sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] and the
 * clover field strength F_{mu nu} = (Q - Q^dagger)/(8i) made traceless.
 */
void orc_clover_A(const int *g, const dc *U, double csw, double kappa, dc *A)
{
    geom_t G;
    geom_from(g, &G);
    init_gamma();
    dc sig[4][4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    dc s = 0;
                    for (int k = 0; k < 4; ++k) s += GAM[mu][i][k] * GAM[nu][k][j] - GAM[nu][i][k] * GAM[mu][k][j];
                    sig[mu][nu][i][j] = 0.5 * I * s;
                }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < G.V; ++n) {
        dc *An = A + 144 * n;
        for (int i = 0; i < 144; ++i) An[i] = 0;
        for (int i = 0; i < 12; ++i) An[13 * i] = 1;
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                dc Q[9], Fmn[9];
                clover_leaves(&G, U, n, mu, nu, Q);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Fmn[3 * a + b] = (Q[3 * a + b] - conj(Q[3 * b + a])) / (8.0 * I);
                dc tr = (Fmn[0] + Fmn[4] + Fmn[8]) / 3.0;
                for (int a = 0; a < 3; ++a) Fmn[4 * a] -= tr;
                for (int al = 0; al < 4; ++al)
                    for (int be = 0; be < 4; ++be) {
                        dc sg = sig[mu][nu][al][be];
                        if (sg == 0) continue;
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                An[12 * (3 * al + a) + 3 * be + b] -= csw * kappa * sg * Fmn[3 * a + b];
                    }
            }
    }
}

/* in-place inverse of an n x n complex matrix by Gauss-Jordan with partial pivoting */
static int cinv(dc *a, int n)
{
    dc inv[36];
    for (int i = 0; i < n * n; ++i) inv[i] = 0;
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (cabs(a[r * n + c]) > cabs(a[p * n + c])) p = r;
        if (cabs(a[p * n + c]) == 0) return -1;
        if (p != c)
            for (int j = 0; j < n; ++j) {
                dc t = a[c * n + j];
                a[c * n + j] = a[p * n + j];
                a[p * n + j] = t;
                t = inv[c * n + j];
                inv[c * n + j] = inv[p * n + j];
                inv[p * n + j] = t;
            }
        dc d = a[c * n + c];
        for (int j = 0; j < n; ++j) {
            a[c * n + j] /= d;
            inv[c * n + j] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            dc f = a[r * n + c];
            if (f == 0) continue;
            for (int j = 0; j < n; ++j) {
                a[r * n + j] -= f * a[c * n + j];
                inv[r * n + j] -= f * inv[c * n + j];
            }
        }
    }
    memcpy(a, inv, sizeof(dc) * n * n);
    return 0;
}

/* F(n) = A(n)^{-1}, stored as its two 6x6 chiral blocks */
int orc_clover_inv(const int *g, const dc *U, double csw, double kappa, dc *F)
{
    geom_t G;
    geom_from(g, &G);
    dc *A = (dc *)malloc(sizeof(dc) * 144 * G.V);
    orc_clover_A(g, U, csw, kappa, A);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (long n = 0; n < G.V; ++n)
        for (int k = 0; k < 2; ++k) {
            dc blk[36];
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) blk[6 * i + j] = A[144 * n + 12 * (6 * k + i) + 6 * k + j];
            if (cinv(blk, 6)) bad++;
            memcpy(F + 72 * n + 36 * k, blk, sizeof(blk));
        }
    free(A);
    return bad;
}

/* average plaquette: mean over n and mu<nu of Re tr(U_mu(n)U_nu(n+mu)U_mu(n+nu)^+U_nu(n)^+)/3 */
double orc_plaquette(const int *g, const dc *U)
{
    geom_t G;
    geom_from(g, &G);
    double sum = 0;
    for (long n = 0; n < G.V; ++n)
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                double ph;
                long a = neighbour(&G, n, mu, 1, &ph), b = neighbour(&G, n, nu, 1, &ph);
                dc t[9], d[9];
                cmat3_mul(link(U, n, mu), link(U, a, nu), t);
                cmat3_dag(link(U, b, mu), d);
                cmat3_mul(t, d, t);
                cmat3_dag(link(U, n, nu), d);
                cmat3_mul(t, d, t);
                sum += creal(t[0] + t[4] + t[8]) / 3.0;
            }
    return sum / (6.0 * G.V);
}

/* ------------------------------------------------------------------ SSOR block inverse */

/*
 * Locally-lexicographic order of the sites of one block: the key is first the
 * local position inside the sub-block (lexicographic, x fastest), then the
 * index of the sub-block.  order[k] is the block-local lexicographic index of
 * the k-th site.
 *
 * A sub-block shape of all zeros selects the even-odd site ordering that section 3 ("Inverse of block operator")
 * compares the ll ordering against: the sites whose block-local coordinates have an
 * even sum, in lexicographic order, then the odd ones.  (Reading: the parity is taken
 * inside the block; the paper does not say, and for SSOR on one block only the
 * relative order of coupled sites matters.)
 */
void orc_ll_order(const int *g, int *order)
{
    geom_t G;
    geom_from(g, &G);
    int Vb = G.B[0] * G.B[1] * G.B[2] * G.B[3];
    if (G.S[0] == 0 && G.S[1] == 0 && G.S[2] == 0 && G.S[3] == 0) {
        int k = 0;
        for (int par = 0; par < 2; ++par)
            for (int l = 0; l < Vb; ++l) {
                int r = l, sum = 0;
                for (int m = 0; m < 4; ++m) {
                    sum += r % G.B[m];
                    r /= G.B[m];
                }
                if ((sum & 1) == par) order[k++] = l;
            }
        return;
    }
    int nsub[4], Vs = 1, Ns = 1;
    for (int m = 0; m < 4; ++m) {
        nsub[m] = G.B[m] / G.S[m];
        Vs *= G.S[m];
        Ns *= nsub[m];
    }
    (void)Vs;
    for (int l = 0; l < Vb; ++l) {
        int c[4], r = l;
        for (int m = 0; m < 4; ++m) {
            c[m] = r % G.B[m];
            r /= G.B[m];
        }
        int pos = 0, sub = 0, pm = 1, sm = 1;
        for (int m = 0; m < 4; ++m) {
            pos += (c[m] % G.S[m]) * pm;
            pm *= G.S[m];
            sub += (c[m] / G.S[m]) * sm;
            sm *= nsub[m];
        }
        order[pos * Ns + sub] = l;
    }
}

/* one relaxation step at site n: x_n <- (1-omega) x_n + omega (v_n + kappa F(n) sum_{m in block} H_nm x_m) */
static void ssor_site(const geom_t *G, const dc *U, const dc *F, double kappa, double omega, const dc *v,
                      dc *x, long n)
{
    dc h[12], fh[12];
    hop_at(G, U, x, n, 1, h);
    clover_site(F + 72 * n, h, fh);
    for (int i = 0; i < 12; ++i)
        x[12 * n + i] = (1.0 - omega) * x[12 * n + i] + omega * (v[12 * n + i] + kappa * fh[i]);
}

/*
 * x = A_cc v on every block of colour `colour`: starting from x = 0 on the block,
 * n_ssor times a forward substitution sweep over the sites in `order` followed by a
 * backward sweep in reverse order, updated in place.  order == NULL means the
 * locally-lexicographic order; any other array is a permutation of the block-local
 * lexicographic indices.  Sites of the other colour get x = 0.
 */
void orc_ssor(const int *g, const dc *U, const dc *F, const orc_params *p, int colour, const int *order,
              const dc *v, dc *x)
{
    geom_t G;
    geom_from(g, &G);
    init_gamma();
    int Vb = G.B[0] * G.B[1] * G.B[2] * G.B[3];
    int *ord = (int *)malloc(sizeof(int) * Vb);
    if (order)
        memcpy(ord, order, sizeof(int) * Vb);
    else
        orc_ll_order(g, ord);
    int nb[4];
    long NB = 1;
    for (int m = 0; m < 4; ++m) {
        nb[m] = G.L[m] / G.B[m];
        NB *= nb[m];
    }
    memset(x, 0, sizeof(dc) * 12 * G.V);
#pragma omp parallel for schedule(dynamic)
    for (long blk = 0; blk < NB; ++blk) {
        int bcrd[4];
        long r = blk;
        int col = 0;
        for (int m = 0; m < 4; ++m) {
            bcrd[m] = (int)(r % nb[m]);
            r /= nb[m];
            col += bcrd[m];
        }
        if ((col & 1) != colour) continue;
        long *sites = (long *)malloc(sizeof(long) * Vb);
        for (int k = 0; k < Vb; ++k) {
            int l = ord[k], c[4];
            for (int m = 0; m < 4; ++m) {
                c[m] = bcrd[m] * G.B[m] + l % G.B[m];
                l /= G.B[m];
            }
            sites[k] = site_of(&G, c);
        }
        for (int sw = 0; sw < p->n_ssor; ++sw) {
            for (int k = 0; k < Vb; ++k) ssor_site(&G, U, F, p->kappa, p->omega, v, x, sites[k]);
            for (int k = Vb - 1; k >= 0; --k) ssor_site(&G, U, F, p->kappa, p->omega, v, x, sites[k]);
        }
        free(sites);
    }
    free(ord);
}

/* parity of the block-local coordinate sum of site n (0 = even) */
static int local_parity(const geom_t *G, long n)
{
    int c[4], s = 0;
    coords(G, n, c);
    for (int m = 0; m < 4; ++m) s += c[m] % G->B[m];
    return s & 1;
}

/* out_n = kappa F(n) sum_{m in block(n)} H_nm in_m on the sites of block colour `colour` and
 * parity `par`; every other site of out is set to 0 */
static void k_block(const geom_t *G, const dc *U, const dc *F, double kappa, int colour, int par, const dc *in,
                    dc *out)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < G->V; ++n) {
        dc h[12], fh[12];
        if (colour_of(G, n) != colour || local_parity(G, n) != par) {
            for (int i = 0; i < 12; ++i) out[12 * n + i] = 0;
            continue;
        }
        hop_at(G, U, in, n, 1, h);
        clover_site(F + 72 * n, h, fh);
        for (int i = 0; i < 12; ++i) out[12 * n + i] = kappa * fh[i];
    }
}

/*
 * x = A_cc v by the even-odd site-preconditioned block solve, on every block of colour
 * `colour` (the block solver of the cited Luscher SAP, which section 3 compares the SSOR
 * against at equal cost).  Inside a block, A = 1 - K with K = kappa F H restricted to the
 * block; a hop changes the parity of the block-local coordinate sum, so with e / o the two
 * parities A x = v reads x_e - K_eo x_o = v_e, x_o - K_oe x_e = v_o.  Eliminating x_o:
 *     (1 - K_eo K_oe) x_e = v_e + K_eo v_o,      x_o = v_o + K_oe x_e.
 * The reduced system is solved by n_mr minimal-residual steps from x_e = 0 (r = rhs):
 *     p = (1 - K_eo K_oe) r,  alpha = <p, r> / <p, p>,  x_e += alpha r,  r -= alpha p,
 * alpha taken per block.  n_mr = 2 n_ssor: a step applies K to the odd and then to the even
 * sites, one application of the block operator, as one SSOR half-sweep does.
 * Readings: the paper names this solver and the equal-cost comparison only; the reduced
 * system, the minimal-residual steps and their count are taken from the cited SAP.
 * Sites of the other colour get x = 0.
 */
void orc_eomr(const int *g, const dc *U, const dc *F, const orc_params *p, int colour, const dc *v, dc *x)
{
    geom_t G;
    geom_from(g, &G);
    init_gamma();
    const long N = 12 * G.V;
    long NB = 1;
    for (int m = 0; m < 4; ++m) NB *= G.L[m] / G.B[m];
    dc *ve = calloc(N, sizeof(dc)), *vo = calloc(N, sizeof(dc)), *r = calloc(N, sizeof(dc));
    dc *t = calloc(N, sizeof(dc)), *q = calloc(N, sizeof(dc)), *xe = calloc(N, sizeof(dc));
    dc *num = calloc(NB, sizeof(dc));
    double *den = calloc(NB, sizeof(double));
    for (long n = 0; n < G.V; ++n) {
        if (colour_of(&G, n) != colour) continue;
        dc *dst = local_parity(&G, n) == 0 ? ve : vo;
        for (int i = 0; i < 12; ++i) dst[12 * n + i] = v[12 * n + i];
    }
    k_block(&G, U, F, p->kappa, colour, 0, vo, t); /* t_e = K_eo v_o */
    for (long i = 0; i < N; ++i) r[i] = ve[i] + t[i];
    const int n_mr = 2 * p->n_ssor;
    for (int k = 0; k < n_mr; ++k) {
        k_block(&G, U, F, p->kappa, colour, 1, r, t); /* t_o = K_oe r_e */
        k_block(&G, U, F, p->kappa, colour, 0, t, q); /* q_e = K_eo t_o */
        for (long i = 0; i < N; ++i) q[i] = r[i] - q[i]; /* p = (1 - K_eo K_oe) r (zero off the even sites) */
        for (long b = 0; b < NB; ++b) {
            num[b] = 0;
            den[b] = 0;
        }
        for (long n = 0; n < G.V; ++n) {
            const long b = block_of(&G, n);
            for (int i = 0; i < 12; ++i) {
                num[b] += conj(q[12 * n + i]) * r[12 * n + i];
                den[b] += creal(conj(q[12 * n + i]) * q[12 * n + i]);
            }
        }
        for (long n = 0; n < G.V; ++n) {
            const long b = block_of(&G, n);
            const dc alpha = den[b] > 0 ? num[b] / den[b] : 0;
            for (int i = 0; i < 12; ++i) {
                xe[12 * n + i] += alpha * r[12 * n + i];
                r[12 * n + i] -= alpha * q[12 * n + i];
            }
        }
    }
    k_block(&G, U, F, p->kappa, colour, 1, xe, t); /* t_o = K_oe x_e */
    for (long i = 0; i < N; ++i) x[i] = xe[i] + vo[i] + t[i];
    free(ve); free(vo); free(r); free(t); free(q); free(xe); free(num); free(den);
}

/* the block inverse the parameters select: SSOR in ll order, or the even-odd MR solve */
static void block_solve(const int *g, const dc *U, const dc *F, const orc_params *p, int colour, const dc *v, dc *x)
{
    if (p->block_solver == 1)
        orc_eomr(g, U, F, p, colour, v, x);
    else
        orc_ssor(g, U, F, p, colour, NULL, v, x);
}

/* ------------------------------------------------------------------ SAP: Algorithm 1 and M_SAP */

static void vzero(dc *a, long n) { memset(a, 0, sizeof(dc) * n); }

/*
 * Algorithm 1 (w = D K v), step by step with E = colour 0 and O = colour 1:
 *   x_E = A_EE v_E;  w_O = D_OE x_E;  w_E = D_EE x_E;  f_O = v_O - w_O;  x_O = A_OO f_O;
 *   f_E = D_EO x_O;  f_O = D_OO x_O;  w_O = w_O + f_O;  w_E = w_E + f_E.
 * Returns x = K v and w = D K v.
 */
void orc_dk(const int *g, const dc *U, const dc *F, const orc_params *p, const dc *v, dc *x, dc *w)
{
    geom_t G;
    geom_from(g, &G);
    long N = 12 * G.V;
    dc *xE = malloc(sizeof(dc) * N), *xO = malloc(sizeof(dc) * N);
    dc *wE = malloc(sizeof(dc) * N), *wO = malloc(sizeof(dc) * N);
    dc *fE = malloc(sizeof(dc) * N), *fO = malloc(sizeof(dc) * N);
    block_solve(g, U, F, p, 0, v, xE);                         /* x_E = A_EE v_E */
    orc_dslash_part(g, U, F, p->kappa, xE, wO, 2, 1);          /* w_O = D_OE x_E */
    orc_dslash_part(g, U, F, p->kappa, xE, wE, 1, 0);          /* w_E = D_EE x_E */
    for (long n = 0; n < G.V; ++n) {                            /* f_O = v_O - w_O */
        int c = colour_of(&G, n);
        for (int i = 0; i < 12; ++i) fO[12 * n + i] = (c == 1) ? v[12 * n + i] - wO[12 * n + i] : 0;
    }
    block_solve(g, U, F, p, 1, fO, xO);                        /* x_O = A_OO f_O */
    orc_dslash_part(g, U, F, p->kappa, xO, fE, 2, 0);          /* f_E = D_EO x_O */
    orc_dslash_part(g, U, F, p->kappa, xO, fO, 1, 1);          /* f_O = D_OO x_O */
    for (long i = 0; i < N; ++i) {
        wO[i] += fO[i];                                         /* w_O = w_O + f_O */
        wE[i] += fE[i];                                         /* w_E = w_E + f_E */
        x[i] = xE[i] + xO[i];
        w[i] = wE[i] + wO[i];
    }
    free(xE); free(xO); free(wE); free(wO); free(fE); free(fO);
}

/*
 * M_SAP of eq. (2.4) as its recurrence: r = v, y = 0; N_SAP times (x, w) = DK(r),
 * y += x, r -= w.  Then y = K sum_{j<N} (1-DK)^j v = M_SAP v and dy = v - r = D M_SAP v.
 */
void orc_msap(const int *g, const dc *U, const dc *F, const orc_params *p, const dc *v, dc *y, dc *dy)
{
    geom_t G;
    geom_from(g, &G);
    long N = 12 * G.V;
    dc *r = malloc(sizeof(dc) * N), *x = malloc(sizeof(dc) * N), *w = malloc(sizeof(dc) * N);
    memcpy(r, v, sizeof(dc) * N);
    vzero(y, N);
    for (int j = 0; j < p->n_sap; ++j) {
        orc_dk(g, U, F, p, r, x, w);
        for (long i = 0; i < N; ++i) {
            y[i] += x[i];
            r[i] -= w[i];
        }
    }
    if (dy)
        for (long i = 0; i < N; ++i) dy[i] = v[i] - r[i];
    free(r); free(x); free(w);
}

/* ------------------------------------------------------------------ Krylov solvers */

static dc vdot(const dc *a, const dc *b, long n) /* <a,b> = sum conj(a) b, in index order */
{
    dc s = 0;
    for (long i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double vnorm(const dc *a, long n) { return sqrt(creal(vdot(a, a, n))); }

/*
 * Inner solver: BiCGStab for D e = r from e = 0, right-preconditioned by M_SAP
 * (it solves (D M) u = r and accumulates e = M u directly).  The products
 * D p^ and D s^ are the D M_SAP outputs of the SAP recurrence.  Stops when
 * |r_i| <= tol_inner |r|, after maxit_inner iterations, or on breakdown.
 * Returns the number of iterations.
 */
int orc_inner_bicgstab(const int *g, const dc *U, const dc *F, const orc_params *p, const dc *rhs, dc *e)
{
    geom_t G;
    geom_from(g, &G);
    long N = 12 * G.V;
    dc *r = malloc(sizeof(dc) * N), *rt = malloc(sizeof(dc) * N), *pv = malloc(sizeof(dc) * N);
    dc *v = malloc(sizeof(dc) * N), *ph = malloc(sizeof(dc) * N), *s = malloc(sizeof(dc) * N);
    dc *sh = malloc(sizeof(dc) * N), *t = malloc(sizeof(dc) * N);
    memcpy(r, rhs, sizeof(dc) * N);
    memcpy(rt, rhs, sizeof(dc) * N);
    vzero(e, N);
    vzero(pv, N);
    vzero(v, N);
    double r0 = vnorm(r, N);
    dc rho_old = 1, alpha = 1, om = 1;
    int it = 0;
    if (r0 == 0) goto done;
    while (it < p->maxit_inner) {
        dc rho = vdot(rt, r, N);
        if (rho == 0) break;
        dc beta = (rho / rho_old) * (alpha / om);
        for (long i = 0; i < N; ++i) pv[i] = r[i] + beta * (pv[i] - om * v[i]);
        orc_msap(g, U, F, p, pv, ph, v);                          /* p^ = M p, v = D p^ */
        dc rv = vdot(rt, v, N);
        if (rv == 0) break;
        alpha = rho / rv;
        for (long i = 0; i < N; ++i) s[i] = r[i] - alpha * v[i];
        ++it;
        if (vnorm(s, N) <= p->tol_inner * r0) {
            for (long i = 0; i < N; ++i) e[i] += alpha * ph[i];
            break;
        }
        orc_msap(g, U, F, p, s, sh, t);                           /* s^ = M s, t = D s^ */
        double tt = creal(vdot(t, t, N));
        if (tt == 0) {
            for (long i = 0; i < N; ++i) e[i] += alpha * ph[i];
            break;
        }
        om = vdot(t, s, N) / tt;
        for (long i = 0; i < N; ++i) {
            e[i] += alpha * ph[i] + om * sh[i];
            r[i] = s[i] - om * t[i];
        }
        rho_old = rho;
        if (vnorm(r, N) <= p->tol_inner * r0) break;
        if (om == 0) break;
    }
done:
    free(r); free(rt); free(pv); free(v); free(ph); free(s); free(sh); free(t);
    return it;
}

/*
 * Outer solver for D x = b to |b - D x| <= tol |b|.
 * outer_kind 0: flexible BiCGStab whose preconditioner is the inner solver
 *   (p^ = Inner(p), v = D p^, s^ = Inner(s), t = D s^), with the true residual
 *   b - D x recomputed when the recursive one passes, and a restart if it fails.
 * outer_kind 1: defect correction  r = b - D x;  x += Inner(r)  until it passes.
 * stats[0..3] = outer iterations, inner iterations in total, true relative residual, restarts.
 * Returns 0 when converged, 1 otherwise.  use_guess != 0 starts from the x passed in.
 */
int orc_solve(const int *g, const dc *U, const dc *F, const orc_params *p, double tol, const dc *b, dc *x,
              int use_guess, double *stats)
{
    geom_t G;
    geom_from(g, &G);
    long N = 12 * G.V;
    dc *r = malloc(sizeof(dc) * N), *rt = malloc(sizeof(dc) * N), *pv = malloc(sizeof(dc) * N);
    dc *v = malloc(sizeof(dc) * N), *ph = malloc(sizeof(dc) * N), *s = malloc(sizeof(dc) * N);
    dc *sh = malloc(sizeof(dc) * N), *t = malloc(sizeof(dc) * N);
    if (!use_guess) vzero(x, N);
    double bn = vnorm(b, N);
    int outer = 0, inner = 0, restarts = 0, conv = 0;
    double relres = 1.0;
    orc_dslash(g, U, F, p->kappa, x, t);
    for (long i = 0; i < N; ++i) r[i] = b[i] - t[i];
    relres = (bn > 0) ? vnorm(r, N) / bn : 0.0;
    if (relres <= tol) conv = 1;
    if (p->outer_kind == 1) {
        while (!conv && outer < p->maxit_outer) {
            inner += orc_inner_bicgstab(g, U, F, p, r, ph);
            for (long i = 0; i < N; ++i) x[i] += ph[i];
            orc_dslash(g, U, F, p->kappa, x, t);
            for (long i = 0; i < N; ++i) r[i] = b[i] - t[i];
            ++outer;
            relres = vnorm(r, N) / bn;
            if (relres <= tol) conv = 1;
        }
    } else {
        while (!conv && outer < p->maxit_outer) {
            memcpy(rt, r, sizeof(dc) * N);
            vzero(pv, N);
            vzero(v, N);
            dc rho_old = 1, alpha = 1, om = 1;
            int restart = 0;
            while (!restart && outer < p->maxit_outer) {
                dc rho = vdot(rt, r, N);
                dc beta = (rho / rho_old) * (alpha / om);
                for (long i = 0; i < N; ++i) pv[i] = r[i] + beta * (pv[i] - om * v[i]);
                inner += orc_inner_bicgstab(g, U, F, p, pv, ph);   /* p^ = Inner(p) */
                orc_dslash(g, U, F, p->kappa, ph, v);               /* v = D p^ */
                alpha = rho / vdot(rt, v, N);
                for (long i = 0; i < N; ++i) s[i] = r[i] - alpha * v[i];
                ++outer;
                if (vnorm(s, N) <= tol * bn) {
                    for (long i = 0; i < N; ++i) x[i] += alpha * ph[i];
                    restart = 1;
                } else {
                    inner += orc_inner_bicgstab(g, U, F, p, s, sh); /* s^ = Inner(s) */
                    orc_dslash(g, U, F, p->kappa, sh, t);            /* t = D s^ */
                    om = vdot(t, s, N) / creal(vdot(t, t, N));
                    for (long i = 0; i < N; ++i) {
                        x[i] += alpha * ph[i] + om * sh[i];
                        r[i] = s[i] - om * t[i];
                    }
                    rho_old = rho;
                    if (vnorm(r, N) <= tol * bn) restart = 1;
                }
                if (restart) {
                    orc_dslash(g, U, F, p->kappa, x, t);            /* true residual */
                    for (long i = 0; i < N; ++i) r[i] = b[i] - t[i];
                    relres = vnorm(r, N) / bn;
                    if (relres <= tol)
                        conv = 1;
                    else
                        ++restarts;
                }
            }
        }
    }
    if (!conv) { /* report the true residual of the iterate that is returned */
        orc_dslash(g, U, F, p->kappa, x, t);
        for (long i = 0; i < N; ++i) r[i] = b[i] - t[i];
        relres = (bn > 0) ? vnorm(r, N) / bn : 0.0;
    }
    if (stats) {
        stats[0] = outer;
        stats[1] = inner;
        stats[2] = relres;
        stats[3] = restarts;
    }
    free(r); free(rt); free(pv); free(v); free(ph); free(s); free(sh); free(t);
    return conv ? 0 : 1;
}
