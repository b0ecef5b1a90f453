/*
 * nn_oracle.c -- plain FP64 CPU oracle of the learned gauge-covariant preconditioner stage
 * (test infrastructure only; shares no code with the GPU library).
 *
 * The paper has no learned part; the stage is defined here as a linear parallel-transport
 * convolution.  One layer maps c_in spinor channels to c_out:
 *
 *   out[c'](n) = sum_{d=0..8} sum_c W[d][c'][c] (T_d in[c])(n)
 *
 * with W[d][c'][c] a 4x4 complex spin matrix and the transports
 *   T_0 psi(n)        = psi(n)
 *   T_{1+2mu} psi(n)  = U_mu(n) psi(n+mu)          (times the boundary sign if the hop wraps)
 *   T_{2+2mu} psi(n)  = U_mu(n-mu)^+ psi(n-mu)     (likewise)
 * so that one layer with W_0 = 1 and W_{1+2mu} = -kappa (1 - gamma_mu), W_{2+2mu} =
 * -kappa (1 + gamma_mu) is the operator D of eq. (2.2) with F = 1.
 *
 * Layouts: fields [c][V][4][3] complex128; weights [9][c_out][c_in][4][4] complex128; links as
 * in sapq_oracle.c; geometry int g[16] = {L[4], B[4], S[4], bc[4]} (only L and bc are used).
 */
#include <complex.h>
#include <string.h>

typedef double complex dc;

static void coords4(const int *L, long n, int c[4])
{
    for (int m = 0; m < 4; ++m) {
        c[m] = (int)(n % L[m]);
        n /= L[m];
    }
}

static long index4(const int *L, const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/* site n + sgn*mu and the boundary sign of that hop */
static long step(const int *g, long n, int mu, int sgn, double *ph)
{
    const int *L = g;
    int c[4];
    coords4(L, n, c);
    int v = c[mu] + sgn;
    *ph = 1.0;
    if (v >= L[mu]) {
        v -= L[mu];
        *ph = g[12 + mu];
    } else if (v < 0) {
        v += L[mu];
        *ph = g[12 + mu];
    }
    c[mu] = v;
    return index4(L, c);
}

/* t = (T_d psi)(n) for one channel field psi [V][4][3] */
static void transport(const int *g, const dc *U, const dc *psi, long n, int d, dc t[12])
{
    if (d == 0) {
        memcpy(t, psi + 12 * n, sizeof(dc) * 12);
        return;
    }
    int mu = (d - 1) / 2, fwd = ((d - 1) % 2) == 0;
    double ph;
    long m = step(g, n, mu, fwd ? 1 : -1, &ph);
    const dc *p = psi + 12 * m;
    const dc *u = U + 9 * (4 * (fwd ? n : m) + mu);
    for (int be = 0; be < 4; ++be)
        for (int a = 0; a < 3; ++a) {
            dc s = 0;
            for (int b = 0; b < 3; ++b) s += (fwd ? u[3 * a + b] : conj(u[3 * b + a])) * p[3 * be + b];
            t[3 * be + a] = ph * s;
        }
}

void orc_nn_layer(const int *g, const dc *U, const dc *W, int cin, int cout, const dc *in, dc *out)
{
    long V = (long)g[0] * g[1] * g[2] * g[3];
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; ++n) {
        for (int co = 0; co < cout; ++co)
            for (int i = 0; i < 12; ++i) out[(co * V + n) * 12 + i] = 0;
        for (int d = 0; d < 9; ++d)
            for (int ci = 0; ci < cin; ++ci) {
                dc t[12];
                transport(g, U, in + (long)ci * V * 12, n, d, t);
                for (int co = 0; co < cout; ++co) {
                    const dc *w = W + (((long)d * cout + co) * cin + ci) * 16;
                    dc *o = out + (co * V + n) * 12;
                    for (int al = 0; al < 4; ++al)
                        for (int a = 0; a < 3; ++a) {
                            dc s = 0;
                            for (int be = 0; be < 4; ++be) s += w[4 * al + be] * t[3 * be + a];
                            o[3 * al + a] += s;
                        }
                }
            }
    }
}

/*
 * gin = layer^+ gout: the adjoint of the layer.  Since T_{1+2mu}^+ = T_{2+2mu} and the
 * spin matrices act on another index than the transports,
 *   gin[c](n) = sum_d sum_c' W[d][c'][c]^+ (T_{rev(d)} gout[c'])(n),  rev swaps +mu and -mu.
 */
void orc_nn_layer_adjoint(const int *g, const dc *U, const dc *W, int cin, int cout, const dc *gout, dc *gin)
{
    long V = (long)g[0] * g[1] * g[2] * g[3];
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; ++n) {
        for (int ci = 0; ci < cin; ++ci)
            for (int i = 0; i < 12; ++i) gin[(ci * V + n) * 12 + i] = 0;
        for (int d = 0; d < 9; ++d) {
            int rd = d == 0 ? 0 : (((d - 1) % 2) == 0 ? d + 1 : d - 1);
            for (int co = 0; co < cout; ++co) {
                dc t[12];
                transport(g, U, gout + (long)co * V * 12, n, rd, t);
                for (int ci = 0; ci < cin; ++ci) {
                    const dc *w = W + (((long)d * cout + co) * cin + ci) * 16;
                    dc *o = gin + (ci * V + n) * 12;
                    for (int be = 0; be < 4; ++be)
                        for (int a = 0; a < 3; ++a) {
                            dc s = 0;
                            for (int al = 0; al < 4; ++al) s += conj(w[4 * al + be]) * t[3 * al + a];
                            o[3 * be + a] += s;
                        }
                }
            }
        }
    }
}

/*
 * Weight gradient of a real loss L with dL/d(out) = gout (meaning dL/dRe + i dL/dIm):
 *   G[d][c'][c][al][be] = sum_n sum_a gout[c'](n)[al][a] conj((T_d in[c])(n)[be][a])
 * which is dL/dRe W + i dL/dIm W.
 */
void orc_nn_layer_wgrad(const int *g, const dc *U, int cin, int cout, const dc *gout, const dc *in, dc *G)
{
    long V = (long)g[0] * g[1] * g[2] * g[3];
    long NG = 9L * cout * cin * 16;
    memset(G, 0, sizeof(dc) * NG);
    for (int d = 0; d < 9; ++d)
        for (int ci = 0; ci < cin; ++ci)
            for (int co = 0; co < cout; ++co) {
                dc acc[16];
                memset(acc, 0, sizeof(acc));
                for (long n = 0; n < V; ++n) {
                    dc t[12];
                    transport(g, U, in + (long)ci * V * 12, n, d, t);
                    const dc *go = gout + (co * V + n) * 12;
                    for (int al = 0; al < 4; ++al)
                        for (int be = 0; be < 4; ++be)
                            for (int a = 0; a < 3; ++a) acc[4 * al + be] += go[3 * al + a] * conj(t[3 * be + a]);
                }
                memcpy(G + (((long)d * cout + co) * cin + ci) * 16, acc, sizeof(acc));
            }
}
