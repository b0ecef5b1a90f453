// Learned gauge-covariant preconditioner stage: linear parallel-transport convolution
// layers, their adjoints and weight gradients, and the Adam update.
//
// A layer maps c_in spinor channels to c_out:
//   out[c'](n) = sum_{d=0..8} sum_c W[d][c'][c] (T_d in[c])(n),  W[d][c'][c] a 4x4 complex spin matrix,
//   T_0 = 1, T_{1+2mu} psi(n) = U_mu(n) psi(n+mu), T_{2+2mu} psi(n) = U_mu(n-mu)^+ psi(n-mu),
// with the fermion boundary sign on hops that wrap.  Activations are FP32 fields in the
// internal layout, one [NB][12][Vb] spinor field per channel.  The forward pass uses the
// weights rounded to BF16 (FP32 arithmetic); Adam keeps an FP32 master copy.
#include "sitecore.h"

namespace sapq {

// (T_d psi)(ib, s) for one FP32 channel field; links in storage precision P
template <int P>
__device__ __forceinline__ void nn_transport(cx<float> t[12], const float2 *__restrict__ psi, const GeomDev &g,
                                             const typename Prec<P>::S2 *__restrict__ U, int ib, int s, int d) {
    if (d == 0) {
        load_spinor(t, psi, g, ib, s);
        return;
    }
    const int mu = (d - 1) >> 1;
    const bool fwd = ((d - 1) & 1) == 0;
    const unsigned w = g.nbr16[mu * g.Vb + s];
    const unsigned half = fwd ? (w & 0xffffu) : (w >> 16);
    const int ns = (int)(half & 0x7fffu);
    const bool inside = (half & 0x8000u) != 0;
    int nb = ib;
    float ph = 1.f;
    if (!inside) {
        const int bl = g.blk_nbr[(2 * mu + (fwd ? 0 : 1)) * g.NB + ib];
        nb = bl & BLK_MASK;
        ph = (bl & WRAP_BIT) ? g.bc[mu] : 1.f;
    }
    cx<float> p[12], u[9];
    load_spinor(p, psi, g, nb, ns);
    if (fwd)
        load_link(u, U, g, ib, s, mu);
    else
        load_link(u, U, g, nb, ns, mu);
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        cx<float> h[3] = {p[3 * be], p[3 * be + 1], p[3 * be + 2]}, o[3];
        su3_mul(o, u, h, !fwd);
#pragma unroll
        for (int a = 0; a < 3; ++a) t[3 * be + a] = ph * o[a];
    }
}

// Neighbour of (ib, s) for transport d (0: the site itself): block, slot and boundary sign.
__device__ __forceinline__ void nn_neighbour(const GeomDev &g, int ib, int s, int d, int &nb, int &ns, float &ph) {
    nb = ib;
    ns = s;
    ph = 1.f;
    if (d == 0) return;
    const int mu = (d - 1) >> 1;
    const bool fwd = ((d - 1) & 1) == 0;
    const unsigned w = g.nbr16[mu * g.Vb + s];
    const unsigned half = fwd ? (w & 0xffffu) : (w >> 16);
    ns = (int)(half & 0x7fffu);
    if (!(half & 0x8000u)) {
        const int bl = g.blk_nbr[(2 * mu + (fwd ? 0 : 1)) * g.NB + ib];
        nb = bl & BLK_MASK;
        ph = (bl & WRAP_BIT) ? g.bc[mu] : 1.f;
    }
}

// (T_d psi)(ib, s) with the neighbour (nb, ns, ph) already known
template <int P>
__device__ __forceinline__ void nn_transport_at(cx<float> t[12], const float2 *__restrict__ psi, const GeomDev &g,
                                                const typename Prec<P>::S2 *__restrict__ U, int ib, int s, int d, int nb,
                                                int ns, float ph) {
    if (d == 0) {
        load_spinor(t, psi, g, ib, s);
        return;
    }
    const int mu = (d - 1) >> 1;
    const bool fwd = ((d - 1) & 1) == 0;
    cx<float> p[12], u[9];
    load_spinor(p, psi, g, nb, ns);
    if (fwd)
        load_link(u, U, g, ib, s, mu);
    else
        load_link(u, U, g, nb, ns, mu);
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        cx<float> h[3] = {p[3 * be], p[3 * be + 1], p[3 * be + 2]}, o[3];
        su3_mul(o, u, h, !fwd);
#pragma unroll
        for (int a = 0; a < 3; ++a) t[3 * be + a] = ph * o[a];
    }
}

// Tile of 16 sites of a layer workgroup.  Workgroups are dealt to the 8 XCDs in turn; with
// a grid that is a multiple of 8, XCD x takes the x-th eighth of the tiles, and tiles run
// through whole blocks in lexicographic block order, so that the neighbours a tile reads
// (mostly in the same block or the next one) were fetched into the same L2.  ib < 0 marks a
// workgroup past the last tile; n_valid sites of the tile exist (blocks need not hold a
// multiple of 16 sites).
__device__ __forceinline__ void nn_tile(const GeomDev &g, int &ib, int &s0, int &n_valid) {
    const long vt = xcd_site_base(1);
    const int tpb = (g.Vb + 15) / 16;
    const long bl = vt / tpb;
    ib = bl < g.NB ? g.lex_blk[bl] : -1;
    s0 = (int)(vt - bl * tpb) * 16;
    n_valid = min(16, g.Vb - s0);
}

unsigned nn_grid(const Ctx *c) {
    const long tiles = (long)c->g.NB * ((c->g.Vb + 15) / 16);
    return (unsigned)((tiles + N_XCD - 1) / N_XCD * N_XCD);
}

// out[c'] for one output channel c' = blockIdx.y; weights W[9][COUT][CIN][16] complex (float2)
template <int P, int CIN, int COUT>
__global__ void __launch_bounds__(256) k_nn_layer(GeomDev g, const float2 *__restrict__ in, float2 *__restrict__ out,
                                                 const float2 *__restrict__ W,
                                                 const typename Prec<P>::S2 *__restrict__ U) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int co = blockIdx.y;
    if (i >= g.V) return;
    const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    const size_t chan = (size_t)g.V * 12;
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
    for (int d = 0; d < 9; ++d) {
#pragma unroll 1
        for (int ci = 0; ci < CIN; ++ci) {
            cx<float> t[12];
            nn_transport<P>(t, in + ci * chan, g, U, ib, s, d);
            const float2 *w = W + (((size_t)d * COUT + co) * CIN + ci) * 16;
#pragma unroll
            for (int al = 0; al < 4; ++al)
#pragma unroll
                for (int be = 0; be < 4; ++be) {
                    const float2 wv = w[4 * al + be];
                    const cx<float> wc{wv.x, wv.y};
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[3 * al + a] = acc[3 * al + a] + cmul(wc, t[3 * be + a]);
                }
        }
    }
    store_spinor(out + co * chan, g, ib, s, acc);
}

// G[d][c'][c] (16 complex) = sum_n sum_a gout[c'](n)[al][a] conj((T_d in[c])(n)[be][a]), added to G.
// One workgroup per (d, c', c); a fixed-order tree finishes the sum.
template <int P>
__global__ void __launch_bounds__(256) k_nn_wgrad(GeomDev g, int cin, int cout, const float2 *__restrict__ gout,
                                                 const float2 *__restrict__ in, const typename Prec<P>::S2 *__restrict__ U,
                                                 float2 *__restrict__ G) {
    __shared__ float sm[32][257];
    const int d = blockIdx.x, co = blockIdx.y, ci = blockIdx.z;
    const size_t chan = (size_t)g.V * 12;
    float acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0.f;
    for (long i = threadIdx.x; i < g.V; i += blockDim.x) {
        const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
        cx<float> t[12], go[12];
        nn_transport<P>(t, in + ci * chan, g, U, ib, s, d);
        load_spinor(go, gout + co * chan, g, ib, s);
#pragma unroll
        for (int al = 0; al < 4; ++al)
#pragma unroll
            for (int be = 0; be < 4; ++be) {
                cx<float> v = cxz<float>();
#pragma unroll
                for (int a = 0; a < 3; ++a) v = v + cmulc(t[3 * be + a], go[3 * al + a]);
                acc[2 * (4 * al + be)] += v.r;
                acc[2 * (4 * al + be) + 1] += v.i;
            }
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 32; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 16) {
        float2 *p = G + (((size_t)d * cout + co) * cin + ci) * 16 + threadIdx.x;
        float2 o = *p;
        *p = make_float2(o.x + sm[2 * threadIdx.x][0], o.y + sm[2 * threadIdx.x + 1][0]);
    }
}

// weights of the adjoint layer (it maps cout channels to cin):
//   Wt[d][c][c'][a][b] = conj(W[rev(d)][c'][c][b][a]),  rev swaps +mu and -mu
__global__ void k_nn_adjoint_weights(int cin, int cout, const float2 *__restrict__ W, float2 *__restrict__ Wt) {
    const int n = 9 * cin * cout * 16;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int r = t;
    const int b = r % 4; r /= 4;
    const int a = r % 4; r /= 4;
    const int cc = r % cout; r /= cout;  // input channel of the adjoint = output channel c' of W
    const int ci = r % cin; r /= cin;    // output channel of the adjoint = input channel c of W
    const int d = r;
    const int rd = d == 0 ? 0 : (((d - 1) & 1) == 0 ? d + 1 : d - 1);
    const float2 w = W[(((size_t)rd * cout + cc) * cin + ci) * 16 + 4 * b + a];
    Wt[t] = make_float2(w.x, -w.y);
}

// Adam (Kingma and Ba) on the FP32 master weights; writes the BF16-rounded copy used by the layers
__global__ void k_nn_adam(int n, float *__restrict__ w, const float *__restrict__ grad, float gscale,
                          float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                          float c2, float *__restrict__ wq) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gr = grad[t] * gscale;
    const float mt = b1 * m[t] + (1.f - b1) * gr;
    const float vt = b2 * v[t] + (1.f - b2) * gr * gr;
    m[t] = mt;
    v[t] = vt;
    const float p = w[t] - lr * (mt / c1) / (sqrtf(vt / c2) + eps);
    w[t] = p;
    wq[t] = __bfloat162float(__float2bfloat16(p));
}

__global__ void k_nn_round(int n, const float *__restrict__ w, float *__restrict__ wq) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) wq[t] = __bfloat162float(__float2bfloat16(w[t]));
}

// ---------------------------------------------------------------- MFMA layer
// For a tile of 16 sites a layer is the real GEMM
//   [out_r; out_i] (2M x 48) = [[W_r, -W_i], [W_i, W_r]] (2M x 2K) * [T_r; T_i] (2K x 48)
// with rows (re/im, c', alpha), M = 4 c_out; reduction index (re/im, d, c, beta), K = 36 c_in;
// columns (site, colour).  The transported inputs T are written to LDS in BF16, the weights
// are pre-arranged in MFMA fragment order (BF16), and v_mfma_f32_16x16x16bf16 accumulates in
// FP32.  Fragment layout of that instruction (wave64): lane l holds A[l % 16][4 (l / 16) + q],
// B[4 (l / 16) + q][l % 16] (q = 0..3) and D[4 (l / 16) + q][l % 16].
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct __attribute__((aligned(8))) bf16x4 { __hip_bfloat16 v[4]; };

__host__ __device__ constexpr int nn_k2p(int cin) { return (72 * cin + 15) / 16 * 16; }
__host__ __device__ constexpr int nn_m2p(int cout) { return 8 * cout < 16 ? 16 : (8 * cout + 15) / 16 * 16; }

// Afrag[mt][ks][lane][q] = A[mt*16 + lane%16][ks*16 + 4*(lane/16) + q] (zero padded)
__global__ void k_nn_afrag(int cin, int cout, const float2 *__restrict__ W, __hip_bfloat16 *__restrict__ A) {
    const int K = 36 * cin, K2 = 2 * K, K2P = nn_k2p(cin), M = 4 * cout, M2 = 2 * M, M2P = nn_m2p(cout);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M2P * K2P) return;
    const int q = t % 4, lane = (t / 4) % 64, rest = t / 256;
    const int ks = rest % (K2P / 16), mt = rest / (K2P / 16);
    const int r = mt * 16 + lane % 16, k = ks * 16 + 4 * (lane / 16) + q;
    float v = 0.f;
    if (r < M2 && k < K2) {
        const bool imr = r >= M, imc = k >= K;
        const int rr = imr ? r - M : r, kk = imc ? k - K : k;
        const int co = rr / 4, al = rr % 4, d = kk / (4 * cin), c = (kk / 4) % cin, be = kk % 4;
        const float2 w = W[(((size_t)d * cout + co) * cin + c) * 16 + 4 * al + be];
        v = !imr ? (!imc ? w.x : -w.y) : (!imc ? w.y : w.x);
    }
    A[t] = __float2bfloat16(v);
}

template <int P, int CIN, int COUT>
__global__ void __launch_bounds__(256) k_nn_layer_mfma(GeomDev g, const float2 *__restrict__ in,
                                                      float2 *__restrict__ out, const short4_t *__restrict__ Afrag,
                                                      const typename Prec<P>::S2 *__restrict__ U) {
    constexpr int K = 36 * CIN, K2 = 2 * K, K2P = nn_k2p(CIN), M = 4 * COUT, M2P = nn_m2p(COUT);
    constexpr int NS = 16, NC = 48, BPAD = K2P + 8, KS = K2P / 16, MT = M2P / 16, NT = 3;
    constexpr int B_BYTES = NC * BPAD * 2, D_BYTES = M2P * (NC + 1) * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[B_BYTES > D_BYTES ? B_BYTES : D_BYTES];
    __shared__ int nb_blk[9][NS], nb_slot[9][NS];
    __shared__ float nb_ph[9][NS];
    __hip_bfloat16 (*Bt)[BPAD] = reinterpret_cast<__hip_bfloat16 (*)[BPAD]>(smem);
    float (*Dt)[NC + 1] = reinterpret_cast<float (*)[NC + 1]>(smem);
    int ib, s0, nv;
    nn_tile(g, ib, s0, nv);
    if (ib < 0) return;
    const size_t chan = (size_t)g.V * 12;
    // 0. the neighbours of the tile's sites, once for all channels (missing sites of a short
    // tile repeat the last one; their columns are not stored)
    for (int w = threadIdx.x; w < NS * 9; w += blockDim.x) {
        const int t = w % NS, d = w / NS;
        const int s = s0 + min(t, nv - 1);
        nn_neighbour(g, ib, s, d, nb_blk[d][t], nb_slot[d][t], nb_ph[d][t]);
    }
    __syncthreads();
    // 1. transported inputs of the tile, BF16, column = 3 * site + colour
    for (int w = threadIdx.x; w < NS * 9 * CIN; w += blockDim.x) {
        const int t = w % NS, rest = w / NS, c = rest % CIN, d = rest / CIN;
        const int s = s0 + min(t, nv - 1);
        cx<float> T[12];
        nn_transport_at<P>(T, in + c * chan, g, U, ib, s, d, nb_blk[d][t], nb_slot[d][t], nb_ph[d][t]);
        const int kb = (d * CIN + c) * 4;
        // the four spins of one (colour, re / im) are adjacent in k: one 8-byte store each
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bf16x4 re, im;
#pragma unroll
            for (int be = 0; be < 4; ++be) {
                re.v[be] = __float2bfloat16(T[3 * be + a].r);
                im.v[be] = __float2bfloat16(T[3 * be + a].i);
            }
            *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][kb]) = re;
            *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][K + kb]) = im;
        }
    }
    if constexpr (K2P > K2) {
        for (int w = threadIdx.x; w < NC * (K2P - K2); w += blockDim.x)
            Bt[w / (K2P - K2)][K2 + w % (K2P - K2)] = __float2bfloat16(0.f);
    }
    __syncthreads();
    // 2. MFMA over the reduction index; each wave owns up to three 16x16 output tiles
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = 4 * (lane >> 4);
    float4_t acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
        const int tile = wave + 4 * j;
        if (tile < MT * NT) {
            const int mt = tile / NT, nt = tile % NT;
            const short4_t *Ap = Afrag + (size_t)mt * KS * 64 + lane;
            const int col = nt * 16 + (lane & 15);
            for (int ks = 0; ks < KS; ++ks) {
                const short4_t a = Ap[(size_t)ks * 64];
                const short4_t b = *reinterpret_cast<const short4_t *>(&Bt[col][ks * 16 + kq]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int tile = wave + 4 * j;
        if (tile < MT * NT) {
            const int mt = tile / NT, nt = tile % NT, col = nt * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) Dt[mt * 16 + kq + q][col] = acc[j][q];
        }
    }
    __syncthreads();
    // 3. complex outputs: out[c'](site)[alpha][a] = D[c' 4 + alpha][col] + i D[M + c' 4 + alpha][col]
    for (int w = threadIdx.x; w < NS * COUT * 12; w += blockDim.x) {
        const int t = w % NS, rest = w / NS, comp = rest % 12, co = rest / 12;
        const int r = co * 4 + comp / 3, col = 3 * t + comp % 3;
        if (t < nv) out[co * chan + ((size_t)ib * 12 + comp) * g.Vb + s0 + t] = make_float2(Dt[r][col], Dt[M + r][col]);
    }
}

// The same layer for 8 input channels, with the reduction index taken in chunks of two
// transport directions (128 rows: re and im of 2 directions x 8 channels x 4 spins).  A chunk
// is one transport per thread, all loads in flight together, written to a 13 KB LDS tile
// that the MFMA consumes before the next chunk; the accumulators stay in registers.  The
// small LDS footprint lets about five workgroups share a CU.
template <int P, int COUT>
__global__ void __launch_bounds__(256) k_nn_layer8_mfma(GeomDev g, const float2 *__restrict__ in,
                                                       float2 *__restrict__ out, const short4_t *__restrict__ Afrag,
                                                       const typename Prec<P>::S2 *__restrict__ U) {
    constexpr int CIN = 8, K = 36 * CIN, K2P = nn_k2p(CIN), M = 4 * COUT, M2P = nn_m2p(COUT);
    constexpr int NS = 16, NC = 48, KS = K2P / 16, MT = M2P / 16, NT = 3;
    constexpr int CR = 128, BPAD = CR + 8;  // rows of a chunk (local: re 0..63, im 64..127)
    static_assert(K2P == 2 * K && K % 16 == 0, "8 input channels fill whole k-tiles");
    __shared__ __attribute__((aligned(16))) __hip_bfloat16 Bt[NC][BPAD];
    __shared__ float Dt[M2P][NC + 1];
    __shared__ int nb_blk[9][NS], nb_slot[9][NS];
    __shared__ float nb_ph[9][NS];
    int ib, s0, nv;
    nn_tile(g, ib, s0, nv);
    if (ib < 0) return;
    const size_t chan = (size_t)g.V * 12;
    for (int w = threadIdx.x; w < NS * 9; w += blockDim.x) {
        const int t = w % NS, d = w / NS;
        const int s = s0 + min(t, nv - 1);
        nn_neighbour(g, ib, s, d, nb_blk[d][t], nb_slot[d][t], nb_ph[d][t]);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = 4 * (lane >> 4);
    float4_t acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    for (int d0 = 0; d0 < 9; d0 += 2) {
        const int nd = d0 == 8 ? 1 : 2;
        // transports of directions d0, d0 + 1 for all channels: one per thread
        for (int w = threadIdx.x; w < NS * CIN * nd; w += blockDim.x) {
            const int t = w % NS, c = (w / NS) % CIN, dd = w / (NS * CIN), d = d0 + dd;
            const int s = s0 + min(t, nv - 1);
            cx<float> T[12];
            nn_transport_at<P>(T, in + c * chan, g, U, ib, s, d, nb_blk[d][t], nb_slot[d][t], nb_ph[d][t]);
            const int lr = (dd * CIN + c) * 4;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                bf16x4 re, im;
#pragma unroll
                for (int be = 0; be < 4; ++be) {
                    re.v[be] = __float2bfloat16(T[3 * be + a].r);
                    im.v[be] = __float2bfloat16(T[3 * be + a].i);
                }
                *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][lr]) = re;
                *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][64 + lr]) = im;
            }
        }
        __syncthreads();
        // k-tiles of the chunk: re rows of d0 (global tile 2 d0 + lt), im rows (K / 16 + 2 d0 + lt)
        const int ntile = 2 * nd;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int tile = wave + 4 * j;
            if (tile < MT * NT) {
                const int mt = tile / NT, nt = tile % NT, col = nt * 16 + (lane & 15);
                const short4_t *Ap = Afrag + (size_t)mt * KS * 64 + lane;
                for (int lt = 0; lt < ntile; ++lt) {
                    const short4_t a_re = Ap[(size_t)(2 * d0 + lt) * 64];
                    const short4_t b_re = *reinterpret_cast<const short4_t *>(&Bt[col][lt * 16 + kq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_re, b_re, acc[j], 0, 0, 0);
                    const short4_t a_im = Ap[(size_t)(K / 16 + 2 * d0 + lt) * 64];
                    const short4_t b_im = *reinterpret_cast<const short4_t *>(&Bt[col][64 + lt * 16 + kq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_im, b_im, acc[j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int tile = wave + 4 * j;
        if (tile < MT * NT) {
            const int mt = tile / NT, nt = tile % NT, col = nt * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) Dt[mt * 16 + kq + q][col] = acc[j][q];
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < NS * COUT * 12; w += blockDim.x) {
        const int t = w % NS, rest = w / NS, comp = rest % 12, co = rest / 12;
        const int r = co * 4 + comp / 3, col = 3 * t + comp % 3;
        if (t < nv) out[co * chan + ((size_t)ib * 12 + comp) * g.Vb + s0 + t] = make_float2(Dt[r][col], Dt[M + r][col]);
    }
}

// ---------------------------------------------------------------- launchers
template <int P>
static void nn_layer_p(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const float2 *W) {
    using S2 = typename Prec<P>::S2;
    dim3 grid((unsigned)((c->V + 255) / 256), (unsigned)cout);
    const S2 *U = (const S2 *)c->Uin;
    if (cin == 1 && cout == 8)
        k_nn_layer<P, 1, 8><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, U);
    else if (cin == 8 && cout == 8)
        k_nn_layer<P, 8, 8><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, U);
    else if (cin == 8 && cout == 1)
        k_nn_layer<P, 8, 1><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, U);
}

template <int P>
static void nn_layer_mfma_p(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const void *Af) {
    using S2 = typename Prec<P>::S2;
    const unsigned grid = nn_grid(c);
    const S2 *U = (const S2 *)c->Uin;
    const short4_t *A = (const short4_t *)Af;
    if (cin == 1 && cout == 8)
        k_nn_layer_mfma<P, 1, 8><<<grid, 256, 0, c->stream>>>(c->g, in, out, A, U);
    else if (cin == 8 && cout == 8)
        k_nn_layer8_mfma<P, 8><<<grid, 256, 0, c->stream>>>(c->g, in, out, A, U);
    else if (cin == 8 && cout == 1)
        k_nn_layer8_mfma<P, 1><<<grid, 256, 0, c->stream>>>(c->g, in, out, A, U);
}

size_t nn_afrag_elems(int cin, int cout) { return (size_t)nn_m2p(cout) * nn_k2p(cin); }

void launch_nn_afrag(Ctx *c, int cin, int cout, const float2 *W, void *A) {
    const int n = (int)nn_afrag_elems(cin, cout);
    k_nn_afrag<<<(n + 255) / 256, 256, 0, c->stream>>>(cin, cout, W, (__hip_bfloat16 *)A);
}

void launch_nn_layer_mfma(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const void *A) {
    switch (c->prm.prec_inner) {
    case SAPQ_FP32: nn_layer_mfma_p<SAPQ_FP32>(c, cin, cout, in, out, A); break;
    case SAPQ_FP16: nn_layer_mfma_p<SAPQ_FP16>(c, cin, cout, in, out, A); break;
    case SAPQ_BF16: nn_layer_mfma_p<SAPQ_BF16>(c, cin, cout, in, out, A); break;
    }
}

void launch_nn_layer(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const float2 *W) {
    switch (c->prm.prec_inner) {
    case SAPQ_FP32: nn_layer_p<SAPQ_FP32>(c, cin, cout, in, out, W); break;
    case SAPQ_FP16: nn_layer_p<SAPQ_FP16>(c, cin, cout, in, out, W); break;
    case SAPQ_BF16: nn_layer_p<SAPQ_BF16>(c, cin, cout, in, out, W); break;
    }
}

void launch_nn_wgrad(Ctx *c, int cin, int cout, const float2 *gout, const float2 *in, float2 *G) {
    dim3 grid(9, (unsigned)cout, (unsigned)cin);
    switch (c->prm.prec_inner) {
    case SAPQ_FP32:
        k_nn_wgrad<SAPQ_FP32><<<grid, 256, 0, c->stream>>>(c->g, cin, cout, gout, in, (const float2 *)c->Uin, G);
        break;
    case SAPQ_FP16:
        k_nn_wgrad<SAPQ_FP16><<<grid, 256, 0, c->stream>>>(c->g, cin, cout, gout, in, (const __half2 *)c->Uin, G);
        break;
    case SAPQ_BF16:
        k_nn_wgrad<SAPQ_BF16><<<grid, 256, 0, c->stream>>>(c->g, cin, cout, gout, in, (const __hip_bfloat162 *)c->Uin, G);
        break;
    }
}

void launch_nn_adjoint_weights(Ctx *c, int cin, int cout, const float2 *W, float2 *Wt) {
    const int n = 9 * cin * cout * 16;
    k_nn_adjoint_weights<<<(n + 255) / 256, 256, 0, c->stream>>>(cin, cout, W, Wt);
}

void launch_nn_adam(Ctx *c, int n, float *w, const float *grad, float gscale, float *m, float *v, float lr, int t,
                    float *wq) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_nn_adam<<<(n + 255) / 256, 256, 0, c->stream>>>(n, w, grad, gscale, m, v, lr, b1, b2, eps, c1, c2, wq);
}

void launch_nn_round(Ctx *c, int n, const float *w, float *wq) {
    k_nn_round<<<(n + 255) / 256, 256, 0, c->stream>>>(n, w, wq);
}

}  // namespace sapq
