// Learned gauge-covariant preconditioner stage: linear parallel-transport convolution
// layers, their adjoints and weight gradients, and the Adam update.
//
// A layer maps c_in spinor channels to c_out:
//   out[c'](n) = sum_{d=0..8} sum_c W[d][c'][c] (T_d in[c])(n),  W[d][c'][c] a 4x4 complex spin matrix,
//   T_0 = 1, T_{1+2mu} psi(n) = U_mu(n) psi(n+mu), T_{2+2mu} psi(n) = U_mu(n-mu)^+ psi(n-mu),
// with the fermion boundary sign on hops that wrap.  Activations are FP32.  A one-channel
// activation is a spinor field in the solver's layout ([NB][12][Vb]); an NN_C-channel one is
// site-major, one record of NN_C x 12 complex per site i = ib Vb + s, so that a transport
// reads all channels of a neighbour as one contiguous record.  The forward pass uses the
// weights rounded to BF16; Adam keeps an FP32 master copy.  Records hold FP32 values on the
// FP32 path and BF16 values on the MFMA path, whose contraction rounds its inputs to BF16
// anyway (the transports and sums stay FP32).  Inside a record the channels are interleaved
// per 16-byte piece: piece k of channel c (components 2k, 2k + 1 in FP32, 4k .. 4k + 3 in
// BF16) sits at piece index (K i + k) NN_C + c (K = 6 or 3), so the 8 channel threads of a
// site read 128 contiguous bytes per load instruction.
#include "sitecore.h"

namespace sapq {

static_assert(NN_C == 8, "the layer kernels are written for 8 hidden channels");

// ---------------------------------------------------------------- activations
enum { REC_F32 = 0, REC_BF16 = 1 };  // value type of the 8-channel activation records

__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ unsigned bf16_pack(float lo, float hi) {
    const __hip_bfloat16 a = __float2bfloat16(lo), b = __float2bfloat16(hi);  // round to nearest even
    return (unsigned)*reinterpret_cast<const unsigned short *>(&a) |
           ((unsigned)*reinterpret_cast<const unsigned short *>(&b) << 16);
}

template <int RT>
__device__ __forceinline__ void load_rec(cx<float> t[12], const void *__restrict__ f, long i, int nch, int c) {
    if constexpr (RT == REC_F32) {
        const float4 *p = reinterpret_cast<const float4 *>(f) + (size_t)i * 6 * nch + c;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const float4 v = p[k * nch];
            t[2 * k] = cx<float>{v.x, v.y};
            t[2 * k + 1] = cx<float>{v.z, v.w};
        }
    } else {
        const uint4 *p = reinterpret_cast<const uint4 *>(f) + (size_t)i * 3 * nch + c;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint4 v = p[k * nch];
            t[4 * k] = cx<float>{bf16_lo(v.x), bf16_hi(v.x)};
            t[4 * k + 1] = cx<float>{bf16_lo(v.y), bf16_hi(v.y)};
            t[4 * k + 2] = cx<float>{bf16_lo(v.z), bf16_hi(v.z)};
            t[4 * k + 3] = cx<float>{bf16_lo(v.w), bf16_hi(v.w)};
        }
    }
}

template <int RT>
__device__ __forceinline__ void store_rec(void *__restrict__ f, long i, int nch, int c, const cx<float> t[12]) {
    if constexpr (RT == REC_F32) {
        float4 *p = reinterpret_cast<float4 *>(f) + (size_t)i * 6 * nch + c;
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k * nch] = make_float4(t[2 * k].r, t[2 * k].i, t[2 * k + 1].r, t[2 * k + 1].i);
    } else {
        uint4 *p = reinterpret_cast<uint4 *>(f) + (size_t)i * 3 * nch + c;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            p[k * nch] = make_uint4(bf16_pack(t[4 * k].r, t[4 * k].i), bf16_pack(t[4 * k + 1].r, t[4 * k + 1].i),
                                    bf16_pack(t[4 * k + 2].r, t[4 * k + 2].i), bf16_pack(t[4 * k + 3].r, t[4 * k + 3].i));
    }
}

// channel c of an nch-channel activation at site (ib, s)
template <int RT>
__device__ __forceinline__ void load_chan(cx<float> t[12], const float2 *__restrict__ f, int nch, const GeomDev &g,
                                          int ib, int s, int c) {
    if (nch == 1)
        load_spinor(t, f, g, ib, s);
    else
        load_rec<RT>(t, f, (long)ib * g.Vb + s, nch, c);
}

template <int RT>
__device__ __forceinline__ void store_chan(float2 *__restrict__ f, int nch, const GeomDev &g, int ib, int s, int c,
                                           const cx<float> t[12]) {
    if (nch == 1)
        store_spinor(f, g, ib, s, t);
    else
        store_rec<RT>(f, (long)ib * g.Vb + s, nch, c, t);
}

// ---------------------------------------------------------------- transports
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

// Transport links L[i][d - 1] (3x3 complex, FP32), with (T_d psi)(i) = L[i][d - 1] psi(nbr_d(i)):
// U_mu(n) for d = 1 + 2 mu and U_mu(n - mu)^+ for d = 2 + 2 mu, times the boundary sign of the
// hop.  Built once per gauge field from the links in storage precision, so a transport reads
// one contiguous link of its own site instead of gathering the backward neighbour's.
template <int P>
__global__ void k_nn_links(GeomDev g, const typename Prec<P>::S2 *__restrict__ U, float2 *__restrict__ L) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)g.V * 8) return;
    const long i = t >> 3;
    const int d = 1 + (int)(t & 7), mu = (d - 1) >> 1;
    const bool fwd = ((d - 1) & 1) == 0;
    const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    int nb, ns;
    float ph;
    nn_neighbour(g, ib, s, d, nb, ns, ph);
    cx<float> u[9];
    if (fwd)
        load_link(u, U, g, ib, s, mu);
    else
        load_link(u, U, g, nb, ns, mu);
    float2 *o = L + (size_t)t * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cx<float> e = fwd ? u[3 * a + b] : conjx(u[3 * b + a]);
            o[3 * a + b] = make_float2(ph * e.r, ph * e.i);
        }
}

__device__ __forceinline__ void nn_link(cx<float> u[9], const float2 *__restrict__ L, long i, int d) {
    const float2 *p = L + ((size_t)i * 8 + d - 1) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const float2 v = p[e];
        u[e] = cx<float>{v.x, v.y};
    }
}

// (T_d f[c])(ib, s) for channel c of an nch-channel activation, the neighbour (nb, ns) of
// (ib, s) for d already known
template <int RT>
__device__ __forceinline__ void nn_transport(cx<float> t[12], const float2 *__restrict__ f, int nch, const GeomDev &g,
                                             const float2 *__restrict__ L, int ib, int s, int d, int c, int nb, int ns) {
    if (d == 0) {
        load_chan<RT>(t, f, nch, g, ib, s, c);
        return;
    }
    cx<float> p[12], u[9];
    load_chan<RT>(p, f, nch, g, nb, ns, c);
    nn_link(u, L, (long)ib * g.Vb + s, d);
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        cx<float> h[3] = {p[3 * be], p[3 * be + 1], p[3 * be + 2]}, o[3];
        su3_mul(o, u, h, false);
#pragma unroll
        for (int a = 0; a < 3; ++a) t[3 * be + a] = o[a];
    }
}

// (T_d in)(ib, s) for a one-channel input in the solver's layout and storage type S2
template <typename S2>
__device__ __forceinline__ void nn_transport1(cx<float> t[12], const S2 *__restrict__ in, const GeomDev &g,
                                              const float2 *__restrict__ L, int ib, int s, int d, int nb, int ns) {
    if (d == 0) {
        load_spinor(t, in, g, ib, s);
        return;
    }
    cx<float> p[12], u[9];
    load_spinor(p, in, g, nb, ns);
    nn_link(u, L, (long)ib * g.Vb + s, d);
#pragma unroll
    for (int be = 0; be < 4; ++be) {
        cx<float> h[3] = {p[3 * be], p[3 * be + 1], p[3 * be + 2]}, o[3];
        su3_mul(o, u, h, false);
#pragma unroll
        for (int a = 0; a < 3; ++a) t[3 * be + a] = o[a];
    }
}

// ---------------------------------------------------------------- FP32 layer, weight gradient
// out[c'] for one output channel c' = blockIdx.y; weights W[9][COUT][CIN][16] complex (float2)
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_nn_layer(GeomDev g, const float2 *__restrict__ in, float2 *__restrict__ out,
                                                 const float2 *__restrict__ W, const float2 *__restrict__ L) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int co = blockIdx.y;
    if (i >= g.V) return;
    const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
    for (int d = 0; d < 9; ++d) {
        int nb, ns;
        float ph;
        nn_neighbour(g, ib, s, d, nb, ns, ph);
#pragma unroll 1
        for (int ci = 0; ci < CIN; ++ci) {
            cx<float> t[12];
            nn_transport<REC_F32>(t, in, CIN, g, L, ib, s, d, ci, nb, ns);
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
    store_chan<REC_F32>(out, COUT, g, ib, s, co, acc);
}

// G[d][c'][c] (16 complex) = sum_n sum_a gout[c'](n)[al][a] conj((T_d in[c])(n)[be][a]), added to G.
// One workgroup per (d, c', c); a fixed-order tree finishes the sum.
template <int RT>
__global__ void __launch_bounds__(256) k_nn_wgrad(GeomDev g, int cin, int cout, const float2 *__restrict__ gout,
                                                 const float2 *__restrict__ in, const float2 *__restrict__ L,
                                                 float2 *__restrict__ G) {
    __shared__ float sm[32][257];
    const int d = blockIdx.x, co = blockIdx.y, ci = blockIdx.z;
    float acc[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[k] = 0.f;
    for (long i = threadIdx.x; i < g.V; i += blockDim.x) {
        const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
        int nb, ns;
        float ph;
        nn_neighbour(g, ib, s, d, nb, ns, ph);
        cx<float> t[12], go[12];
        nn_transport<RT>(t, in, cin, g, L, ib, s, d, ci, nb, ns);
        load_chan<RT>(go, gout, cout, g, ib, s, co);
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

// ---------------------------------------------------------------- MFMA layers
// For a tile of NN_TILE sites a layer is the real GEMM
//   [out_r; out_i] (2M x 3 NN_TILE) = [[W_r, -W_i], [W_i, W_r]] (2M x 2K) * [T_r; T_i] (2K x 3 NN_TILE)
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


// Tile of NN_TILE sites of a layer workgroup.  Workgroups are dealt to the 8 XCDs in turn;
// with a grid that is a multiple of 8, XCD x takes the x-th eighth of the tiles, and tiles
// run through whole blocks in lexicographic block order, so that the neighbours a tile reads
// (mostly in the same block or the next one) were fetched into the same L2.  ib < 0 marks a
// workgroup past the last tile; n_valid sites of the tile exist (blocks need not hold a
// multiple of NN_TILE sites).
constexpr int NN_TILE = 32;

__device__ __forceinline__ void nn_tile(const GeomDev &g, int &ib, int &s0, int &n_valid) {
    const long vt = xcd_site_base(1);
    const int tpb = (g.Vb + NN_TILE - 1) / NN_TILE;
    const long bl = vt / tpb;
    ib = bl < g.NB ? g.zord_blk[bl] : -1;
    s0 = (int)(vt - bl * tpb) * NN_TILE;
    n_valid = min(NN_TILE, g.Vb - s0);
}

unsigned nn_grid(const Ctx *c) {
    const long tiles = (long)c->g.NB * ((c->g.Vb + NN_TILE - 1) / NN_TILE);
    return (unsigned)((tiles + N_XCD - 1) / N_XCD * N_XCD);
}

// Output tiles of a wave: with four 16-row tiles (c_out = 8) wave w owns row tile w and all
// column tiles, so it reads each A fragment once for all of them; with one row tile (c_out = 1)
// the waves share it and take every fourth column tile.
template <int MT, int NT> struct WaveTiles {
    static_assert(MT == 4 || MT == 1, "four row tiles or one");
    static constexpr int N = MT == 4 ? NT : (NT + 3) / 4;
    __device__ static int mt(int wave) { return MT == 4 ? wave : 0; }
    __device__ static int nt(int wave, int j) { return MT == 4 ? j : wave + 4 * j; }
};

// the tile of D (rows (re/im, c', alpha), columns (site, colour)) to the output activation
template <int COUT, int RT, int POUT>
__device__ __forceinline__ void nn_store_tile(void *__restrict__ out_, const GeomDev &g, int ib, int s0, int nv,
                                              const float (*Dt)[3 * NN_TILE + 1]) {
    constexpr int M = 4 * COUT;
    float2 *out = reinterpret_cast<float2 *>(out_);
    if constexpr (COUT == 1) {
        // one channel: the solver's spinor layout in storage precision POUT
        using S2 = typename Prec<POUT>::S2;
        S2 *o = reinterpret_cast<S2 *>(out_);
        for (int w = threadIdx.x; w < NN_TILE * 12; w += blockDim.x) {
            const int t = w % NN_TILE, comp = w / NN_TILE, r = comp / 3, col = 3 * t + comp % 3;
            if (t < nv) st(o + ((size_t)ib * 12 + comp) * g.Vb + s0 + t, cx<float>{Dt[r][col], Dt[M + r][col]});
        }
    } else if constexpr (RT == REC_F32) {
        // the tile's records are contiguous: one coalesced sweep of 16-byte pieces (two
        // components of one channel each, in the record's interleaved order)
        float4 *o = reinterpret_cast<float4 *>(out) + ((size_t)ib * g.Vb + s0) * 6 * COUT;
        for (int w = threadIdx.x; w < nv * 6 * COUT; w += blockDim.x) {
            const int co = w % COUT, k = (w / COUT) % 6, t = w / (6 * COUT);
            const int r0 = co * 4 + (2 * k) / 3, c0 = 3 * t + (2 * k) % 3;
            const int r1 = co * 4 + (2 * k + 1) / 3, c1 = 3 * t + (2 * k + 1) % 3;
            o[w] = make_float4(Dt[r0][c0], Dt[M + r0][c0], Dt[r1][c1], Dt[M + r1][c1]);
        }
    } else {
        // BF16 records: pieces of four components of one channel
        uint4 *o = reinterpret_cast<uint4 *>(out) + ((size_t)ib * g.Vb + s0) * 3 * COUT;
        for (int w = threadIdx.x; w < nv * 3 * COUT; w += blockDim.x) {
            const int co = w % COUT, k = (w / COUT) % 3, t = w / (3 * COUT);
            unsigned q[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int comp = 4 * k + j, r = co * 4 + comp / 3, col = 3 * t + comp % 3;
                q[j] = bf16_pack(Dt[r][col], Dt[M + r][col]);
            }
            o[w] = make_uint4(q[0], q[1], q[2], q[3]);
        }
    }
}

// the transported spinor T (12 complex) of tile column group t, written as BF16 to rows
// kre.. (real parts) and kim.. (imaginary parts) of the B tile: the four spins of one
// (colour, re / im) are adjacent in k, one 8-byte store each
template <int BPAD>
__device__ __forceinline__ void nn_put_b(__hip_bfloat16 (*Bt)[BPAD], int t, int kre, int kim, const cx<float> T[12]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bf16x4 re, im;
#pragma unroll
        for (int be = 0; be < 4; ++be) {
            re.v[be] = __float2bfloat16(T[3 * be + a].r);
            im.v[be] = __float2bfloat16(T[3 * be + a].i);
        }
        *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][kre]) = re;
        *reinterpret_cast<bf16x4 *>(&Bt[3 * t + a][kim]) = im;
    }
}

// One input channel (the first layer, and the adjoint of the last): the whole reduction
// index (9 directions x 4 spins, re / im) is one LDS tile.
// (skip: nullable flag read at the start; nonzero leaves the output untouched, for sources a
// batched solve has finished)
template <int COUT, int RT, int PIN>
__global__ void __launch_bounds__(256) k_nn_layer1_mfma(GeomDev g, const typename Prec<PIN>::S2 *__restrict__ in,
                                                       float2 *__restrict__ out, const short4_t *__restrict__ Afrag,
                                                       const float2 *__restrict__ L, const int *__restrict__ skip) {
    if (skip && *skip) return;
    constexpr int K = 36, K2 = 2 * K, K2P = nn_k2p(1), M2P = nn_m2p(COUT);
    constexpr int NS = NN_TILE, NC = 3 * NS, BPAD = K2P + 8, KS = K2P / 16, MT = M2P / 16, NT = NC / 16;
    using WT = WaveTiles<MT, NT>;
    constexpr int B_BYTES = NC * BPAD * 2, D_BYTES = M2P * (NC + 1) * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[B_BYTES > D_BYTES ? B_BYTES : D_BYTES];
    __shared__ int nb_blk[9][NS], nb_slot[9][NS];
    __hip_bfloat16 (*Bt)[BPAD] = reinterpret_cast<__hip_bfloat16 (*)[BPAD]>(smem);
    float (*Dt)[NC + 1] = reinterpret_cast<float (*)[NC + 1]>(smem);
    int ib, s0, nv;
    nn_tile(g, ib, s0, nv);
    if (ib < 0) return;
    // 0. the neighbours of the tile's sites (missing sites of a short tile repeat the last
    // one; their columns are not stored)
    for (int w = threadIdx.x; w < NS * 9; w += blockDim.x) {
        const int t = w % NS, d = w / NS;
        float ph;
        nn_neighbour(g, ib, s0 + min(t, nv - 1), d, nb_blk[d][t], nb_slot[d][t], ph);
    }
    __syncthreads();
    // 1. transported inputs, column = 3 * site + colour
    for (int w = threadIdx.x; w < NS * 9; w += blockDim.x) {
        const int t = w % NS, d = w / NS;
        cx<float> T[12];
        nn_transport1(T, in, g, L, ib, s0 + min(t, nv - 1), d, nb_blk[d][t], nb_slot[d][t]);
        nn_put_b<BPAD>(Bt, t, 4 * d, K + 4 * d, T);
    }
    for (int w = threadIdx.x; w < NC * (K2P - K2); w += blockDim.x)
        Bt[w / (K2P - K2)][K2 + w % (K2P - K2)] = __float2bfloat16(0.f);
    __syncthreads();
    // 2. MFMA over the reduction index
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kq = 4 * (lane >> 4);
    const short4_t *Ap = Afrag + (size_t)WT::mt(wave) * KS * 64 + lane;
    float4_t acc[WT::N];
#pragma unroll
    for (int j = 0; j < WT::N; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KS; ++ks) {
        const short4_t a = Ap[(size_t)ks * 64];
#pragma unroll
        for (int j = 0; j < WT::N; ++j) {
            const int nt = WT::nt(wave, j);
            if (nt < NT) {
                const short4_t b = *reinterpret_cast<const short4_t *>(&Bt[nt * 16 + (lane & 15)][ks * 16 + kq]);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[j], 0, 0, 0);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < WT::N; ++j) {
        const int nt = WT::nt(wave, j);
        if (nt < NT)
#pragma unroll
            for (int q = 0; q < 4; ++q) Dt[WT::mt(wave) * 16 + kq + q][nt * 16 + (lane & 15)] = acc[j][q];
    }
    __syncthreads();
    // 3. complex outputs: out[c'](site)[alpha][a] = D[c' 4 + alpha][col] + i D[M + c' 4 + alpha][col]
    nn_store_tile<COUT, RT, SAPQ_FP32>(out, g, ib, s0, nv, Dt);
}

// Eight input channels: the reduction index is taken in chunks of two transport directions
// (128 rows: re and im of 2 directions x 8 channels x 4 spins).  In a chunk each thread
// transports one channel of one site along both directions; the eight threads of a site read
// the neighbour's record as one contiguous 768-byte piece.  The MFMA consumes the chunk from
// LDS before the next one; the accumulators stay in registers.
template <int COUT, int RT, int POUT>
__global__ void __launch_bounds__(256, 4) k_nn_layer8_mfma(GeomDev g, const float2 *__restrict__ in,
                                                       void *__restrict__ out, const short4_t *__restrict__ Afrag,
                                                       const float2 *__restrict__ L, const int *__restrict__ skip) {
    if (skip && *skip) return;
    constexpr int CIN = 8, K = 36 * CIN, K2P = nn_k2p(CIN), M2P = nn_m2p(COUT);
    constexpr int NS = NN_TILE, NC = 3 * NS, KS = K2P / 16, MT = M2P / 16, NT = NC / 16;
    constexpr int CR = 128, BPAD = CR + 8;  // rows of a chunk (local: re 0..63, im 64..127)
    static_assert(K2P == 2 * K && K % 16 == 0, "8 input channels fill whole k-tiles");
    static_assert(NS * CIN == 256, "one (site, channel) per thread");
    using WT = WaveTiles<MT, NT>;
    constexpr int B_BYTES = NC * BPAD * 2, D_BYTES = M2P * (NC + 1) * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[B_BYTES > D_BYTES ? B_BYTES : D_BYTES];
    __shared__ int nb_blk[9][NS], nb_slot[9][NS];
    __hip_bfloat16 (*Bt)[BPAD] = reinterpret_cast<__hip_bfloat16 (*)[BPAD]>(smem);
    float (*Dt)[NC + 1] = reinterpret_cast<float (*)[NC + 1]>(smem);
    int ib, s0, nv;
    nn_tile(g, ib, s0, nv);
    if (ib < 0) return;
    for (int w = threadIdx.x; w < NS * 9; w += blockDim.x) {
        const int t = w % NS, d = w / NS;
        float ph;
        nn_neighbour(g, ib, s0 + min(t, nv - 1), d, nb_blk[d][t], nb_slot[d][t], ph);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kq = 4 * (lane >> 4);
    const int c = threadIdx.x % CIN, t = threadIdx.x / CIN, s = s0 + min(t, nv - 1);
    const short4_t *Ap = Afrag + (size_t)WT::mt(wave) * KS * 64 + lane;
    float4_t acc[WT::N];
#pragma unroll
    for (int j = 0; j < WT::N; ++j) acc[j] = float4_t{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
    // unrolled, so that both transports of a chunk have their loads in flight together
#pragma unroll
    for (int d0 = 0; d0 < 9; d0 += 2) {
        const int nd = d0 == 8 ? 1 : 2;
        cx<float> T[2][12];
#pragma unroll
        for (int dd = 0; dd < 2; ++dd)
            if (dd < nd) nn_transport<RT>(T[dd], in, CIN, g, L, ib, s, d0 + dd, c, nb_blk[d0 + dd][t], nb_slot[d0 + dd][t]);
#pragma unroll
        for (int dd = 0; dd < 2; ++dd)
            if (dd < nd) nn_put_b<BPAD>(Bt, t, (dd * CIN + c) * 4, 64 + (dd * CIN + c) * 4, T[dd]);
        __syncthreads();
        // k-tiles of the chunk: re rows of d0 (global tile 2 d0 + lt), im rows (K / 16 + 2 d0 + lt)
#pragma unroll
        for (int lt = 0; lt < 2 * nd; ++lt) {
            const short4_t a_re = Ap[(size_t)(2 * d0 + lt) * 64];
            const short4_t a_im = Ap[(size_t)(K / 16 + 2 * d0 + lt) * 64];
#pragma unroll
            for (int j = 0; j < WT::N; ++j) {
                const int nt = WT::nt(wave, j);
                if (nt < NT) {
                    const int col = nt * 16 + (lane & 15);
                    const short4_t b_re = *reinterpret_cast<const short4_t *>(&Bt[col][lt * 16 + kq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_re, b_re, acc[j], 0, 0, 0);
                    const short4_t b_im = *reinterpret_cast<const short4_t *>(&Bt[col][64 + lt * 16 + kq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_im, b_im, acc[j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < WT::N; ++j) {
        const int nt = WT::nt(wave, j);
        if (nt < NT)
#pragma unroll
            for (int q = 0; q < 4; ++q) Dt[WT::mt(wave) * 16 + kq + q][nt * 16 + (lane & 15)] = acc[j][q];
    }
    __syncthreads();
    nn_store_tile<COUT, RT, POUT>(out, g, ib, s0, nv, Dt);
}

// ---------------------------------------------------------------- launchers
size_t nn_link_elems(const Ctx *c) { return (size_t)c->V * 72; }

void launch_nn_links(Ctx *c) {
    const long n = (long)c->V * 8;
    const unsigned grid = (unsigned)((n + 255) / 256);
    switch (c->prm.prec_inner) {
    case SAPQ_FP32: k_nn_links<SAPQ_FP32><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)c->Uin, c->nn_L); break;
    case SAPQ_FP16: k_nn_links<SAPQ_FP16><<<grid, 256, 0, c->stream>>>(c->g, (const __half2 *)c->Uin, c->nn_L); break;
    case SAPQ_BF16:
        k_nn_links<SAPQ_BF16><<<grid, 256, 0, c->stream>>>(c->g, (const __hip_bfloat162 *)c->Uin, c->nn_L);
        break;
    }
}

size_t nn_afrag_elems(int cin, int cout) { return (size_t)nn_m2p(cout) * nn_k2p(cin); }

void launch_nn_afrag(Ctx *c, int cin, int cout, const float2 *W, void *A) {
    const int n = (int)nn_afrag_elems(cin, cout);
    k_nn_afrag<<<(n + 255) / 256, 256, 0, c->stream>>>(cin, cout, W, (__hip_bfloat16 *)A);
}

void launch_nn_layer_mfma(Ctx *c, int cin, int cout, const void *in, void *out, const void *Af, int p_in, int p_out,
                          const int *skip) {
    const unsigned grid = nn_grid(c);
    const short4_t *A = (const short4_t *)Af;
    const float2 *L = c->nn_L;
    if (cin == 1 && cout == NN_C) {
        switch (p_in) {
        case SAPQ_FP32:
            k_nn_layer1_mfma<NN_C, REC_BF16, SAPQ_FP32><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)in, (float2 *)out, A, L, skip);
            break;
        case SAPQ_FP16:
            k_nn_layer1_mfma<NN_C, REC_BF16, SAPQ_FP16><<<grid, 256, 0, c->stream>>>(c->g, (const __half2 *)in, (float2 *)out, A, L, skip);
            break;
        case SAPQ_BF16:
            k_nn_layer1_mfma<NN_C, REC_BF16, SAPQ_BF16><<<grid, 256, 0, c->stream>>>(
                c->g, (const __hip_bfloat162 *)in, (float2 *)out, A, L, skip);
            break;
        }
    } else if (cin == NN_C && cout == NN_C) {
        k_nn_layer8_mfma<NN_C, REC_BF16, SAPQ_FP32><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)in, out, A, L, skip);
    } else if (cin == NN_C && cout == 1) {
        switch (p_out) {
        case SAPQ_FP32:
            k_nn_layer8_mfma<1, REC_BF16, SAPQ_FP32><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)in, out, A, L, skip);
            break;
        case SAPQ_FP16:
            k_nn_layer8_mfma<1, REC_BF16, SAPQ_FP16><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)in, out, A, L, skip);
            break;
        case SAPQ_BF16:
            k_nn_layer8_mfma<1, REC_BF16, SAPQ_BF16><<<grid, 256, 0, c->stream>>>(c->g, (const float2 *)in, out, A, L, skip);
            break;
        }
    }
}

void launch_nn_layer(Ctx *c, int cin, int cout, const float2 *in, float2 *out, const float2 *W) {
    dim3 grid((unsigned)((c->V + 255) / 256), (unsigned)cout);
    if (cin == 1 && cout == NN_C)
        k_nn_layer<1, NN_C><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, c->nn_L);
    else if (cin == NN_C && cout == NN_C)
        k_nn_layer<NN_C, NN_C><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, c->nn_L);
    else if (cin == NN_C && cout == 1)
        k_nn_layer<NN_C, 1><<<grid, 256, 0, c->stream>>>(c->g, in, out, W, c->nn_L);
}

void launch_nn_wgrad(Ctx *c, int cin, int cout, const float2 *gout, const float2 *in, float2 *G, bool bf16_records) {
    dim3 grid(9, (unsigned)cout, (unsigned)cin);
    if (bf16_records)
        k_nn_wgrad<REC_BF16><<<grid, 256, 0, c->stream>>>(c->g, cin, cout, gout, in, c->nn_L, G);
    else
        k_nn_wgrad<REC_F32><<<grid, 256, 0, c->stream>>>(c->g, cin, cout, gout, in, c->nn_L, G);
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
