// Per-site device building blocks shared by the operator, SAP and batched kernels:
// four lanes per site, lane j = direction mu, quad reductions, row-split clover.
#pragma once

#include "sapq_impl.h"

namespace sapq {

// ================================================================ site index
// lexicographic site index of internal site (ib, s)
__device__ __forceinline__ long lex_site(const GeomDev &g, int ib, int s) {
    int bl = g.blk_lex[ib], l = g.slot_lex[s];
    long n = 0, stride = 1;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        int bc = bl % g.nbk[m];
        bl /= g.nbk[m];
        int c = l % g.B[m];
        l /= g.B[m];
        n += (long)(bc * g.B[m] + c) * stride;
        stride *= (long)g.B[m] * g.nbk[m];
    }
    return n;
}


// ================================================================ XCD-aware site order
// Workgroups are dealt to the 8 XCDs in turn, each XCD with its own L2.  For a grid that is
// a multiple of 8, XCD x gets workgroups x, x + 8, ...; mapping them to the x-th eighth of
// the sites keeps the sites an XCD works on (and most of their neighbours) contiguous.
constexpr int N_XCD = 8;

__device__ __forceinline__ long xcd_site_base(int sites_per_wg) {
    const unsigned per = gridDim.x / N_XCD;
    const unsigned v = (blockIdx.x % N_XCD) * per + blockIdx.x / N_XCD;
    return (long)v * sites_per_wg;
}

// ================================================================ four lanes per site
// A site is handled by a group of four adjacent lanes; lane j takes direction mu = j
// (its forward and its backward hop), the four partial hopping sums are added with a
// quad butterfly, and lane j then owns spin j (components 3j..3j+2) of the result.
// The spin projection is written with per-lane coefficients so that the four lanes
// run the same instructions:
//   (1 - s gamma_mu) W psi:  h0 = p0 + c0 p[a0],  h1 = p1 + c1 p[a1],  g = W h,
//   spins (0, 1) += (g0, g1),  spin a0 += conj(c0) g0,  spin a1 += conj(c1) g1,
// with a0 = 3, a1 = 2 for mu = x, y and a0 = 2, a1 = 3 for mu = z, t, and (c0, c1) =
// (s i, s i), (s, -s), (s i, -s i), (-s, -s) for mu = x, y, z, t.
template <typename C> struct LaneDir {
    int mu;
    bool a0_is3;
    cx<C> c0, c1;  // forward hop (s = +1); the backward hop uses -c0, -c1
};

template <typename C> __device__ __forceinline__ LaneDir<C> lane_dir(int j) {
    LaneDir<C> d;
    d.mu = j;
    d.a0_is3 = j < 2;
    const C one = C(1), zero = C(0);
    d.c0 = (j == 0 || j == 2) ? cx<C>{zero, one} : (j == 1 ? cx<C>{one, zero} : cx<C>{-one, zero});
    d.c1 = (j == 0) ? cx<C>{zero, one} : (j == 1 ? cx<C>{-one, zero} : (j == 2 ? cx<C>{zero, -one} : cx<C>{-one, zero}));
    return d;
}

template <typename T> __device__ __forceinline__ cx<T> sel(bool p, cx<T> a, cx<T> b) { return {p ? a.r : b.r, p ? a.i : b.i}; }

template <typename C>
__device__ __forceinline__ void lane_hop(cx<C> acc[12], const cx<C> psi[12], const cx<C> u[9], bool dag, cx<C> c0,
                                         cx<C> c1, bool a0_is3, C phase) {
    cx<C> h0[3], h1[3], g0[3], g1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<C> pa0 = sel(a0_is3, psi[9 + a], psi[6 + a]);
        cx<C> pa1 = sel(a0_is3, psi[6 + a], psi[9 + a]);
        h0[a] = cfma(c0, pa0, psi[a]);
        h1[a] = cfma(c1, pa1, psi[3 + a]);
    }
    su3_mul(g0, u, h0, dag);
    su3_mul(g1, u, h1, dag);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<C> q0 = phase * g0[a], q1 = phase * g1[a];
        acc[a] = rfma(phase, g0[a], acc[a]);
        acc[3 + a] = rfma(phase, g1[a], acc[3 + a]);
        cx<C> t0 = cmulc(c0, q0), t1 = cmulc(c1, q1);
        acc[6 + a] = acc[6 + a] + sel(a0_is3, t1, t0);
        acc[9 + a] = acc[9 + a] + sel(a0_is3, t0, t1);
    }
}

// Spinor sources for the hops.
template <typename S2, typename C> struct FieldSrc {  // a field in storage precision
    const S2 *f;
    __device__ __forceinline__ void get(cx<C> psi[12], const GeomDev &g, int ib, int s) const { load_spinor(psi, f, g, ib, s); }
};
struct BlockSrc {  // the float2 [12][Vb] SSOR iterate of the current block (LDS or scratch)
    const float2 *x;
    __device__ __forceinline__ void get(cx<float> psi[12], const GeomDev &g, int, int s) const {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            float2 v = x[c * g.Vb + s];
            psi[c] = {v.x, v.y};
        }
    }
};

enum { HOP_ALL = 0, HOP_IN = 1, HOP_OUT = 2 };

// value of the lane (lane ^ 1) or (lane ^ 2) of the same quad, by DPP quad permutes
template <int CTRL> __device__ __forceinline__ float quad_get(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double quad_get(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int QUAD_XOR1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int QUAD_XOR2 = 0x4E;  // quad_perm [2, 3, 0, 1]

template <typename C> __device__ __forceinline__ void quad_reduce(cx<C> acc[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        acc[c].r += quad_get<QUAD_XOR1>(acc[c].r);
        acc[c].i += quad_get<QUAD_XOR1>(acc[c].i);
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        acc[c].r += quad_get<QUAD_XOR2>(acc[c].r);
        acc[c].i += quad_get<QUAD_XOR2>(acc[c].i);
    }
}

// The two neighbours of a lane (direction j, forward and backward) of site (ib, s).
// nbr16[j][s] packs the forward slot in bits 0..14 and the backward slot in bits 16..30,
// with bit 15 / bit 31 set when that neighbour lies inside the block; outside
// neighbours give the slot in the adjacent block.
struct LaneNbr {
    int s_f, s_b, ib_f, ib_b;
    bool in_f, in_b;
    float ph_f, ph_b;
};

__device__ __forceinline__ LaneNbr lane_nbr(unsigned w, int ib, int bl_f, int bl_b, float bc) {
    LaneNbr n;
    n.s_f = (int)(w & 0x7fffu);
    n.in_f = (w & 0x8000u) != 0;
    n.s_b = (int)((w >> 16) & 0x7fffu);
    n.in_b = (w & 0x80000000u) != 0;
    n.ib_f = n.in_f ? ib : (bl_f & BLK_MASK);
    n.ib_b = n.in_b ? ib : (bl_b & BLK_MASK);
    n.ph_f = (!n.in_f && (bl_f & WRAP_BIT)) ? bc : 1.f;
    n.ph_b = (!n.in_b && (bl_b & WRAP_BIT)) ? bc : 1.f;
    return n;
}

// Lane part of sum_m H_nm psi(m) over the selected neighbours (direction j) of (ib, s),
// followed by the quad reduction: on return every lane of the group holds the full sum.
// Excluded neighbours are read from a valid address and their spinor is set to zero.
// The two links a lane needs: U_j(n) for the forward hop, U_j(n - j) for the backward hop.
template <typename C> struct LaneLinks { cx<C> uf[9], ub[9]; };

template <typename S2, typename C>
__device__ __forceinline__ void lane_links(LaneLinks<C> &l, const GeomDev &g, int ib, int s, int j, const LaneNbr &n,
                                           const S2 *__restrict__ U) {
    load_link(l.uf, U, g, ib, s, j);
    load_link(l.ub, U, g, n.ib_b, n.s_b, j);
}

// Lane part of sum_m H_nm psi(m) over the selected neighbours (direction j) of (ib, s),
// followed by the quad reduction: on return every lane of the group holds the full sum.
// Excluded neighbours are read from a valid address and their spinor is set to zero.
template <int MODE, typename C, typename Src>
__device__ __forceinline__ void quad_hop_apply(cx<C> acc[12], const GeomDev &g, int j, const LaneNbr &n,
                                               const LaneLinks<C> &l, const Src &src) {
    const LaneDir<C> d = lane_dir<C>(j);
    const bool use_f = MODE == HOP_ALL || (MODE == HOP_IN ? n.in_f : !n.in_f);
    const bool use_b = MODE == HOP_ALL || (MODE == HOP_IN ? n.in_b : !n.in_b);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<C>();
    {
        cx<C> pf[12];
        src.get(pf, g, n.ib_f, n.s_f);
#pragma unroll
        for (int c = 0; c < 12; ++c) pf[c] = sel(use_f, pf[c], cxz<C>());
        lane_hop(acc, pf, l.uf, false, d.c0, d.c1, d.a0_is3, C(n.ph_f));
    }
    {
        cx<C> pb[12];
        src.get(pb, g, n.ib_b, n.s_b);
#pragma unroll
        for (int c = 0; c < 12; ++c) pb[c] = sel(use_b, pb[c], cxz<C>());
        lane_hop(acc, pb, l.ub, true, C(-1) * d.c0, C(-1) * d.c1, d.a0_is3, C(n.ph_b));
    }
    quad_reduce(acc);
}

template <int MODE, bool LEAN, typename S2, typename C, typename Src>
__device__ __forceinline__ void quad_hop_sum(cx<C> acc[12], const GeomDev &g, int ib, int s, int j, const LaneNbr &n,
                                             const S2 *__restrict__ U, const Src &src) {
    LaneLinks<C> l;
    lane_links(l, g, ib, s, j, n, U);
    if (LEAN) __builtin_amdgcn_sched_barrier(0);
    quad_hop_apply<MODE>(acc, g, j, n, l, src);
}

// Rows of F(n) owned by lane j (spin j): with k = j >> 1 and hi = j & 1 the lane needs
// rows 3*hi .. 3*hi+2 of chiral block k = [[A, B], [B^+, C]]:
//   hi = 0:  A h_u + B h_l        hi = 1:  B^+ h_u + C h_l
template <typename C> struct LaneClover {
    C dg[3];
    cx<C> h10, h20, h21;  // strict lower triangle of A (hi = 0) or C (hi = 1)
    cx<C> m[9];           // B (hi = 0) or B^+ (hi = 1)
};

template <typename S2, typename C>
__device__ __forceinline__ void lane_clover_load(LaneClover<C> &L, const S2 *__restrict__ F, const GeomDev &g, int ib,
                                                 int s, int j) {
    const int k = j >> 1;
    const bool hi = (j & 1) != 0;
    const S2 *p = F + ((size_t)ib * 2 + k) * 18 * g.Vb + s;
    const cx<C> d01 = ld(p), d23 = ld(p + g.Vb), d45 = ld(p + 2 * (size_t)g.Vb);
    L.dg[0] = hi ? d23.i : d01.r;
    L.dg[1] = hi ? d45.r : d01.i;
    L.dg[2] = hi ? d45.i : d23.r;
    const S2 *ph = p + (size_t)(hi ? 6 : 3) * g.Vb;
    L.h10 = ld(ph);
    L.h20 = ld(ph + g.Vb);
    L.h21 = ld(ph + 2 * (size_t)g.Vb);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int slot = hi ? 9 + 3 * b + a : 9 + 3 * a + b;
            cx<C> v = ld(p + (size_t)slot * g.Vb);
            L.m[3 * a + b] = {v.r, hi ? -v.i : v.i};
        }
}

template <typename C>
__device__ __forceinline__ void lane_clover_apply(cx<C> out[3], const cx<C> h[12], const LaneClover<C> &L, int j) {
    const int k = j >> 1;
    const bool hi = (j & 1) != 0;
    cx<C> own[3], oth[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<C> u = sel(k != 0, h[6 + a], h[a]), l = sel(k != 0, h[9 + a], h[3 + a]);
        own[a] = sel(hi, l, u);
        oth[a] = sel(hi, u, l);
    }
    out[0] = cfmac(L.h20, own[2], cfmac(L.h10, own[1], L.dg[0] * own[0]));
    out[1] = cfmac(L.h21, own[2], cfma(L.h10, own[0], L.dg[1] * own[1]));
    out[2] = cfma(L.h21, own[1], cfma(L.h20, own[0], L.dg[2] * own[2]));
#pragma unroll
    for (int a = 0; a < 3; ++a)
        out[a] = cfma(L.m[3 * a + 2], oth[2], cfma(L.m[3 * a + 1], oth[1], cfma(L.m[3 * a], oth[0], out[a])));
}

template <typename S2, typename C>
__device__ __forceinline__ void lane_clover(cx<C> out[3], const cx<C> h[12], const S2 *__restrict__ F, const GeomDev &g,
                                            int ib, int s, int j) {
    LaneClover<C> L;
    lane_clover_load(L, F, g, ib, s, j);
    lane_clover_apply(out, h, L, j);
}

// spin j (components 3j..3j+2) of a field site
template <typename S2, typename C>
__device__ __forceinline__ void load_spin(cx<C> v[3], const S2 *f, const GeomDev &g, int ib, int s, int j) {
    const S2 *p = f + ((size_t)ib * 12 + 3 * j) * g.Vb + s;
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = ld(p + (size_t)a * g.Vb);
}
template <typename S2, typename C>
__device__ __forceinline__ void store_spin(S2 *f, const GeomDev &g, int ib, int s, int j, const cx<C> v[3]) {
    S2 *p = f + ((size_t)ib * 12 + 3 * j) * g.Vb + s;
#pragma unroll
    for (int a = 0; a < 3; ++a) st(p + (size_t)a * g.Vb, v[a]);
}


}  // namespace sapq
