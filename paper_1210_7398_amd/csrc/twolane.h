// Two lanes per site: the per-site building blocks of the two-lane SAP phase kernels (one
// source, csrc/sap_parts.hip; several sources, csrc/batch.hip).  Lane d = 0 of a pair takes
// the four forward hops (1 - gamma_mu) U_mu(n) psi(n + mu), lane d = 1 the four backward hops
// (1 + gamma_mu) U_mu(n - mu)^+ psi(n - mu), with U_mu(n - mu) read at the neighbour and
// daggered in registers; both lanes run the same instructions (projection sign s = +1 / -1).
// A pair butterfly adds the two halves, and lane d then owns chiral half d (spins 2d, 2d + 1).
#pragma once

#include "sitecore.h"

namespace sapq {

// (1 - s gamma_mu) M psi accumulated into acc, M a full SU(3) matrix; the projection and
// the rebuild of the lower spins follow the chiral-basis gamma matrices (see sitecore.h).
// The helpers below are written for the compute type C (float, or double for the FP64
// operator); the SSOR iterate in LDS is always float.
template <int MU, typename C>
__device__ __forceinline__ void hop_lane(cx<C> acc[12], const cx<C> psi[12], const cx<C> u[9], C s) {
    cx<C> h0[3], h1[3], g0[3], g1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<C> p0 = psi[a], p1 = psi[3 + a], p2 = psi[6 + a], p3 = psi[9 + a];
        if (MU == 0) { h0[a] = rfma(s, itimes(p3), p0);  h1[a] = rfma(s, itimes(p2), p1); }
        if (MU == 1) { h0[a] = rfma(s, p3, p0);          h1[a] = rfma(-s, p2, p1); }
        if (MU == 2) { h0[a] = rfma(s, itimes(p2), p0);  h1[a] = rfma(-s, itimes(p3), p1); }
        if (MU == 3) { h0[a] = rfma(-s, p2, p0);         h1[a] = rfma(-s, p3, p1); }
    }
    su3_mul(g0, u, h0, false);
    su3_mul(g1, u, h1, false);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + g0[a];
        acc[3 + a] = acc[3 + a] + g1[a];
        if (MU == 0) { acc[6 + a] = rfma(-s, itimes(g1[a]), acc[6 + a]); acc[9 + a] = rfma(-s, itimes(g0[a]), acc[9 + a]); }
        if (MU == 1) { acc[6 + a] = rfma(-s, g1[a], acc[6 + a]);         acc[9 + a] = rfma(s, g0[a], acc[9 + a]); }
        if (MU == 2) { acc[6 + a] = rfma(-s, itimes(g0[a]), acc[6 + a]); acc[9 + a] = rfma(s, itimes(g1[a]), acc[9 + a]); }
        if (MU == 3) { acc[6 + a] = rfma(-s, g0[a], acc[6 + a]);         acc[9 + a] = rfma(-s, g1[a], acc[9 + a]); }
    }
}

// rows 0, 1 of a stored link and row 2 = conj(row0 x row1)
template <typename C> __device__ __forceinline__ void link_rebuild(cx<C> u[9]) { su3_row2(u); }
template <typename S2, typename C>
__device__ __forceinline__ void link_rows(cx<C> u[9], const S2 *p, int Vb) {
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = ld(p + (size_t)e * Vb);
    link_rebuild(u);
}

// u <- u^+ on the lanes with dag set, u unchanged on the others (same instructions on both)
template <typename C> __device__ __forceinline__ void dagger_if(cx<C> u[9], bool dag) {
    cx<C> t[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t[3 * a + b] = sel(dag, u[3 * b + a], u[3 * a + b]);
    const C sg = dag ? C(-1) : C(1);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = {t[e].r, sg * t[e].i};
}

// one hermitian chiral block [[A, B], [B^+, C]] of F (18 slots, see k_pack_clover)
template <typename C = float> struct Clov { cx<C> f[18]; };

template <typename S2, typename C>
__device__ __forceinline__ void load_clov(Clov<C> &F, const S2 *p, int Vb) {
#pragma unroll
    for (int e = 0; e < 18; ++e) F.f[e] = ld(p + (size_t)e * Vb);
}

// out = F_k in:  slots 0-2 the six real diagonal entries pairwise, 3-5 / 6-8 the strict
// lower triangles of A / C, 9-17 B row by row
template <typename C> __device__ __forceinline__ void clover_apply(cx<C> out[6], const cx<C> in[6], const Clov<C> &F) {
    const cx<C> d01 = F.f[0], d23 = F.f[1], d45 = F.f[2];
    const cx<C> a10 = F.f[3], a20 = F.f[4], a21 = F.f[5], c10 = F.f[6], c20 = F.f[7], c21 = F.f[8];
    const cx<C> *B = F.f + 9;
    const cx<C> u0 = in[0], u1 = in[1], u2 = in[2], l0 = in[3], l1 = in[4], l2 = in[5];
    out[0] = cfma(B[2], l2, cfma(B[1], l1, cfma(B[0], l0, cfmac(a20, u2, cfmac(a10, u1, d01.r * u0)))));
    out[1] = cfma(B[5], l2, cfma(B[4], l1, cfma(B[3], l0, cfmac(a21, u2, cfma(a10, u0, d01.i * u1)))));
    out[2] = cfma(B[8], l2, cfma(B[7], l1, cfma(B[6], l0, cfma(a21, u1, cfma(a20, u0, d23.r * u2)))));
    out[3] = cfmac(c20, l2, cfmac(c10, l1, cfmac(B[6], u2, cfmac(B[3], u1, cfmac(B[0], u0, d23.i * l0)))));
    out[4] = cfmac(c21, l2, cfma(c10, l0, cfmac(B[7], u2, cfmac(B[4], u1, cfmac(B[1], u0, d45.r * l1)))));
    out[5] = cfma(c21, l1, cfma(c20, l0, cfmac(B[8], u2, cfmac(B[5], u1, cfmac(B[2], u0, d45.i * l2)))));
}

template <typename S2, typename C>
__device__ __forceinline__ void clover_block(cx<C> out[6], const cx<C> in[6], const S2 *p, int Vb) {
    Clov<C> F;
    load_clov(F, p, Vb);
    clover_apply(out, in, F);
}

template <typename C> __device__ __forceinline__ void pair_reduce(cx<C> acc[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        acc[c].r += quad_get<QUAD_XOR1>(acc[c].r);
        acc[c].i += quad_get<QUAD_XOR1>(acc[c].i);
    }
}

// the six components (spins 2d, 2d + 1) of site (ib, s) owned by lane d
template <typename S2, typename C>
__device__ __forceinline__ void load6(cx<C> v[6], const S2 *f, int ib, int s, int d, int Vb) {
    const S2 *p = f + ((size_t)ib * 12 + 6 * d) * Vb + s;
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = ld(p + (size_t)e * Vb);
}
template <typename S2, typename C>
__device__ __forceinline__ void store6(S2 *f, int ib, int s, int d, int Vb, const cx<C> v[6]) {
    S2 *p = f + ((size_t)ib * 12 + 6 * d) * Vb + s;
#pragma unroll
    for (int e = 0; e < 6; ++e) st(p + (size_t)e * Vb, v[e]);
}

// iterate in LDS: float4 [6][NS], float4 q holding components 2q and 2q + 1
__device__ __forceinline__ void lds_spinor(cx<float> psi[12], const float4 *xs, int NS, int slot) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float4 f = xs[q * NS + slot];
        psi[2 * q] = {f.x, f.y};
        psi[2 * q + 1] = {f.z, f.w};
    }
}

// One in-block hop of the lane: the neighbour spinor from LDS slot `slot` and the lane's
// link rows u (U_mu at the site for lane 0, at the backward neighbour for lane 1, where they
// are daggered), already loaded.
template <int MU>
__device__ __forceinline__ void lds_hop(cx<float> acc[12], const float4 *xs, int NS, unsigned slot, cx<float> u[9],
                                        float sg) {
    cx<float> psi[12];
    lds_spinor(psi, xs, NS, (int)slot);
    link_rebuild(u);
    dagger_if(u, sg < 0.f);
    hop_lane<MU>(acc, psi, u, sg);
}

// the six stored rows of link U_mu at block slot sl of block ib
template <typename S2>
__device__ __forceinline__ void link_load(cx<float> u[9], const S2 *U, int ib, int mu, int sl, int Vb) {
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = ld(U + ((size_t)ib * 4 + mu) * 6 * Vb + sl + (size_t)e * Vb);
}

// sum over the lane's in-block hops of site (ib, s), reduced over the pair, and F of the
// lane's chiral half:  out = (F sum_{m in block} H_nm x_m) restricted to spins 2d, 2d + 1;
// with WITH_V also the lane's six components of the field vf at the site.
// gl: block slots of the backward neighbours, where lane 1 finds its links.
// Load order (STAGED): the link rows of all four hops before any product, the clover rows
// after the second hop, v after the third, so that each group arrives while earlier hops
// compute.  A wait on a load also waits on every load issued before it, so the groups are
// issued in the order they are used; issuing everything at once, or each hop's links just
// before the hop (the unstaged order, for kernels short of registers), leaves more of the
// latency exposed.  Both orders compute the same values.
template <bool WITH_V, bool STAGED, typename S2>
__device__ __forceinline__ void block_hop_clover_impl(cx<float> out[6], cx<float> v[6], const S2 *vf, const float4 *xs,
                                                      int NS, uint2 nb, uint2 gl, const S2 *U, const S2 *Fk, int ib,
                                                      int s, int d, int Vb, float sg) {
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
    const bool at_site = d == 0;
    const int sl[4] = {at_site ? s : (int)(gl.x & 0xffffu), at_site ? s : (int)(gl.x >> 16),
                       at_site ? s : (int)(gl.y & 0xffffu), at_site ? s : (int)(gl.y >> 16)};
    cx<float> u[4][9];
    Clov<float> F;
    if constexpr (STAGED) {
#pragma unroll
        for (int m = 0; m < 4; ++m) link_load(u[m], U, ib, m, sl[m], Vb);
    }
    if constexpr (!STAGED) link_load(u[0], U, ib, 0, sl[0], Vb);
    lds_hop<0>(acc, xs, NS, nb.x & 0xffffu, u[0], sg);
    if constexpr (!STAGED) link_load(u[1], U, ib, 1, sl[1], Vb);
    lds_hop<1>(acc, xs, NS, nb.x >> 16, u[1], sg);
    if constexpr (STAGED) load_clov(F, Fk + s, Vb);
    if constexpr (!STAGED) link_load(u[2], U, ib, 2, sl[2], Vb);
    lds_hop<2>(acc, xs, NS, nb.y & 0xffffu, u[2], sg);
    if constexpr (STAGED && WITH_V) load6(v, vf, ib, s, d, Vb);
    if constexpr (!STAGED) link_load(u[3], U, ib, 3, sl[3], Vb);
    lds_hop<3>(acc, xs, NS, nb.y >> 16, u[3], sg);
    pair_reduce(acc);
    if constexpr (!STAGED) {
        load_clov(F, Fk + s, Vb);
        if constexpr (WITH_V) load6(v, vf, ib, s, d, Vb);
    }
    cx<float> own[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
    clover_apply(out, own, F);
}
template <typename S2>
__device__ __forceinline__ void block_hop_clover(cx<float> out[6], const float4 *xs, int NS, uint2 nb, uint2 gl,
                                                 const S2 *U, const S2 *Fk, int ib, int s, int d, int Vb, float sg) {
    block_hop_clover_impl<false, true>(out, (cx<float> *)nullptr, (const S2 *)nullptr, xs, NS, nb, gl, U, Fk, ib, s, d,
                                       Vb, sg);
}
// the unstaged order
template <typename S2>
__device__ __forceinline__ void block_hop_clover_seq(cx<float> out[6], const float4 *xs, int NS, uint2 nb, uint2 gl,
                                                     const S2 *U, const S2 *Fk, int ib, int s, int d, int Vb, float sg) {
    block_hop_clover_impl<false, false>(out, (cx<float> *)nullptr, (const S2 *)nullptr, xs, NS, nb, gl, U, Fk, ib, s, d,
                                        Vb, sg);
}
// the same and v = the lane's six components of vf at (ib, s), in either order
template <bool STAGED, typename S2>
__device__ __forceinline__ void block_hop_clover_v(cx<float> out[6], cx<float> v[6], const S2 *vf, const float4 *xs,
                                                   int NS, uint2 nb, uint2 gl, const S2 *U, const S2 *Fk, int ib, int s,
                                                   int d, int Vb, float sg) {
    block_hop_clover_impl<true, STAGED>(out, v, vf, xs, NS, nb, gl, U, Fk, ib, s, d, Vb, sg);
}

// one hop leaving the block (neighbour in another block, from the global iterate x)
template <int MU, typename S2>
__device__ __forceinline__ void gather_hop(cx<float> acc[12], const GeomDev &g, const S2 *x, const S2 *U, int ib,
                                           int s, int d, int bl, float sg) {
    const unsigned w = g.nbr16[MU * g.Vb + s];
    const unsigned hw = d ? (w >> 16) : (w & 0xffffu);
    if (hw & 0x8000u) return;  // inside the block: not part of the gather
    const int sn = (int)(hw & 0x7fffu), ibn = bl & BLK_MASK;
    const float ph = (bl & WRAP_BIT) ? g.bc[MU] : 1.f;
    cx<float> psi[12], u[9];
    load_spinor(psi, x, g, ibn, sn);
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = ph * psi[c];
    const bool at_site = d == 0;
    link_rows(u, U + ((size_t)(at_site ? ib : ibn) * 4 + MU) * 6 * g.Vb + (at_site ? s : sn), g.Vb);
    dagger_if(u, d != 0);
    hop_lane<MU>(acc, psi, u, sg);
}

// one hop of the lane to a neighbour inside or outside the block, read from the global field x
// (the full operator); outside neighbours across the lattice boundary take the fermion phase
template <int MU, typename S2, typename C>
__device__ __forceinline__ void hop_any(cx<C> acc[12], const GeomDev &g, const S2 *x, const S2 *U, int ib, int s, int d,
                                        C sg) {
    const unsigned w = g.nbr16[MU * g.Vb + s];
    const unsigned hw = d ? (w >> 16) : (w & 0xffffu);
    const int sn = (int)(hw & 0x7fffu);
    int ibn = ib;
    C ph = C(1);
    if (!(hw & 0x8000u)) {
        const int bl = g.blk_nbr[(2 * MU + d) * g.NB + ib];
        ibn = bl & BLK_MASK;
        ph = (bl & WRAP_BIT) ? C(g.bc[MU]) : C(1);
    }
    cx<C> psi[12], u[9];
    load_spinor(psi, x, g, ibn, sn);
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = ph * psi[c];
    const bool at_site = d == 0;
    link_rows(u, U + ((size_t)(at_site ? ib : ibn) * 4 + MU) * 6 * g.Vb + (at_site ? s : sn), g.Vb);
    dagger_if(u, d != 0);
    hop_lane<MU>(acc, psi, u, sg);
}

}  // namespace sapq
