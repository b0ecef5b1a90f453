// SAP phase kernel with two lanes per site, for blocks whose SSOR iterate does not fit
// LDS as a whole: the block is split along t into two workgroups ("parts"), each holding
// the iterate of its own half in LDS.  It computes exactly what k_sap_phase computes
// (Algorithm 1 fused with the M_SAP update, the locally-lexicographic SSOR in hyperplane
// order of the sub-block-local coordinates, Sec. 3.2 and Fig. 2):
//   v_c = r_c + kappa F sum_{hops leaving the block} H x_other
//   x_c = n_ssor forward + backward sweeps from 0,  y_c += x_c,  r_c = v_c - D_cc x_c.
//
// Lanes.  Lane d = 0 of a pair takes the four forward hops of its site, lane d = 1 the
// four backward hops.  Both run the same instructions: the projection sign is s = +1 / -1,
// and lane 1 reads U_mu at its backward neighbour and turns it into U^+ with selects (a
// daggered copy of the links at the site would cost a quarter more bytes per sweep).  After
// a pair butterfly each lane owns one chiral half (spins 2d and 2d + 1), applies its 6x6
// block of F and updates those six components.
//
// Parts.  The sub-block layers along t are split in halves.  Only hops in t cross between
// the halves, and they connect the last t-layer of a sub-block to the first one of the
// next, whose hyperplanes differ by S_t - 1: the data one part needs from the other were
// produced S_t - 1 steps earlier (new values) or in the previous sweep (old values).
// Each part publishes its boundary layer after every update into a global array of
// 64-bit words (value, tag), the tag naming launch and sweep; the other part copies the
// words it needs for its next step into LDS halo slots, waiting (bounded) on the tag.
// Sweep w's words go to slot w mod 3, which a part can only reuse after the reader has
// moved on (writing sweep w + 3 needs the reader's sweep w + 2 data).  The two parts of a
// block take their block from a ticket counter in start order, so a part only ever waits
// on a part that is already running; the last workgroup resets the counter.
#include "sitecore.h"

namespace sapq {

struct PartArgs {
    int colour, gather, first, ssor_only, n_ssor;
    float kappa, omega;
    int NP, Vp, Hp;
    const int *gslot;         // [NP][Vp] block slot of each part-local site
    const uint2 *pnb;         // [NP][Vp][2] LDS slots of the 4 neighbours of lane d (16 bits each)
    const uint2 *gnb;         // [NP][Vp] block slots of the 4 backward neighbours (16 bits each)
    const int *pstart;        // [MAX_PLANES + 1] part-local hyperplane starts
    const int *exp_idx;       // [NP][Vp] index in the part's boundary layer, or -1
    const int *imp;           // [NP][Hp] halo slots, ordered by the hyperplane that reads them
    const int *imp_start;     // [NP][MAX_PLANES + 1]
    unsigned long long *xch;  // [NBc][NP][3][24][Hp]
    unsigned *sync;           // [0] ticket, [1] done, [2] epoch, [3] error
};

constexpr int IMP_REGS = 4;          // halo words a thread keeps in flight during a step
constexpr int SPIN_LIMIT = 1 << 20;  // bounded wait on a halo word (about a second)

__device__ __forceinline__ unsigned xch_tag(unsigned epoch, int sweep) {
    return 0x80000000u | ((epoch & 0x1ffffffu) << 6) | (unsigned)(sweep & 63);
}
__device__ __forceinline__ void xch_put(unsigned long long *p, float v, unsigned tag) {
    const unsigned long long w = ((unsigned long long)tag << 32) | __float_as_uint(v);
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long xch_get(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the word at p once it carries `tag`; on time-out the error flag is raised and the caller
// stops waiting for the rest of the launch (the result is then discarded by the host)
__device__ __forceinline__ float xch_wait(unsigned long long w, unsigned long long *p, unsigned tag, bool &gave_up,
                                          unsigned *sync) {
    if ((unsigned)(w >> 32) != tag && !gave_up) {
        int it = 0;
        do {
            __builtin_amdgcn_s_sleep(2);
            w = xch_get(p);
        } while ((unsigned)(w >> 32) != tag && ++it < SPIN_LIMIT);
        if ((unsigned)(w >> 32) != tag) {
            gave_up = true;
            __hip_atomic_store(&sync[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return __uint_as_float((unsigned)w);
}

// barrier for LDS traffic only: global loads (halo words) and stores stay in flight
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// (1 - s gamma_mu) M psi accumulated into acc, M a full SU(3) matrix; the projection and
// the rebuild of the lower spins follow the chiral-basis gamma matrices (see sitecore.h)
template <int MU>
__device__ __forceinline__ void hop_lane(cx<float> acc[12], const cx<float> psi[12], const cx<float> u[9], float s) {
    cx<float> h0[3], h1[3], g0[3], g1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<float> p0 = psi[a], p1 = psi[3 + a], p2 = psi[6 + a], p3 = psi[9 + a];
        if (MU == 0) { h0[a] = p0 + s * itimes(p3); h1[a] = p1 + s * itimes(p2); }
        if (MU == 1) { h0[a] = p0 + s * p3;         h1[a] = p1 - s * p2; }
        if (MU == 2) { h0[a] = p0 + s * itimes(p2); h1[a] = p1 - s * itimes(p3); }
        if (MU == 3) { h0[a] = p0 - s * p2;         h1[a] = p1 - s * p3; }
    }
    su3_mul(g0, u, h0, false);
    su3_mul(g1, u, h1, false);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[a] = acc[a] + g0[a];
        acc[3 + a] = acc[3 + a] + g1[a];
        if (MU == 0) { acc[6 + a] = acc[6 + a] - s * itimes(g1[a]); acc[9 + a] = acc[9 + a] - s * itimes(g0[a]); }
        if (MU == 1) { acc[6 + a] = acc[6 + a] - s * g1[a];         acc[9 + a] = acc[9 + a] + s * g0[a]; }
        if (MU == 2) { acc[6 + a] = acc[6 + a] - s * itimes(g0[a]); acc[9 + a] = acc[9 + a] + s * itimes(g1[a]); }
        if (MU == 3) { acc[6 + a] = acc[6 + a] - s * g0[a];         acc[9 + a] = acc[9 + a] - s * g1[a]; }
    }
}

// rows 0, 1 of a stored link and row 2 = conj(row0 x row1)
__device__ __forceinline__ void link_rebuild(cx<float> u[9]) {
    u[6] = conjx(cmul(u[1], u[5]) - cmul(u[2], u[4]));
    u[7] = conjx(cmul(u[2], u[3]) - cmul(u[0], u[5]));
    u[8] = conjx(cmul(u[0], u[4]) - cmul(u[1], u[3]));
}
template <typename S2>
__device__ __forceinline__ void link_rows(cx<float> u[9], const S2 *p, int Vb) {
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = ld(p + (size_t)e * Vb);
    link_rebuild(u);
}

// u <- u^+ on the lanes with dag set, u unchanged on the others (same instructions on both)
__device__ __forceinline__ void dagger_if(cx<float> u[9], bool dag) {
    cx<float> t[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t[3 * a + b] = sel(dag, u[3 * b + a], u[3 * a + b]);
    const float sg = dag ? -1.f : 1.f;
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = {t[e].r, sg * t[e].i};
}

// one hermitian chiral block [[A, B], [B^+, C]] of F (18 slots, see k_pack_clover)
struct Clov { cx<float> f[18]; };

template <typename S2>
__device__ __forceinline__ void load_clov(Clov &F, const S2 *p, int Vb) {
#pragma unroll
    for (int e = 0; e < 18; ++e) F.f[e] = ld(p + (size_t)e * Vb);
}

// out = F_k in:  slots 0-2 the six real diagonal entries pairwise, 3-5 / 6-8 the strict
// lower triangles of A / C, 9-17 B row by row
__device__ __forceinline__ void clover_apply(cx<float> out[6], const cx<float> in[6], const Clov &F) {
    const cx<float> d01 = F.f[0], d23 = F.f[1], d45 = F.f[2];
    const cx<float> a10 = F.f[3], a20 = F.f[4], a21 = F.f[5], c10 = F.f[6], c20 = F.f[7], c21 = F.f[8];
    const cx<float> *B = F.f + 9;
    const cx<float> u0 = in[0], u1 = in[1], u2 = in[2], l0 = in[3], l1 = in[4], l2 = in[5];
    out[0] = d01.r * u0 + cmulc(a10, u1) + cmulc(a20, u2) + cmul(B[0], l0) + cmul(B[1], l1) + cmul(B[2], l2);
    out[1] = cmul(a10, u0) + d01.i * u1 + cmulc(a21, u2) + cmul(B[3], l0) + cmul(B[4], l1) + cmul(B[5], l2);
    out[2] = cmul(a20, u0) + cmul(a21, u1) + d23.r * u2 + cmul(B[6], l0) + cmul(B[7], l1) + cmul(B[8], l2);
    out[3] = cmulc(B[0], u0) + cmulc(B[3], u1) + cmulc(B[6], u2) + d23.i * l0 + cmulc(c10, l1) + cmulc(c20, l2);
    out[4] = cmulc(B[1], u0) + cmulc(B[4], u1) + cmulc(B[7], u2) + cmul(c10, l0) + d45.r * l1 + cmulc(c21, l2);
    out[5] = cmulc(B[2], u0) + cmulc(B[5], u1) + cmulc(B[8], u2) + cmul(c20, l0) + cmul(c21, l1) + d45.i * l2;
}

template <typename S2>
__device__ __forceinline__ void clover_block(cx<float> out[6], const cx<float> in[6], const S2 *p, int Vb) {
    Clov F;
    load_clov(F, p, Vb);
    clover_apply(out, in, F);
}

__device__ __forceinline__ void pair_reduce(cx<float> acc[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        acc[c].r += quad_get<QUAD_XOR1>(acc[c].r);
        acc[c].i += quad_get<QUAD_XOR1>(acc[c].i);
    }
}

// the six components (spins 2d, 2d + 1) of site (ib, s) owned by lane d
template <typename S2>
__device__ __forceinline__ void load6(cx<float> v[6], const S2 *f, int ib, int s, int d, int Vb) {
    const S2 *p = f + ((size_t)ib * 12 + 6 * d) * Vb + s;
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = ld(p + (size_t)e * Vb);
}
template <typename S2>
__device__ __forceinline__ void store6(S2 *f, int ib, int s, int d, int Vb, const cx<float> v[6]) {
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

// One in-block hop of the lane: the neighbour spinor from LDS slot `slot`, the link U_mu
// at block slot sl (the site for lane 0, the backward neighbour for lane 1, daggered there).
template <int MU, typename S2>
__device__ __forceinline__ void lds_hop(cx<float> acc[12], const float4 *xs, int NS, unsigned slot, const S2 *U,
                                        int ib, int sl, int Vb, float sg) {
    cx<float> psi[12], u[9];
    lds_spinor(psi, xs, NS, (int)slot);
    link_rows(u, U + ((size_t)ib * 4 + MU) * 6 * Vb + sl, Vb);
    dagger_if(u, sg < 0.f);
    hop_lane<MU>(acc, psi, u, sg);
}

// sum over the lane's in-block hops of site (ib, s), reduced over the pair, and F of the
// lane's chiral half:  out = (F sum_{m in block} H_nm x_m) restricted to spins 2d, 2d + 1
// gl: block slots of the backward neighbours, where lane 1 finds its links
template <typename S2>
__device__ __forceinline__ void block_hop_clover(cx<float> out[6], const float4 *xs, int NS, uint2 nb, uint2 gl,
                                                 const S2 *U, const S2 *Fk, int ib, int s, int d, int Vb, float sg) {
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
    const bool at_site = d == 0;
    lds_hop<0>(acc, xs, NS, nb.x & 0xffffu, U, ib, at_site ? s : (int)(gl.x & 0xffffu), Vb, sg);
    lds_hop<1>(acc, xs, NS, nb.x >> 16, U, ib, at_site ? s : (int)(gl.x >> 16), Vb, sg);
    lds_hop<2>(acc, xs, NS, nb.y & 0xffffu, U, ib, at_site ? s : (int)(gl.y & 0xffffu), Vb, sg);
    lds_hop<3>(acc, xs, NS, nb.y >> 16, U, ib, at_site ? s : (int)(gl.y >> 16), Vb, sg);
    pair_reduce(acc);
    cx<float> own[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
    clover_block(out, own, Fk + s, Vb);
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

template <int P>
__global__ void __launch_bounds__(512) k_sap_phase_parts(GeomDev g, PartArgs a, const typename Prec<P>::S2 *rsrc,
                                                         typename Prec<P>::S2 *r, typename Prec<P>::S2 *x,
                                                         typename Prec<P>::S2 *y,
                                                         const typename Prec<P>::S2 *__restrict__ U,
                                                         const typename Prec<P>::S2 *__restrict__ F) {
    using S2 = typename Prec<P>::S2;
    extern __shared__ float4 xs[];
    __shared__ unsigned sh_ticket;
    const int Vb = g.Vb, Vp = a.Vp, Hp = a.Hp, NS = Vp + Hp + 1;
    int blk = blockIdx.x, part = 0;
    unsigned epoch = 0;
    if (a.NP == 2) {
        if (threadIdx.x == 0) sh_ticket = atomicAdd(&a.sync[0], 1u);
        __syncthreads();
        const unsigned t = sh_ticket;
        if (t >= gridDim.x) {  // counter out of step with the launch: flag it and do nothing
            if (threadIdx.x == 0) __hip_atomic_store(&a.sync[3], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        blk = (int)(t >> 1);
        part = (int)(t & 1u);
        epoch = __hip_atomic_load(&a.sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int ib = a.colour * g.NBc + blk;
    const int d = threadIdx.x & 1;
    const int q0 = threadIdx.x >> 1, nq = blockDim.x >> 1;
    const float sg = d ? -1.f : 1.f;
    const float kappa = a.kappa, omega = a.omega;
    const int *gslot = a.gslot + (size_t)part * Vp;
    const uint2 *pnb = a.pnb + (size_t)part * Vp * 2;
    const int *expi = a.exp_idx + (size_t)part * Vp;
    const int *imp = a.imp + (size_t)part * Hp;
    const int *imps = a.imp_start + (size_t)part * (MAX_PLANES + 1);
    const size_t xstride = (size_t)3 * 24 * Hp;
    unsigned long long *xo = a.xch + ((size_t)blk * a.NP + part) * xstride;
    unsigned long long *xi = a.xch + ((size_t)blk * a.NP + (part ^ 1)) * xstride;
    const uint2 *gnb = a.gnb + (size_t)part * Vp;
    const S2 *Fk = F + ((size_t)ib * 2 + d) * 18 * Vb;
    const S2 *vb = a.ssor_only ? rsrc : r;
    float *xsf = reinterpret_cast<float *>(xs);
    bool gave_up = false;

    // 1. v_c (gathering the other colour), zero the iterate, the halo slots and the zero slot
    {
        int bl[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) bl[mu] = g.blk_nbr[(2 * mu + d) * g.NB + ib];
        for (int i = q0; i < Vp; i += nq) {
            const int s = gslot[i];
            if (!a.ssor_only) {
                cx<float> v[6];
                load6(v, rsrc, ib, s, d, Vb);
                if (a.gather) {
                    cx<float> acc[12];
#pragma unroll
                    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
                    gather_hop<0>(acc, g, x, U, ib, s, d, bl[0], sg);
                    gather_hop<1>(acc, g, x, U, ib, s, d, bl[1], sg);
                    gather_hop<2>(acc, g, x, U, ib, s, d, bl[2], sg);
                    gather_hop<3>(acc, g, x, U, ib, s, d, bl[3], sg);
                    pair_reduce(acc);
                    cx<float> own[6], out[6];
#pragma unroll
                    for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
                    clover_block(out, own, Fk + s, Vb);
#pragma unroll
                    for (int e = 0; e < 6; ++e) v[e] = v[e] + kappa * out[e];
                }
                store6(r, ib, s, d, Vb, v);
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) xs[(3 * d + q) * NS + i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        for (int t = threadIdx.x; t < 6 * (Hp + 1); t += blockDim.x)
            xs[(t / (Hp + 1)) * NS + Vp + t % (Hp + 1)] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();

    // 2. sweeps: x_n <- (1 - omega) x_n + omega (v_n + kappa F(n) sum_{m in block} H_nm x_m).
    // A hyperplane has at most blockDim.x / 2 sites of the part, so a lane pair updates at
    // most one site per step.
    const int H = g.nplanes, nsw = 2 * a.n_ssor;
    const int *pst = a.pstart;
    for (int w = 0; w < nsw; ++w) {
        const bool fwd = (w & 1) == 0;
        for (int pi = 0; pi < H; ++pi) {
            const int h = fwd ? pi : H - 1 - pi;
            const int i = pst[h] + q0;
            const bool ok = i < pst[h + 1];
            // block slot of the site: each part owns one contiguous slot range of every
            // hyperplane, part 0 first
            const int s = a.NP == 2 ? i + pst[h] + part * (pst[h + 1] - pst[h]) : i;
            const int kx = (ok && a.NP == 2) ? expi[i] : -1;
            // (1) halo words for the next step, stored to LDS after this step's updates.  At
            // the turn of a sweep the plane repeats and its halo slots already hold the right
            // sweep (or the plane reads none), so nothing is fetched.
            int nw = 0, ne = 0, e0 = 0;
            unsigned tag = 0;
            unsigned long long *src = nullptr;
            unsigned long long pre[IMP_REGS];
            if (a.NP == 2 && pi + 1 < H) {
                const int nh = fwd ? h + 1 : h - 1;
                // part 0 reads part 1 through +t (lower hyperplane: this sweep's values in a
                // forward sweep); part 1 reads part 0 through -t (higher hyperplane)
                const int ver = ((part == 0) == fwd) ? w : w - 1;
                if (ver >= 0) {  // before the first sweep the halo is zero
                    e0 = imps[nh];
                    ne = imps[nh + 1] - e0;
                    nw = 24 * ne;
                    tag = xch_tag(epoch, ver);
                    src = xi + (size_t)(ver % 3) * 24 * Hp;
#pragma unroll
                    for (int u = 0; u < IMP_REGS; ++u) {
                        const int t = threadIdx.x + u * blockDim.x;
                        if (t < nw) {
                            const int c = t / ne, e = t - c * ne;
                            pre[u] = xch_get(src + (size_t)c * Hp + imp[e0 + e]);
                        }
                    }
                }
            }
            // (2) the update
            if (ok) {
                cx<float> out[6], v[6];
                block_hop_clover(out, xs, NS, pnb[2 * i + d], gnb[i], U, Fk, ib, s, d, Vb, sg);
                load6(v, vb, ib, s, d, Vb);
                cx<float> xn[6];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    float4 *o = &xs[(3 * d + q) * NS + i];
                    const float4 ov = *o;
                    const cx<float> n0 = v[2 * q] + kappa * out[2 * q], n1 = v[2 * q + 1] + kappa * out[2 * q + 1];
                    xn[2 * q] = {(1.f - omega) * ov.x + omega * n0.r, (1.f - omega) * ov.y + omega * n0.i};
                    xn[2 * q + 1] = {(1.f - omega) * ov.z + omega * n1.r, (1.f - omega) * ov.w + omega * n1.i};
                    *o = make_float4(xn[2 * q].r, xn[2 * q].i, xn[2 * q + 1].r, xn[2 * q + 1].i);
                }
                if (kx >= 0) {
                    const unsigned wt = xch_tag(epoch, w);
                    unsigned long long *dst = xo + (size_t)(w % 3) * 24 * Hp + kx;
#pragma unroll
                    for (int e = 0; e < 6; ++e) {
                        xch_put(dst + (size_t)(12 * d + 2 * e) * Hp, xn[e].r, wt);
                        xch_put(dst + (size_t)(12 * d + 2 * e + 1) * Hp, xn[e].i, wt);
                    }
                }
            }
            // (3) the halo words into LDS
            if (nw) {
#pragma unroll
                for (int u = 0; u < IMP_REGS; ++u) {
                    const int t = threadIdx.x + u * blockDim.x;
                    if (t < nw) {
                        const int c = t / ne, e = t - c * ne, k = imp[e0 + e];
                        unsigned long long *p = src + (size_t)c * Hp + k;
                        xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(pre[u], p, tag, gave_up, a.sync);
                    }
                }
                for (int t = threadIdx.x + IMP_REGS * blockDim.x; t < nw; t += blockDim.x) {
                    const int c = t / ne, e = t - c * ne, k = imp[e0 + e];
                    unsigned long long *p = src + (size_t)c * Hp + k;
                    xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(xch_get(p), p, tag, gave_up, a.sync);
                }
            }
            lds_barrier();
        }
    }

    // 3. the whole halo at the last sweep, then outputs
    if (a.NP == 2) {
        const unsigned tag = xch_tag(epoch, nsw - 1);
        unsigned long long *src = xi + (size_t)((nsw - 1) % 3) * 24 * Hp;
        for (int t = threadIdx.x; t < 24 * Hp; t += blockDim.x) {
            const int c = t / Hp, k = t - c * Hp;
            unsigned long long *p = src + (size_t)c * Hp + k;
            xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(xch_get(p), p, tag, gave_up, a.sync);
        }
        __syncthreads();
    }
    for (int i = q0; i < Vp; i += nq) {
        const int s = gslot[i];
        cx<float> xv[6];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float4 f = xs[(3 * d + q) * NS + i];
            xv[2 * q] = {f.x, f.y};
            xv[2 * q + 1] = {f.z, f.w};
        }
        store6(x, ib, s, d, Vb, xv);
        if (a.ssor_only) continue;
        cx<float> yv[6];
        if (a.first) {
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = xv[e];
        } else {
            load6(yv, y, ib, s, d, Vb);
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = yv[e] + xv[e];
        }
        store6(y, ib, s, d, Vb, yv);
        cx<float> out[6], v[6];
        block_hop_clover(out, xs, NS, pnb[2 * i + d], gnb[i], U, Fk, ib, s, d, Vb, sg);
        load6(v, r, ib, s, d, Vb);
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = v[e] - xv[e] + kappa * out[e];
        store6(r, ib, s, d, Vb, v);
    }

    // 4. the last workgroup to finish resets the ticket counter and advances the epoch
    if (a.NP == 2) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned done = atomicAdd(&a.sync[1], 1u);
            if (done == gridDim.x - 1) {
                __hip_atomic_store(&a.sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.sync[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.sync[2], epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

void launch_sap_phase_parts(Ctx *c, int colour, int gather, int first, int ssor_only, const void *rsrc, void *r,
                            void *x, void *y) {
    PartArgs a;
    a.colour = colour;
    a.gather = gather;
    a.first = first;
    a.ssor_only = ssor_only;
    a.n_ssor = c->prm.n_ssor;
    a.kappa = (float)c->prm.kappa;
    a.omega = (float)c->prm.omega;
    a.NP = c->sap_np;
    a.Vp = c->part_Vp;
    a.Hp = c->part_Hp;
    a.gslot = c->part_gslot;
    a.pnb = c->part_nb;
    a.gnb = c->part_gnb;
    a.pstart = c->part_pstart;
    a.exp_idx = c->part_exp;
    a.imp = c->part_imp;
    a.imp_start = c->part_imps;
    a.xch = c->xch;
    a.sync = c->xsync;
    const dim3 grid(c->g.NBc * c->sap_np), block(c->part_threads);
    INNER_SWITCH(c->prm.prec_inner, ({
                     using S2 = typename Prec<P_>::S2;
                     k_sap_phase_parts<P_><<<grid, block, c->parts_lds, c->stream>>>(
                         c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin);
                 }));
}

int set_parts_lds_limit(Ctx *c) {
    if (!c->use_parts || c->parts_lds <= 65536) return 0;
    const int bytes = (int)c->parts_lds;
    INNER_SWITCH(c->prm.prec_inner, (void)hipFuncSetAttribute((const void *)k_sap_phase_parts<P_>,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sapq
