// SAP phase kernel with two lanes per site, for blocks whose SSOR iterate does not fit
// LDS as a whole: the block is split along t into two workgroups ("parts"), each holding
// the iterate of its own half in LDS.  It computes exactly what k_sap_phase computes
// (Algorithm 1 fused with the M_SAP update, the locally-lexicographic SSOR in hyperplane
// order of the sub-block-local coordinates, section 3 "Inverse of block operator" and Fig. 1):
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
#include "twolane.h"

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
    int spin_limit;           // bounded wait on a halo word, in polls
    unsigned wait_xor;        // 0; nonzero only where a test forces the time-out path (no
                              // written word then carries the awaited tag)
};

constexpr int IMP_REGS = 4;          // halo words a thread keeps in flight during a step
constexpr int SPIN_LIMIT = 1 << 20;  // default bounded wait on a halo word (about a second)

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
                                          const PartArgs &a) {
    tag ^= a.wait_xor;
    if ((unsigned)(w >> 32) != tag && !gave_up) {
        int it = 0;
        do {
            __builtin_amdgcn_s_sleep(2);
            w = xch_get(p);
        } while ((unsigned)(w >> 32) != tag && ++it < a.spin_limit);
        if ((unsigned)(w >> 32) != tag) {
            gave_up = true;
            __hip_atomic_store(&a.sync[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return __uint_as_float((unsigned)w);
}

// barrier for LDS traffic only: global loads (halo words) and stores stay in flight
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// STAGED: the load order of a site update (block_hop_clover_impl); the staged order holds
// about 40 more registers, which costs nothing where a workgroup's LDS already keeps the CU
// to one workgroup, and occupancy where several workgroups share a CU
template <int P, bool STAGED>
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
    int *xsi = reinterpret_cast<int *>(xs);
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
        // the hyperplane and halo-import starts into LDS behind the iterate: every step reads
        // them, and from global memory (which the kernel writes, so they cannot go through the
        // scalar cache) each read would be a load round trip at the head of the step
        for (int t = threadIdx.x; t < MAX_PLANES + 1; t += blockDim.x) {
            xsi[6 * 4 * NS + t] = a.pstart[t];
            xsi[6 * 4 * NS + MAX_PLANES + 1 + t] = imps[t];
        }
    }
    __syncthreads();

    // 2. sweeps: x_n <- (1 - omega) x_n + omega (v_n + kappa F(n) sum_{m in block} H_nm x_m)
    const int H = g.nplanes, nsw = 2 * a.n_ssor;
    const int *pst = xsi + 6 * 4 * NS;  // the hyperplane starts, copied to LDS in step 1
    imps = pst + MAX_PLANES + 1;         // and this part's halo-import starts
    // The table entries of a site (LDS slots of its neighbours, block slots of its backward
    // neighbours, boundary index) are read one step ahead, for this thread's first site of
    // the coming hyperplane, right after its current update: read at the start of their own
    // step they would put a load round trip ahead of every other load of the step.
    uint2 nb_n = make_uint2(0u, 0u), gl_n = make_uint2(0u, 0u);
    int kx_n = -1;
    auto tables_for = [&](int hh) {
        const int i = pst[hh] + q0;
        if (i < pst[hh + 1]) {
            nb_n = pnb[2 * i + d];
            gl_n = gnb[i];
            kx_n = a.NP == 2 ? expi[i] : -1;
        }
    };
    tables_for(0);
    for (int w = 0; w < nsw; ++w) {
        const bool fwd = (w & 1) == 0;
        for (int pi = 0; pi < H; ++pi) {
            const int h = fwd ? pi : H - 1 - pi;
            // (1) halo words for the next step, stored to LDS after this step's updates.  At
            // the turn of a sweep the plane repeats and its halo slots already hold the right
            // sweep (or the plane reads none), so nothing is fetched.
            int nw = 0, ne = 0, e0 = 0;
            unsigned tag = 0;
            unsigned long long *src = nullptr;
            unsigned long long pre[IMP_REGS];
            // every thread issues IMP_REGS loads in every step (a harmless read of the hyperplane
            // table where there is no word to fetch), so that the number of loads in flight after
            // the tables read a step ahead is fixed and waiting for those does not wait for these
            const unsigned long long *pre_p[IMP_REGS];
#pragma unroll
            for (int u = 0; u < IMP_REGS; ++u) pre_p[u] = reinterpret_cast<const unsigned long long *>(pst);
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
                            pre_p[u] = src + (size_t)c * Hp + imp[e0 + e];
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < IMP_REGS; ++u) pre[u] = xch_get(const_cast<unsigned long long *>(pre_p[u]));
            // (2) the updates; a part-local site i of plane h sits at block slot
            // i + pst[h] + part (pst[h + 1] - pst[h]) (each part owns one contiguous slot
            // range of every hyperplane, part 0 first)
            const int shift = a.NP == 2 ? pst[h] + part * (pst[h + 1] - pst[h]) : 0;
            // At the turn of a sweep (w > 0, pi = 0) the plane repeats: the top corner of the
            // sub-blocks after a forward sweep, the bottom corner after a backward one.  Every
            // neighbour of such a site lies on the side just swept and has not changed since the
            // site's last update, so with omega = 1 (no (1 - omega) x term) the update would give
            // the same value bit for bit: it is skipped and only the boundary words are
            // published again under the new sweep's tag.
            const bool repeat = omega == 1.f && w > 0 && pi == 0;
            auto update = [&](int i, uint2 nb, uint2 gl, int kx) {
                const int s = i + shift;
                cx<float> xn[6];
                if (repeat) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const float4 f = xs[(3 * d + q) * NS + i];
                        xn[2 * q] = {f.x, f.y};
                        xn[2 * q + 1] = {f.z, f.w};
                    }
                } else {
                cx<float> out[6], v[6];
                block_hop_clover_v<STAGED>(out, v, vb, xs, NS, nb, gl, U, Fk, ib, s, d, Vb, sg);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    float4 *o = &xs[(3 * d + q) * NS + i];
                    const float4 ov = *o;
                    const cx<float> n0 = v[2 * q] + kappa * out[2 * q], n1 = v[2 * q + 1] + kappa * out[2 * q + 1];
                    xn[2 * q] = {(1.f - omega) * ov.x + omega * n0.r, (1.f - omega) * ov.y + omega * n0.i};
                    xn[2 * q + 1] = {(1.f - omega) * ov.z + omega * n1.r, (1.f - omega) * ov.w + omega * n1.i};
                    *o = make_float4(xn[2 * q].r, xn[2 * q].i, xn[2 * q + 1].r, xn[2 * q + 1].i);
                }
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
            };
            // this thread's first site with the tables read a step ahead, then those of the
            // coming step (at a turn the plane repeats, and so do its tables), then any further
            // sites (a hyperplane with more sites than the workgroup has lane pairs)
            const uint2 nb0 = nb_n, gl0 = gl_n;
            const int kx0 = kx_n, i0 = pst[h] + q0;
            if (i0 < pst[h + 1]) update(i0, nb0, gl0, kx0);
            if (pi + 1 < H) tables_for(fwd ? h + 1 : h - 1);
            for (int i = i0 + nq; i < pst[h + 1]; i += nq)
                update(i, pnb[2 * i + d], gnb[i], a.NP == 2 ? expi[i] : -1);
            // (3) the halo words into LDS
            if (nw) {
#pragma unroll
                for (int u = 0; u < IMP_REGS; ++u) {
                    const int t = threadIdx.x + u * blockDim.x;
                    if (t < nw) {
                        const int c = t / ne, e = t - c * ne, k = imp[e0 + e];
                        unsigned long long *p = src + (size_t)c * Hp + k;
                        xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(pre[u], p, tag, gave_up, a);
                    }
                }
                for (int t = threadIdx.x + IMP_REGS * blockDim.x; t < nw; t += blockDim.x) {
                    const int c = t / ne, e = t - c * ne, k = imp[e0 + e];
                    unsigned long long *p = src + (size_t)c * Hp + k;
                    xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(xch_get(p), p, tag, gave_up, a);
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
            xsf[(((c >> 2) * NS) + Vp + k) * 4 + (c & 3)] = xch_wait(xch_get(p), p, tag, gave_up, a);
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
        block_hop_clover_v<STAGED>(out, v, r, xs, NS, pnb[2 * i + d], gnb[i], U, Fk, ib, s, d, Vb, sg);
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

// r_c += kappa F sum_{hops leaving the block} H x  (r_c -= D_{c,other} x_other, the last step
// of M_SAP), two lanes per site; a site with no hop leaving its block is left alone.
template <int P>
__global__ void __launch_bounds__(256) k_sap_face_2l(GeomDev g, int colour, float kappa, typename Prec<P>::S2 *r,
                                                     const typename Prec<P>::S2 *x,
                                                     const typename Prec<P>::S2 *__restrict__ U,
                                                     const typename Prec<P>::S2 *__restrict__ F) {
    const long i = xcd_site_base(128) + (threadIdx.x >> 1);
    const int d = threadIdx.x & 1;
    const long nc = (long)g.NBc * g.Vb;
    if (i >= nc) return;
    const int ib = colour * g.NBc + (int)(i / g.Vb), s = (int)(i % g.Vb);
    int outside = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const unsigned w = g.nbr16[mu * g.Vb + s];
        outside |= ((d ? (w >> 16) : w) & 0x8000u) ? 0 : 1;
    }
    outside |= __builtin_amdgcn_update_dpp(0, outside, QUAD_XOR1, 0xF, 0xF, true);
    if (!outside) return;  // both lanes of the pair leave together
    const float sg = d ? -1.f : 1.f;
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
    gather_hop<0>(acc, g, x, U, ib, s, d, g.blk_nbr[(2 * 0 + d) * g.NB + ib], sg);
    gather_hop<1>(acc, g, x, U, ib, s, d, g.blk_nbr[(2 * 1 + d) * g.NB + ib], sg);
    gather_hop<2>(acc, g, x, U, ib, s, d, g.blk_nbr[(2 * 2 + d) * g.NB + ib], sg);
    gather_hop<3>(acc, g, x, U, ib, s, d, g.blk_nbr[(2 * 3 + d) * g.NB + ib], sg);
    pair_reduce(acc);
    cx<float> own[6], out[6], v[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
    clover_block(out, own, F + ((size_t)ib * 2 + d) * 18 * g.Vb + s, g.Vb);
    load6(v, r, ib, s, d, g.Vb);
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = v[e] + kappa * out[e];
    store6(r, ib, s, d, g.Vb, v);
}

void launch_sap_face_2l(Ctx *c, int colour, void *r, const void *x) {
    const long nc = (long)c->g.NBc * c->g.Vb;
    const unsigned grid = (unsigned)((2 * nc + 255) / 256 + N_XCD - 1) / N_XCD * N_XCD;
    INNER_SWITCH(c->prm.prec_inner, (k_sap_face_2l<P_><<<grid, 256, 0, c->stream>>>(
                                         c->g, colour, (float)c->prm.kappa, (typename Prec<P_>::S2 *)r,
                                         (const typename Prec<P_>::S2 *)x, (const typename Prec<P_>::S2 *)c->Uin,
                                         (const typename Prec<P_>::S2 *)c->Fin)));
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
    a.spin_limit = c->halo_spin_limit;
    a.wait_xor = c->halo_wait_xor;
    const dim3 grid(c->g.NBc * c->sap_np), block(c->part_threads);
    INNER_SWITCH(c->prm.prec_inner, ({
                     using S2 = typename Prec<P_>::S2;
                     if (c->parts_staged)
                         k_sap_phase_parts<P_, true><<<grid, block, c->parts_lds, c->stream>>>(
                             c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin);
                     else
                         k_sap_phase_parts<P_, false><<<grid, block, c->parts_lds, c->stream>>>(
                             c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin);
                 }));
}

int set_parts_lds_limit(Ctx *c) {
    if (!c->use_parts || c->parts_lds <= 65536) return 0;
    const int bytes = (int)c->parts_lds;
    INNER_SWITCH(c->prm.prec_inner, ({
                     (void)hipFuncSetAttribute((const void *)k_sap_phase_parts<P_, true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
                     (void)hipFuncSetAttribute((const void *)k_sap_phase_parts<P_, false>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
                 }));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sapq
