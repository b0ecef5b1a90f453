// Batched solver: several gauge fields (lattices of any size, one SAP block and sub-block
// shape) with several right-hand sides each, solved together.  Every inner BiCGStab
// iteration of all fields and right-hand sides is one hipGraph replay; each SAP phase is one
// kernel launch over a work list of (field, block, group of right-hand sides), whose
// workgroup loads the links and clover rows of a site once and applies them to every
// right-hand side of the group.  Krylov scalars live on the device, one set per right-hand
// side; converged right-hand sides are masked.  The outer iteration is FP64 defect
// correction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "twolane.h"

namespace sapq {

// inner vector slots (storage precision), rhs-major: slot base + k * nvec
enum { IV_R, IV_RT, IV_P, IV_V, IV_S, IV_T, IV_E, IV_PH, IV_SH, IV_SAPR, IV_SAPX, IV_RIN, IV_Z, IV_RP, NIV };
// outer vector slots (FP64)
enum { DV_B, DV_X, DV_R, DV_T, NDV };

constexpr int MAX_FIELDS = 16;

struct BField {
    GeomDev g;
    const void *Uin, *Fin;
    const double2 *U64, *F64;
    float kappa, omega;
    int n_ssor;
    int nrhs, rhs0;       // right-hand sides of this field and the index of its first one
    int ngroups;          // groups of NR right-hand sides
    size_t nvec;
    void *iv[NIV];
    double2 *dv[NDV];
    // two-lane kernel (contexts with one workgroup per block): neighbour LDS slots, block
    // slots of the backward neighbours, hyperplane starts, threads per right-hand side
    const uint2 *pnb, *gnb;
    const int *pst;
    int tpr;
};

struct BatchDev {
    int nf, total_rhs;
    int work0[MAX_FIELDS + 1];  // prefix sums of 8 ceil(NBc / 8) ngroups over fields (work_item)
    BField f[MAX_FIELDS];
};

// per right-hand-side Krylov state on the device; bad: a scalar of the inner solve was not
// finite (the source stops, its solution keeps the last finite iterate)
struct BState {
    double2 rho, rho_old, alpha, omega, beta;
    double r0, rr;
    int done, its, bad, pad;
};

// per right-hand-side outer state on the device
enum { OS_RUNNING = 0, OS_CONVERGED = 1, OS_BREAKDOWN = 2 };
struct BOuter {
    double bnorm, relres, scale;
    int status, outer_its, inner_its, pad;
};

// ---------------------------------------------------------------- work list decode
__device__ __forceinline__ int field_of_work(const BatchDev &B, int w) {
    int f = 0;
    while (f + 1 < B.nf && w >= B.work0[f + 1]) ++f;
    return f;
}

// Work item w of a phase launch: its field fi, block ib of colour `colour` (-1: an idle
// workgroup) and group index. Workgroups are dealt to the 8 XCDs in turn. A field's items
// (8 ceil(NBc / 8) ngroups of them, from a multiple of 8) deal its blocks round robin to the
// XCDs, and an XCD takes all groups of one block in a row. So the groups share the block's
// links and clover rows in one L2, while the blocks, and with them the uneven work of
// converged sources and differently sized fields, stay spread evenly over the XCDs.
__device__ __forceinline__ int work_item(const BatchDev &B, int w, int colour, int &fi, int &group) {
    fi = field_of_work(B, w);
    const BField &F = B.f[fi];
    const int local = w - B.work0[fi], pos = local / N_XCD;
    const int b = (pos / F.ngroups) * N_XCD + local % N_XCD;
    group = pos % F.ngroups;
    return b < F.g.NBc ? colour * F.g.NBc + b : -1;
}

// ---------------------------------------------------------------- multi-RHS SAP phase
// As the single-source phase kernel, for NR right-hand sides at once (iterates in LDS).
template <int P, int NR>
__global__ void __launch_bounds__(512) k_bsap_phase(const BatchDev *__restrict__ Bd, int colour, int first, int s_src,
                                                    int s_r, int s_x, int s_y, const BState *__restrict__ bst) {
    using S2 = typename Prec<P>::S2;
    using C = float;
    extern __shared__ float2 lds[];
    const BatchDev &B = *Bd;
    if ((int)blockIdx.x >= B.work0[B.nf]) return;
    int fi, grp;
    const int ib = work_item(B, blockIdx.x, colour, fi, grp);
    if (ib < 0) return;
    const BField &F = B.f[fi];
    const GeomDev &g = F.g;
    const int k0 = grp * NR;
    // skip groups whose right-hand sides are all finished (uniform over the workgroup)
    bool any = false;
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (k0 + k < F.nrhs && !bst[F.rhs0 + k0 + k].done) any = true;
    if (!any) return;
    float2 *xs = lds;  // [NR][12][Vb]
    unsigned *nb_lds = reinterpret_cast<unsigned *>(lds + NR * 12 * g.Vb);
    int *ps_lds = reinterpret_cast<int *>(nb_lds + 4 * g.Vb);
    const S2 *U = (const S2 *)F.Uin;
    const S2 *Fc = (const S2 *)F.Fin;
    const C kappa = F.kappa, omega = F.omega;
    const int j = threadIdx.x & 3;
    const int q0 = threadIdx.x >> 2, nq = blockDim.x >> 2;
    const int bl_f = g.blk_nbr[(2 * j) * g.NB + ib], bl_b = g.blk_nbr[(2 * j + 1) * g.NB + ib];
    const float bc = g.bc[j];
    const S2 *src = (const S2 *)F.iv[s_src];
    S2 *r = (S2 *)F.iv[s_r];
    S2 *x = (S2 *)F.iv[s_x];
    S2 *y = (S2 *)F.iv[s_y];
    const size_t nv = F.nvec;
    const int nk = min(NR, F.nrhs - k0);

    for (int t = threadIdx.x; t < 4 * g.Vb; t += blockDim.x) nb_lds[t] = g.nbr16[t];
    for (int t = threadIdx.x; t <= g.nplanes; t += blockDim.x) ps_lds[t] = g.plane_start[t];
    __syncthreads();

    const bool gather = colour == 1 || !first;
    for (int s = q0; s < g.Vb; s += nq) {
        const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
        LaneLinks<C> lk;
        LaneClover<C> lc;
        if (gather) {
            lane_links(lk, g, ib, s, j, n, U);
            lane_clover_load(lc, Fc, g, ib, s, j);
        }
        for (int k = 0; k < nk; ++k) {
            const size_t ko = (size_t)(k0 + k) * nv;
            cx<C> v[3];
            load_spin(v, src + ko, g, ib, s, j);
            if (gather) {
                cx<C> h[12], fh[3];
                quad_hop_apply<HOP_OUT>(h, g, j, n, lk, FieldSrc<S2, C>{x + ko});
                lane_clover_apply(fh, h, lc, j);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = v[c] + kappa * fh[c];
            }
            store_spin(r + ko, g, ib, s, j, v);
#pragma unroll
            for (int c = 0; c < 3; ++c) xs[(k * 12 + 3 * j + c) * g.Vb + s] = make_float2(0.f, 0.f);
        }
    }
    __syncthreads();

    for (int sw = 0; sw < F.n_ssor; ++sw) {
        for (int dir = 0; dir < 2; ++dir) {
            for (int pi = 0; pi < g.nplanes; ++pi) {
                // omega = 1: the repeated plane at a sweep turn keeps its values (as above)
                if (omega == 1.f && (sw > 0 || dir > 0) && pi == 0) continue;
                const int p = dir == 0 ? pi : g.nplanes - 1 - pi;
                const int s0 = ps_lds[p], s1 = ps_lds[p + 1];
                for (int s = s0 + q0; s < s1; s += nq) {
                    const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
                    LaneLinks<C> lk;
                    LaneClover<C> lc;
                    lane_links(lk, g, ib, s, j, n, U);
                    lane_clover_load(lc, Fc, g, ib, s, j);
                    for (int k = 0; k < nk; ++k) {
                        const BlockSrc bs{xs + (size_t)k * 12 * g.Vb};
                        cx<C> h[12], fh[3], v[3];
                        quad_hop_apply<HOP_IN>(h, g, j, n, lk, bs);
                        lane_clover_apply(fh, h, lc, j);
                        load_spin(v, r + (size_t)(k0 + k) * nv, g, ib, s, j);
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            float2 *o = &xs[(k * 12 + 3 * j + c) * g.Vb + s];
                            float2 ov = *o;
                            cx<C> nx = v[c] + kappa * fh[c];
                            *o = make_float2((1.f - omega) * ov.x + omega * nx.r, (1.f - omega) * ov.y + omega * nx.i);
                        }
                    }
                }
                __syncthreads();
            }
        }
    }

    for (int s = q0; s < g.Vb; s += nq) {
        const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
        LaneLinks<C> lk;
        LaneClover<C> lc;
        lane_links(lk, g, ib, s, j, n, U);
        lane_clover_load(lc, Fc, g, ib, s, j);
        for (int k = 0; k < nk; ++k) {
            const size_t ko = (size_t)(k0 + k) * nv;
            const float2 *xk = xs + (size_t)k * 12 * g.Vb;
            cx<C> xv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float2 t = xk[(3 * j + c) * g.Vb + s];
                xv[c] = {t.x, t.y};
            }
            store_spin(x + ko, g, ib, s, j, xv);
            cx<C> yv[3];
            if (first) {
#pragma unroll
                for (int c = 0; c < 3; ++c) yv[c] = xv[c];
            } else {
                load_spin(yv, y + ko, g, ib, s, j);
#pragma unroll
                for (int c = 0; c < 3; ++c) yv[c] = yv[c] + xv[c];
            }
            store_spin(y + ko, g, ib, s, j, yv);
            cx<C> h[12], fh[3], v[3];
            quad_hop_apply<HOP_IN>(h, g, j, n, lk, BlockSrc{xk});
            lane_clover_apply(fh, h, lc, j);
            load_spin(v, r + ko, g, ib, s, j);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = v[c] - xv[c] + kappa * fh[c];
            store_spin(r + ko, g, ib, s, j, v);
        }
    }
}

// The multi-source phase kernel with two lanes per site, for blocks whose iterate fits LDS:
// the workgroup is NR slices of a single-source workgroup (k_sap_phase_parts with one part),
// slice k working on right-hand side k0 + k of its group with its own iterate in LDS.  The
// slices read the same links and clover rows at the same time, so the group fetches them
// from HBM once and the other slices find them in L1/L2.
template <int P, int NR>
__global__ void __launch_bounds__(768) k_bsap_phase_2l(const BatchDev *__restrict__ Bd, int colour, int first,
                                                        int s_src, int s_r, int s_x, int s_y,
                                                        const BState *__restrict__ bst) {
    using S2 = typename Prec<P>::S2;
    extern __shared__ float4 xb[];
    const BatchDev &B = *Bd;
    if ((int)blockIdx.x >= B.work0[B.nf]) return;
    int fi, grp;
    const int ib = work_item(B, blockIdx.x, colour, fi, grp);
    if (ib < 0) return;
    const BField &F = B.f[fi];
    const GeomDev &g = F.g;
    const int k0 = grp * NR;
    bool any = false;
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (k0 + k < F.nrhs && !bst[F.rhs0 + k0 + k].done) any = true;
    if (!any) return;  // uniform over the workgroup
    const int tpr = F.tpr;
    const int k = threadIdx.x / tpr, tt = threadIdx.x - k * tpr;
    const int d = tt & 1, q0 = tt >> 1, nq = tpr >> 1;
    const int Vb = g.Vb, NS = Vb + 1;
    const bool live = k < NR && k0 + k < F.nrhs;
    float4 *xs = xb + (size_t)min(k, NR - 1) * 6 * NS;
    const size_t ko = (size_t)(k0 + min(k, NR - 1)) * F.nvec;
    const S2 *U = (const S2 *)F.Uin;
    const S2 *Fk = (const S2 *)F.Fin + ((size_t)ib * 2 + d) * 18 * Vb;
    const S2 *src = (const S2 *)F.iv[s_src] + ko;
    S2 *r = (S2 *)F.iv[s_r] + ko;
    S2 *x = (S2 *)F.iv[s_x] + ko;
    S2 *y = (S2 *)F.iv[s_y] + ko;
    const float sg = d ? -1.f : 1.f, kappa = F.kappa, omega = F.omega;
    const bool gather = colour == 1 || !first;

    // 1. v_c (gathering the other colour), zero the iterate and the zero slot
    if (live) {
        int bl[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) bl[mu] = g.blk_nbr[(2 * mu + d) * g.NB + ib];
        for (int i = q0; i < Vb; i += nq) {
            cx<float> v[6];
            load6(v, src, ib, i, d, Vb);
            if (gather) {
                cx<float> acc[12];
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = cxz<float>();
                gather_hop<0>(acc, g, x, U, ib, i, d, bl[0], sg);
                gather_hop<1>(acc, g, x, U, ib, i, d, bl[1], sg);
                gather_hop<2>(acc, g, x, U, ib, i, d, bl[2], sg);
                gather_hop<3>(acc, g, x, U, ib, i, d, bl[3], sg);
                pair_reduce(acc);
                cx<float> own[6], out[6];
#pragma unroll
                for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
                clover_block(out, own, Fk + i, Vb);
#pragma unroll
                for (int e = 0; e < 6; ++e) v[e] = v[e] + kappa * out[e];
            }
            store6(r, ib, i, d, Vb, v);
#pragma unroll
            for (int q = 0; q < 3; ++q) xs[(3 * d + q) * NS + i] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        for (int t = tt; t < 6; t += tpr) xs[t * NS + Vb] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();

    // 2. sweeps, one hyperplane per step; with omega = 1 the repeated plane at the turn of a
    // sweep would get bit-identical values (its neighbours all lie on the side just swept and
    // are unchanged), so that step is skipped (uniform over the workgroup: one field)
    const int H = g.nplanes;
    for (int sw = 0; sw < 2 * F.n_ssor; ++sw) {
        for (int pi = 0; pi < H; ++pi) {
            if (omega == 1.f && sw > 0 && pi == 0) continue;
            const int h = (sw & 1) == 0 ? pi : H - 1 - pi;
            for (int i = F.pst[h] + q0; live && i < F.pst[h + 1]; i += nq) {
                cx<float> out[6], v[6];
                block_hop_clover(out, xs, NS, F.pnb[2 * i + d], F.gnb[i], U, Fk, ib, i, d, Vb, sg);
                load6(v, r, ib, i, d, Vb);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    float4 *o = &xs[(3 * d + q) * NS + i];
                    const float4 ov = *o;
                    const cx<float> n0 = v[2 * q] + kappa * out[2 * q], n1 = v[2 * q + 1] + kappa * out[2 * q + 1];
                    *o = make_float4((1.f - omega) * ov.x + omega * n0.r, (1.f - omega) * ov.y + omega * n0.i,
                                     (1.f - omega) * ov.z + omega * n1.r, (1.f - omega) * ov.w + omega * n1.i);
                }
            }
            __syncthreads();
        }
    }

    // 3. outputs: x_c, y_c += x_c, r_c = v_c - D_cc x_c
    if (!live) return;
    for (int i = q0; i < Vb; i += nq) {
        cx<float> xv[6], yv[6];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float4 f = xs[(3 * d + q) * NS + i];
            xv[2 * q] = {f.x, f.y};
            xv[2 * q + 1] = {f.z, f.w};
        }
        store6(x, ib, i, d, Vb, xv);
        if (first) {
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = xv[e];
        } else {
            load6(yv, y, ib, i, d, Vb);
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = yv[e] + xv[e];
        }
        store6(y, ib, i, d, Vb, yv);
        cx<float> out[6], v[6];
        block_hop_clover(out, xs, NS, F.pnb[2 * i + d], F.gnb[i], U, Fk, ib, i, d, Vb, sg);
        load6(v, r, ib, i, d, Vb);
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = v[e] - xv[e] + kappa * out[e];
        store6(r, ib, i, d, Vb, v);
    }
}

// allow the batched phase kernels the dynamic LDS they are launched with
static void batch_lds_attr(int bytes) {
    const void *fns[] = {
        (const void *)k_bsap_phase<SAPQ_FP32, 1>,    (const void *)k_bsap_phase<SAPQ_FP32, 2>,
        (const void *)k_bsap_phase<SAPQ_FP32, 3>,    (const void *)k_bsap_phase<SAPQ_FP32, 4>,
        (const void *)k_bsap_phase<SAPQ_FP16, 1>,    (const void *)k_bsap_phase<SAPQ_FP16, 2>,
        (const void *)k_bsap_phase<SAPQ_FP16, 3>,    (const void *)k_bsap_phase<SAPQ_FP16, 4>,
        (const void *)k_bsap_phase<SAPQ_BF16, 1>,    (const void *)k_bsap_phase<SAPQ_BF16, 2>,
        (const void *)k_bsap_phase<SAPQ_BF16, 3>,    (const void *)k_bsap_phase<SAPQ_BF16, 4>,
        (const void *)k_bsap_phase_2l<SAPQ_FP32, 1>, (const void *)k_bsap_phase_2l<SAPQ_FP32, 2>,
        (const void *)k_bsap_phase_2l<SAPQ_FP32, 3>, (const void *)k_bsap_phase_2l<SAPQ_FP32, 4>,
        (const void *)k_bsap_phase_2l<SAPQ_FP16, 1>, (const void *)k_bsap_phase_2l<SAPQ_FP16, 2>,
        (const void *)k_bsap_phase_2l<SAPQ_FP16, 3>, (const void *)k_bsap_phase_2l<SAPQ_FP16, 4>,
        (const void *)k_bsap_phase_2l<SAPQ_BF16, 1>, (const void *)k_bsap_phase_2l<SAPQ_BF16, 2>,
        (const void *)k_bsap_phase_2l<SAPQ_BF16, 3>, (const void *)k_bsap_phase_2l<SAPQ_BF16, 4>};
    for (const void *f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// r_c += kappa F sum_{hops leaving the block} H x for every field and right-hand side
template <int P>
__global__ void __launch_bounds__(256) k_bsap_face(const BatchDev *__restrict__ Bd, int colour, int s_r, int s_x,
                                                  const BState *__restrict__ bst) {
    using S2 = typename Prec<P>::S2;
    using C = float;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs || bst[F.rhs0 + k].done) return;
    const GeomDev &g = F.g;
    const long gt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long i = gt >> 2;
    const int j = (int)(gt & 3);
    if (i >= (long)g.NBc * g.Vb) return;
    const int ib = colour * g.NBc + (int)(i / g.Vb), s = (int)(i % g.Vb);
    const size_t ko = (size_t)k * F.nvec;
    S2 *r = (S2 *)F.iv[s_r] + ko;
    const S2 *x = (const S2 *)F.iv[s_x] + ko;
    const LaneNbr n = lane_nbr(g.nbr16[j * g.Vb + s], ib, g.blk_nbr[(2 * j) * g.NB + ib],
                               g.blk_nbr[(2 * j + 1) * g.NB + ib], g.bc[j]);
    cx<C> h[12], fh[3], v[3];
    quad_hop_sum<HOP_OUT, false>(h, g, ib, s, j, n, (const S2 *)F.Uin, FieldSrc<S2, C>{x});
    lane_clover(fh, h, (const S2 *)F.Fin, g, ib, s, j);
    load_spin(v, r, g, ib, s, j);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = v[c] + F.kappa * fh[c];
    store_spin(r, g, ib, s, j, v);
}

// The same face update with two lanes per site (the single-source k_sap_face_2l), for every
// field and right-hand side; sites with no hop out of their block leave at once.
template <int P>
__global__ void __launch_bounds__(256) k_bsap_face_2l(const BatchDev *__restrict__ Bd, int colour, int s_r, int s_x,
                                                     const BState *__restrict__ bst) {
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs || bst[F.rhs0 + k].done) return;
    const GeomDev &g = F.g;
    const long i = xcd_site_base(128) + (threadIdx.x >> 1);
    const int d = threadIdx.x & 1;
    if (i >= (long)g.NBc * g.Vb) return;  // both lanes of a site together
    const int ib = colour * g.NBc + (int)(i / g.Vb), s = (int)(i % g.Vb);
    int outside = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const unsigned w = g.nbr16[mu * g.Vb + s];
        outside |= ((d ? (w >> 16) : w) & 0x8000u) ? 0 : 1;
    }
    outside |= __builtin_amdgcn_update_dpp(0, outside, QUAD_XOR1, 0xF, 0xF, true);
    if (!outside) return;
    const size_t ko = (size_t)k * F.nvec;
    S2 *r = (S2 *)F.iv[s_r] + ko;
    const S2 *x = (const S2 *)F.iv[s_x] + ko;
    const S2 *U = (const S2 *)F.Uin;
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
    clover_block(out, own, (const S2 *)F.Fin + ((size_t)ib * 2 + d) * 18 * g.Vb + s, g.Vb);
    load6(v, r, ib, s, d, g.Vb);
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = v[e] + F.kappa * out[e];
    store6(r, ib, s, d, g.Vb, v);
}

// out = D in in FP64 for every field and right-hand side (outer slots)
__global__ void __launch_bounds__(256) k_bdslash64(const BatchDev *__restrict__ Bd, int s_out, int s_in) {
    using C = double;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const GeomDev &g = F.g;
    const long gt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long i = gt >> 2;
    const int j = (int)(gt & 3);
    if (i >= g.V) return;
    const int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    const size_t ko = (size_t)k * F.nvec;
    const double2 *in = F.dv[s_in] + ko;
    double2 *out = F.dv[s_out] + ko;
    const LaneNbr n = lane_nbr(g.nbr16[j * g.Vb + s], ib, g.blk_nbr[(2 * j) * g.NB + ib],
                               g.blk_nbr[(2 * j + 1) * g.NB + ib], g.bc[j]);
    cx<C> h[12], fh[3], v[3];
    quad_hop_sum<HOP_ALL, false>(h, g, ib, s, j, n, F.U64, FieldSrc<double2, C>{in});
    lane_clover(fh, h, F.F64, g, ib, s, j);
    load_spin(v, in, g, ib, s, j);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = v[c] - (double)F.kappa * fh[c];
    store_spin(out, g, ib, s, j, v);
}

// ---------------------------------------------------------------- batched vector updates
// Coefficients are per right-hand side: a table index selects which BState entry (or 1, -1).
enum { CF_ONE, CF_MONE, CF_MALPHA, CF_MOMEGA, CF_ALPHA, CF_OMEGA };

__device__ __forceinline__ cx<double> coef(const BState &s, int which) {
    switch (which) {
    case CF_ONE: return {1.0, 0.0};
    case CF_MONE: return {-1.0, 0.0};
    case CF_MALPHA: return {-s.alpha.x, -s.alpha.y};
    case CF_MOMEGA: return {-s.omega.x, -s.omega.y};
    case CF_ALPHA: return {s.alpha.x, s.alpha.y};
    default: return {s.omega.x, s.omega.y};
    }
}

// z = x + c y, skipped for finished right-hand sides when masked
template <int P>
__global__ void k_bxpay(const BatchDev *__restrict__ Bd, int s_z, int s_x, int which, int s_y,
                        const BState *__restrict__ bst, int masked) {
    using C = typename Prec<P>::C;
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const BState &S = bst[F.rhs0 + k];
    if (masked && S.done) return;
    const cx<double> cd = coef(S, which);
    const cx<C> c{C(cd.r), C(cd.i)};
    const size_t ko = (size_t)k * F.nvec;
    S2 *z = (S2 *)F.iv[s_z] + ko;
    const S2 *x = (const S2 *)F.iv[s_x] + ko;
    const S2 *y = (const S2 *)F.iv[s_y] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x)
        st(z + i, ld(x + i) + cmul(c, ld(y + i)));
}

// p = r + beta (p - omega v)
template <int P>
__global__ void k_bbicg_p(const BatchDev *__restrict__ Bd, const BState *__restrict__ bst) {
    using C = typename Prec<P>::C;
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const BState &S = bst[F.rhs0 + k];
    if (S.done) return;
    const cx<C> beta{C(S.beta.x), C(S.beta.y)}, om{C(S.omega.x), C(S.omega.y)};
    const size_t ko = (size_t)k * F.nvec;
    S2 *p = (S2 *)F.iv[IV_P] + ko;
    const S2 *r = (const S2 *)F.iv[IV_R] + ko;
    const S2 *v = (const S2 *)F.iv[IV_V] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x)
        st(p + i, ld(r + i) + cmul(beta, ld(p + i) - cmul(om, ld(v + i))));
}

// e += alpha ph + omega sh
template <int P>
__global__ void k_bupdate_e(const BatchDev *__restrict__ Bd, const BState *__restrict__ bst) {
    using C = typename Prec<P>::C;
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const BState &S = bst[F.rhs0 + k];
    if (S.done) return;
    const cx<C> a{C(S.alpha.x), C(S.alpha.y)}, o{C(S.omega.x), C(S.omega.y)};
    const size_t ko = (size_t)k * F.nvec;
    S2 *e = (S2 *)F.iv[IV_E] + ko;
    const S2 *ph = (const S2 *)F.iv[IV_PH] + ko;
    const S2 *sh = (const S2 *)F.iv[IV_SH] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x)
        st(e + i, ld(e + i) + cmul(a, ld(ph + i)) + cmul(o, ld(sh + i)));
}

template <int P>
__global__ void k_bzero(const BatchDev *__restrict__ Bd, int slot) {
    using C = typename Prec<P>::C;
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    S2 *z = (S2 *)F.iv[slot];
    const size_t n = F.nvec * F.nrhs;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(z + i, cxz<C>());
}

// dot products <a_q, b_q> (q < nd) per right-hand side: partial sums per workgroup
constexpr int BDOT_BLOCKS = 64;
template <int P, bool OUTER>
__global__ void __launch_bounds__(256) k_bdots(const BatchDev *__restrict__ Bd, int nd, int a0, int b0, int a1, int b1,
                                               double *__restrict__ partials /* [rhs][BDOT_BLOCKS][4] */) {
    using S2 = typename Prec<P>::S2;
    __shared__ double sm[4][4];
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const size_t ko = (size_t)k * F.nvec;
    const S2 *A0 = (const S2 *)(OUTER ? (const void *)F.dv[a0] : F.iv[a0]) + ko;
    const S2 *B0 = (const S2 *)(OUTER ? (const void *)F.dv[b0] : F.iv[b0]) + ko;
    const S2 *A1 = (const S2 *)(OUTER ? (const void *)F.dv[a1] : F.iv[a1]) + ko;
    const S2 *B1 = (const S2 *)(OUTER ? (const void *)F.dv[b1] : F.iv[b1]) + ko;
    double acc[4] = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x) {
        auto x = ld(A0 + i), y = ld(B0 + i);
        acc[0] += (double)x.r * y.r + (double)x.i * y.i;
        acc[1] += (double)x.r * y.i - (double)x.i * y.r;
        if (nd > 1) {
            auto u = ld(A1 + i), w = ld(B1 + i);
            acc[2] += (double)u.r * w.r + (double)u.i * w.i;
            acc[3] += (double)u.r * w.i - (double)u.i * w.r;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = acc[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sm[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] + sm[3][threadIdx.x];
        partials[((size_t)(F.rhs0 + k) * BDOT_BLOCKS + blockIdx.x) * 4 + threadIdx.x] = v;
    }
}

// scalar steps of BiCGStab, one thread per right-hand side (partials summed in fixed order)
enum { SC_INIT, SC_BETA, SC_ALPHA, SC_OMEGA, SC_UPDATE, SC_OUTER };

__device__ __forceinline__ double2 sum_part(const double *partials, int rhs, int q) {
    double re = 0, im = 0;
    for (int b = 0; b < BDOT_BLOCKS; ++b) {
        re += partials[((size_t)rhs * BDOT_BLOCKS + b) * 4 + 2 * q];
        im += partials[((size_t)rhs * BDOT_BLOCKS + b) * 4 + 2 * q + 1];
    }
    return make_double2(re, im);
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }

__global__ void k_bscalar(int step, int total, const double *__restrict__ partials, BState *__restrict__ st, double tol,
                          int maxit) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    BState &S = st[k];
    if (step == SC_INIT) {
        // partials hold <rt, r> and <r, r>; S.done was set by k_bouter for stopped sources
        S.rho = sum_part(partials, k, 0);
        S.rr = sum_part(partials, k, 1).x;
        S.r0 = sqrt(S.rr);
        S.rho_old = make_double2(1, 0);
        S.alpha = make_double2(1, 0);
        S.omega = make_double2(1, 0);
        S.its = 0;
        S.bad = 0;
        if (!S.done && (!finite2(S.rho) || !isfinite(S.r0))) { S.done = 1; S.bad = 1; }
        if (S.r0 == 0) S.done = 1;
    } else if (!S.done) {
        if (step == SC_BETA) {
            S.beta = cmul2(cdiv(S.rho, S.rho_old), cdiv(S.alpha, S.omega));
        } else if (step == SC_ALPHA) {
            const double2 rv = sum_part(partials, k, 0);
            if (!finite2(rv)) { S.done = 1; S.bad = 1; }
            else if (rv.x == 0 && rv.y == 0) { S.done = 1; S.alpha = make_double2(0, 0); }
            else S.alpha = cdiv(S.rho, rv);
        } else if (step == SC_OMEGA) {
            const double2 ts = sum_part(partials, k, 0);
            const double tt = sum_part(partials, k, 1).x;
            if (!finite2(ts) || !isfinite(tt)) { S.done = 1; S.bad = 1; }
            else S.omega = tt > 0 ? make_double2(ts.x / tt, ts.y / tt) : make_double2(0, 0);
        } else if (step == SC_UPDATE) {
            S.rho_old = S.rho;
            S.rho = sum_part(partials, k, 0);
            S.rr = sum_part(partials, k, 1).x;
            S.its += 1;
            if (!finite2(S.rho) || !isfinite(S.rr)) { S.done = 1; S.bad = 1; }
            else if (sqrt(S.rr) <= tol * S.r0 || S.its >= maxit || (S.omega.x == 0 && S.omega.y == 0) ||
                     (S.rho.x == 0 && S.rho.y == 0))
                S.done = 1;
        }
    }
}

// the number of right-hand sides whose inner solve is still running, after every k_bscalar
// of the launch has ended (one thread, in a launch of its own)
__global__ void k_bcount(const BState *__restrict__ st, int total, int *__restrict__ active) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int n = 0;
        for (int q = 0; q < total; ++q) n += st[q].done ? 0 : 1;
        *active = n;
    }
}

// |b| per right-hand side from the partial sums of <b, b> (start of a batched solve)
__global__ void k_bouter_start(int total, const double *__restrict__ partials, BOuter *__restrict__ os,
                               BState *__restrict__ st) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    BOuter &O = os[k];
    O.bnorm = sqrt(sum_part(partials, k, 0).x);
    O.relres = 1.0;
    O.scale = 0.0;
    O.status = isfinite(O.bnorm) ? OS_RUNNING : OS_BREAKDOWN;
    O.outer_its = O.inner_its = 0;
    st[k].done = 1;
    st[k].bad = 0;
    st[k].its = 0;
}

// The outer step of the FP64 defect correction per right-hand side, from the partial sums of
// |r|^2 for r = b - D x: count the inner solve just applied, the relative residual, the
// status (converged, or breakdown on a non-finite residual or inner scalar), and for the
// running sources the scale of the next inner right-hand side (unit RMS per complex
// component of that field) and a fresh inner state.
__global__ void k_bouter(const BatchDev *__restrict__ Bd, const double *__restrict__ partials, BOuter *__restrict__ os,
                         BState *__restrict__ st, double tol) {
    const BatchDev &B = *Bd;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B.total_rhs) return;
    int f = 0;
    while (f + 1 < B.nf && k >= B.f[f + 1].rhs0) ++f;
    BOuter &O = os[k];
    BState &S = st[k];
    if (O.status == OS_RUNNING && O.scale != 0) {  // an inner solve ran for this source
        O.outer_its += 1;
        O.inner_its += S.its;
        if (S.bad) O.status = OS_BREAKDOWN;
    }
    const double rr = sum_part(partials, k, 0).x;
    if (O.bnorm == 0) {
        O.relres = 0.0;
        if (O.status == OS_RUNNING) O.status = OS_CONVERGED;
    } else {
        O.relres = sqrt(rr) / O.bnorm;
        if (O.status == OS_RUNNING && !isfinite(O.relres)) O.status = OS_BREAKDOWN;
        if (O.status == OS_RUNNING && O.relres <= tol) O.status = OS_CONVERGED;
    }
    const bool run = O.status == OS_RUNNING;
    O.scale = run ? sqrt((double)B.f[f].nvec) / sqrt(rr) : 0.0;
    S.done = run ? 0 : 1;
    S.bad = 0;
    S.its = 0;
}

// inner storage <-> FP64 outer, with a per-right-hand-side scale from the outer norms
template <int P>
__global__ void k_bconvert_in(const BatchDev *__restrict__ Bd, const BOuter *__restrict__ os) {
    using C = typename Prec<P>::C;
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const double sc = os[F.rhs0 + k].scale;
    if (sc == 0) return;
    const size_t ko = (size_t)k * F.nvec;
    S2 *d = (S2 *)F.iv[IV_RIN] + ko;
    const double2 *s = F.dv[DV_R] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x) {
        double2 v = s[i];
        st(d + i, cx<C>{C(v.x * sc), C(v.y * sc)});
    }
}

// x += e / scale after an inner solve (not for a source whose inner solve broke down)
template <int P>
__global__ void k_bconvert_out(const BatchDev *__restrict__ Bd, const BOuter *__restrict__ os,
                               const BState *__restrict__ st) {
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const BOuter &O = os[F.rhs0 + k];
    const double sc = O.scale;
    if (sc == 0 || O.status != OS_RUNNING || st[F.rhs0 + k].bad) return;
    const size_t ko = (size_t)k * F.nvec;
    double2 *x = F.dv[DV_X] + ko;
    const S2 *e = (const S2 *)F.iv[IV_E] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x) {
        auto v = ld(e + i);
        double2 o = x[i];
        x[i] = make_double2(o.x + (double)v.r / sc, o.y + (double)v.i / sc);
    }
}

// r = b - t (FP64)
__global__ void k_bresid(const BatchDev *__restrict__ Bd) {
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y, k = blockIdx.z;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    if (k >= F.nrhs) return;
    const size_t ko = (size_t)k * F.nvec;
    const double2 *b = F.dv[DV_B] + ko, *t = F.dv[DV_T] + ko;
    double2 *r = F.dv[DV_R] + ko;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < F.nvec; i += (size_t)gridDim.x * blockDim.x)
        r[i] = make_double2(b[i].x - t[i].x, b[i].y - t[i].y);
}

template <int P>
__global__ void k_bcopy(const BatchDev *__restrict__ Bd, int s_d, int s_s) {
    using S2 = typename Prec<P>::S2;
    const BatchDev &B = *Bd;
    const int fi = blockIdx.y;
    if (fi >= B.nf) return;
    const BField &F = B.f[fi];
    S2 *d = (S2 *)F.iv[s_d];
    const S2 *s = (const S2 *)F.iv[s_s];
    const size_t n = F.nvec * F.nrhs;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}

// ---------------------------------------------------------------- host driver
struct Batch {
    std::vector<Ctx *> ctx;
    int nf = 0, total = 0, max_rhs = 0;
    long max_V = 0;
    int prec = SAPQ_FP32, NR = 1;
    bool two_lane = false;  // k_bsap_phase_2l (else the four-lane k_bsap_phase)
    bool use_nn = false;    // every context has the learned stage on
    int threads = 0;
    size_t lds = 0;
    hipStream_t stream = nullptr;
    BatchDev host;
    BatchDev *dev = nullptr;
    BState *st = nullptr;
    BOuter *os = nullptr;
    double *partials = nullptr;
    int *active = nullptr;
    int k_inner = 2;  // inner iterations per graph replay (one host check each)
};

static size_t rhs_bytes(Ctx *c, int prec) { return c->nvec * elem_bytes(prec); }

static size_t layout_batch(Batch &B, char *base) {
    size_t used = 0;
    auto take = [&](size_t n) -> void * {
        size_t off = (used + 255) & ~(size_t)255;
        used = off + n;
        return base ? (void *)(base + off) : nullptr;
    };
    B.dev = (BatchDev *)take(sizeof(BatchDev));
    B.st = (BState *)take(sizeof(BState) * B.total);
    B.partials = (double *)take(sizeof(double) * 4 * BDOT_BLOCKS * B.total);
    B.os = (BOuter *)take(sizeof(BOuter) * B.total);
    B.active = (int *)take(sizeof(int) * 4);
    for (int f = 0; f < B.nf; ++f) {
        BField &F = B.host.f[f];
        for (int s = 0; s < NIV; ++s)
            F.iv[s] = (s == IV_Z || s == IV_RP) && !B.use_nn ? nullptr : take(rhs_bytes(B.ctx[f], B.prec) * F.nrhs);
        for (int s = 0; s < NDV; ++s) F.dv[s] = (double2 *)take(B.ctx[f]->nvec * 16 * F.nrhs);
    }
    return used + 256;
}


static int setup_batch(Batch &B, sapq_ctx *const *ctxs, int nctx, const int *nrhs, std::string &why) {
    if (nctx < 1 || nctx > MAX_FIELDS) { why = "between 1 and 16 contexts"; return SAPQ_EINVAL; }
    B.nf = nctx;
    B.total = 0;
    int work = 0;
    for (int f = 0; f < nctx; ++f) {
        if (!ctxs[f] || nrhs[f] < 1) { why = "null context or nrhs < 1"; return SAPQ_EINVAL; }
        Ctx *c = &ctxs[f]->c;
        B.ctx.push_back(c);
        if (f > 0) {
            Ctx *c0 = B.ctx[0];
            for (int m = 0; m < 4; ++m)
                if (c->geom.block[m] != c0->geom.block[m] || c->geom.subblock[m] != c0->geom.subblock[m]) {
                    why = "all contexts need the same block and sub-block shape";
                    return SAPQ_EINVAL;
                }
            if (c->prm.prec_inner != c0->prm.prec_inner) { why = "all contexts need the same prec_inner"; return SAPQ_EINVAL; }
        }
        if (!c->have_U || !c->have_F) { why = "fields must be loaded in every context"; return SAPQ_ESTATE; }
        if (c->prm.flags & SAPQ_FLAG_EOMR) { why = "the batched solver runs the SSOR block inverses only"; return SAPQ_EINVAL; }
        B.max_rhs = std::max(B.max_rhs, nrhs[f]);
        B.max_V = std::max(B.max_V, c->V);
    }
    Ctx *c0 = B.ctx[0];
    B.prec = c0->prm.prec_inner;
    B.stream = c0->stream;
    B.use_nn = true;
    for (Ctx *c : B.ctx) B.use_nn = B.use_nn && c->have_nn && (c->prm.flags & SAPQ_FLAG_NN);
    int max_lds = 65536, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    // two lanes per site when every context runs the one-workgroup two-lane kernel (same
    // block and sub-block shape, so the same decision and tables in all of them)
    B.two_lane = true;
    for (Ctx *c : B.ctx) B.two_lane = B.two_lane && c->use_parts && c->sap_np == 1;
    const size_t per = B.two_lane ? (size_t)(c0->g.Vb + 1) * 6 * sizeof(float4) : (size_t)c0->g.Vb * 12 * sizeof(float2);
    const size_t extra = B.two_lane ? 0 : c0->lds_extra;
    const int tpr = B.two_lane ? c0->part_threads : c0->ssor_threads;
    // right-hand sides per workgroup: one by default.  Larger groups (up to 4, as the LDS and
    // the thread limit allow; SAPQ_BATCH_NR=n, read here, permits them) load a site's links
    // once for all their sources, but their slices wait for each other at every barrier.
    // With the groups of a block consecutive on one XCD (work_item) the links are shared
    // through its L2 anyway, and one source per workgroup measured fastest.  Among the
    // permitted sizes the one that leaves the fewest empty slots in the groups of all fields
    // wins (ties to the larger).
    // sapq_autotune_batch's choice (batch_nr > 0) is taken as it is where the LDS allows it
    int nr_cap = c0->batch_nr > 0 ? c0->batch_nr : 1;
    if (const char *e = getenv("SAPQ_BATCH_NR")) nr_cap = std::max(1, std::min(4, atoi(e)));
    const int nr_only = (c0->batch_nr > 0 && !getenv("SAPQ_BATCH_NR")) ? c0->batch_nr : 0;
    B.k_inner = c0->batch_k > 0 ? c0->batch_k : 2;
    B.NR = 0;
    long best_slots = 0;
    for (int nr : {4, 3, 2, 1}) {
        if (nr > nr_cap || nr > std::max(1, B.max_rhs) || per * nr + extra > (size_t)max_lds ||
            (B.two_lane && nr * tpr > 768) || (nr_only && nr != nr_only))
            continue;
        long slots = 0;
        for (int f = 0; f < nctx; ++f) slots += (long)(nrhs[f] + nr - 1) / nr * nr;
        if (B.NR == 0 || slots < best_slots) {
            B.NR = nr;
            best_slots = slots;
        }
    }
    if (B.NR == 0) { why = "the SAP block is too large for the batched kernel's LDS"; return SAPQ_ESHAPE; }
    B.lds = per * B.NR + extra;
    B.threads = B.two_lane ? B.NR * tpr : c0->ssor_threads;
    if (B.lds > 65536) {
        batch_lds_attr((int)B.lds);
        (void)hipGetLastError();  // clears the runtime's last-error slot
    }
    if (c0->ssor_threads > 512) { why = "hyperplanes too large for the batched kernel"; return SAPQ_ESHAPE; }
    memset(&B.host, 0, sizeof(B.host));
    B.host.nf = nctx;
    for (int f = 0; f < nctx; ++f) {
        Ctx *c = B.ctx[f];
        BField &F = B.host.f[f];
        F.g = c->g;
        F.Uin = c->Uin;
        F.Fin = c->Fin;
        F.U64 = c->U64;
        F.F64 = c->F64;
        F.kappa = (float)c->prm.kappa;
        F.omega = (float)c->prm.omega;
        F.n_ssor = c->prm.n_ssor;
        F.nrhs = nrhs[f];
        F.rhs0 = B.total;
        F.ngroups = (nrhs[f] + B.NR - 1) / B.NR;
        F.nvec = c->nvec;
        F.pnb = c->part_nb;
        F.gnb = c->part_gnb;
        F.pst = c->part_pstart;
        F.tpr = c->part_threads;
        B.host.work0[f] = work;
        work += (c->g.NBc + N_XCD - 1) / N_XCD * N_XCD * F.ngroups;  // a multiple of 8 (work_item)
        B.total += nrhs[f];
    }
    B.host.work0[nctx] = work;
    B.host.total_rhs = B.total;
    return SAPQ_OK;
}

#define BPREC(prec, BODY)                                          \
    switch (prec) {                                                \
    case SAPQ_FP32: { constexpr int P_ = SAPQ_FP32; BODY; } break; \
    case SAPQ_FP16: { constexpr int P_ = SAPQ_FP16; BODY; } break; \
    case SAPQ_BF16: { constexpr int P_ = SAPQ_BF16; BODY; } break; \
    default: break;                                                \
    }

static dim3 vgrid(const Batch &B) { return dim3(256, (unsigned)B.nf, (unsigned)B.max_rhs); }

template <int P, int NR>
static void bphase(Batch &B, int colour, int first, int src, int r, int x, int y) {
    const unsigned nw = (unsigned)B.host.work0[B.nf];
    if (B.two_lane)
        k_bsap_phase_2l<P, NR><<<nw, B.threads, B.lds, B.stream>>>(B.dev, colour, first, src, r, x, y, B.st);
    else
        k_bsap_phase<P, NR><<<nw, B.threads, B.lds, B.stream>>>(B.dev, colour, first, src, r, x, y, B.st);
}

static void bmsap(Batch &B, int src, int y) {
    Ctx *c0 = B.ctx[0];
    for (int j = 0; j < c0->prm.n_sap; ++j) {
        const int s = j == 0 ? src : IV_SAPR;
        for (int colour = 0; colour < 2; ++colour) {
            BPREC(B.prec, ({
                      if (B.NR == 4) bphase<P_, 4>(B, colour, j == 0, s, IV_SAPR, IV_SAPX, y);
                      else if (B.NR == 3) bphase<P_, 3>(B, colour, j == 0, s, IV_SAPR, IV_SAPX, y);
                      else if (B.NR == 2) bphase<P_, 2>(B, colour, j == 0, s, IV_SAPR, IV_SAPX, y);
                      else bphase<P_, 1>(B, colour, j == 0, s, IV_SAPR, IV_SAPX, y);
                  }));
        }
    }
    long maxc = 0;
    for (Ctx *c : B.ctx) maxc = std::max(maxc, (long)c->g.NBc * c->g.Vb);
    if (B.two_lane) {
        const unsigned gx = (unsigned)((2 * maxc + 255) / 256 + N_XCD - 1) / N_XCD * N_XCD;
        dim3 g(gx, (unsigned)B.nf, (unsigned)B.max_rhs);
        BPREC(B.prec, (k_bsap_face_2l<P_><<<g, 256, 0, B.stream>>>(B.dev, 0, IV_SAPR, IV_SAPX, B.st)));
    } else {
        dim3 g((unsigned)((4 * maxc + 255) / 256), (unsigned)B.nf, (unsigned)B.max_rhs);
        BPREC(B.prec, (k_bsap_face<P_><<<g, 256, 0, B.stream>>>(B.dev, 0, IV_SAPR, IV_SAPX, B.st)));
    }
}

static void bdots(Batch &B, int nd, int a0, int b0, int a1, int b1) {
    dim3 g(BDOT_BLOCKS, (unsigned)B.nf, (unsigned)B.max_rhs);
    BPREC(B.prec, (k_bdots<P_, false><<<g, 256, 0, B.stream>>>(B.dev, nd, a0, b0, a1, b1, B.partials)));
}

static void bscalar(Batch &B, int step, double tol, int maxit) {
    k_bscalar<<<(B.total + 63) / 64, 64, 0, B.stream>>>(step, B.total, B.partials, B.st, tol, maxit);
}

static void bcount(Batch &B) { k_bcount<<<1, 64, 0, B.stream>>>(B.st, B.total, B.active); }

static void bxpay(Batch &B, int z, int x, int which, int y, int masked) {
    BPREC(B.prec, (k_bxpay<P_><<<vgrid(B), 256, 0, B.stream>>>(B.dev, z, x, which, y, B.st, masked)));
}

// The inner preconditioner for every field and right-hand side: dst = M_SAP src, or with the
// learned stage dst = z + M_SAP (src - D z), z = N src (the network runs per right-hand side
// on its field's context, the SAP phases batched).  Either way the SAP recurrence leaves
// D dst = src - r_N in IV_SAPR.
static void bprecondition(Batch &B, int src, int dst) {
    if (!B.use_nn) {
        bmsap(B, src, dst);
        return;
    }
    for (int f = 0; f < B.nf; ++f) {
        Ctx *c = B.ctx[f];
        const BField &F = B.host.f[f];
        const size_t stride = rhs_bytes(c, B.prec);
        // the network skips sources that have finished (their done flag, read on the device)
        for (int k = 0; k < F.nrhs; ++k)
            nn_apply(c, (const char *)F.iv[src] + k * stride, (char *)F.iv[IV_Z] + k * stride,
                     (char *)F.iv[IV_RP] + k * stride, &B.st[F.rhs0 + k].done);
    }
    bmsap(B, IV_RP, dst);
    bxpay(B, dst, dst, CF_ONE, IV_Z, 1);
}

// one inner BiCGStab iteration for every active right-hand side (captured in a graph)
static void inner_iteration(Batch &B, double tol, int maxit) {
    bscalar(B, SC_BETA, tol, maxit);
    BPREC(B.prec, (k_bbicg_p<P_><<<vgrid(B), 256, 0, B.stream>>>(B.dev, B.st)));
    bprecondition(B, IV_P, IV_PH);
    bxpay(B, IV_V, IV_P, CF_MONE, IV_SAPR, 1);       // v = D p^ = p - r_N
    bdots(B, 1, IV_RT, IV_V, IV_RT, IV_V);
    bscalar(B, SC_ALPHA, tol, maxit);
    bxpay(B, IV_S, IV_R, CF_MALPHA, IV_V, 1);        // s = r - alpha v
    bprecondition(B, IV_S, IV_SH);
    bxpay(B, IV_T, IV_S, CF_MONE, IV_SAPR, 1);       // t = D s^
    bdots(B, 2, IV_T, IV_S, IV_T, IV_T);
    bscalar(B, SC_OMEGA, tol, maxit);
    BPREC(B.prec, (k_bupdate_e<P_><<<vgrid(B), 256, 0, B.stream>>>(B.dev, B.st)));
    bxpay(B, IV_R, IV_S, CF_MOMEGA, IV_T, 1);        // r = s - omega t
    bdots(B, 2, IV_RT, IV_R, IV_R, IV_R);
    bscalar(B, SC_UPDATE, tol, maxit);
}

// What a batched solve keeps between calls, per device: its stream (graphs cannot be captured
// on the legacy default stream), an event, a pinned host buffer, and the two instantiated
// graphs with the identity of the batch they were captured for (contexts, their versions and
// right-hand sides, arena, tolerances, kernel choices).  A call on the same batch replays them.
struct BatchCache {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    std::vector<unsigned long long> key;
    hipGraphExec_t g_outer = nullptr, g_inner = nullptr;
};
constexpr int BATCH_MAX_DEVICES = 64;
static BatchCache g_bcache[BATCH_MAX_DEVICES];
static std::mutex g_bcache_mu;

static void drop_graphs(BatchCache &C) {
    if (C.g_outer) (void)hipGraphExecDestroy(C.g_outer);
    if (C.g_inner) (void)hipGraphExecDestroy(C.g_inner);
    C.g_outer = C.g_inner = nullptr;
    C.key.clear();
}

static std::vector<unsigned long long> batch_key(const Batch &B, const void *arena, size_t bytes, double tol) {
    std::vector<unsigned long long> k;
    auto dbl = [](double v) { unsigned long long u; memcpy(&u, &v, sizeof u); return u; };
    k.push_back((unsigned long long)(uintptr_t)arena);
    k.push_back(bytes);
    k.push_back(dbl(tol));
    k.push_back((unsigned long long)B.prec | (unsigned long long)B.NR << 8 | (unsigned long long)B.k_inner << 16 |
                (unsigned long long)B.use_nn << 24 | (unsigned long long)B.two_lane << 25);
    for (int f = 0; f < B.nf; ++f) {
        const Ctx *c = B.ctx[f];
        k.push_back(c->serial);
        k.push_back(c->version);
        k.push_back((unsigned long long)B.host.f[f].nrhs);
        k.push_back(dbl(c->prm.tol_inner));
        k.push_back((unsigned long long)c->prm.maxit_inner | (unsigned long long)c->prm.n_sap << 32);
    }
    return k;
}

// The outer step of every right-hand side, on the device (captured once as a graph): apply the
// inner solve just finished (x += e / scale), the true residual r = b - D x in FP64, its norms,
// the status and scale of each source (k_bouter), the count of the running ones, and a fresh
// inner BiCGStab on the scaled residual for those.
static void outer_step(Batch &B, double tol, double tol_in, int maxit_in) {
    dim3 vg = vgrid(B);
    dim3 dg((unsigned)((4 * B.max_V + 255) / 256), (unsigned)B.nf, (unsigned)B.max_rhs);
    dim3 bd(BDOT_BLOCKS, (unsigned)B.nf, (unsigned)B.max_rhs);
    BPREC(B.prec, (k_bconvert_out<P_><<<vg, 256, 0, B.stream>>>(B.dev, B.os, B.st)));
    k_bdslash64<<<dg, 256, 0, B.stream>>>(B.dev, DV_T, DV_X);
    k_bresid<<<vg, 256, 0, B.stream>>>(B.dev);
    k_bdots<SAPQ_FP64, true><<<bd, 256, 0, B.stream>>>(B.dev, 1, DV_R, DV_R, DV_R, DV_R, B.partials);
    k_bouter<<<(B.total + 63) / 64, 64, 0, B.stream>>>(B.dev, B.partials, B.os, B.st, tol);
    bcount(B);
    BPREC(B.prec, (k_bconvert_in<P_><<<vg, 256, 0, B.stream>>>(B.dev, B.os)));
    BPREC(B.prec, (k_bcopy<P_><<<dim3(256, B.nf), 256, 0, B.stream>>>(B.dev, IV_R, IV_RIN)));
    BPREC(B.prec, (k_bcopy<P_><<<dim3(256, B.nf), 256, 0, B.stream>>>(B.dev, IV_RT, IV_RIN)));
    BPREC(B.prec, (k_bzero<P_><<<dim3(256, B.nf), 256, 0, B.stream>>>(B.dev, IV_P)));
    BPREC(B.prec, (k_bzero<P_><<<dim3(256, B.nf), 256, 0, B.stream>>>(B.dev, IV_V)));
    BPREC(B.prec, (k_bzero<P_><<<dim3(256, B.nf), 256, 0, B.stream>>>(B.dev, IV_E)));
    bdots(B, 2, IV_RT, IV_R, IV_R, IV_R);
    bscalar(B, SC_INIT, tol_in, maxit_in);
}

// k_inner inner iterations of every running right-hand side and the count of those still
// running (captured once as a graph; finished sources are masked inside the kernels)
static void inner_steps(Batch &B, double tol_in, int maxit_in) {
    for (int i = 0; i < B.k_inner; ++i) inner_iteration(B, tol_in, maxit_in);
    bcount(B);
}

static int hipok(hipError_t e, const char *what) {
    if (e == hipSuccess) return SAPQ_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return SAPQ_EHIP;
}

}  // namespace sapq

using namespace sapq;

extern "C" {

size_t sapq_batch_arena_bytes(sapq_ctx *const *ctxs, int nctx, const int *nrhs) {
    if (!ctxs || !nrhs) return 0;
    Batch B;
    std::string why;
    if (setup_batch(B, ctxs, nctx, nrhs, why) != SAPQ_OK) return 0;
    return layout_batch(B, nullptr);
}

int sapq_solve_batch(sapq_ctx *const *ctxs, int nctx, const int *nrhs, double *const *x, const double *const *b,
                     double tol, void *arena, size_t arena_bytes, sapq_stats *stats) {
    if (!ctxs || !nrhs || !x || !b || !arena || !(tol > 0)) { set_error("null argument"); return SAPQ_EINVAL; }
    Batch B;
    std::string why;
    int rc = setup_batch(B, ctxs, nctx, nrhs, why);
    if (rc) { set_error(why); return rc; }
    if (((uintptr_t)arena) & 255) { set_error("arena must be 256-byte aligned"); return SAPQ_EINVAL; }
    size_t need = layout_batch(B, nullptr);
    if (arena_bytes < need) { set_error("batch arena too small: need " + std::to_string(need)); return SAPQ_ENOMEM; }
    layout_batch(B, (char *)arena);
    auto t0 = std::chrono::steady_clock::now();
    Ctx *c0 = B.ctx[0];
    const int dev = c0->device;
    if (dev < 0 || dev >= BATCH_MAX_DEVICES) { set_error("device index beyond the batch cache"); return SAPQ_EINVAL; }
    std::lock_guard<std::mutex> lock(g_bcache_mu);
    BatchCache &C = g_bcache[dev];
    // the batch's own stream (default priority) and pinned buffer, kept for later calls
    if (!C.stream && (rc = hipok(hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking), "hipStreamCreate"))) return rc;
    if (!C.ev && (rc = hipok(hipEventCreateWithFlags(&C.ev, hipEventDisableTiming), "hipEventCreate"))) return rc;
    const size_t pin_need = sizeof(int) * 4 + sizeof(BOuter) * B.total;
    if (C.pinned_bytes < pin_need) {
        if (C.pinned) (void)hipHostFree(C.pinned);
        C.pinned = nullptr;
        C.pinned_bytes = 0;
        if ((rc = hipok(hipHostMalloc(&C.pinned, pin_need, hipHostMallocDefault), "hipHostMalloc"))) return rc;
        C.pinned_bytes = pin_need;
    }
    int *host_active = (int *)C.pinned;
    BOuter *host_os = (BOuter *)((char *)C.pinned + sizeof(int) * 4);
    hipStream_t caller = B.stream, s = C.stream;
    // ordered after the work already queued on the caller's stream
    (void)hipEventRecord(C.ev, caller);
    (void)hipStreamWaitEvent(s, C.ev, 0);
    B.stream = s;
    // the context launchers below (pack / unpack, the network) use the context's stream
    std::vector<hipStream_t> saved;
    for (Ctx *c : B.ctx) {
        saved.push_back(c->stream);
        c->stream = s;
    }
    auto restore = [&]() {
        (void)hipStreamSynchronize(s);
        for (size_t f = 0; f < B.ctx.size(); ++f) B.ctx[f]->stream = saved[f];
    };
    const double tol_in = c0->prm.tol_inner;
    const int maxit_in = c0->prm.maxit_inner;
    rc = hipok(hipMemcpyAsync(B.dev, &B.host, sizeof(BatchDev), hipMemcpyHostToDevice, s), "copy batch descriptor");
    if (rc) { restore(); return rc; }
    // pack the sources, zero the solutions and the inner state, |b| per source
    for (int f = 0; f < B.nf; ++f) {
        Ctx *c = B.ctx[f];
        BField &F = B.host.f[f];
        for (int k = 0; k < F.nrhs; ++k) {
            launch_pack_spinor(c, SAPQ_FP64, F.dv[DV_B] + (size_t)k * c->nvec, b[f] + (size_t)k * c->V * 24, 1.0);
            (void)hipMemsetAsync(F.dv[DV_X] + (size_t)k * c->nvec, 0, c->nvec * 16, s);
        }
    }
    (void)hipMemsetAsync(B.st, 0, sizeof(BState) * B.total, s);
    {
        dim3 bd(BDOT_BLOCKS, (unsigned)B.nf, (unsigned)B.max_rhs);
        k_bdots<SAPQ_FP64, true><<<bd, 256, 0, s>>>(B.dev, 1, DV_B, DV_B, DV_B, DV_B, B.partials);
        k_bouter_start<<<(B.total + 63) / 64, 64, 0, s>>>(B.total, B.partials, B.os, B.st);
    }
    // the outer step and k_inner inner iterations as two graphs, captured on the first call for
    // this batch and replayed after
    const std::vector<unsigned long long> key = batch_key(B, arena, arena_bytes, tol);
    if (C.key != key || !C.g_outer || !C.g_inner) {
        drop_graphs(C);
        for (int which = 0; which < 2 && rc == SAPQ_OK; ++which) {
            hipGraph_t graph = nullptr;
            rc = hipok(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            if (rc) break;
            if (which == 0) outer_step(B, tol, tol_in, maxit_in);
            else inner_steps(B, tol_in, maxit_in);
            rc = hipok(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
            if (rc == SAPQ_OK)
                rc = hipok(hipGraphInstantiate(which == 0 ? &C.g_outer : &C.g_inner, graph, nullptr, nullptr, 0),
                           "hipGraphInstantiate");
            if (graph) (void)hipGraphDestroy(graph);
        }
        if (rc) { drop_graphs(C); restore(); return rc; }
        C.key = key;
    }
    // the host reads one count per graph replay: running sources after an outer step, sources
    // whose inner solve still runs after k_inner inner iterations
    auto replay = [&](hipGraphExec_t g, int *count) {
        int r = hipok(hipGraphLaunch(g, s), "hipGraphLaunch");
        if (r == SAPQ_OK) r = hipok(hipMemcpyAsync(host_active, B.active, sizeof(int), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        if (r == SAPQ_OK) r = hipok(hipStreamSynchronize(s), "hipStreamSynchronize");
        *count = *host_active;
        return r;
    };
    int outer = 0, running = 0, left = 0;
    for (;;) {
        if ((rc = replay(C.g_outer, &running))) break;
        if (running == 0 || outer == c0->prm.maxit_outer) break;
        ++outer;
        for (int it = 0; it < maxit_in; it += B.k_inner) {
            if ((rc = replay(C.g_inner, &left))) break;
            if (left == 0) break;
        }
        if (rc) break;
    }
    if (rc == SAPQ_OK) {
        rc = hipok(hipMemcpyAsync(host_os, B.os, sizeof(BOuter) * B.total, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        for (int f = 0; f < B.nf && rc == SAPQ_OK; ++f) {
            Ctx *c = B.ctx[f];
            BField &F = B.host.f[f];
            for (int k = 0; k < F.nrhs; ++k)
                launch_unpack_spinor(c, SAPQ_FP64, x[f] + (size_t)k * c->V * 24, F.dv[DV_X] + (size_t)k * c->nvec, 1.0);
        }
        if (rc == SAPQ_OK) rc = hipok(hipStreamSynchronize(s), "sapq_solve_batch");
        if (rc == SAPQ_OK) rc = hipok(hipGetLastError(), "sapq_solve_batch");
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = rc == SAPQ_OK, broke = false;
    for (int q = 0; q < B.total && rc == SAPQ_OK; ++q) {
        const BOuter &O = host_os[q];
        all = all && O.status == OS_CONVERGED;
        broke = broke || O.status == OS_BREAKDOWN;
        if (stats) {
            memset(&stats[q], 0, sizeof(sapq_stats));
            stats[q].outer_its = O.outer_its;
            stats[q].inner_its = O.inner_its;
            stats[q].true_relres = O.relres;
            stats[q].breakdowns = O.status == OS_BREAKDOWN ? 1 : 0;
            stats[q].time_s = secs;
        }
    }
    restore();
    if (rc) return rc;
    if (broke) { set_error("some right-hand sides broke down (a non-finite source, residual or inner scalar)"); return SAPQ_EBREAKDOWN; }
    if (!all) { set_error("some right-hand sides did not reach the tolerance"); return SAPQ_ENOTCONV; }
    return SAPQ_OK;
}

static std::string batch_tune_key(sapq_ctx *const *ctxs, int nctx, const int *nrhs) {
    std::string k = "batch";
    for (int f = 0; f < nctx; ++f) {
        const Ctx *c = &ctxs[f]->c;
        char b[160];
        snprintf(b, sizeof b, ";L=%dx%dx%dx%d,nrhs=%d", c->geom.L[0], c->geom.L[1], c->geom.L[2], c->geom.L[3], nrhs[f]);
        k += b;
    }
    const Ctx *c = &ctxs[0]->c;
    char b[160];
    snprintf(b, sizeof b, ";B=%dx%dx%dx%d;S=%dx%dx%dx%d;prec=%d;nn=%d", c->geom.block[0], c->geom.block[1],
             c->geom.block[2], c->geom.block[3], c->geom.subblock[0], c->geom.subblock[1], c->geom.subblock[2],
             c->geom.subblock[3], c->prm.prec_inner, (c->prm.flags & SAPQ_FLAG_NN) ? 1 : 0);
    return k + b;
}

int sapq_autotune_batch(sapq_ctx *const *ctxs, int nctx, const int *nrhs, double *const *x, const double *const *b,
                        double tol, void *arena, size_t arena_bytes, const char *cache_json_path, int *nr_out,
                        int *k_out) {
    if (!ctxs || !nrhs || !x || !b || !arena || nctx < 1 || nctx > MAX_FIELDS) { set_error("bad argument"); return SAPQ_EINVAL; }
    for (int f = 0; f < nctx; ++f)
        if (!ctxs[f]) { set_error("null context"); return SAPQ_EINVAL; }
    auto set_all = [&](int nr, int k) {
        for (int f = 0; f < nctx; ++f) {
            ctxs[f]->c.batch_nr = nr;
            ctxs[f]->c.batch_k = k;
        }
    };
    const std::string key = batch_tune_key(ctxs, nctx, nrhs);
    if (cache_json_path) {
        if (FILE *fp = fopen(cache_json_path, "r")) {
            char line[2048];
            int nr = 0, k = 0;
            while (fgets(line, sizeof line, fp)) {
                const char *q = strstr(line, "\"key\": \"");
                if (!q || strncmp(q + 8, key.c_str(), key.size()) != 0 || q[8 + key.size()] != '"') continue;
                const char *a = strstr(line, "\"nr\": "), *c = strstr(line, "\"k_inner\": ");
                if (a && c) { nr = atoi(a + 6); k = atoi(c + 11); }
            }
            fclose(fp);
            if (nr >= 1 && nr <= 4 && k >= 1) {
                set_all(nr, k);
                if (nr_out) *nr_out = nr;
                if (k_out) *k_out = k;
                return SAPQ_OK;
            }
        }
    }
    // every candidate times three batched solves of the sources; the median counts (the first
    // call of a candidate also captures its graphs)
    double best_t = 1e300;
    int best_nr = 1, best_k = 2, rc = SAPQ_OK;
    const int K[3] = {1, 2, 4};
    std::string cand;  // every timed candidate, for the cache record

    for (int nr = 1; nr <= 4; ++nr)
        for (int ki = 0; ki < 3; ++ki) {
            set_all(nr, K[ki]);
            Batch B;
            std::string why;
            if (setup_batch(B, ctxs, nctx, nrhs, why) != SAPQ_OK || B.NR != nr) continue;
            double t[3];
            bool ok = true;
            for (int r = 0; r < 3 && ok; ++r) {
                auto t0 = std::chrono::steady_clock::now();
                const int rr = sapq_solve_batch(ctxs, nctx, nrhs, x, b, tol, arena, arena_bytes, nullptr);
                t[r] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (rr == SAPQ_EHIP || rr == SAPQ_EINVAL || rr == SAPQ_ENOMEM || rr == SAPQ_ESTATE) { rc = rr; ok = false; }
                else if (rr != SAPQ_OK) ok = false;
            }
            if (rc) { set_all(0, 0); return rc; }
            if (!ok) continue;
            std::sort(t, t + 3);
            char cb[64];
            snprintf(cb, sizeof cb, "%s[%d, %d, %.6f]", cand.empty() ? "" : ", ", nr, K[ki], t[1]);
            cand += cb;
            if (t[1] < best_t) {
                best_t = t[1];
                best_nr = nr;
                best_k = K[ki];
            }
        }
    if (best_t >= 1e300) { set_all(0, 0); set_error("no candidate of the batched solver reached the tolerance"); return SAPQ_ENOTCONV; }
    set_all(best_nr, best_k);
    if (nr_out) *nr_out = best_nr;
    if (k_out) *k_out = best_k;
    if (cache_json_path) {
        if (FILE *fp = fopen(cache_json_path, "a")) {
            fprintf(fp, "{\"key\": \"%s\", \"nr\": %d, \"k_inner\": %d, \"time_s\": %.6f, \"candidates\": [%s]}\n",
                    key.c_str(), best_nr, best_k, best_t, cand.c_str());
            fclose(fp);
        }
    }
    return SAPQ_OK;
}

}  // extern "C"
