// SAP phase kernel with the even-odd site-preconditioned block solve in place of the SSOR:
// the block solver of the cited Luscher SAP, which section 3 measures the ll-ordered SSOR
// against at equal cost.  One workgroup per block of the phase's colour, two lanes per site
// (lane d = 0 the forward hops, d = 1 the backward ones, as in k_sap_phase_parts), the block
// vector in LDS in the even-odd site order: slots [0, Ve) hold the sites with an even sum of
// block-local coordinates, [Ve, Vb) the odd ones, slot Vb stays zero (hops leaving the block).
//
// Inside a block A = 1 - K, K = kappa F H restricted to the block.  A hop changes the parity,
// so A x = v reduces to the even sites,
//     (1 - K_eo K_oe) x_e = v_e + K_eo v_o,        x_o = v_o + K_oe x_e,
// and the reduced system gets 2 n_ssor minimal-residual steps from x_e = 0:
//     p = (1 - K_eo K_oe) r,  alpha = <p, r> / <p, p>,  x_e += alpha r,  r -= alpha p.
// Each step applies K to the odd sites (reading the even slots) and then to the even ones
// (reading the odd slots): one application of the block operator, the cost of one SSOR
// half-sweep.  Since a hop never reads a slot of its own parity, a step writes the slots of
// the parity it updates while the other half is read, with one barrier in between.
// The phase around the block solve is that of k_sap_phase_parts (Algorithm 1 fused with the
// M_SAP update): v_c = r_c + kappa F sum_{hops leaving the block} H x_other,
// x_c = A_cc^-1 v_c (approximately), y_c += x_c, r_c = v_c - A_cc x_c.
#include "sapq_impl.h"
#include "twolane.h"

namespace sapq {

struct EomrArgs {
    int colour, gather, first, ssor_only, n_mr;
    float kappa;
    const uint2 *pnb;   // [Vb][2] LDS slots of the 4 neighbours of lane d (16 bits each)
    const uint2 *gnb;   // [Vb] block slots of the 4 backward neighbours (16 bits each)
    const int *pstart;  // [0] = 0, [1] = Ve, [2] = Vb
};

constexpr int EOMR_MAXK = 4;   // sites of one parity per lane pair (the kernel's K, at most)
constexpr int EOMR_WAVES = 8;  // at most 512 threads

// sums of a, b, c over the workgroup, the same values (same order) in every thread
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[3 * wv] = a;
        red[3 * wv + 1] = b;
        red[3 * wv + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int k = 0; k < nw; ++k) {
        a += red[3 * k];
        b += red[3 * k + 1];
        c += red[3 * k + 2];
    }
}

__device__ __forceinline__ void lds_put6(float4 *xs, int NS, int d, int i, const cx<float> v[6]) {
#pragma unroll
    for (int q = 0; q < 3; ++q) xs[(3 * d + q) * NS + i] = make_float4(v[2 * q].r, v[2 * q].i, v[2 * q + 1].r, v[2 * q + 1].i);
}
__device__ __forceinline__ void lds_get6(cx<float> v[6], const float4 *xs, int NS, int d, int i) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float4 f = xs[(3 * d + q) * NS + i];
        v[2 * q] = {f.x, f.y};
        v[2 * q + 1] = {f.z, f.w};
    }
}

// K: sites of one parity per lane pair, the smallest that covers the block (x_e and p of
// those sites stay in registers across the steps)
template <int P, int K>
__global__ void __launch_bounds__(512) k_sap_phase_eomr(GeomDev g, EomrArgs a, const typename Prec<P>::S2 *rsrc,
                                                        typename Prec<P>::S2 *r, typename Prec<P>::S2 *x,
                                                        typename Prec<P>::S2 *y,
                                                        const typename Prec<P>::S2 *__restrict__ U,
                                                        const typename Prec<P>::S2 *__restrict__ F) {
    using S2 = typename Prec<P>::S2;
    extern __shared__ float4 xs[];
    __shared__ double red[3 * EOMR_WAVES];
    const int Vb = g.Vb, NS = Vb + 1, Ve = a.pstart[1];
    const int ib = a.colour * g.NBc + blockIdx.x;
    const int d = threadIdx.x & 1;
    const int q0 = threadIdx.x >> 1, nq = blockDim.x >> 1;
    const float sg = d ? -1.f : 1.f;
    const float kappa = a.kappa;
    const S2 *Fk = F + ((size_t)ib * 2 + d) * 18 * Vb;
    const S2 *vb = a.ssor_only ? rsrc : r;

    // 1. v_c (gathering the other colour) into r; the LDS vector: v on the odd slots, zero on
    //    the even slots and the zero slot
    {
        int bl[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) bl[mu] = g.blk_nbr[(2 * mu + d) * g.NB + ib];
        for (int i = q0; i < Vb; i += nq) {
            cx<float> v[6];
            load6(v, rsrc, ib, i, d, Vb);
            if (!a.ssor_only) {
                if (a.gather) {
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
            }
            if (i < Ve)
#pragma unroll
                for (int e = 0; e < 6; ++e) v[e] = cxz<float>();
            lds_put6(xs, NS, d, i, v);
        }
        if (threadIdx.x < 6) xs[threadIdx.x * NS + Vb] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();

    // 2. the reduced right-hand side r_e = v_e + K_eo v_o onto the even slots (the even-site
    //    hops read only odd slots, so the even slots can be written in the same pass)
    cx<float> xe[K][6];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + k * nq;
#pragma unroll
        for (int e = 0; e < 6; ++e) xe[k][e] = cxz<float>();
        if (i < Ve) {
            cx<float> out[6], v[6];
            block_hop_clover_seq(out, xs, NS, a.pnb[2 * i + d], a.gnb[i], U, Fk, ib, i, d, Vb, sg);
            load6(v, vb, ib, i, d, Vb);
#pragma unroll
            for (int e = 0; e < 6; ++e) v[e] = v[e] + kappa * out[e];
            lds_put6(xs, NS, d, i, v);
        }
    }
    __syncthreads();

    // 3. minimal-residual steps on the reduced system
    for (int it = 0; it < a.n_mr; ++it) {
        // (a) t_o = K_oe r_e onto the odd slots
        for (int i = Ve + q0; i < Vb; i += nq) {
            cx<float> out[6];
            block_hop_clover_seq(out, xs, NS, a.pnb[2 * i + d], a.gnb[i], U, Fk, ib, i, d, Vb, sg);
#pragma unroll
            for (int e = 0; e < 6; ++e) out[e] = kappa * out[e];
            lds_put6(xs, NS, d, i, out);
        }
        __syncthreads();
        // (b) p = r_e - K_eo t_o and the partial sums of <p, r> and <p, p>
        cx<float> pe[K][6];
        double pr = 0.0, pi = 0.0, pp = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = q0 + k * nq;
#pragma unroll
            for (int e = 0; e < 6; ++e) pe[k][e] = cxz<float>();
            if (i < Ve) {
                cx<float> out[6], rv[6];
                block_hop_clover_seq(out, xs, NS, a.pnb[2 * i + d], a.gnb[i], U, Fk, ib, i, d, Vb, sg);
                lds_get6(rv, xs, NS, d, i);
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    pe[k][e] = rv[e] - kappa * out[e];
                    const double p_r = pe[k][e].r, p_i = pe[k][e].i, r_r = rv[e].r, r_i = rv[e].i;
                    pr += p_r * r_r + p_i * r_i;
                    pi += p_r * r_i - p_i * r_r;
                    pp += p_r * p_r + p_i * p_i;
                }
            }
        }
        block_sum3(pr, pi, pp, red);  // its barrier also ends every read of the odd slots
        const float ar = pp > 0.0 ? (float)(pr / pp) : 0.f, ai = pp > 0.0 ? (float)(pi / pp) : 0.f;
        // (c) x_e += alpha r_e,  r_e -= alpha p  (the new r_e onto the even slots)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = q0 + k * nq;
            if (i < Ve) {
                cx<float> rv[6];
                lds_get6(rv, xs, NS, d, i);
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    xe[k][e] = {xe[k][e].r + ar * rv[e].r - ai * rv[e].i, xe[k][e].i + ar * rv[e].i + ai * rv[e].r};
                    rv[e] = {rv[e].r - (ar * pe[k][e].r - ai * pe[k][e].i), rv[e].i - (ar * pe[k][e].i + ai * pe[k][e].r)};
                }
                lds_put6(xs, NS, d, i, rv);
            }
        }
        __syncthreads();
    }

    // 4. x_e onto the even slots, then x_o = v_o + K_oe x_e onto the odd ones
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int i = q0 + k * nq;
        if (i < Ve) lds_put6(xs, NS, d, i, xe[k]);
    }
    __syncthreads();
    for (int i = Ve + q0; i < Vb; i += nq) {
        cx<float> out[6], v[6];
        block_hop_clover_seq(out, xs, NS, a.pnb[2 * i + d], a.gnb[i], U, Fk, ib, i, d, Vb, sg);
        load6(v, vb, ib, i, d, Vb);
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = v[e] + kappa * out[e];
        lds_put6(xs, NS, d, i, v);
    }
    __syncthreads();

    // 5. outputs: x_c, y_c += x_c, r_c = v_c - A_cc x_c
    for (int i = q0; i < Vb; i += nq) {
        cx<float> xv[6];
        lds_get6(xv, xs, NS, d, i);
        store6(x, ib, i, d, Vb, xv);
        if (a.ssor_only) continue;
        cx<float> yv[6];
        if (a.first) {
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = xv[e];
        } else {
            load6(yv, y, ib, i, d, Vb);
#pragma unroll
            for (int e = 0; e < 6; ++e) yv[e] = yv[e] + xv[e];
        }
        store6(y, ib, i, d, Vb, yv);
        cx<float> out[6], v[6];
        block_hop_clover_seq(out, xs, NS, a.pnb[2 * i + d], a.gnb[i], U, Fk, ib, i, d, Vb, sg);
        load6(v, r, ib, i, d, Vb);
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] = v[e] - xv[e] + kappa * out[e];
        store6(r, ib, i, d, Vb, v);
    }
}

// sites per block, from the geometry (valid from planning on, before the device tables)
static int eomr_vb(const Ctx *c) {
    return c->geom.block[0] * c->geom.block[1] * c->geom.block[2] * c->geom.block[3];
}

// sites of one parity per lane pair (Vb even: Vb / 2 sites of each parity)
static int eomr_k(const Ctx *c) {
    const int nq = c->part_threads / 2, nh = eomr_vb(c) / 2;
    return (nh + nq - 1) / nq;
}

bool eomr_supported(const Ctx *c, std::string &why) {
    const sapq_geom &G = c->geom;
    if (G.subblock[0] || G.subblock[1] || G.subblock[2] || G.subblock[3]) {
        why = "the even-odd MR block solver needs the even-odd site order (sub-block {0, 0, 0, 0})";
        return false;
    }
    if (eomr_vb(c) % 2) {
        why = "the even-odd MR block solver needs an even number of sites per block";
        return false;
    }
    if (!c->use_parts || c->sap_np != 1) {
        why = "the even-odd MR block solver needs a block whose vector fits one workgroup's LDS";
        return false;
    }
    if (c->part_threads > 64 * EOMR_WAVES || c->part_threads % 64 || eomr_k(c) > EOMR_MAXK ||
        c->parts_lds + 3 * EOMR_WAVES * sizeof(double) > 160 * 1024) {
        why = "block too large for the even-odd MR block solver";
        return false;
    }
    return true;
}

void launch_sap_phase_eomr(Ctx *c, int colour, int gather, int first, int ssor_only, const void *rsrc, void *r,
                           void *x, void *y) {
    EomrArgs a;
    a.colour = colour;
    a.gather = gather;
    a.first = first;
    a.ssor_only = ssor_only;
    a.n_mr = 2 * c->prm.n_ssor;
    a.kappa = (float)c->prm.kappa;
    a.pnb = c->part_nb;
    a.gnb = c->part_gnb;
    a.pstart = c->part_pstart;
    const dim3 grid(c->g.NBc), block(c->part_threads);
    const int K = eomr_k(c);
    INNER_SWITCH(c->prm.prec_inner, ({
                     using S2 = typename Prec<P_>::S2;
                     const S2 *rs = (const S2 *)rsrc, *Uc = (const S2 *)c->Uin, *Fc = (const S2 *)c->Fin;
                     S2 *rr = (S2 *)r, *xx = (S2 *)x, *yy = (S2 *)y;
                     if (K == 1)
                         k_sap_phase_eomr<P_, 1><<<grid, block, c->parts_lds, c->stream>>>(c->g, a, rs, rr, xx, yy, Uc, Fc);
                     else if (K == 2)
                         k_sap_phase_eomr<P_, 2><<<grid, block, c->parts_lds, c->stream>>>(c->g, a, rs, rr, xx, yy, Uc, Fc);
                     else if (K == 3)
                         k_sap_phase_eomr<P_, 3><<<grid, block, c->parts_lds, c->stream>>>(c->g, a, rs, rr, xx, yy, Uc, Fc);
                     else
                         k_sap_phase_eomr<P_, 4><<<grid, block, c->parts_lds, c->stream>>>(c->g, a, rs, rr, xx, yy, Uc, Fc);
                 }));
}

int set_eomr_lds_limit(Ctx *c) {
    if (!c->use_parts || c->parts_lds <= 65536) return 0;
    const int bytes = (int)c->parts_lds;
    INNER_SWITCH(c->prm.prec_inner, ({
                     const void *fn[4] = {(const void *)k_sap_phase_eomr<P_, 1>, (const void *)k_sap_phase_eomr<P_, 2>,
                                          (const void *)k_sap_phase_eomr<P_, 3>, (const void *)k_sap_phase_eomr<P_, 4>};
                     for (const void *f : fn) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
                 }));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace sapq
