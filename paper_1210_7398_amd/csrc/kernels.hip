// HIP kernels of libsapq for gfx950: layout conversion, the clover-Wilson operator,
// the SAP phase kernels (gather, SSOR in hyperplane order, block hop) and BLAS-1.
#include "twolane.h"

namespace sapq {

// ================================================================ layout conversion
template <int P>
__global__ void k_pack_spinor(GeomDev g, typename Prec<P>::S2 *dst, const double2 *src, double scale) {
    using C = typename Prec<P>::C;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    const double2 *p = src + lex_site(g, ib, s) * 12;
    typename Prec<P>::S2 *q = dst + (size_t)ib * 12 * g.Vb + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 v = p[c];
        st(q + (size_t)c * g.Vb, cx<C>{C(v.x * scale), C(v.y * scale)});
    }
}

// FP32 (re, im) pairs in the interchange layout -> FP32 internal layout
__global__ void k_pack_spinor_f32(GeomDev g, float2 *dst, const float2 *src) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    const float2 *p = src + lex_site(g, ib, s) * 12;
    float2 *q = dst + (size_t)ib * 12 * g.Vb + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) q[(size_t)c * g.Vb] = p[c];
}

// FP64 internal layout -> FP32 (re, im) pairs in the interchange layout (rounded)
__global__ void k_unpack_spinor_f32(GeomDev g, float2 *dst, const double2 *src) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    float2 *p = dst + lex_site(g, ib, s) * 12;
    const double2 *q = src + (size_t)ib * 12 * g.Vb + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const double2 v = q[(size_t)c * g.Vb];
        p[c] = make_float2((float)v.x, (float)v.y);
    }
}

template <int P>
__global__ void k_unpack_spinor(GeomDev g, double2 *dst, const typename Prec<P>::S2 *src, double scale) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    double2 *p = dst + lex_site(g, ib, s) * 12;
    const typename Prec<P>::S2 *q = src + (size_t)ib * 12 * g.Vb + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        auto v = ld(q + (size_t)c * g.Vb);
        p[c] = make_double2((double)v.r * scale, (double)v.i * scale);
    }
}

// links: keep rows 0 and 1; record max(|U^+U - 1|, |det U - 1|) per workgroup
template <int P>
__global__ void k_pack_links(GeomDev g, const double2 *src, double2 *U64, typename Prec<P>::S2 *Uin, double *dev) {
    using C = typename Prec<P>::C;
    __shared__ double red[256];
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double worst = 0.0;
    if (i < g.V) {
        int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
        const double2 *p = src + lex_site(g, ib, s) * 36;
        for (int mu = 0; mu < 4; ++mu) {
            cx<double> u[9];
            for (int e = 0; e < 9; ++e) u[e] = {p[9 * mu + e].x, p[9 * mu + e].y};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    cx<double> t = cmulc(u[a], u[b]) + cmulc(u[3 + a], u[3 + b]) + cmulc(u[6 + a], u[6 + b]);
                    double re = t.r - (a == b ? 1.0 : 0.0);
                    worst = fmax(worst, sqrt(re * re + t.i * t.i));
                }
            cx<double> det = cmul(u[0], cmul(u[4], u[8]) - cmul(u[5], u[7])) -
                             cmul(u[1], cmul(u[3], u[8]) - cmul(u[5], u[6])) +
                             cmul(u[2], cmul(u[3], u[7]) - cmul(u[4], u[6]));
            worst = fmax(worst, sqrt((det.r - 1) * (det.r - 1) + det.i * det.i));
            size_t base = ((size_t)ib * 4 + mu) * 6 * g.Vb + s;
            for (int e = 0; e < 6; ++e) {
                U64[base + (size_t)e * g.Vb] = make_double2(u[e].r, u[e].i);
                st(Uin + base + (size_t)e * g.Vb, cx<C>{C(u[e].r), C(u[e].i)});
            }
        }
    }
    red[threadIdx.x] = worst;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dev[blockIdx.x] = red[0];
}

// clover: each hermitian chiral block [[A, B], [B^+, C]] (A, C hermitian 3x3) is stored as
// 18 complex slots: the six real diagonal entries pairwise (3 slots), the strict lower
// triangles of A and of C (3 + 3 slots), and B row by row (9 slots).
template <int P>
__global__ void k_pack_clover(GeomDev g, const double2 *src, double2 *F64, typename Prec<P>::S2 *Fin) {
    using C = typename Prec<P>::C;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int ib = (int)(i / g.Vb), s = (int)(i - (long)ib * g.Vb);
    const double2 *p = src + lex_site(g, ib, s) * 72;
    for (int k = 0; k < 2; ++k) {
        const double2 *m = p + 36 * k;
        size_t base = ((size_t)ib * 2 + k) * 18 * g.Vb + s;
        cx<double> e[18];
        for (int d = 0; d < 3; ++d) e[d] = {m[7 * (2 * d)].x, m[7 * (2 * d + 1)].x};
        const int lo[3][2] = {{1, 0}, {2, 0}, {2, 1}};
        for (int q = 0; q < 3; ++q) {
            e[3 + q] = {m[6 * lo[q][0] + lo[q][1]].x, m[6 * lo[q][0] + lo[q][1]].y};
            e[6 + q] = {m[6 * (3 + lo[q][0]) + 3 + lo[q][1]].x, m[6 * (3 + lo[q][0]) + 3 + lo[q][1]].y};
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) e[9 + 3 * a + b] = {m[6 * a + 3 + b].x, m[6 * a + 3 + b].y};
        for (int t = 0; t < 18; ++t) {
            F64[base + (size_t)t * g.Vb] = make_double2(e[t].r, e[t].i);
            st(Fin + base + (size_t)t * g.Vb, cx<C>{C(e[t].r), C(e[t].i)});
        }
    }
}

// ================================================================ full operator D
// out = in - kappa F H in; two lanes per site (lane 0 the four forward hops, lane 1 the four
// backward ones, as in the SAP phase kernels), DSLASH_SITES(P) sites per workgroup (64 in FP64,
// whose 248 VGPRs allow two waves per SIMD, else 128).  Workgroups are dealt
// to the 8 XCDs in turn (each with its own L2); the grid is a multiple of 8 and XCD x takes
// the x-th eighth of the sites, blocks in lexicographic order, so that most neighbours a
// workgroup reads were fetched into the same L2 by its neighbouring workgroups.
constexpr int dslash_sites(int P) { return P == SAPQ_FP64 ? 64 : 128; }

template <int P>
__global__ void __launch_bounds__(2 * dslash_sites(P)) k_dslash(GeomDev g, typename Prec<P>::S2 *__restrict__ out,
                                               const typename Prec<P>::S2 *__restrict__ in,
                                               const typename Prec<P>::S2 *__restrict__ U,
                                               const typename Prec<P>::S2 *__restrict__ F, double kappa) {
    using C = typename Prec<P>::C;
    const long i = xcd_site_base(dslash_sites(P)) + (threadIdx.x >> 1);
    const int d = threadIdx.x & 1;
    if (i >= g.V) return;
    const int bl = (int)(i / g.Vb), s = (int)(i - (long)bl * g.Vb);
    const int ib = g.lex_blk[bl];
    const C sg = d ? C(-1) : C(1);
    cx<C> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cxz<C>();
    hop_any<0>(acc, g, in, U, ib, s, d, sg);
    hop_any<1>(acc, g, in, U, ib, s, d, sg);
    hop_any<2>(acc, g, in, U, ib, s, d, sg);
    hop_any<3>(acc, g, in, U, ib, s, d, sg);
    pair_reduce(acc);
    cx<C> own[6], fh[6], v[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) own[e] = sel(d != 0, acc[6 + e], acc[e]);
    clover_block(fh, own, F + ((size_t)ib * 2 + d) * 18 * g.Vb + s, g.Vb);
    load6(v, in, ib, s, d, g.Vb);
    const C k = C(kappa);
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = rfma(-k, fh[e], v[e]);
    store6(out, ib, s, d, g.Vb, v);
}

// ================================================================ SAP phase kernel
// One workgroup per block of colour `colour` (Algorithm 1 fused with the M_SAP update):
//   v_c = r_c + kappa F sum_{hops leaving the block} H x_other   (= r_c - D_{c,other} x_other)
//   x_c = SSOR block inverse of v_c (n_ssor forward+backward sweeps from 0; the sweeps walk
//         the hyperplanes of the sub-block-local coordinates, whose sites are independent)
//   y_c = (first ? 0 : y_c) + x_c,   r_c = v_c - D_cc x_c,   x_c kept for the other colour.
// ssor_only: v_c = rsrc and only x_c is written.  Four lanes per site throughout.
struct SapArgs {
    int colour, gather, first, ssor_only, n_ssor;
    float kappa, omega;
};

template <int P, bool XLDS, int NT>
__global__ void __launch_bounds__(NT) k_sap_phase(GeomDev g, SapArgs a, const typename Prec<P>::S2 *rsrc,
                                                  typename Prec<P>::S2 *r, typename Prec<P>::S2 *x,
                                                  typename Prec<P>::S2 *y, const typename Prec<P>::S2 *__restrict__ U,
                                                  const typename Prec<P>::S2 *__restrict__ F, float2 *scratch) {
    using S2 = typename Prec<P>::S2;
    using C = float;
    // LDS: [iterate x (XLDS only): 12 Vb float2][neighbour words: 4 Vb][plane starts: MAX_PLANES + 1]
    extern __shared__ float2 lds[];
    const int ib = a.colour * g.NBc + blockIdx.x;
    float2 *xs = XLDS ? lds : scratch + (size_t)ib * 12 * g.Vb;
    unsigned *nb_lds = reinterpret_cast<unsigned *>(lds + (XLDS ? 12 * g.Vb : 0));
    int *ps_lds = reinterpret_cast<int *>(nb_lds + 4 * g.Vb);
    const C kappa = a.kappa, omega = a.omega;
    const S2 *vb = a.ssor_only ? rsrc : r;  // where v_c lives during the sweeps
    const int j = threadIdx.x & 3;
    const int q0 = threadIdx.x >> 2, nq = blockDim.x >> 2;
    const BlockSrc bs{xs};
    const int bl_f = g.blk_nbr[(2 * j) * g.NB + ib], bl_b = g.blk_nbr[(2 * j + 1) * g.NB + ib];
    const float bc = g.bc[j];

    for (int t = threadIdx.x; t < 4 * g.Vb; t += blockDim.x) nb_lds[t] = g.nbr16[t];
    for (int t = threadIdx.x; t <= g.nplanes; t += blockDim.x) ps_lds[t] = g.plane_start[t];
    __syncthreads();

    // 1. v_c (gathering the other colour), zero the iterate
    for (int s = q0; s < g.Vb; s += nq) {
        if (!a.ssor_only) {
            cx<C> v[3];
            load_spin(v, rsrc, g, ib, s, j);
            if (a.gather) {
                const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
                cx<C> h[12], fh[3];
                quad_hop_sum<HOP_OUT, (NT > 512)>(h, g, ib, s, j, n, U, FieldSrc<S2, C>{x});
                lane_clover(fh, h, F, g, ib, s, j);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = v[c] + kappa * fh[c];
            }
            store_spin(r, g, ib, s, j, v);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) xs[(3 * j + c) * g.Vb + s] = make_float2(0.f, 0.f);
    }
    __syncthreads();

    // 2. sweeps: x_n <- (1-omega) x_n + omega (v_n + kappa F(n) sum_{m in block} H_nm x_m)
    for (int sw = 0; sw < a.n_ssor; ++sw) {
        for (int dir = 0; dir < 2; ++dir) {
            for (int pi = 0; pi < g.nplanes; ++pi) {
                const int p = dir == 0 ? pi : g.nplanes - 1 - pi;
                const int s0 = ps_lds[p], s1 = ps_lds[p + 1];
                for (int s = s0 + q0; s < s1; s += nq) {
                    const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
                    cx<C> h[12], fh[3], v[3];
                    quad_hop_sum<HOP_IN, (NT > 512)>(h, g, ib, s, j, n, U, bs);
                    if (NT > 512) __builtin_amdgcn_sched_barrier(0);
                    lane_clover(fh, h, F, g, ib, s, j);
                    load_spin(v, vb, g, ib, s, j);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float2 *o = &xs[(3 * j + c) * g.Vb + s];
                        float2 ov = *o;
                        cx<C> nx = v[c] + kappa * fh[c];
                        *o = make_float2((1.f - omega) * ov.x + omega * nx.r, (1.f - omega) * ov.y + omega * nx.i);
                    }
                }
                __syncthreads();
            }
        }
    }

    // 3. outputs
    for (int s = q0; s < g.Vb; s += nq) {
        cx<C> xv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float2 t = xs[(3 * j + c) * g.Vb + s];
            xv[c] = {t.x, t.y};
        }
        store_spin(x, g, ib, s, j, xv);
        if (a.ssor_only) continue;
        cx<C> yv[3];
        if (a.first) {
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = xv[c];
        } else {
            load_spin(yv, y, g, ib, s, j);
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = yv[c] + xv[c];
        }
        store_spin(y, g, ib, s, j, yv);
        const LaneNbr n = lane_nbr(nb_lds[j * g.Vb + s], ib, bl_f, bl_b, bc);
        cx<C> h[12], fh[3], v[3];
        quad_hop_sum<HOP_IN, (NT > 512)>(h, g, ib, s, j, n, U, bs);
        lane_clover(fh, h, F, g, ib, s, j);
        load_spin(v, r, g, ib, s, j);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = v[c] - xv[c] + kappa * fh[c];
        store_spin(r, g, ib, s, j, v);
    }
}

// Neighbours of lane j inside the block, for fields staged in LDS (block index 0 there);
// outside neighbours keep their wrapped slot, a valid LDS address, and are masked by the hop.
__device__ __forceinline__ LaneNbr lane_nbr_local(unsigned w) {
    LaneNbr n;
    n.s_f = (int)(w & 0x7fffu);
    n.in_f = (w & 0x8000u) != 0;
    n.s_b = (int)((w >> 16) & 0x7fffu);
    n.in_b = (w & 0x80000000u) != 0;
    n.ib_f = n.ib_b = 0;
    n.ph_f = n.ph_b = 1.f;
    return n;
}

// The phase kernel for blocks whose links and clover field fit in LDS next to the iterate:
// they are copied in once and all sweeps and the block hop read LDS only.
// LDS: [x 12 Vb float2][links 24 Vb S2][clover 36 Vb S2][neighbour words 4 Vb][plane starts]
template <int P, int NT>
__global__ void __launch_bounds__(NT) k_sap_phase_staged(GeomDev g, SapArgs a, const typename Prec<P>::S2 *rsrc,
                                                         typename Prec<P>::S2 *r, typename Prec<P>::S2 *x,
                                                         typename Prec<P>::S2 *y, const typename Prec<P>::S2 *__restrict__ U,
                                                         const typename Prec<P>::S2 *__restrict__ F) {
    using S2 = typename Prec<P>::S2;
    using C = float;
    extern __shared__ float2 lds[];
    const int ib = a.colour * g.NBc + blockIdx.x;
    const int Vb = g.Vb;
    float2 *xs = lds;
    S2 *Ul = reinterpret_cast<S2 *>(xs + 12 * Vb);
    S2 *Fl = Ul + 24 * Vb;
    unsigned *nb_lds = reinterpret_cast<unsigned *>(Fl + 36 * Vb);
    int *ps_lds = reinterpret_cast<int *>(nb_lds + 4 * Vb);
    const C kappa = a.kappa, omega = a.omega;
    const S2 *vb = a.ssor_only ? rsrc : r;
    const int j = threadIdx.x & 3;
    const int q0 = threadIdx.x >> 2, nq = blockDim.x >> 2;
    const BlockSrc bs{xs};
    const int bl_f = g.blk_nbr[(2 * j) * g.NB + ib], bl_b = g.blk_nbr[(2 * j + 1) * g.NB + ib];
    const float bc = g.bc[j];

    {
        const S2 *Ug = U + (size_t)ib * 24 * Vb;
        const S2 *Fg = F + (size_t)ib * 36 * Vb;
        for (int t = threadIdx.x; t < 24 * Vb; t += blockDim.x) Ul[t] = Ug[t];
        for (int t = threadIdx.x; t < 36 * Vb; t += blockDim.x) Fl[t] = Fg[t];
        for (int t = threadIdx.x; t < 4 * Vb; t += blockDim.x) nb_lds[t] = g.nbr16[t];
        for (int t = threadIdx.x; t <= g.nplanes; t += blockDim.x) ps_lds[t] = g.plane_start[t];
    }
    __syncthreads();

    // 1. v_c (gathering the other colour from global memory), zero the iterate
    for (int s = q0; s < Vb; s += nq) {
        if (!a.ssor_only) {
            cx<C> v[3];
            load_spin(v, rsrc, g, ib, s, j);
            if (a.gather) {
                const LaneNbr n = lane_nbr(nb_lds[j * Vb + s], ib, bl_f, bl_b, bc);
                cx<C> h[12], fh[3];
                quad_hop_sum<HOP_OUT, false>(h, g, ib, s, j, n, U, FieldSrc<S2, C>{x});
                lane_clover(fh, h, Fl, g, 0, s, j);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = v[c] + kappa * fh[c];
            }
            store_spin(r, g, ib, s, j, v);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) xs[(3 * j + c) * Vb + s] = make_float2(0.f, 0.f);
    }
    __syncthreads();

    // 2. sweeps, from LDS
    for (int sw = 0; sw < a.n_ssor; ++sw) {
        for (int dir = 0; dir < 2; ++dir) {
            for (int pi = 0; pi < g.nplanes; ++pi) {
                const int p = dir == 0 ? pi : g.nplanes - 1 - pi;
                const int s0 = ps_lds[p], s1 = ps_lds[p + 1];
                for (int s = s0 + q0; s < s1; s += nq) {
                    cx<C> v[3];
                    load_spin(v, vb, g, ib, s, j);
                    const LaneNbr n = lane_nbr_local(nb_lds[j * Vb + s]);
                    cx<C> h[12], fh[3];
                    quad_hop_sum<HOP_IN, false>(h, g, 0, s, j, n, Ul, bs);
                    lane_clover(fh, h, Fl, g, 0, s, j);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float2 *o = &xs[(3 * j + c) * Vb + s];
                        float2 ov = *o;
                        cx<C> nx = v[c] + kappa * fh[c];
                        *o = make_float2((1.f - omega) * ov.x + omega * nx.r, (1.f - omega) * ov.y + omega * nx.i);
                    }
                }
                __syncthreads();
            }
        }
    }

    // 3. outputs
    for (int s = q0; s < Vb; s += nq) {
        cx<C> xv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float2 t = xs[(3 * j + c) * Vb + s];
            xv[c] = {t.x, t.y};
        }
        store_spin(x, g, ib, s, j, xv);
        if (a.ssor_only) continue;
        cx<C> yv[3];
        if (a.first) {
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = xv[c];
        } else {
            load_spin(yv, y, g, ib, s, j);
#pragma unroll
            for (int c = 0; c < 3; ++c) yv[c] = yv[c] + xv[c];
        }
        store_spin(y, g, ib, s, j, yv);
        const LaneNbr n = lane_nbr_local(nb_lds[j * Vb + s]);
        cx<C> h[12], fh[3], v[3];
        quad_hop_sum<HOP_IN, false>(h, g, 0, s, j, n, Ul, bs);
        lane_clover(fh, h, Fl, g, 0, s, j);
        load_spin(v, r, g, ib, s, j);
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = v[c] - xv[c] + kappa * fh[c];
        store_spin(r, g, ib, s, j, v);
    }
}

// r_c += kappa F sum_{hops leaving the block} H x   (r_c -= D_{c,other} x_other); four lanes per site
template <int P>
__global__ void __launch_bounds__(256) k_sap_face(GeomDev g, int colour, float kappa, typename Prec<P>::S2 *r,
                                                 const typename Prec<P>::S2 *x, const typename Prec<P>::S2 *__restrict__ U,
                                                 const typename Prec<P>::S2 *__restrict__ F) {
    using S2 = typename Prec<P>::S2;
    using C = float;
    const long gt = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long i = gt >> 2;
    const int j = (int)(gt & 3);
    const long nc = (long)g.NBc * g.Vb;
    if (i >= nc) return;
    const int ib = colour * g.NBc + (int)(i / g.Vb), s = (int)(i % g.Vb);
    const LaneNbr n = lane_nbr(g.nbr16[j * g.Vb + s], ib, g.blk_nbr[(2 * j) * g.NB + ib], g.blk_nbr[(2 * j + 1) * g.NB + ib],
                               g.bc[j]);
    cx<C> h[12], fh[3], v[3];
    quad_hop_sum<HOP_OUT, false>(h, g, ib, s, j, n, U, FieldSrc<S2, C>{x});
    lane_clover(fh, h, F, g, ib, s, j);
    load_spin(v, r, g, ib, s, j);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = v[c] + kappa * fh[c];
    store_spin(r, g, ib, s, j, v);
}

// ================================================================ BLAS-1
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial sums of <a_k, b_k> (k < nd) per workgroup, in double
template <int P>
__global__ void __launch_bounds__(RED_THREADS) k_dots(size_t n, int nd, const typename Prec<P>::S2 *a0,
                                                     const typename Prec<P>::S2 *b0, const typename Prec<P>::S2 *a1,
                                                     const typename Prec<P>::S2 *b1, const typename Prec<P>::S2 *a2,
                                                     const typename Prec<P>::S2 *b2, double2 *partials) {
    __shared__ double sm[RED_THREADS / 64][6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        {
            auto x = ld(a0 + i), y = ld(b0 + i);
            acc[0] += (double)x.r * y.r + (double)x.i * y.i;
            acc[1] += (double)x.r * y.i - (double)x.i * y.r;
        }
        if (nd > 1) {
            auto x = ld(a1 + i), y = ld(b1 + i);
            acc[2] += (double)x.r * y.r + (double)x.i * y.i;
            acc[3] += (double)x.r * y.i - (double)x.i * y.r;
        }
        if (nd > 2) {
            auto x = ld(a2 + i), y = ld(b2 + i);
            acc[4] += (double)x.r * y.r + (double)x.i * y.i;
            acc[5] += (double)x.r * y.i - (double)x.i * y.r;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) sm[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0;
        for (int j = 0; j < RED_THREADS / 64; ++j) v += sm[j][threadIdx.x];
        double *pp = reinterpret_cast<double *>(partials + (size_t)blockIdx.x * 3);
        pp[threadIdx.x] = v;
    }
}

// the value a store rounds v to (the storage precision), as a later load would read it
__device__ __forceinline__ cx<double> as_stored(const double2 *, cx<double> v) { return v; }
__device__ __forceinline__ cx<float> as_stored(const float2 *, cx<float> v) { return v; }
__device__ __forceinline__ cx<float> as_stored(const __half2 *, cx<float> v) {
    const float2 f = __half22float2(__floats2half2_rn(v.r, v.i));
    return {f.x, f.y};
}
__device__ __forceinline__ cx<float> as_stored(const __hip_bfloat162 *, cx<float> v) {
    return {__bfloat162float(__float2bfloat16(v.r)), __bfloat162float(__float2bfloat16(v.i))};
}

// z = x + a y, and in the same pass the partial sums per workgroup, in double, of <w, z> (w
// not null), <z, z> (zz) and <z, x> (zx), taken on z as stored: the Krylov update and the inner
// products that follow it read the vectors once
template <int P>
__global__ void __launch_bounds__(RED_THREADS) k_xpay_dots(size_t n, typename Prec<P>::S2 *z,
                                                          const typename Prec<P>::S2 *x, double ar, double ai,
                                                          const typename Prec<P>::S2 *y,
                                                          const typename Prec<P>::S2 *w, int zz, int zx,
                                                          double2 *partials) {
    using C = typename Prec<P>::C;
    const cx<C> a{C(ar), C(ai)};
    __shared__ double sm[RED_THREADS / 64][6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cx<C> xv = ld(x + i);
        const cx<C> zn = as_stored(z, xv + cmul(a, ld(y + i)));
        st(z + i, zn);
        if (w) {
            const cx<C> wv = ld(w + i);
            acc[0] += (double)wv.r * zn.r + (double)wv.i * zn.i;
            acc[1] += (double)wv.r * zn.i - (double)wv.i * zn.r;
        }
        if (zz) acc[2] += (double)zn.r * zn.r + (double)zn.i * zn.i;
        if (zx) {
            acc[4] += (double)zn.r * xv.r + (double)zn.i * xv.i;
            acc[5] += (double)zn.r * xv.i - (double)zn.i * xv.r;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = wave_sum(acc[k]);
        if (lane == 0) sm[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = 0;
        for (int j = 0; j < RED_THREADS / 64; ++j) v += sm[j][threadIdx.x];
        double *pp = reinterpret_cast<double *>(partials + (size_t)blockIdx.x * 3);
        pp[threadIdx.x] = v;
    }
}

// final sum of the partials: a fixed pairwise tree (256 threads)
__global__ void __launch_bounds__(256) k_dots_final(int nblocks, const double2 *partials, double2 *out) {
    __shared__ double sm[6][256];
    const double *pp = reinterpret_cast<const double *>(partials);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] += pp[(size_t)b * 6 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < 6; ++k) sm[k][threadIdx.x] += sm[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) reinterpret_cast<double *>(out)[threadIdx.x] = sm[threadIdx.x][0];
}

template <int P>
__global__ void k_xpay(size_t n, typename Prec<P>::S2 *z, const typename Prec<P>::S2 *x, double ar, double ai,
                       const typename Prec<P>::S2 *y) {
    using C = typename Prec<P>::C;
    const cx<C> a{C(ar), C(ai)};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(z + i, ld(x + i) + cmul(a, ld(y + i)));
}

template <int P>
__global__ void k_bicg_p(size_t n, typename Prec<P>::S2 *p, const typename Prec<P>::S2 *r, double br, double bi,
                         double omr, double omi, const typename Prec<P>::S2 *v) {
    using C = typename Prec<P>::C;
    const cx<C> beta{C(br), C(bi)}, om{C(omr), C(omi)};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(p + i, ld(r + i) + cmul(beta, ld(p + i) - cmul(om, ld(v + i))));
}

template <int P>
__global__ void k_axpbypz(size_t n, typename Prec<P>::S2 *e, double ar, double ai, const typename Prec<P>::S2 *ph,
                          double br, double bi, const typename Prec<P>::S2 *sh) {
    using C = typename Prec<P>::C;
    const cx<C> a{C(ar), C(ai)}, b{C(br), C(bi)};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(e + i, ld(e + i) + cmul(a, ld(ph + i)) + cmul(b, ld(sh + i)));
}

template <int PD, int PS>
__global__ void k_convert(size_t n, typename Prec<PD>::S2 *d, const typename Prec<PS>::S2 *s, double scale) {
    using CD = typename Prec<PD>::C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        auto v = ld(s + i);
        st(d + i, cx<CD>{CD((double)v.r * scale), CD((double)v.i * scale)});
    }
}

template <int P>
__global__ void k_zero(size_t n, typename Prec<P>::S2 *d) {
    using C = typename Prec<P>::C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        st(d + i, cxz<C>());
}

// ================================================================ launchers
static inline unsigned grid_for(long n, int t) { return (unsigned)((n + t - 1) / t); }
static constexpr unsigned BLAS_GRID = 1024;

void launch_pack_spinor(Ctx *c, int prec, void *dst, const double *src, double scale) {
    PREC_SWITCH(prec, (k_pack_spinor<P_><<<grid_for(c->V, 256), 256, 0, c->stream>>>(
                          c->g, (typename Prec<P_>::S2 *)dst, (const double2 *)src, scale)));
}

void launch_pack_spinor_f32(Ctx *c, void *dst, const float *src) {
    k_pack_spinor_f32<<<grid_for(c->V, 256), 256, 0, c->stream>>>(c->g, (float2 *)dst, (const float2 *)src);
}

void launch_unpack_spinor_f32(Ctx *c, float *dst, const double2 *src) {
    k_unpack_spinor_f32<<<grid_for(c->V, 256), 256, 0, c->stream>>>(c->g, (float2 *)dst, src);
}

void launch_unpack_spinor(Ctx *c, int prec, double *dst, const void *src, double scale) {
    PREC_SWITCH(prec, (k_unpack_spinor<P_><<<grid_for(c->V, 256), 256, 0, c->stream>>>(
                          c->g, (double2 *)dst, (const typename Prec<P_>::S2 *)src, scale)));
}

int launch_pack_links(Ctx *c, const double *U, double *max_dev) {
    unsigned nb = grid_for(c->V, 256);
    INNER_SWITCH(c->prm.prec_inner, (k_pack_links<P_><<<nb, 256, 0, c->stream>>>(
                                        c->g, (const double2 *)U, c->U64, (typename Prec<P_>::S2 *)c->Uin, c->dev_dev)));
    double *h = (double *)malloc(sizeof(double) * nb);
    hipError_t e = hipMemcpyAsync(h, c->dev_dev, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double w = 0;
    for (unsigned i = 0; i < nb; ++i) w = fmax(w, h[i]);
    free(h);
    *max_dev = w;
    return e == hipSuccess ? 0 : -1;
}

void launch_pack_clover(Ctx *c, const double *F) {
    INNER_SWITCH(c->prm.prec_inner, (k_pack_clover<P_><<<grid_for(c->V, 256), 256, 0, c->stream>>>(
                                         c->g, (const double2 *)F, c->F64, (typename Prec<P_>::S2 *)c->Fin)));
}

// ================================================================ slot re-ordering
// f is [rows][Vb]; each row becomes row[s] = old row[perm[s]] (one workgroup per row, the row
// staged in LDS)
template <typename T>
__global__ void __launch_bounds__(256) k_permute_rows(T *__restrict__ f, int Vb, const int *__restrict__ perm) {
    extern __shared__ __attribute__((aligned(16))) unsigned char perm_lds[];
    T *row = reinterpret_cast<T *>(perm_lds);
    T *p = f + (size_t)blockIdx.x * Vb;
    for (int s = threadIdx.x; s < Vb; s += blockDim.x) row[s] = p[s];
    __syncthreads();
    for (int s = threadIdx.x; s < Vb; s += blockDim.x) p[s] = row[perm[s]];
}

template <typename T>
static bool permute_rows(Ctx *c, void *f, long rows, const int *perm) {
    const size_t bytes = (size_t)c->g.Vb * sizeof(T);
    if (bytes > 65536 &&
        hipFuncSetAttribute((const void *)k_permute_rows<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
            hipSuccess)
        return false;
    k_permute_rows<T><<<(unsigned)rows, 256, bytes, c->stream>>>((T *)f, c->g.Vb, perm);
    return true;
}

// The packed links and clover field (FP64 and inner precision) re-laid out for a new slot
// order inside the blocks: new slot s holds what old slot perm[s] held.  False if a block row
// does not fit the LDS.
bool launch_permute_fields(Ctx *c, const int *perm) {
    const long NB = c->g.NB;
    const bool half = elem_bytes(c->prec_created) == 4;
    bool ok = true;
    if (c->have_U) {
        ok = ok && permute_rows<uint4>(c, c->U64, NB * 24, perm);
        ok = ok && (half ? permute_rows<unsigned>(c, c->Uin_lp, NB * 24, perm) : permute_rows<uint2>(c, c->Uin_lp, NB * 24, perm));
        if (c->fb_fp32) ok = ok && permute_rows<uint2>(c, c->Uin32, NB * 24, perm);
    }
    if (c->have_F) {
        ok = ok && permute_rows<uint4>(c, c->F64, NB * 36, perm);
        ok = ok && (half ? permute_rows<unsigned>(c, c->Fin_lp, NB * 36, perm) : permute_rows<uint2>(c, c->Fin_lp, NB * 36, perm));
        if (c->fb_fp32) ok = ok && permute_rows<uint2>(c, c->Fin32, NB * 36, perm);
    }
    return ok;
}

void launch_dslash(Ctx *c, int prec, void *out, const void *in) {
    if (prec == SAPQ_FP64) {
        constexpr int nt = 2 * dslash_sites(SAPQ_FP64);
        const unsigned grid = (grid_for(2 * c->V, nt) + N_XCD - 1) / N_XCD * N_XCD;
        k_dslash<SAPQ_FP64><<<grid, nt, 0, c->stream>>>(c->g, (double2 *)out, (const double2 *)in, c->U64, c->F64,
                                                         c->prm.kappa);
        return;
    }
    const unsigned grid = (grid_for(2 * c->V, 256) + N_XCD - 1) / N_XCD * N_XCD;
    INNER_SWITCH(prec, (k_dslash<P_><<<grid, 2 * dslash_sites(P_), 0, c->stream>>>(
                           c->g, (typename Prec<P_>::S2 *)out, (const typename Prec<P_>::S2 *)in,
                           (const typename Prec<P_>::S2 *)c->Uin, (const typename Prec<P_>::S2 *)c->Fin, c->prm.kappa)));
}

template <int P, int NT>
static void sap_phase_nt(Ctx *c, const SapArgs &a, const void *rsrc, void *r, void *x, void *y) {
    using S2 = typename Prec<P>::S2;
    dim3 grid(c->g.NBc), block(c->ssor_threads);
    if (c->ssor_lds)
        k_sap_phase<P, true, NT><<<grid, block, c->lds_bytes + c->lds_extra, c->stream>>>(
            c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin, c->ssor_scratch);
    else
        k_sap_phase<P, false, NT><<<grid, block, c->lds_extra, c->stream>>>(
            c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin, c->ssor_scratch);
}

template <int P>
static void sap_phase_t(Ctx *c, const SapArgs &a, const void *rsrc, void *r, void *x, void *y) {
    if (c->ssor_staged) {
        using S2 = typename Prec<P>::S2;
        k_sap_phase_staged<P, 512><<<dim3(c->g.NBc), dim3(c->ssor_threads), c->staged_bytes, c->stream>>>(
            c->g, a, (const S2 *)rsrc, (S2 *)r, (S2 *)x, (S2 *)y, (const S2 *)c->Uin, (const S2 *)c->Fin);
        return;
    }
    if (c->ssor_threads <= 512)
        sap_phase_nt<P, 512>(c, a, rsrc, r, x, y);
    else
        sap_phase_nt<P, 1024>(c, a, rsrc, r, x, y);
}

template <int P>
static void set_lds_limit(Ctx *c) {
    // only sizes the device can grant are requested; the variant that is not used is left alone
    if (c->ssor_lds) {
        const int bytes = (int)(c->lds_bytes + c->lds_extra);
        (void)hipFuncSetAttribute((const void *)k_sap_phase<P, true, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute((const void *)k_sap_phase<P, true, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    } else {
        const int bytes = (int)c->lds_extra;
        (void)hipFuncSetAttribute((const void *)k_sap_phase<P, false, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        (void)hipFuncSetAttribute((const void *)k_sap_phase<P, false, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    }
}

int set_sap_lds_limits(Ctx *c) {
    if (c->ssor_staged && c->staged_bytes > 65536) {
        const int bytes = (int)c->staged_bytes;
        switch (c->prm.prec_inner) {
        case SAPQ_FP32: (void)hipFuncSetAttribute((const void *)k_sap_phase_staged<SAPQ_FP32, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes); break;
        case SAPQ_FP16: (void)hipFuncSetAttribute((const void *)k_sap_phase_staged<SAPQ_FP16, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes); break;
        case SAPQ_BF16: (void)hipFuncSetAttribute((const void *)k_sap_phase_staged<SAPQ_BF16, 512>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes); break;
        }
    }
    const size_t need = c->ssor_lds ? c->lds_bytes + c->lds_extra : c->lds_extra;
    if (need <= 65536) return 0;
    set_lds_limit<SAPQ_FP32>(c);
    set_lds_limit<SAPQ_FP16>(c);
    set_lds_limit<SAPQ_BF16>(c);
    return hipGetLastError() == hipSuccess ? 0 : -1;  // also clears the runtime's last-error slot
}

void launch_sap_phase(Ctx *c, int colour, bool first, const void *rsrc, void *r, void *x, void *y) {
    if (c->prm.flags & SAPQ_FLAG_EOMR) {
        launch_sap_phase_eomr(c, colour, (colour == 1 || !first) ? 1 : 0, first ? 1 : 0, 0, rsrc, r, x, y);
        return;
    }
    if (c->use_parts) {
        launch_sap_phase_parts(c, colour, (colour == 1 || !first) ? 1 : 0, first ? 1 : 0, 0, rsrc, r, x, y);
        return;
    }
    SapArgs a;
    a.colour = colour;
    a.gather = (colour == 1 || !first) ? 1 : 0;
    a.first = first ? 1 : 0;
    a.ssor_only = 0;
    a.n_ssor = c->prm.n_ssor;
    a.kappa = (float)c->prm.kappa;
    a.omega = (float)c->prm.omega;
    INNER_SWITCH(c->prm.prec_inner, sap_phase_t<P_>(c, a, rsrc, r, x, y));
}

void launch_ssor_only(Ctx *c, int colour, const void *v, void *x) {
    if (c->prm.flags & SAPQ_FLAG_EOMR) {
        launch_sap_phase_eomr(c, colour, 0, 1, 1, v, nullptr, x, nullptr);
        return;
    }
    if (c->use_parts) {
        launch_sap_phase_parts(c, colour, 0, 1, 1, v, nullptr, x, nullptr);
        return;
    }
    SapArgs a;
    a.colour = colour;
    a.gather = 0;
    a.first = 1;
    a.ssor_only = 1;
    a.n_ssor = c->prm.n_ssor;
    a.kappa = (float)c->prm.kappa;
    a.omega = (float)c->prm.omega;
    INNER_SWITCH(c->prm.prec_inner, sap_phase_t<P_>(c, a, v, nullptr, x, nullptr));
}

void launch_sap_face(Ctx *c, int colour, void *r, const void *x) {
    if (c->use_parts) {
        launch_sap_face_2l(c, colour, r, x);
        return;
    }
    long nc = (long)c->g.NBc * c->g.Vb;
    INNER_SWITCH(c->prm.prec_inner, (k_sap_face<P_><<<grid_for(4 * nc, 256), 256, 0, c->stream>>>(
                                         c->g, colour, (float)c->prm.kappa, (typename Prec<P_>::S2 *)r,
                                         (const typename Prec<P_>::S2 *)x, (const typename Prec<P_>::S2 *)c->Uin,
                                         (const typename Prec<P_>::S2 *)c->Fin)));
}

void blas_dots(Ctx *c, int prec, int nd, const void *const *a, const void *const *b, double2 *host_out) {
    PREC_SWITCH(prec, ({
                    using S2 = typename Prec<P_>::S2;
                    k_dots<P_><<<c->red_blocks, RED_THREADS, 0, c->stream>>>(
                        c->nvec, nd, (const S2 *)a[0], (const S2 *)b[0], (const S2 *)(nd > 1 ? a[1] : a[0]),
                        (const S2 *)(nd > 1 ? b[1] : b[0]), (const S2 *)(nd > 2 ? a[2] : a[0]),
                        (const S2 *)(nd > 2 ? b[2] : b[0]), c->partials);
                }));
    k_dots_final<<<1, 256, 0, c->stream>>>(c->red_blocks, c->partials, c->dev_res);
    (void)hipMemcpyAsync(c->host_res, c->dev_res, sizeof(double2) * 3, hipMemcpyDeviceToHost, c->stream);
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < nd; ++k) host_out[k] = c->host_res[k];
    prof_harvest(c);
}

void blas_xpay_dots(Ctx *c, int prec, void *z, const void *x, double2 a, const void *y, const void *w, int zz, int zx,
                    double2 host_out[3]) {
    PREC_SWITCH(prec, ({
                    using S2 = typename Prec<P_>::S2;
                    k_xpay_dots<P_><<<c->red_blocks, RED_THREADS, 0, c->stream>>>(
                        c->nvec, (S2 *)z, (const S2 *)x, a.x, a.y, (const S2 *)y, (const S2 *)w, zz, zx, c->partials);
                }));
    k_dots_final<<<1, 256, 0, c->stream>>>(c->red_blocks, c->partials, c->dev_res);
    (void)hipMemcpyAsync(c->host_res, c->dev_res, sizeof(double2) * 3, hipMemcpyDeviceToHost, c->stream);
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 3; ++k) host_out[k] = c->host_res[k];
    prof_harvest(c);
}

void blas_copy(Ctx *c, int prec, void *dst, const void *src) {
    hipMemcpyAsync(dst, src, c->nvec * elem_bytes(prec), hipMemcpyDeviceToDevice, c->stream);
}

void blas_zero(Ctx *c, int prec, void *dst) {
    PREC_SWITCH(prec, (k_zero<P_><<<BLAS_GRID, 256, 0, c->stream>>>(c->nvec, (typename Prec<P_>::S2 *)dst)));
}

void blas_xpay(Ctx *c, int prec, void *z, const void *x, double2 a, const void *y) {
    PREC_SWITCH(prec, (k_xpay<P_><<<BLAS_GRID, 256, 0, c->stream>>>(c->nvec, (typename Prec<P_>::S2 *)z,
                                                                      (const typename Prec<P_>::S2 *)x, a.x, a.y,
                                                                      (const typename Prec<P_>::S2 *)y)));
}

void blas_bicg_p(Ctx *c, int prec, void *p, const void *r, double2 beta, double2 om, const void *v) {
    PREC_SWITCH(prec, (k_bicg_p<P_><<<BLAS_GRID, 256, 0, c->stream>>>(c->nvec, (typename Prec<P_>::S2 *)p,
                                                                        (const typename Prec<P_>::S2 *)r, beta.x, beta.y,
                                                                        om.x, om.y, (const typename Prec<P_>::S2 *)v)));
}

void blas_axpbypz(Ctx *c, int prec, void *e, double2 a, const void *ph, double2 b, const void *sh) {
    PREC_SWITCH(prec, (k_axpbypz<P_><<<BLAS_GRID, 256, 0, c->stream>>>(c->nvec, (typename Prec<P_>::S2 *)e, a.x, a.y,
                                                                         (const typename Prec<P_>::S2 *)ph, b.x, b.y,
                                                                         (const typename Prec<P_>::S2 *)sh)));
}

void blas_convert(Ctx *c, int pd, void *dst, int ps, const void *src, double scale) {
    if (pd == SAPQ_FP32 && ps != SAPQ_FP64) {
        INNER_SWITCH(ps, (k_convert<SAPQ_FP32, P_><<<BLAS_GRID, 256, 0, c->stream>>>(
                             c->nvec, (float2 *)dst, (const typename Prec<P_>::S2 *)src, scale)));
    } else if (ps == SAPQ_FP32 && pd != SAPQ_FP64) {
        INNER_SWITCH(pd, (k_convert<P_, SAPQ_FP32><<<BLAS_GRID, 256, 0, c->stream>>>(
                             c->nvec, (typename Prec<P_>::S2 *)dst, (const float2 *)src, scale)));
    } else if (pd == SAPQ_FP64) {
        INNER_SWITCH(ps, (k_convert<SAPQ_FP64, P_><<<BLAS_GRID, 256, 0, c->stream>>>(
                             c->nvec, (double2 *)dst, (const typename Prec<P_>::S2 *)src, scale)));
    } else if (ps == SAPQ_FP64) {
        INNER_SWITCH(pd, (k_convert<P_, SAPQ_FP64><<<BLAS_GRID, 256, 0, c->stream>>>(
                             c->nvec, (typename Prec<P_>::S2 *)dst, (const double2 *)src, scale)));
    }
}

}  // namespace sapq
