// Host emulation of the two-workgroup SAP phase kernel's protocol (k_sap_phase_parts):
// the split tables of tables.h, the halo exchange through tagged words in three sweep
// slots, the choice of the sweep each halo copy must carry, and the skipped copy at the
// turn of a sweep.  A scalar toy operator x_n <- v_n + sum_k c_k(n) x_{n+k} over the
// in-block neighbours is swept in hyperplane order (n_ssor forward + backward sweeps
// from 0) once on the whole block and once by two emulated workgroups advancing in a
// random interleaving; the results must agree bit for bit and no interleaving may leave
// both workgroups waiting.
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1210_7398_amd/csrc/tables.h"

using namespace sapq;

struct Word { double v; unsigned tag; };

static unsigned tagof(int sweep) { return 0x80000000u | (1u << 6) | (unsigned)(sweep & 63); }

struct Part {
    int p;
    std::vector<double> xl;  // own sites, halo slots, zero slot
    int w = 0, pi = 0;       // current step
    int phase = 0;           // 0: compute + export, 1: halo copy for the next step, 2: final copy, 3: done
};

static int run(const int B[4], const int S[4], int n_ssor, unsigned seed, std::string &msg) {
    sapq_geom G;
    for (int m = 0; m < 4; ++m) { G.L[m] = 2 * B[m]; G.block[m] = B[m]; G.subblock[m] = S[m]; G.bc_sign[m] = 1; }
    HostTables T;
    build_tables(&G, T);
    PartTables P;
    if (!build_parts(&G, T, 2, P)) { msg = "build_parts refused the geometry"; return 2; }
    const int Vb = T.Vb, Vp = P.Vp, Hp = P.Hp, H = T.nplanes, NS = Vp + Hp + 1, nsw = 2 * n_ssor;
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(-0.3, 0.3);
    std::vector<double> c((size_t)8 * Vb), v(Vb);
    for (auto &e : c) e = U(rng);
    for (auto &e : v) e = 1.0 + U(rng);
    // the update of one site from a neighbour lookup, forward hops summed before backward
    auto update = [&](int s, auto &&nbr_value) {
        double f = 0.0, b = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
            f += c[(size_t)(2 * mu) * Vb + s] * nbr_value(2 * mu);
            b += c[(size_t)(2 * mu + 1) * Vb + s] * nbr_value(2 * mu + 1);
        }
        return v[s] + (f + b);
    };
    // reference: whole block
    std::vector<double> xr(Vb, 0.0);
    for (int w = 0; w < nsw; ++w)
        for (int pi = 0; pi < H; ++pi) {
            const int h = (w & 1) == 0 ? pi : H - 1 - pi;
            for (int s = T.plane_start[h]; s < T.plane_start[h + 1]; ++s)
                xr[s] = update(s, [&](int k) { int t = T.loc_nbr[(size_t)k * Vb + s]; return t >= 0 ? xr[t] : 0.0; });
        }
    // emulated workgroups
    std::vector<Word> xch((size_t)2 * 3 * Hp, Word{0.0, 0u});
    Part parts[2];
    for (int p = 0; p < 2; ++p) { parts[p].p = p; parts[p].xl.assign(NS, 0.0); }
    auto slot_word = [&](int q, int sweep, int k) -> Word & { return xch[((size_t)q * 3 + sweep % 3) * Hp + k]; };
    auto try_copy = [&](Part &A, int h_next, int ver) {
        const int q = A.p ^ 1;
        const int *st = &P.imp_start[(size_t)A.p * (MAX_PLANES + 1)];
        for (int e = st[h_next]; e < st[h_next + 1]; ++e)
            if (slot_word(q, ver, P.imp[(size_t)A.p * Hp + e]).tag != tagof(ver)) return false;
        for (int e = st[h_next]; e < st[h_next + 1]; ++e) {
            const int k = P.imp[(size_t)A.p * Hp + e];
            A.xl[Vp + k] = slot_word(q, ver, k).v;
        }
        return true;
    };
    auto advance = [&](Part &A) -> bool {  // one action; false when blocked
        const int p = A.p;
        const bool fwd = (A.w & 1) == 0;
        const int h = fwd ? A.pi : H - 1 - A.pi;
        if (A.phase == 0) {
            for (int i = P.pstart[h]; i < P.pstart[h + 1]; ++i) {
                const int s = P.gslot[(size_t)p * Vp + i];
                const double xn = update(s, [&](int k) {
                    const int mu = k >> 1, d = k & 1;
                    const unsigned wd = P.pnb[(((size_t)p * Vp + i) * 2 + d) * 2 + (mu >> 1)];
                    const unsigned sl = (mu & 1) ? wd >> 16 : wd & 0xffffu;
                    if (sl >= (unsigned)NS) { fprintf(stderr, "slot out of range\n"); exit(3); }
                    return A.xl[sl];
                });
                A.xl[i] = xn;
                const int kx = P.exp_idx[(size_t)p * Vp + i];
                if (kx >= 0) slot_word(p, A.w, kx) = Word{xn, tagof(A.w)};
            }
            A.phase = 1;
            return true;
        }
        if (A.phase == 1) {
            if (A.pi + 1 < H) {
                const int nh = fwd ? h + 1 : h - 1;
                const int ver = ((p == 0) == fwd) ? A.w : A.w - 1;
                if (ver >= 0 && !try_copy(A, nh, ver)) return false;
            }
            A.phase = 0;
            if (++A.pi == H) { A.pi = 0; if (++A.w == nsw) A.phase = 2; }
            return true;
        }
        if (A.phase == 2) {
            const int q = p ^ 1;
            for (int k = 0; k < Hp; ++k)
                if (slot_word(q, nsw - 1, k).tag != tagof(nsw - 1)) return false;
            for (int k = 0; k < Hp; ++k) A.xl[Vp + k] = slot_word(q, nsw - 1, k).v;
            A.phase = 3;
            return true;
        }
        return false;
    };
    std::uniform_int_distribution<int> coin(0, 1);
    long guard = 0;
    while (parts[0].phase != 3 || parts[1].phase != 3) {
        const int first = coin(rng);
        // a workgroup may run ahead for a while: take a random burst of actions
        const int burst = (rng() % 4 == 0) ? 1 + (int)(rng() % 400) : 1 + (int)(rng() % 7);
        bool moved = false;
        for (int t = 0; t < 2 && !moved; ++t) {
            Part &A = parts[(first + t) & 1];
            for (int r = 0; r < burst && A.phase != 3; ++r) {
                if (!advance(A)) break;
                moved = true;
            }
        }
        if (!moved) { msg = "both workgroups wait: deadlock"; return 1; }
        if (++guard > 100000000L) { msg = "no progress"; return 1; }
    }
    for (int p = 0; p < 2; ++p)
        for (int i = 0; i < Vp; ++i) {
            const int s = P.gslot[(size_t)p * Vp + i];
            if (memcmp(&parts[p].xl[i], &xr[s], sizeof(double)) != 0) {
                char b[256];
                snprintf(b, sizeof b, "part %d site %d (slot %d): %.17g vs whole-block %.17g", p, i, s, parts[p].xl[i], xr[s]);
                msg = b;
                return 1;
            }
        }
    return 0;
}

int main() {
    struct Case { int B[4], S[4], n_ssor; } cases[] = {
        {{6, 6, 6, 12}, {3, 3, 3, 6}, 4},  // 24^3x48 workload blocks
        {{6, 6, 6, 12}, {3, 3, 3, 6}, 1},
        {{4, 4, 4, 4}, {2, 2, 2, 2}, 4},   // neighbouring hyperplanes across the split (S_t = 2)
        {{4, 4, 4, 8}, {2, 2, 2, 2}, 3},   // two sub-block layers per part
        {{6, 6, 6, 6}, {3, 3, 3, 3}, 2},
        {{4, 6, 4, 12}, {2, 3, 2, 3}, 4},  // uneven sub-block shape
        {{8, 4, 4, 8}, {4, 2, 2, 4}, 2},
    };
    int fails = 0;
    for (auto &cs : cases)
        for (unsigned seed = 1; seed <= 6; ++seed) {
            std::string msg;
            const int rc = run(cs.B, cs.S, cs.n_ssor, seed, msg);
            if (rc) {
                printf("FAIL B=%dx%dx%dx%d S=%dx%dx%dx%d n_ssor=%d seed=%u: %s\n", cs.B[0], cs.B[1], cs.B[2], cs.B[3], cs.S[0],
                       cs.S[1], cs.S[2], cs.S[3], cs.n_ssor, seed, msg.c_str());
                ++fails;
            }
        }
    // geometries the split must refuse: an odd number of sub-block layers in t
    {
        sapq_geom G;
        const int B[4] = {4, 4, 4, 6}, S[4] = {2, 2, 2, 2};
        for (int m = 0; m < 4; ++m) { G.L[m] = 2 * B[m]; G.block[m] = B[m]; G.subblock[m] = S[m]; G.bc_sign[m] = 1; }
        HostTables T;
        build_tables(&G, T);
        PartTables P;
        if (build_parts(&G, T, 2, P)) { printf("FAIL: split accepted 3 sub-block layers in t\n"); ++fails; }
    }
    // even-odd site order (all-zero sub-block): two hyperplanes, the even and the odd sites of
    // the block, no coupled pair inside a plane, one-workgroup tables only
    for (const auto &Bv : {std::array<int, 4>{4, 4, 4, 4}, std::array<int, 4>{6, 6, 6, 6}, std::array<int, 4>{3, 4, 5, 6}}) {
        sapq_geom G;
        for (int m = 0; m < 4; ++m) { G.L[m] = 2 * Bv[m]; G.block[m] = Bv[m]; G.subblock[m] = 0; G.bc_sign[m] = 1; }
        HostTables T;
        build_tables(&G, T);
        const int Vb = T.Vb;
        bool ok = T.nplanes == 2 && T.plane_start[0] == 0 && T.plane_start[2] == Vb;
        std::vector<int> plane(Vb);
        for (int s = 0; s < Vb && ok; ++s) {
            plane[s] = s < T.plane_start[1] ? 0 : 1;
            int l = T.slot_lex[s], sum = 0;
            for (int m = 0; m < 4; ++m) { sum += l % Bv[m]; l /= Bv[m]; }
            ok = ok && (sum & 1) == plane[s];
        }
        for (int k = 0; k < 8 && ok; ++k)
            for (int s = 0; s < Vb && ok; ++s) {
                const int t = T.loc_nbr[(size_t)k * Vb + s];
                if (t >= 0) ok = plane[t] != plane[s];
            }
        PartTables P1, P2;
        ok = ok && build_parts(&G, T, 1, P1) && !build_parts(&G, T, 2, P2);
        if (!ok) {
            printf("FAIL: even-odd tables for B=%dx%dx%dx%d\n", Bv[0], Bv[1], Bv[2], Bv[3]);
            ++fails;
        }
    }
    printf(fails ? "%d failures\n" : "all protocol cases agree\n", fails);
    return fails ? 1 : 0;
}
