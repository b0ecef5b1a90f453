// Host emulation of the two-workgroup SAP phase kernel's protocol (k_sap_phase_parts):
// the split tables of tables.h, the halo exchange through tagged words in three sweep
// slots, the choice of the sweep each halo copy must carry, and the skipped copy at the
// turn of a sweep.  A scalar toy operator x_n <- v_n + sum_k c_k(n) x_{n+k} over the
// in-block neighbours is swept in hyperplane order (n_ssor forward + backward sweeps
// from 0) once on the whole block and once by two emulated workgroups advancing in a
// random interleaving; the results must agree bit for bit and no interleaving may leave
// both workgroups waiting.  A launch whose waits time out is followed by a second launch on
// the same exchange array, with the sync words reset as the library resets them after an
// error (parts_sync_after_error): the second launch must not take the failed launch's words.
// Half of the interleavings run with the omega = 1 shortcut at the turn of a sweep (the repeated
// plane keeps its values and republishes its boundary words), whose recomputation the emulator
// checks to be bit-identical.
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

// the tag of a halo word, as the kernel forms it from the launch epoch and the sweep
static unsigned tagof(unsigned epoch, int sweep) {
    return 0x80000000u | ((epoch & 0x1ffffffu) << 6) | (unsigned)(sweep & 63);
}

struct Part {
    int p;
    std::vector<double> xl;  // own sites, halo slots, zero slot
    int w = 0, pi = 0;       // current step
    int phase = 0;           // 0: compute + export, 1: halo copy for the next step, 2: final copy, 3: done
    bool gave_up = false;    // a wait timed out: from then on the part waits no more (as the kernel)
};

struct Problem {
    HostTables T;
    PartTables P;
    int n_ssor;
    std::vector<double> c;   // toy operator coefficients [8][Vb]
};

// the update of one site from a neighbour lookup, forward hops summed before backward
template <typename F>
static double update(const Problem &Q, const std::vector<double> &v, int s, F &&nbr_value) {
    const int Vb = Q.T.Vb;
    double f = 0.0, b = 0.0;
    for (int mu = 0; mu < 4; ++mu) {
        f += Q.c[(size_t)(2 * mu) * Vb + s] * nbr_value(2 * mu);
        b += Q.c[(size_t)(2 * mu + 1) * Vb + s] * nbr_value(2 * mu + 1);
    }
    return v[s] + (f + b);
}

// reference: hyperplane-order sweeps of the whole block
static std::vector<double> whole_block(const Problem &Q, const std::vector<double> &v) {
    const HostTables &T = Q.T;
    const int Vb = T.Vb, H = T.nplanes;
    std::vector<double> xr(Vb, 0.0);
    for (int w = 0; w < 2 * Q.n_ssor; ++w)
        for (int pi = 0; pi < H; ++pi) {
            const int h = (w & 1) == 0 ? pi : H - 1 - pi;
            for (int s = T.plane_start[h]; s < T.plane_start[h + 1]; ++s)
                xr[s] = update(Q, v, s, [&](int k) { int t = T.loc_nbr[(size_t)k * Vb + s]; return t >= 0 ? xr[t] : 0.0; });
        }
    return xr;
}

// One launch of the two emulated workgroups at `epoch` on the exchange array xch (kept
// between launches, as the context keeps it).  stall_part >= 0 emulates a launch whose
// waits time out: that part does nothing until the other has given up on a wait, then both
// run to the end taking whatever the halo words hold.  Returns 1 on a deadlock; *timed_out
// tells whether any wait gave up; xs receives the block's result by block slot.
// skip_turns: the kernel's omega = 1 shortcut, the repeated plane at the turn of a sweep keeps
// its values (checked here to equal a recomputation bit for bit) and only republishes its
// boundary words under the new sweep's tag.
static int launch(const Problem &Q, const std::vector<double> &v, unsigned epoch, std::vector<Word> &xch, int stall_part,
                  std::mt19937 &rng, std::vector<double> &xs, bool *timed_out, std::string &msg, bool skip_turns = false) {
    const HostTables &T = Q.T;
    const PartTables &P = Q.P;
    const int Vp = P.Vp, Hp = P.Hp, H = T.nplanes, NS = Vp + Hp + 1, nsw = 2 * Q.n_ssor;
    Part parts[2];
    for (int p = 0; p < 2; ++p) { parts[p].p = p; parts[p].xl.assign(NS, 0.0); }
    auto slot_word = [&](int q, int sweep, int k) -> Word & { return xch[((size_t)q * 3 + sweep % 3) * Hp + k]; };
    // copy the halo words of plane h_next; false while one does not carry the awaited tag
    // (unless the part has given up, when it takes them as they are)
    auto try_copy = [&](Part &A, int h_next, int ver) {
        const int q = A.p ^ 1;
        const int *st = &P.imp_start[(size_t)A.p * (MAX_PLANES + 1)];
        if (!A.gave_up)
            for (int e = st[h_next]; e < st[h_next + 1]; ++e)
                if (slot_word(q, ver, P.imp[(size_t)A.p * Hp + e]).tag != tagof(epoch, ver)) return false;
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
            const bool repeat = skip_turns && A.w > 0 && A.pi == 0;
            for (int i = P.pstart[h]; i < P.pstart[h + 1]; ++i) {
                const int s = P.gslot[(size_t)p * Vp + i];
                const double xn = update(Q, v, s, [&](int k) {
                    const int mu = k >> 1, d = k & 1;
                    const unsigned wd = P.pnb[(((size_t)p * Vp + i) * 2 + d) * 2 + (mu >> 1)];
                    const unsigned sl = (mu & 1) ? wd >> 16 : wd & 0xffffu;
                    if (sl >= (unsigned)NS) { fprintf(stderr, "slot out of range\n"); exit(3); }
                    return A.xl[sl];
                });
                if (repeat && memcmp(&xn, &A.xl[i], sizeof xn) != 0 && !A.gave_up) {
                    fprintf(stderr, "the repeated plane at a sweep turn changed (part %d, site %d)\n", p, i);
                    exit(4);
                }
                if (!repeat) A.xl[i] = xn;
                const int kx = P.exp_idx[(size_t)p * Vp + i];
                if (kx >= 0) slot_word(p, A.w, kx) = Word{xn, tagof(epoch, A.w)};
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
            if (!A.gave_up)
                for (int k = 0; k < Hp; ++k)
                    if (slot_word(q, nsw - 1, k).tag != tagof(epoch, nsw - 1)) return false;
            for (int k = 0; k < Hp; ++k) A.xl[Vp + k] = slot_word(q, nsw - 1, k).v;
            A.phase = 3;
            return true;
        }
        return false;
    };
    std::uniform_int_distribution<int> coin(0, 1);
    long guard = 0;
    *timed_out = false;
    while (parts[0].phase != 3 || parts[1].phase != 3) {
        const int first = coin(rng);
        // a workgroup may run ahead for a while: take a random burst of actions
        const int burst = (rng() % 4 == 0) ? 1 + (int)(rng() % 400) : 1 + (int)(rng() % 7);
        bool moved = false;
        for (int t = 0; t < 2 && !moved; ++t) {
            Part &A = parts[(first + t) & 1];
            if (A.p == stall_part && !parts[A.p ^ 1].gave_up) continue;  // the slow part
            for (int r = 0; r < burst && A.phase != 3; ++r) {
                if (!advance(A)) break;
                moved = true;
            }
        }
        if (!moved) {
            // a blocked part whose partner makes no progress times out
            Part *W = nullptr;
            for (int p = 0; p < 2; ++p)
                if (parts[p].phase != 3 && !parts[p].gave_up && (stall_part >= 0 || parts[p ^ 1].phase == 3)) W = &parts[p];
            if (stall_part < 0 || !W) { msg = "both workgroups wait: deadlock"; return 1; }
            W->gave_up = true;
            *timed_out = true;
        }
        if (++guard > 100000000L) { msg = "no progress"; return 1; }
    }
    xs.assign(T.Vb, 0.0);
    for (int p = 0; p < 2; ++p)
        for (int i = 0; i < Vp; ++i) xs[P.gslot[(size_t)p * Vp + i]] = parts[p].xl[i];
    return 0;
}

static bool make_problem(const int B[4], const int S[4], int n_ssor, unsigned seed, Problem &Q, std::string &msg) {
    sapq_geom G;
    for (int m = 0; m < 4; ++m) { G.L[m] = 2 * B[m]; G.block[m] = B[m]; G.subblock[m] = S[m]; G.bc_sign[m] = 1; }
    build_tables(&G, Q.T);
    if (!build_parts(&G, Q.T, 2, Q.P)) { msg = "build_parts refused the geometry"; return false; }
    Q.n_ssor = n_ssor;
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(-0.3, 0.3);
    Q.c.resize((size_t)8 * Q.T.Vb);
    for (auto &e : Q.c) e = U(rng);
    return true;
}

static std::vector<double> source(int Vb, unsigned seed) {
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(-0.3, 0.3);
    std::vector<double> v(Vb);
    for (auto &e : v) e = 1.0 + U(rng);
    return v;
}

static int compare(const std::vector<double> &got, const std::vector<double> &want, std::string &msg) {
    for (size_t s = 0; s < want.size(); ++s)
        if (memcmp(&got[s], &want[s], sizeof(double)) != 0) {
            char b[256];
            snprintf(b, sizeof b, "block slot %zu: %.17g vs whole-block %.17g", s, got[s], want[s]);
            msg = b;
            return 1;
        }
    return 0;
}

// one launch at epoch 1 against the whole-block sweeps, bit for bit
static int run(const int B[4], const int S[4], int n_ssor, unsigned seed, std::string &msg, bool skip_turns = false) {
    Problem Q;
    if (!make_problem(B, S, n_ssor, seed, Q, msg)) return 2;
    const std::vector<double> v = source(Q.T.Vb, seed + 1000);
    std::vector<Word> xch((size_t)2 * 3 * Q.P.Hp, Word{0.0, 0u});
    std::mt19937 rng(seed);
    std::vector<double> xs;
    bool to = false;
    if (launch(Q, v, 1u, xch, -1, rng, xs, &to, msg, skip_turns)) return 1;
    if (to) { msg = "a wait timed out in a launch without a slow part"; return 1; }
    return compare(xs, whole_block(Q, v), msg);
}

// A launch whose waits time out (epoch 0, the context's first split launch), then the next
// launch on the same exchange array with another source.  The sync words after the failed
// launch: its last workgroup reset the counters and advanced the epoch, and the error word
// is set; the host then applies reset(sync).  The second launch must match the whole-block
// sweeps of its own source bit for bit.  Returns 1 on a mismatch or a deadlock.
template <typename Reset>
static int run_after_failure(const int B[4], const int S[4], int n_ssor, unsigned seed, Reset &&reset, std::string &msg) {
    Problem Q;
    if (!make_problem(B, S, n_ssor, seed, Q, msg)) return 2;
    const std::vector<double> v1 = source(Q.T.Vb, seed + 2000), v2 = source(Q.T.Vb, seed + 3000);
    std::vector<Word> xch((size_t)2 * 3 * Q.P.Hp, Word{0.0, 0u});
    std::mt19937 rng(seed);
    std::vector<double> xs;
    bool to = false;
    const unsigned epoch0 = 0u;
    if (launch(Q, v1, epoch0, xch, (int)(seed & 1u), rng, xs, &to, msg)) return 1;
    if (!to) { msg = "the slow part did not make a wait time out"; return 1; }
    const unsigned after[4] = {0u, 0u, epoch0 + 1u, 1u};
    unsigned next[4];
    reset(after, next);
    if (next[0] || next[1] || next[3]) { msg = "counters or error word not cleared"; return 1; }
    if (launch(Q, v2, next[2], xch, -1, rng, xs, &to, msg)) return 1;
    if (to) { msg = "a wait timed out in the launch after the failure"; return 1; }
    return compare(xs, whole_block(Q, v2), msg);
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
        for (unsigned seed = 1; seed <= 12; ++seed) {
            std::string msg;
            const bool skip = seed > 6;  // seeds 7-12: the omega = 1 turn-plane shortcut
            const int rc = run(cs.B, cs.S, cs.n_ssor, seed, msg, skip);
            if (rc) {
                printf("FAIL B=%dx%dx%dx%d S=%dx%dx%dx%d n_ssor=%d seed=%u: %s\n", cs.B[0], cs.B[1], cs.B[2], cs.B[3], cs.S[0],
                       cs.S[1], cs.S[2], cs.S[3], cs.n_ssor, seed, msg.c_str());
                ++fails;
            }
        }
    // a failed launch, then the context reused: with the reset rule of the library
    // (parts_sync_after_error) every second launch agrees; zeroing all four words, which puts
    // the epoch back to that of the failed launch, must be caught by some interleaving
    {
        int stale_caught = 0;
        for (auto &cs : cases)
            for (unsigned seed = 1; seed <= 6; ++seed) {
                std::string msg;
                if (run_after_failure(cs.B, cs.S, cs.n_ssor, seed, parts_sync_after_error, msg)) {
                    printf("FAIL after a failed launch, B=%dx%dx%dx%d S=%dx%dx%dx%d n_ssor=%d seed=%u: %s\n", cs.B[0], cs.B[1],
                           cs.B[2], cs.B[3], cs.S[0], cs.S[1], cs.S[2], cs.S[3], cs.n_ssor, seed, msg.c_str());
                    ++fails;
                }
                auto zero_all = [](const unsigned *, unsigned *o) { o[0] = o[1] = o[2] = o[3] = 0u; };
                std::string m2;
                if (run_after_failure(cs.B, cs.S, cs.n_ssor, seed, zero_all, m2)) ++stale_caught;
            }
        printf("zeroing the epoch after a failure: %d of %d cases read stale halo words\n", stale_caught,
               (int)(sizeof cases / sizeof cases[0]) * 6);
        if (stale_caught == 0) { printf("FAIL: the emulator does not see stale halo words\n"); ++fails; }
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
