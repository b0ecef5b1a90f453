// Host-side geometry tables of libsapq (no HIP dependency): the slot order of a block
// (hyperplanes of the locally-lexicographic SSOR, section 3 "Inverse of block operator", Fig. 1), neighbour tables, the block
// colouring, and the split of a block into two workgroups for the two-lanes-per-site
// phase kernel.  Used by api.hip and compiled on its own by the host-logic tests.
#pragma once

#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/sapq.h"

namespace sapq {

constexpr int WRAP_BIT = 1 << 30;  // in blk_nbr: the hop crosses the lattice boundary
constexpr int BLK_MASK = WRAP_BIT - 1;
constexpr int MAX_PLANES = 64;

// ---------------------------------------------------------------- geometry tables (host)
struct HostTables {
    int Vb = 0, NB = 0, nplanes = 0, max_plane = 0;
    int nbk[4];
    std::vector<int> loc_nbr, blk_nbr, plane_start, slot_lex, blk_lex, lex_blk, zord_blk;
    std::vector<int> nbr16;  // packed forward/backward slots per direction (stored as unsigned)
};

// An all-zero sub-block shape asks for the even-odd site order instead of the ll order:
// first the sites of the block whose block-local coordinates have an even sum, then the odd
// ones, each in lexicographic order.  This is the ordering the paper compares the ll order
// against (section 3, "Inverse of block operator"); its two hyperplanes are the two parities.
inline bool eo_order(const sapq_geom *G) {
    return G->subblock[0] == 0 && G->subblock[1] == 0 && G->subblock[2] == 0 && G->subblock[3] == 0;
}

// Slots sorted by hyperplane h = sum_mu (x_mu mod S_mu) (the site parity for the even-odd
// order); inside a plane first by the half of the block in t that the site lies in (when
// the sub-block layers in t split evenly), then by the ll key.  The order inside a
// hyperplane is free (its sites are independent); this one gives each half of the block one
// contiguous slot range per hyperplane.
inline void build_tables(const sapq_geom *G, HostTables &T) {
    const int *B = G->block, *S = G->subblock;
    const bool eo = eo_order(G);
    int Vb = B[0] * B[1] * B[2] * B[3];
    int ns[4];
    for (int m = 0; m < 4; ++m) { ns[m] = eo ? 1 : B[m] / S[m]; T.nbk[m] = G->L[m] / B[m]; }
    int Nsub = ns[0] * ns[1] * ns[2] * ns[3];
    struct Key { int h, half; long ll; int lex; };
    std::vector<Key> keys(Vb);
    for (int l = 0; l < Vb; ++l) {
        int c[4], r = l;
        for (int m = 0; m < 4; ++m) { c[m] = r % B[m]; r /= B[m]; }
        if (eo) {
            keys[l] = {(c[0] + c[1] + c[2] + c[3]) & 1, B[3] % 2 == 0 ? c[3] * 2 / B[3] : 0, l, l};
            continue;
        }
        int h = 0; long pos = 0, sub = 0, pm = 1, sm = 1;
        for (int m = 0; m < 4; ++m) {
            h += c[m] % S[m];
            pos += (c[m] % S[m]) * pm; pm *= S[m];
            sub += (c[m] / S[m]) * sm; sm *= ns[m];
        }
        const int half = ns[3] % 2 == 0 ? (c[3] / S[3]) * 2 / ns[3] : 0;
        keys[l] = {h, half, pos * Nsub + sub, l};
    }
    std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) {
        return a.h != b.h ? a.h < b.h : a.half != b.half ? a.half < b.half : a.ll < b.ll;
    });
    T.Vb = Vb;
    T.slot_lex.resize(Vb);
    std::vector<int> slot_of(Vb);
    for (int s = 0; s < Vb; ++s) { T.slot_lex[s] = keys[s].lex; slot_of[keys[s].lex] = s; }
    int H = keys.back().h + 1;
    T.nplanes = H;
    T.plane_start.assign(H + 1, 0);
    for (auto &k : keys) T.plane_start[k.h + 1]++;
    for (int p = 0; p < H; ++p) T.plane_start[p + 1] += T.plane_start[p];
    T.max_plane = 0;
    for (int p = 0; p < H; ++p) T.max_plane = std::max(T.max_plane, T.plane_start[p + 1] - T.plane_start[p]);
    // in-block neighbours
    T.loc_nbr.resize(8 * Vb);
    for (int s = 0; s < Vb; ++s) {
        int c[4], r = T.slot_lex[s];
        for (int m = 0; m < 4; ++m) { c[m] = r % B[m]; r /= B[m]; }
        for (int mu = 0; mu < 4; ++mu)
            for (int dir = 0; dir < 2; ++dir) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] += dir == 0 ? 1 : -1;
                bool inside = cc[mu] >= 0 && cc[mu] < B[mu];
                cc[mu] = (cc[mu] + B[mu]) % B[mu];
                int l = cc[0] + B[0] * (cc[1] + B[1] * (cc[2] + B[2] * cc[3]));
                int t = slot_of[l];
                T.loc_nbr[(2 * mu + dir) * Vb + s] = inside ? t : -1 - t;
            }
    }
    T.nbr16.resize(4 * Vb);
    for (int mu = 0; mu < 4; ++mu)
        for (int s = 0; s < Vb; ++s) {
            int f = T.loc_nbr[(2 * mu) * Vb + s], b = T.loc_nbr[(2 * mu + 1) * Vb + s];
            unsigned wf = f >= 0 ? (unsigned)f | 0x8000u : (unsigned)(-1 - f);
            unsigned wb = b >= 0 ? (unsigned)b | 0x8000u : (unsigned)(-1 - b);
            T.nbr16[mu * Vb + s] = (int)(wf | (wb << 16));
        }
    // blocks: E (colour 0) first, then O, each in lexicographic order
    int NB = T.nbk[0] * T.nbk[1] * T.nbk[2] * T.nbk[3];
    T.NB = NB;
    T.blk_lex.clear();
    for (int col = 0; col < 2; ++col)
        for (int b = 0; b < NB; ++b) {
            int r = b, sum = 0;
            for (int m = 0; m < 4; ++m) { sum += r % T.nbk[m]; r /= T.nbk[m]; }
            if ((sum & 1) == col) T.blk_lex.push_back(b);
        }
    std::vector<int> ib_of(NB);
    for (int i = 0; i < NB; ++i) ib_of[T.blk_lex[i]] = i;
    T.lex_blk = ib_of;
    // blocks in Z (Morton) order of their block coordinates: each aligned group of 2^k blocks
    // per dimension is contiguous in it, so a run of it is a compact piece of the lattice
    {
        std::vector<std::pair<unsigned long long, int>> key(NB);
        for (int b = 0; b < NB; ++b) {
            int c[4], r = b;
            for (int m = 0; m < 4; ++m) { c[m] = r % T.nbk[m]; r /= T.nbk[m]; }
            unsigned long long k = 0;
            for (int bit = 0; bit < 15; ++bit)
                for (int m = 0; m < 4; ++m) k |= (unsigned long long)((c[m] >> bit) & 1) << (4 * bit + m);
            key[b] = {k, b};
        }
        std::sort(key.begin(), key.end());
        T.zord_blk.resize(NB);
        for (int i = 0; i < NB; ++i) T.zord_blk[i] = ib_of[key[i].second];
    }
    T.blk_nbr.resize(8 * NB);
    for (int i = 0; i < NB; ++i) {
        int c[4], r = T.blk_lex[i];
        for (int m = 0; m < 4; ++m) { c[m] = r % T.nbk[m]; r /= T.nbk[m]; }
        for (int mu = 0; mu < 4; ++mu)
            for (int dir = 0; dir < 2; ++dir) {
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] += dir == 0 ? 1 : -1;
                bool wrap = cc[mu] < 0 || cc[mu] >= T.nbk[mu];
                cc[mu] = (cc[mu] + T.nbk[mu]) % T.nbk[mu];
                int l = cc[0] + T.nbk[0] * (cc[1] + T.nbk[1] * (cc[2] + T.nbk[2] * cc[3]));
                T.blk_nbr[(2 * mu + dir) * NB + i] = ib_of[l] | (wrap ? WRAP_BIT : 0);
            }
    }
}

// Split of a block along t into NP parts for the two-lanes-per-site phase kernel: the
// sub-block layers in t are divided in halves, and the slots of each part keep the block's
// order, so every hyperplane of the block contributes the same number of sites to each part.
struct PartTables {
    int NP = 1, Vp = 0, Hp = 0, max_plane = 0;
    std::vector<int> gslot, pstart, exp_idx, imp, imp_start;
    std::vector<unsigned> pnb;  // [NP][Vp][2 lanes][2 words]
    std::vector<unsigned> gnb;  // [NP][Vp][2 words]: block slots of the backward neighbours
};

inline bool build_parts(const sapq_geom *G, const HostTables &T, int NP, PartTables &P) {
    const int *B = G->block, *S = G->subblock;
    // the split of a block in two is written for the ll order's sub-block layers in t
    if (eo_order(G) && NP != 1) return false;
    const int Vb = T.Vb, nst = eo_order(G) ? 1 : B[3] / S[3], H = T.nplanes;
    if (NP < 1 || NP > 2 || nst % NP) return false;
    const int Vp = Vb / NP, slab = B[0] * B[1] * B[2];
    std::vector<int> part_of(Vb), loc_of(Vb), plane_of(Vb), cnt(NP, 0);
    for (int h = 0; h < H; ++h)
        for (int s = T.plane_start[h]; s < T.plane_start[h + 1]; ++s) plane_of[s] = h;
    P = PartTables();
    P.NP = NP;
    P.Vp = Vp;
    P.gslot.assign((size_t)NP * Vp, 0);
    for (int s = 0; s < Vb; ++s) {
        const int t = T.slot_lex[s] / slab;
        const int p = eo_order(G) ? 0 : (t / S[3]) * NP / nst;
        if (cnt[p] >= Vp) return false;
        part_of[s] = p;
        loc_of[s] = cnt[p];
        P.gslot[(size_t)p * Vp + cnt[p]++] = s;
    }
    P.pstart.assign(MAX_PLANES + 1, 0);
    for (int h = 0; h <= H; ++h) {
        if (T.plane_start[h] % NP) return false;
        P.pstart[h] = T.plane_start[h] / NP;
    }
    for (int h = 0; h < H; ++h) P.max_plane = std::max(P.max_plane, P.pstart[h + 1] - P.pstart[h]);
    // the kernel computes the block slot of part-local site i in hyperplane h as
    // i + pstart[h] + p (pstart[h + 1] - pstart[h]) for NP = 2, and i for NP = 1
    for (int p = 0; p < NP; ++p)
        for (int i = 0; i < Vp; ++i) {
            const int s = P.gslot[(size_t)p * Vp + i], h = plane_of[s];
            if (i < P.pstart[h] || i >= P.pstart[h + 1]) return false;
            const int want = NP == 2 ? i + P.pstart[h] + p * (P.pstart[h + 1] - P.pstart[h]) : i;
            if (s != want) return false;
        }
    // boundary layer of each part: its sites with a neighbour in the other part
    P.exp_idx.assign((size_t)NP * Vp, -1);
    std::vector<int> nexp(NP, 0);
    for (int p = 0; p < NP; ++p)
        for (int i = 0; i < Vp; ++i) {
            const int s = P.gslot[(size_t)p * Vp + i];
            for (int k = 0; k < 8; ++k) {
                const int t = T.loc_nbr[(size_t)k * Vb + s];
                if (t >= 0 && part_of[t] != p) { P.exp_idx[(size_t)p * Vp + i] = nexp[p]++; break; }
            }
        }
    P.Hp = nexp[0];
    for (int p = 0; p < NP; ++p)
        if (nexp[p] != P.Hp) return false;
    if (Vp + P.Hp + 1 > 65535) return false;
    // LDS slots of the neighbours (own site, halo slot Vp + k, or the zero slot Vp + Hp) and
    // the halo slots each hyperplane reads, in the order of the hyperplanes
    const unsigned zero = (unsigned)(Vp + P.Hp);
    P.pnb.assign((size_t)NP * Vp * 4, 0);
    P.gnb.assign((size_t)NP * Vp * 2, 0);
    if (Vb > 65535) return false;
    P.imp.assign((size_t)NP * std::max(P.Hp, 1), 0);
    P.imp_start.assign((size_t)NP * (MAX_PLANES + 1), 0);
    for (int p = 0; p < NP; ++p) {
        std::vector<std::pair<int, int>> li;
        for (int i = 0; i < Vp; ++i) {
            const int s = P.gslot[(size_t)p * Vp + i];
            for (int d = 0; d < 2; ++d) {
                unsigned sl[4];
                for (int mu = 0; mu < 4; ++mu) {
                    const int t = T.loc_nbr[(size_t)(2 * mu + d) * Vb + s];
                    if (t < 0) {
                        sl[mu] = zero;
                    } else if (part_of[t] == p) {
                        sl[mu] = (unsigned)loc_of[t];
                    } else {
                        const int k = P.exp_idx[(size_t)part_of[t] * Vp + loc_of[t]];
                        if (k < 0 || mu != 3) return false;
                        // part 0 reads part 1 through +t at a lower hyperplane, part 1 reads
                        // part 0 through -t at a higher one (the kernel's choice of sweep)
                        if ((p == 0) != (d == 0) || (p == 0) != (plane_of[t] < plane_of[s])) return false;
                        sl[mu] = (unsigned)(Vp + k);
                        li.push_back({plane_of[s], k});
                    }
                }
                const size_t o = (((size_t)p * Vp + i) * 2 + d) * 2;
                P.pnb[o] = sl[0] | (sl[1] << 16);
                P.pnb[o + 1] = sl[2] | (sl[3] << 16);
                if (d == 1) {
                    // the link of a backward hop sits at the neighbour (the site itself when
                    // the neighbour is outside the block: that hop is masked)
                    unsigned gs[4];
                    for (int mu = 0; mu < 4; ++mu) {
                        const int t = T.loc_nbr[(size_t)(2 * mu + 1) * Vb + s];
                        gs[mu] = (unsigned)(t >= 0 ? t : s);
                    }
                    P.gnb[((size_t)p * Vp + i) * 2] = gs[0] | (gs[1] << 16);
                    P.gnb[((size_t)p * Vp + i) * 2 + 1] = gs[2] | (gs[3] << 16);
                }
            }
        }
        if ((int)li.size() != P.Hp) return false;  // every halo slot is read by exactly one site
        std::stable_sort(li.begin(), li.end(), [](const std::pair<int, int> &a, const std::pair<int, int> &b) { return a.first < b.first; });
        std::vector<int> seen(P.Hp, 0);
        int *st = &P.imp_start[(size_t)p * (MAX_PLANES + 1)];
        for (size_t j = 0; j < li.size(); ++j) {
            if (seen[li[j].second]++) return false;
            P.imp[(size_t)p * P.Hp + j] = li[j].second;
            st[li[j].first + 1]++;
        }
        for (int h = 0; h < H; ++h) st[h + 1] += st[h];
        for (int h = H + 1; h <= MAX_PLANES; ++h) st[h] = st[H];
    }
    if (NP == 2) {
        // at the turn of a sweep the kernel keeps the halo of the repeated plane: part 0 must
        // read nothing at plane 0 and part 1 nothing at plane H - 1
        const int *s0 = &P.imp_start[0], *s1 = &P.imp_start[MAX_PLANES + 1];
        if (s0[1] != s0[0] || s1[H] != s1[H - 1]) return false;
    }
    return true;
}

// Sync words of the split phase kernel ([0] ticket, [1] done, [2] epoch, [3] error) to use
// after a launch that raised the error word.  The halo words that launch left in the
// exchange array carry its epoch (or an earlier one), so the epoch only moves forward: the
// next launch must never tag its words like the failed one, or a part could take a stale
// word for a current one.  Ticket and done counts restart from zero (a workgroup that found
// the ticket counter out of step returned without counting itself done).
inline void parts_sync_after_error(const unsigned in[4], unsigned out[4]) {
    out[0] = 0u;
    out[1] = 0u;
    out[2] = in[2] + 1u;
    out[3] = 0u;
}

}  // namespace sapq
