// Host builder of the paired-half move table for the int8 search (layout and
// position order in group.h).
//
// Every move is classified by its direction space D (the span of x ^ x0 over
// its support, x0 its smallest point; for a flat a + V of EG(m, 2), D = V).
// A normal u can carry the move iff u is orthogonal to D and 0 < u < N/4.  All moves with the same D go to the same normal u;
// those in the half u.x = 0 become rows, and each row's partner, the move
// translated by e_i, must be in the table too (true for the minimum-weight
// tables: the translate of a flat is a flat with the same direction).
//
// Normals are chosen greedily so that most of them carry a multiple of 128
// rows (whole chunks): repeatedly the normal with the most rows still
// available takes whole chunks' worth of directions, those with the fewest
// alternative normals first; what is left is spread the same way into
// partly filled chunks, padded with all-zero rows, and a repair pass then
// moves directions between normals to empty partly filled chunks.  Only
// normals below N/4 are used (the same split in every lane group); they
// cover every direction space of codimension 3 or more.  The moves of a
// direction space without one (codimension 2: e.g. 4096 of the 10668 moves
// of RM(2, 7)) are listed apart, with their indices, for the plain search.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"
#include "group.h"

namespace {

inline int par(uint32_t x) { return __builtin_popcount(x) & 1; }
inline uint32_t ins(uint32_t e, int i, uint32_t v) { return ((e >> i) << (i + 1)) | (v << i) | (e & ((1u << i) - 1u)); }

inline bool has(const uint8_t* row, int x) { return (row[x >> 3] >> (x & 7)) & 1; }

// Reduced echelon basis of the direction space, one byte per pivot (the
// highest set bit); the packed bytes identify the space.
uint64_t direction_key(const uint8_t* row, int N, int32_t* x0_out)
{
    uint32_t b[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int x0 = -1;
    for (int x = 0; x < N; ++x) {
        if (!has(row, x)) continue;
        if (x0 < 0) {
            x0 = x;
            continue;
        }
        uint32_t v = (uint32_t)(x ^ x0);
        for (int j = 7; j >= 0 && v; --j) {
            if (!((v >> j) & 1u)) continue;
            if (b[j]) {
                v ^= b[j];
            } else {
                b[j] = v;
                v = 0;
            }
        }
    }
    for (int j = 0; j < 8; ++j)
        if (b[j])
            for (int k = j + 1; k < 8; ++k)
                if ((b[k] >> j) & 1u) b[k] ^= b[j];
    uint64_t key = 0;
    for (int j = 0; j < 8; ++j) key |= (uint64_t)b[j] << (8 * j);
    *x0_out = x0;
    return key;
}

constexpr int64_t kGroupRowsLocal = mpwsd::kGroupRows;

struct Dir {
    int64_t begin, end;  // members in order[begin, end), ascending index
    uint64_t cand[4];    // candidate normals (bit u)
    int ncand;
    int64_t rows;        // moves in one half
    bool taken;
};

struct Round {
    uint32_t u;
    std::vector<int64_t> dirs;
};

// Fewer partly filled chunks: when every direction has the same number of
// rows R and R divides 128, the chunk count of a normal is ceil(load / per),
// per = 128 / R directions.  For normals with a partial chunk (smallest
// remainder first) the capacity is lowered by one chunk and the surplus
// directions are pushed along augmenting paths (a direction moves to another
// of its candidate normals, displacing one there, ...) to normals with spare
// capacity; an attempt that cannot place all of them is undone.  Only worth
// it, and only run, when padding exceeds 2% of the rows.
void repack(std::vector<Dir>& dirs, std::vector<Round>& rounds, int N)
{
    if (dirs.empty()) return;
    const int64_t R = dirs[0].rows;
    for (const Dir& d : dirs)
        if (d.rows != R) return;
    if (R <= 0 || kGroupRowsLocal % R) return;
    const int64_t per = kGroupRowsLocal / R;
    const int nr = (int)rounds.size();
    std::vector<std::vector<int64_t>> mem(nr);
    std::vector<int> owner(dirs.size());
    std::vector<int64_t> posn(dirs.size());
    std::vector<int> ridx((size_t)N, -1);
    for (int k = 0; k < nr; ++k) ridx[rounds[k].u] = k;
    int64_t total = 0, chunks = 0;
    for (int k = 0; k < nr; ++k) {
        for (int64_t di : rounds[k].dirs) {
            owner[di] = k;
            posn[di] = (int64_t)mem[k].size();
            mem[k].push_back(di);
        }
        total += (int64_t)mem[k].size();
        chunks += ((int64_t)mem[k].size() + per - 1) / per;
    }
    if ((chunks * per - total) * 50 <= total) return;
    std::vector<int64_t> cap(nr);
    for (int k = 0; k < nr; ++k) cap[k] = ((int64_t)mem[k].size() + per - 1) / per * per;
    auto move_dir = [&](int64_t di, int to) {
        const int from = owner[di];
        const int64_t last = mem[from].back();
        mem[from][posn[di]] = last;
        posn[last] = posn[di];
        mem[from].pop_back();
        owner[di] = to;
        posn[di] = (int64_t)mem[to].size();
        mem[to].push_back(di);
    };
    struct Step {
        int64_t di;
        int from;
    };
    // one direction out of normal k0, along a shortest path of moves
    auto augment = [&](int k0, std::vector<Step>& log) {
        std::vector<int> par(nr, -2);
        std::vector<int64_t> via(nr, -1);
        std::vector<int> q{k0};
        par[k0] = -1;
        for (size_t h = 0; h < q.size(); ++h) {
            const int k = q[h];
            for (int64_t di : mem[k]) {
                const Dir& d = dirs[di];
                for (int w = 0; w < 4; ++w) {
                    uint64_t bits = d.cand[w];
                    while (bits) {
                        const int u = 64 * w + __builtin_ctzll(bits);
                        bits &= bits - 1;
                        const int k2 = ridx[u];
                        if (k2 < 0 || par[k2] != -2) continue;
                        par[k2] = k;
                        via[k2] = di;
                        if ((int64_t)mem[k2].size() < cap[k2]) {
                            for (int t = k2; par[t] >= 0; t = par[t]) {
                                log.push_back(Step{via[t], owner[via[t]]});
                                move_dir(via[t], t);
                            }
                            return true;
                        }
                        q.push_back(k2);
                    }
                }
            }
        }
        return false;
    };
    std::vector<int> order(nr);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)mem[a].size() % per < (int64_t)mem[b].size() % per;
    });
    for (int k : order) {
        const int64_t rem = (int64_t)mem[k].size() % per;
        if (rem == 0) continue;
        cap[k] -= per;
        std::vector<Step> log;
        bool ok = true;
        for (int64_t t = 0; t < rem && ok; ++t) ok = augment(k, log);
        if (!ok) {
            for (size_t j = log.size(); j-- > 0;) move_dir(log[j].di, log[j].from);
            cap[k] += per;
        }
    }
    for (int k = 0; k < nr; ++k) rounds[k].dirs = mem[k];
}

}  // namespace

extern "C" int mpwsd_group_moves(int m, const uint8_t* moves, int64_t P, uint8_t* out, size_t cap_bytes,
                                 int64_t* chunks_out, int64_t* extras_out, size_t* bytes_out)
{
    using namespace mpwsd;
    clear_error();
    if (m != 7 && m != 8) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: needs m = 7 or 8 (m=%d)", m);
    if (!moves || P < 2 || P > kMaxMoves)
        return fail(MPWSD_ERR_ARG, "mpwsd_group_moves: need a table of 2 .. %lld moves", (long long)kMaxMoves);
    const int N = 1 << m, NB = N / 8, LB = N / 4, KW = N / 2;

    // direction space of every move; members of a space sorted by index
    std::vector<uint64_t> key((size_t)P);
    std::vector<int32_t> x0((size_t)P);
    for (int64_t p = 0; p < P; ++p) {
        key[p] = direction_key(moves + (size_t)p * NB, N, &x0[p]);
        if (x0[p] < 0) return fail(MPWSD_ERR_ARG, "mpwsd_group_moves: move %lld is empty", (long long)p);
    }
    std::vector<int64_t> order((size_t)P);
    std::iota(order.begin(), order.end(), int64_t(0));
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });

    // only normals inside the lane groups (u < N/4): every lane group splits
    // alike, and fewer normals fill their chunks better; they exist for every
    // direction space of codimension 3 or more.  The moves of a direction
    // space without one are kept apart (searched with plain rows).
    std::vector<Dir> dirs;
    std::vector<int64_t> extra;
    for (int64_t s = 0; s < P;) {
        int64_t e = s;
        while (e < P && key[order[e]] == key[order[s]]) ++e;
        Dir d{};
        d.begin = s;
        d.end = e;
        const uint64_t k = key[order[s]];
        for (uint32_t u = 1; u < (uint32_t)LB; ++u) {
            bool ok = true;
            for (int j = 0; j < 8 && ok; ++j) ok = !par(u & (uint32_t)((k >> (8 * j)) & 0xFFu));
            if (ok) {
                d.cand[u >> 6] |= 1ull << (u & 63);
                ++d.ncand;
            }
        }
        if (d.ncand == 0) {
            for (int64_t a = s; a < e; ++a) extra.push_back(order[a]);
        } else {
            if ((e - s) % 2)
                return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: move %lld has no translate partner",
                            (long long)order[s]);
            d.rows = (e - s) / 2;
            dirs.push_back(d);
        }
        s = e;
    }
    std::sort(extra.begin(), extra.end());
    const int64_t E = (int64_t)extra.size();
    auto cand = [](const Dir& d, uint32_t u) { return (d.cand[u >> 6] >> (u & 63)) & 1ull; };

    // greedy choice of normals: rounds of (normal, directions)
    std::vector<int64_t> byflex(dirs.size());
    std::iota(byflex.begin(), byflex.end(), int64_t(0));
    std::stable_sort(byflex.begin(), byflex.end(), [&](int64_t a, int64_t b) { return dirs[a].ncand < dirs[b].ncand; });
    std::vector<int64_t> avail((size_t)N, 0);
    for (const Dir& d : dirs)
        for (uint32_t u = 1; u < (uint32_t)N; ++u)
            if (cand(d, u)) avail[u] += d.rows;
    std::vector<Round> rounds;
    int64_t left = (int64_t)dirs.size();
    for (int whole = 1; whole >= 0 && left > 0; --whole) {
        while (left > 0) {
            uint32_t best = 1;
            for (uint32_t u = 1; u < (uint32_t)N; ++u)
                if (avail[u] > avail[best]) best = u;
            const int64_t target = whole ? avail[best] / kGroupRows * kGroupRows : avail[best];
            if (target == 0) break;
            Round rd{best, {}};
            int64_t got = 0;
            for (int64_t di : byflex) {
                Dir& d = dirs[di];
                if (d.taken || !cand(d, best) || got + d.rows > target) continue;
                d.taken = true;
                got += d.rows;
                rd.dirs.push_back(di);
                --left;
                for (uint32_t u = 1; u < (uint32_t)N; ++u)
                    if (cand(d, u)) avail[u] -= d.rows;
            }
            if (rd.dirs.empty()) break;
            rounds.push_back(std::move(rd));
        }
    }
    if (left > 0) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: %lld directions left unplaced", (long long)left);
    // one round per normal from here on
    {
        std::vector<Round> merged;
        std::vector<int> at((size_t)N, -1);
        for (Round& rd : rounds) {
            if (at[rd.u] < 0) {
                at[rd.u] = (int)merged.size();
                merged.push_back(Round{rd.u, {}});
            }
            std::vector<int64_t>& v = merged[at[rd.u]].dirs;
            v.insert(v.end(), rd.dirs.begin(), rd.dirs.end());
        }
        rounds.swap(merged);
    }
    repack(dirs, rounds, N);

    // rows of each round: (move in half 0, its translate), ascending index
    struct Row {
        int64_t p, q;
    };
    std::vector<std::vector<Row>> rrows(rounds.size());
    int64_t chunks = 0;
    for (size_t ri = 0; ri < rounds.size(); ++ri) {
        const uint32_t u = rounds[ri].u, ulo = u & (uint32_t)(LB - 1);
        const int i = __builtin_ctz(ulo);
        for (int64_t di : rounds[ri].dirs) {
            const Dir& d = dirs[di];
            for (int64_t a = d.begin; a < d.end; ++a) {
                const int64_t p = order[a];
                if (par(u & (uint32_t)x0[p])) continue;  // half 1: somebody's partner
                const uint8_t* rp = moves + (size_t)p * NB;
                int64_t q = -1;
                for (int64_t b = d.begin; b < d.end && q < 0; ++b) {
                    const uint8_t* rq = moves + (size_t)order[b] * NB;
                    if (!has(rq, x0[p] ^ (1 << i))) continue;
                    bool same = true;
                    for (int x = 0; x < N && same; ++x) same = has(rp, x) == has(rq, x ^ (1 << i));
                    if (same) q = order[b];
                }
                if (q < 0)
                    return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: move %lld has no translate partner",
                                (long long)p);
                rrows[ri].push_back(Row{p, q});
            }
        }
        if ((int64_t)rrows[ri].size() * 2 != [&] {
                int64_t n = 0;
                for (int64_t di : rounds[ri].dirs) n += dirs[di].end - dirs[di].begin;
                return n;
            }())
            return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: halves of normal %u do not pair up", u);
        std::sort(rrows[ri].begin(), rrows[ri].end(), [](const Row& a, const Row& b) { return a.p < b.p; });
        chunks += ((int64_t)rrows[ri].size() + kGroupRows - 1) / kGroupRows;
    }

    const GroupLayout g = group_layout(m, chunks, E);
    if (chunks_out) *chunks_out = chunks;
    if (extras_out) *extras_out = E;
    if (bytes_out) *bytes_out = g.bytes;
    if (!out) return MPWSD_OK;
    if (cap_bytes < g.bytes)
        return fail(MPWSD_ERR_SIZE, "mpwsd_group_moves: needs %zu bytes, got %zu", g.bytes, cap_bytes);

    std::memset(out, 0, g.bytes);
    GroupHeader h{kGroupMagic, kGroupVersion, m, N, P, chunks, KW, 0, E};
    std::memcpy(out, &h, sizeof h);
    for (int64_t x = 0; x < E; ++x) {
        std::memcpy(out + g.xrows_off + (size_t)x * NB, moves + (size_t)extra[x] * NB, (size_t)NB);
        ((int32_t*)(out + g.xcanon_off))[x] = (int32_t)extra[x];
    }
    int32_t* uo = (int32_t*)(out + g.u_off);
    uint8_t* ro = out + g.rows_off;
    int32_t* co = (int32_t*)(out + g.canon_off);
    // selectors of every normal below N/4 (the search's byte gathers)
    {
        const int LDW = LB / 4, WDW = LDW / 2;
        int32_t* so = (int32_t*)(out + g.sel_off);
        for (uint32_t u = 1; u < (uint32_t)LB; ++u) {
            int32_t* t = so + (size_t)u * g.SELW;
            const int i = __builtin_ctz(u);
            const int S = i > 2 ? i - 2 : 0;
            t[0] = S;
            for (int k = 0; k < WDW; ++k) {
                const int lo = ((k >> S) << (S + 1)) | (k & ((1 << S) - 1));
                for (int h = 0; h < 2; ++h) {
                    uint32_t sel = 0;
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t e = (uint32_t)(4 * k + j);
                        const uint32_t b = (uint32_t)par(u & ins(e, i, 0)) ^ (uint32_t)h;
                        const uint32_t tb = ins(e, i, b);
                        sel |= (((int)(tb >> 2) == lo ? 0u : 4u) + (tb & 3u)) << (8 * j);
                    }
                    t[1 + h * WDW + k] = (int32_t)sel;
                }
            }
            for (int d = 0; d < LDW; ++d) {
                uint32_t sel = 0;
                for (int b = 0; b < 4; ++b) {
                    const uint32_t tb = (uint32_t)(4 * d + b);
                    const uint32_t bit = (tb >> i) & 1u;
                    const uint32_t e = ((tb >> (i + 1)) << i) | (tb & ((1u << i) - 1u));
                    const uint32_t h = bit ^ (uint32_t)par(u & ins(e, i, 0));
                    sel |= (4u * h + (e & 3u)) << (8 * b);
                }
                t[1 + 2 * WDW + d] = (int32_t)sel;
            }
        }
    }
    int64_t c = 0;
    for (size_t ri = 0; ri < rounds.size(); ++ri) {
        const uint32_t u = rounds[ri].u, ulo = u & (uint32_t)(LB - 1), uhi = u / (uint32_t)LB;
        const int i = __builtin_ctz(ulo);
        const std::vector<Row>& rows = rrows[ri];
        for (size_t r0 = 0; r0 < rows.size(); r0 += kGroupRows, ++c) {
            uo[c] = (int32_t)u;
            for (int r = 0; r < kGroupRows; ++r) {
                int32_t* cc = co + (size_t)c * 2 * kGroupRows;
                if (r0 + r >= rows.size()) {
                    cc[r] = cc[kGroupRows + r] = (int32_t)P;
                    continue;
                }
                const Row& rw = rows[r0 + r];
                if (r > 0 && rw.q <= rows[r0 + r - 1].q)
                    return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_group_moves: translates of normal %u out of order", u);
                cc[r] = (int32_t)rw.p;
                cc[kGroupRows + r] = (int32_t)rw.q;
                const uint8_t* rp = moves + (size_t)rw.p * NB;
                uint8_t* dst = ro + ((size_t)c * kGroupRows + r) * KW;
                const int sw = group_swizzle(KW, r);
                for (int k = 0; k < KW; ++k) {
                    const uint32_t lg = (uint32_t)k / (uint32_t)(KW / 4), e = (uint32_t)k % (uint32_t)(KW / 4);
                    const uint32_t b = (uint32_t)(par(ulo & ins(e, i, 0)) ^ par(uhi & lg));
                    const int x = (int)(lg * (uint32_t)LB + ins(e, i, b));
                    if (has(rp, x)) dst[16 * ((k / 16) ^ sw) + k % 16] = 0x80;
                }
            }
        }
    }
    return MPWSD_OK;
}
