// Host side of the library: error state, code parameters and the move table
// S_1(0) \ {0} of RM(r, m) (Sec. II-C, Eq. (2)-(3)).
//
// The minimum-weight codewords of RM(r, m) are the incidence vectors of the
// (m-r)-dimensional flats of EG(m, 2).  This file enumerates each flat as the
// solution set of r independent affine equations a_i . x = b_i over F_2: the
// coefficient rows run over all r x m matrices in reduced echelon form (each
// row's lowest set bit is its pivot, pivots increase down the rows, and no
// row has a bit at another row's pivot), and b over F_2^r.  Distinct (matrix,
// b) pairs give distinct flats, and every flat arises once.  The table is
// then sorted canonically: sorted supports compared lexicographically, which
// for equal-weight sets is decided by the smallest point of the symmetric
// difference (the set holding it comes first).
//
// Larger spheres S_rho(0), rho >= 2 (Eq. (1)-(2)), hold every nonzero
// codeword whose weight is one of the rho smallest nonzero weights of the
// code.  For codes of dimension K <= 30 they are found by walking all 2^K
// codewords: the message space is cut into one block per host thread, each
// block is walked in Gray-code order (one generator row XORed per step, the
// weight taken by popcount of the bit-packed word), a first walk counts the
// weights and a second keeps the words of the wanted weights.  The table is
// sorted by weight, then canonically.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"

namespace mpwsd {

namespace {
thread_local std::string g_last_error;

struct Mask256 {
    uint64_t w[4];
};

bool canonical_less(const Mask256& x, const Mask256& y)
{
    for (int i = 0; i < 4; ++i) {
        uint64_t d = x.w[i] ^ y.w[i];
        if (d) return (x.w[i] & (d & (~d + 1))) != 0;
    }
    return false;
}

void enumerate_rows(int m, int r, int row, int last_pivot, std::vector<int>& pivots,
                    std::vector<uint32_t>& rows, std::vector<Mask256>& out)
{
    if (row == r) {
        // rows[] are complete only now: free bits of a row may sit at
        // positions that later rows choose as pivots, so reduce first.
        for (int i = 0; i < r; ++i)
            for (int k = 0; k < r; ++k)
                if (k != i && (rows[i] >> pivots[k] & 1u)) return;  // not reduced
        const int n = 1 << m;
        for (uint32_t b = 0; b < (1u << r); ++b) {
            Mask256 f{};
            for (int x = 0; x < n; ++x) {
                bool in = true;
                for (int i = 0; i < r && in; ++i)
                    in = ((__builtin_popcount(rows[i] & (uint32_t)x) & 1) == (int)((b >> i) & 1u));
                if (in) f.w[x >> 6] |= 1ull << (x & 63);
            }
            out.push_back(f);
        }
        return;
    }
    for (int p = last_pivot + 1; p <= m - (r - row); ++p) {
        pivots[row] = p;
        // free bits: positions above p; pivots of later rows are excluded by
        // the reduction check at the leaf
        int nfree = m - 1 - p;
        for (uint32_t fb = 0; fb < (1u << nfree); ++fb) {
            rows[row] = (1u << p) | (fb << (p + 1));
            // earlier rows must not touch this pivot
            bool ok = true;
            for (int i = 0; i < row; ++i)
                if (rows[i] >> p & 1u) { ok = false; break; }
            if (!ok) continue;
            enumerate_rows(m, r, row + 1, p, pivots, rows, out);
        }
    }
}
// ---- exhaustive walk of RM(r, m), bit-packed
struct Walk {
    int n = 0, nw = 0, K = 0;
    std::vector<Mask256> rows;  // generator rows of the information positions, ascending
};

Walk make_walk(int r, int m)
{
    Walk w;
    w.n = 1 << m;
    w.nw = w.n >= 64 ? w.n / 64 : 1;
    for (int i = 0; i < w.n; ++i) {
        if (__builtin_popcount((unsigned)i) < m - r) continue;
        Mask256 row{};
        for (int j = 0; j < w.n; ++j)
            if ((j & ~i) == 0) row.w[j >> 6] |= 1ull << (j & 63);
        w.rows.push_back(row);
    }
    w.K = (int)w.rows.size();
    return w;
}

int weight_of(const Mask256& c, int nw)
{
    int t = 0;
    for (int i = 0; i < nw; ++i) t += __builtin_popcountll(c.w[i]);
    return t;
}

// Visits the codewords of messages [lo, hi) in Gray-code order: fn(word, weight).
template <class Fn>
void walk_block(const Walk& wk, uint64_t lo, uint64_t hi, Fn&& fn)
{
    if (lo >= hi) return;
    Mask256 c{};
    const uint64_t g0 = lo ^ (lo >> 1);
    for (int b = 0; b < wk.K; ++b)
        if (g0 >> b & 1)
            for (int i = 0; i < wk.nw; ++i) c.w[i] ^= wk.rows[b].w[i];
    fn(c, weight_of(c, wk.nw));
    for (uint64_t g = lo + 1; g < hi; ++g) {
        const Mask256& row = wk.rows[__builtin_ctzll(g)];
        for (int i = 0; i < wk.nw; ++i) c.w[i] ^= row.w[i];
        fn(c, weight_of(c, wk.nw));
    }
}

// Host threads for a walk: one for small codes, else one per hardware thread (<= 64).
int walk_threads(const Walk& wk)
{
    if ((1ull << wk.K) < (1ull << 16)) return 1;
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h ? h : 1u, 64u));
}

// per_thread(t, lo, hi) for t < walk_threads(wk), the blocks tiling [0, 2^K).
template <class Fn>
void parallel_walk(const Walk& wk, Fn&& per_thread)
{
    const uint64_t total = 1ull << wk.K;
    const int nt = walk_threads(wk);
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const uint64_t lo = total * t / nt, hi = total * (t + 1) / nt;
        th.emplace_back([&, t, lo, hi] { per_thread(t, lo, hi); });
    }
    for (auto& x : th) x.join();
}

constexpr int kMaxWalkK = 30;

std::vector<int64_t> walk_distribution(int r, int m)
{
    const Walk wk = make_walk(r, m);
    const int nt = walk_threads(wk);
    std::vector<std::vector<int64_t>> part(nt, std::vector<int64_t>(wk.n + 1, 0));
    parallel_walk(wk, [&](int t, uint64_t lo, uint64_t hi) {
        auto& h = part[t];
        walk_block(wk, lo, hi, [&](const Mask256&, int w) { ++h[w]; });
    });
    std::vector<int64_t> A(wk.n + 1, 0);
    for (auto& h : part)
        for (int w = 0; w <= wk.n; ++w) A[w] += h[w];
    return A;
}

std::mutex g_dist_mu;
std::map<std::pair<int, int>, std::vector<int64_t>> g_dist;

const std::vector<int64_t>& cached_distribution(int r, int m)
{
    std::lock_guard<std::mutex> lk(g_dist_mu);
    auto key = std::make_pair(r, m);
    auto it = g_dist.find(key);
    if (it == g_dist.end()) it = g_dist.emplace(key, walk_distribution(r, m)).first;
    return it->second;
}

// The rho smallest nonzero weights [wlo, whi] and the number of words with
// them; false when the code has fewer nonzero weights.
bool sphere_weights(const std::vector<int64_t>& A, int rho, int& wlo, int& whi, int64_t& P)
{
    int got = 0;
    wlo = whi = -1;
    P = 0;
    for (int w = 1; w < (int)A.size() && got < rho; ++w)
        if (A[w]) {
            if (wlo < 0) wlo = w;
            whi = w;
            P += A[w];
            ++got;
        }
    return got == rho;
}
}  // namespace

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

int rm_dimension(int r, int m)
{
    int k = 0;
    for (int d = 0; d <= r; ++d) {
        int64_t c = 1;
        for (int i = 1; i <= d; ++i) c = c * (m - d + i) / i;
        k += (int)c;
    }
    return k;
}

int64_t rm_min_weight_count(int r, int m)
{
    // Gaussian binomial [m, r]_2 times the 2^r cosets of each direction space
    int64_t num = 1, den = 1;
    for (int i = 0; i < r; ++i) {
        num *= (int64_t(1) << (m - i)) - 1;
        den *= (int64_t(1) << (i + 1)) - 1;
    }
    return (num / den) << r;
}

bool valid_move_count(int r, int m, int64_t P)
{
    if (P == rm_min_weight_count(r, m)) return true;
    if (rm_dimension(r, m) > kMaxWalkK || P <= 0) return false;
    const std::vector<int64_t>& A = cached_distribution(r, m);
    int64_t cum = 0;
    for (int w = 1; w < (int)A.size(); ++w) {
        cum += A[w];
        if (A[w] && cum == P) return true;
    }
    return false;
}

}  // namespace mpwsd

extern "C" const char* mpwsd_last_error(void) { return mpwsd::g_last_error.c_str(); }

extern "C" int mpwsd_build_moves(int r, int m, uint8_t* moves, size_t cap_bytes,
                                 int64_t* P_out, int* N_out, int* w_out)
{
    using namespace mpwsd;
    clear_error();
    if (m < 2 || m > 8 || r < 1 || r >= m)
        return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_build_moves: need 1 <= r < m <= 8 (r=%d m=%d)", r, m);
    const int n = 1 << m;
    const int64_t P = rm_min_weight_count(r, m);
    if (P_out) *P_out = P;
    if (N_out) *N_out = n;
    if (w_out) *w_out = 1 << (m - r);
    if (!moves) return MPWSD_OK;
    const size_t row_bytes = (size_t)n / 8 ? (size_t)n / 8 : 1;
    if (cap_bytes < (size_t)P * row_bytes)
        return fail(MPWSD_ERR_SIZE, "mpwsd_build_moves: need %zu bytes, got %zu",
                    (size_t)P * row_bytes, cap_bytes);
    std::vector<Mask256> flats;
    flats.reserve((size_t)P);
    std::vector<int> pivots(r);
    std::vector<uint32_t> rows(r);
    enumerate_rows(m, r, 0, -1, pivots, rows, flats);
    if ((int64_t)flats.size() != P)
        return fail(MPWSD_ERR_ARG, "mpwsd_build_moves: internal count mismatch (%zu vs %lld)",
                    flats.size(), (long long)P);
    std::sort(flats.begin(), flats.end(), canonical_less);
    for (int64_t p = 0; p < P; ++p)
        std::memcpy(moves + (size_t)p * row_bytes, flats[(size_t)p].w, row_bytes);
    return MPWSD_OK;
}

extern "C" int mpwsd_build_sphere(int r, int m, int radius, uint8_t* moves, size_t cap_bytes,
                                  int64_t* P_out, int* N_out, int* w_max)
{
    using namespace mpwsd;
    clear_error();
    if (radius == 1) return mpwsd_build_moves(r, m, moves, cap_bytes, P_out, N_out, w_max);
    if (m < 2 || m > 8 || r < 1 || r >= m || radius < 1)
        return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_build_sphere: need 1 <= r < m <= 8, radius >= 1 (r=%d m=%d radius=%d)",
                    r, m, radius);
    if (rm_dimension(r, m) > kMaxWalkK)
        return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_build_sphere: radius %d needs K <= %d (RM(%d,%d) has K=%d)",
                    radius, kMaxWalkK, r, m, rm_dimension(r, m));
    const std::vector<int64_t>& A = cached_distribution(r, m);
    int wlo, whi;
    int64_t P;
    if (!sphere_weights(A, radius, wlo, whi, P))
        return fail(MPWSD_ERR_ARG, "mpwsd_build_sphere: RM(%d,%d) has fewer than %d nonzero weights", r, m, radius);
    const int n = 1 << m;
    if (P_out) *P_out = P;
    if (N_out) *N_out = n;
    if (w_max) *w_max = whi;
    if (!moves) return MPWSD_OK;
    const size_t row_bytes = (size_t)n / 8;
    if (cap_bytes < (size_t)P * row_bytes)
        return fail(MPWSD_ERR_SIZE, "mpwsd_build_sphere: need %zu bytes, got %zu", (size_t)P * row_bytes, cap_bytes);
    const Walk wk = make_walk(r, m);
    std::vector<std::vector<Mask256>> part(walk_threads(wk));
    parallel_walk(wk, [&](int t, uint64_t lo, uint64_t hi) {
        auto& out = part[t];
        walk_block(wk, lo, hi, [&](const Mask256& c, int w) {
            if (w >= wlo && w <= whi) out.push_back(c);
        });
    });
    std::vector<std::pair<int, Mask256>> all;
    all.reserve((size_t)P);
    for (auto& v : part) {
        for (auto& c : v) all.emplace_back(weight_of(c, wk.nw), c);
        std::vector<Mask256>().swap(v);
    }
    if ((int64_t)all.size() != P)
        return fail(MPWSD_ERR_ARG, "mpwsd_build_sphere: internal count mismatch (%zu vs %lld)", all.size(),
                    (long long)P);
    std::sort(all.begin(), all.end(), [](const std::pair<int, Mask256>& a, const std::pair<int, Mask256>& b) {
        if (a.first != b.first) return a.first < b.first;
        return canonical_less(a.second, b.second);
    });
    for (int64_t p = 0; p < P; ++p) std::memcpy(moves + (size_t)p * row_bytes, all[(size_t)p].second.w, row_bytes);
    return MPWSD_OK;
}
