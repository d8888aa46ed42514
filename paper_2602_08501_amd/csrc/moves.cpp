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
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
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
