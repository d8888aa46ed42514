// Stage 1 by ordered-statistics decoding of order k (Sec. III-A; the OSD
// initialisation of the RM experiment, Sec. IV-A): per frame, the L
// candidates of smallest metric become the anchors of stage 2, which then
// runs on every frame (always-on mode, Sec. III-C).
//
// One wavefront per frame (workgroup of 64 lanes):
//   1. reliability order by the key (|llr| descending, then position): int8
//      keys fit 16 bits and are sorted in registers by a bitonic network; a
//      binary32 position's rank is the number of positions with a smaller
//      key, counted against all keys in LDS; position j goes to slot rank(j);
//   2. most reliable basis: lane i holds generator row i (row A[i] of
//      F^{(x)m}, bit-packed).  Positions are visited in reliability order;
//      a ballot finds the unpivoted rows with a 1 there, the lowest such
//      lane becomes the pivot, its row is broadcast and cleared from every
//      other row holding a 1 there (Gauss-Jordan).  After K pivots row t is
//      the codeword that is 1 at the t-th basis position and 0 at the others;
//   3. candidates: for every set e of at most k basis indices (numbered by
//      |e|, then lexicographically), c(e) = c0 xor sum_{i in e} g_i, c0 the
//      codeword agreeing with the hard decisions on the basis.  The lanes
//      split the numbering into 64 contiguous ranges.  Integer metric
//      M(c) = sum_{c_j = 1} q_j from eight bit planes of q (ballots), one
//      AND + popcount per plane and word; binary32 metric ||y - x(c)||^2
//      summed in ascending position order;
//   4. every lane keeps its L best (metric, number) keys in LDS; L rounds of
//      a wave-wide minimum merge them, and lanes 0..L-1 rebuild and store the
//      winners.
//
// Integer metric, order k <= 2 and K <= 32 (the OSD(2) of RM(2,7)): step 3
// is a Gram matrix on the matrix cores instead.  With z_j = q_j (1 - 2 c0_j),
// M(c0 xor x) = M(c0) + sum_j x_j z_j for any x, so with T = G diag(z) G^T
// over the K basis rows g_a:
//     M(c0 xor g_a)         = M(c0) + T_aa,
//     M(c0 xor g_a xor g_b) = M(c0) + T_aa + T_bb - 2 T_ab,
// exact in integers.  T is a K x N x K int8 product (|z_j| <= 127, rows 0/1)
// with int32 sums: 16 x 16 tiles of v_mfma_i32_16x16x64_i8, three tiles
// (two row blocks, the upper triangle) times N / 64 position chunks for
// RM(2,7).  Every candidate then sits in one accumulator slot of one lane
// (pairs a < b above the diagonal, singles on it, c0 in one slot below
// it); L rounds of a wave minimum over 32-bit (metric, number) keys pick
// the anchors.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstring>

#include "apply.h"
#include "common.h"

namespace {

constexpr int WAVE = 64;
constexpr int MAXN = 256;
constexpr int MAXK = 64;
constexpr int MAX_ORDER = 4;

__device__ __host__ inline uint32_t binom_small(int n, int k)
{
    // C(n, k) for 0 <= k <= 4, n <= 64 (fits 32 bits)
    if (k < 0 || n < k) return 0;
    switch (k) {
    case 0: return 1;
    case 1: return (uint32_t)n;
    case 2: return (uint32_t)n * (n - 1) / 2;
    case 3: return (uint32_t)n * (n - 1) * (n - 2) / 6;
    default: return (uint32_t)n * (n - 1) * (n - 2) * (n - 3) / 24;
    }
}

// Set of j in [0, 64) with j a subset of a (bitwise): the low word of row a of F^{(x)6}.
__device__ inline uint64_t subset_mask64(uint32_t a)
{
    uint64_t mk = 1;
    for (int t = 0; t < 6; ++t)
        if ((a >> t) & 1u) mk |= mk << (1 << t);
    return mk;
}

// Value of lane `src` (wave-uniform) to every lane, through scalar registers.
__device__ inline uint64_t readlane_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// v combined with the value of a partner lane inside its row of 16 (DPP).
template <int CTRL>
__device__ inline uint64_t dpp_partner(uint64_t v)
{
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

constexpr int DPP_QUAD_1032 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;      // lane i <-> 15 - i within 16

// Minimum over the wave: inside each row of 16 lanes by DPP, then across the
// four rows through scalar reads.  Every lane returns the minimum.
__device__ inline uint64_t wave_min_u64(uint64_t v)
{
    uint64_t o;
    o = dpp_partner<DPP_QUAD_1032>(v); v = o < v ? o : v;
    o = dpp_partner<DPP_QUAD_2301>(v); v = o < v ? o : v;
    o = dpp_partner<DPP_HALF_MIRROR>(v); v = o < v ? o : v;
    o = dpp_partner<DPP_MIRROR>(v); v = o < v ? o : v;
    const uint64_t a = readlane_u64(v, 0), b = readlane_u64(v, 16), c = readlane_u64(v, 32), d = readlane_u64(v, 48);
    const uint64_t ab = a < b ? a : b, cd = c < d ? c : d;
    return ab < cd ? ab : cd;
}

// Exclusive-or over the wave, returned to every lane.
__device__ inline uint64_t wave_xor_u64(uint64_t v)
{
    v ^= dpp_partner<DPP_QUAD_1032>(v);
    v ^= dpp_partner<DPP_QUAD_2301>(v);
    v ^= dpp_partner<DPP_HALF_MIRROR>(v);
    v ^= dpp_partner<DPP_MIRROR>(v);
    return readlane_u64(v, 0) ^ readlane_u64(v, 16) ^ readlane_u64(v, 32) ^ readlane_u64(v, 48);
}

// Minimum over the wave of a 32-bit value (every lane returns it).
__device__ inline uint32_t wave_min_u32(uint32_t v)
{
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_1032, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_QUAD_2301, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_HALF_MIRROR, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, DPP_MIRROR, 0xF, 0xF, false));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(a, b), min(c, d));
}

// Sum over the wave (every lane returns it).
__device__ inline int wave_sum_i32(int v)
{
    v += __builtin_amdgcn_update_dpp(v, v, DPP_QUAD_1032, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(v, v, DPP_QUAD_2301, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(v, v, DPP_HALF_MIRROR, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(v, v, DPP_MIRROR, 0xF, 0xF, false);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
           __builtin_amdgcn_readlane(v, 48);
}

// Bytes 0 / 1 of the four bits of nibble t of x: byte i is bit 4 t + i.
__device__ inline uint32_t nibble_bytes(uint32_t x, int t) { return mpwsd::bit_bytes(x >> (4 * t)); }

// Ascending bitonic sort of the 64 E keys of a wave, E per lane (element
// lane * E + h in x[h]): partners closer than E in registers, the others by
// lane exchanges.
template <int E>
__device__ inline void wave_sort(uint32_t (&x)[E], int lane)
{
    constexpr int M = WAVE * E;
#pragma unroll
    for (int ks = 2; ks <= M; ks <<= 1) {
#pragma unroll
        for (int j = ks >> 1; j > 0; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int h = 0; h < E; ++h) {
                    if (h & j) continue;
                    const bool up = ((lane * E + h) & ks) == 0;
                    const uint32_t lo = min(x[h], x[h | j]), hi = max(x[h], x[h | j]);
                    x[h] = up ? lo : hi;
                    x[h | j] = up ? hi : lo;
                }
            } else {
#pragma unroll
                for (int h = 0; h < E; ++h) {
                    const uint32_t y = (uint32_t)__shfl_xor((int)x[h], j / E);
                    const int e = lane * E + h;
                    const bool keep_min = ((e & j) == 0) == ((e & ks) == 0);
                    x[h] = keep_min ? min(x[h], y) : max(x[h], y);
                }
            }
        }
    }
}

// Pattern e = {e_0 < e_1 < ...} of size s (s <= 4), one byte per element.
struct Pattern {
    int s;
    uint32_t e;
    __device__ int at(int t) const { return (int)((e >> (8 * t)) & 0xFFu); }
    __device__ void set(int t, int v) { e = (e & ~(0xFFu << (8 * t))) | ((uint32_t)v << (8 * t)); }
};

// Candidate number -> pattern (numbering: by size, then lexicographic).
__device__ inline Pattern unrank(uint32_t num, int K)
{
    Pattern p{0, 0};
    int s = 0;
    while (num >= binom_small(K, s)) {
        num -= binom_small(K, s);
        ++s;
    }
    p.s = s;
    // element t is the largest x whose patterns starting below it number at
    // most num: those are sum_{x' = a}^{x - 1} C(K-1-x', r) = C(K-a, r+1) -
    // C(K-x, r+1) (a = first allowed value, r = elements after t), found by
    // bisection on the decreasing C(K-x, r+1)
    int x = 0;
    for (int t = 0; t < s; ++t) {
        const int r = s - 1 - t;
        const uint32_t tot = binom_small(K - x, r + 1);
        const uint32_t tgt = tot - num;
        int lo = x, hi = K - 1 - r;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (binom_small(K - mid, r + 1) >= tgt) lo = mid;
            else hi = mid - 1;
        }
        num -= tot - binom_small(K - lo, r + 1);
        p.set(t, lo);
        x = lo + 1;
    }
    return p;
}

// The pattern numbered one higher.
__device__ inline void next_pattern(Pattern& p, int K)
{
    int t = p.s - 1;
    while (t >= 0 && p.at(t) == K - p.s + t) --t;
    if (t < 0) {
        ++p.s;
        p.e = 0;
        for (int u = 0; u < p.s; ++u) p.set(u, u);
        return;
    }
    const int v = p.at(t) + 1;
    p.set(t, v);
    for (int u = t + 1; u < p.s; ++u) p.set(u, v + (u - t));
}

template <int W>
__device__ inline void build_candidate(uint64_t (&c)[W], const uint64_t (&c0)[W], const uint64_t* rows, const Pattern& p)
{
#pragma unroll
    for (int w = 0; w < W; ++w) c[w] = c0[w];
    for (int t = 0; t < p.s; ++t) {
        const uint64_t* g = rows + (size_t)p.at(t) * W;
#pragma unroll
        for (int w = 0; w < W; ++w) c[w] ^= g[w];
    }
}

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ inline int pick4(const v4i& x, int j)
{
    return j == 0 ? x[0] : j == 1 ? x[1] : j == 2 ? x[2] : x[3];
}

// Candidate key of the Gram form: (metric - M(c0) + 2^15) << 10 | number.
// |metric - M(c0)| <= 127 N <= 32512 and numbers < 2^10 (K <= 32, order
// <= 2), so the keys order as (metric, number) and fit 26 bits.
__device__ inline uint32_t gram_key(int delta, int num) { return ((uint32_t)(delta + 32768) << 10) | (uint32_t)num; }

// Steps 3-4 of the Gram form (integer metric, order <= 2, K <= 16 GB):
// T = G diag(z) G^T on the matrix cores, one key per candidate in the
// accumulator slots, L rounds of a wave minimum, winners rebuilt by lanes
// 0 .. L-1.  Lane (li, lg) supplies row (and column) 16 X + li of block X
// at its 16 positions 64 w + 16 lg + e of chunk w: the A operand carries
// z_j g_a(j), the B operand g_b(j) (0 / 1), so both use the same position
// for a given byte and the sums do not depend on how the matrix core maps
// bytes to the reduction index.  Slot j of the (R, C) tile holds
// T[16 R + 4 lg + j][16 C + li].
template <int W, int GB>
__device__ __forceinline__ void gram_anchors(int lane, int64_t f, int N, int K, int order, int L,
                                             const int8_t* qs, const int8_t* nqs, const uint64_t* rows,
                                             const uint64_t (&c0)[W], int32_t* dT, uint64_t* win,
                                             uint8_t* __restrict__ anchors, int32_t* __restrict__ metric_out)
{
    const int li = lane & 15, lg = lane >> 4;
    const uint32_t* q4 = reinterpret_cast<const uint32_t*>(qs);
    const uint32_t* nq4 = reinterpret_cast<const uint32_t*>(nqs);
    v4i za[GB][W], gb[GB][W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        // z = q where c0 is 0, -q where it is 1 (byte select: v_perm picks
        // byte i of q, or byte i of -q when c0's byte is 1)
        const uint32_t cb = (uint32_t)(c0[w] >> (16 * lg)) & 0xFFFFu;
        uint32_t zw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t ct = nibble_bytes(cb, t);
            const int qi = 16 * w + 4 * lg + t;
            zw[t] = __builtin_amdgcn_perm(nq4[qi], q4[qi], 0x03020100u + (ct << 2));
        }
#pragma unroll
        for (int X = 0; X < GB; ++X) {
            const int a = 16 * X + li;
            const uint64_t rw = a < K ? rows[a * W + w] : 0ull;
            const uint32_t bits = (uint32_t)(rw >> (16 * lg)) & 0xFFFFu;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t e = nibble_bytes(bits, t);
                gb[X][w][t] = (int)e;
                za[X][w][t] = (int)(zw[t] & ((e << 8) - e));  // bytes 0xFF where e is 1
            }
        }
    }
    // tiles (0, 0), (0, 1), (1, 1)
    constexpr int NT = GB == 2 ? 3 : 1;
    v4i tt[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) tt[i] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int w = 0; w < W; ++w) {
        tt[0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(za[0][w], gb[0][w], tt[0], 0, 0, 0);
        if constexpr (GB == 2) {
            tt[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(za[0][w], gb[1][w], tt[1], 0, 0, 0);
            tt[2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(za[1][w], gb[1][w], tt[2], 0, 0, 0);
        }
    }
    // the diagonal, for every lane
    {
        const int j = li - 4 * lg;
        if (j >= 0 && j < 4) {
            dT[li] = pick4(tt[0], j);
            if constexpr (GB == 2) dT[16 + li] = pick4(tt[NT - 1], j);
        }
    }
    int M0 = 0;  // M(c0), for the metrics returned
    if (metric_out) {
        int part = 0;
#pragma unroll
        for (int h = 0; h < W; ++h)
            if (64 * h + lane < N && ((c0[h] >> lane) & 1ull)) part += qs[64 * h + lane];
        M0 = wave_sum_i32(part);
    }
    __syncthreads();
    uint32_t key[NT][4];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int R = i == 2 ? 1 : 0, C = i == 0 ? 0 : 1;
        const v4i da = *reinterpret_cast<const v4i*>(dT + 16 * R + 4 * lg);
        const int b = 16 * C + li, db = dT[b];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = 16 * R + 4 * lg + j;
            const int tv = tt[i][j];
            uint32_t k = 0xFFFFFFFFu;
            if (a == b) {
                if (order >= 1 && a < K) k = gram_key(tv, 1 + a);                    // {a}
            } else if (a < b) {
                if (order >= 2 && b < K)                                              // {a, b}
                    k = gram_key(da[j] + db - 2 * tv, 1 + K + a * (2 * K - a - 1) / 2 + b - a - 1);
            } else if (i == 0 && a == 1 && b == 0) {
                k = gram_key(0, 0);                                                   // c0
            }
            key[i][j] = k;
        }
    }
    // L rounds: the smallest key above the last winner (keys are distinct;
    // subtracting last + 1 sends the taken ones and the empty slots past 2^31)
    uint32_t last = 0xFFFFFFFFu;
    for (int t = 0; t < L; ++t) {
        const uint32_t off = last + 1u;
        uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) mn = min(mn, key[i][j] - off);
        last = wave_min_u32(mn) + off;
        if (lane == 0) win[t] = last;
    }
    __syncthreads();
    if (lane < L) {
        const uint32_t k = (uint32_t)win[lane];
        const Pattern p = unrank(k & 0x3FFu, K);
        uint64_t c[W];
        build_candidate<W>(c, c0, rows, p);
        uint8_t* dst = anchors + ((size_t)f * L + lane) * (N / 8);
        for (int b = 0; b < N / 8; ++b) dst[b] = (uint8_t)(c[b >> 3] >> (8 * (b & 7)));
        if (metric_out) metric_out[f * L + lane] = M0 + ((int)(k >> 10) - 32768);
    }
}

// W: 64-bit words per codeword (N = 32 uses the low half of one word).
// GB: 0 = enumerate the candidates; 1 or 2 = integer metric of order <= 2
// from the Gram matrix over GB blocks of 16 basis rows (K <= 16 GB).
template <int W, bool FLOAT, int GB>
__global__ __launch_bounds__(WAVE) void osd_kernel(const void* __restrict__ llr, int64_t F, int m, int r, int K,
                                                   int order, int L, uint8_t* __restrict__ anchors,
                                                   int32_t* __restrict__ metric_out)
{
    static_assert(GB == 0 || !FLOAT, "the Gram form is exact in integers only");
    const int N = 1 << m;
    const int NB = N / 8;
    const int lane = threadIdx.x;
    const int64_t f = blockIdx.x;
    if (f >= F) return;  // whole workgroup: no barrier is skipped by part of it

    __shared__ float ys[FLOAT ? MAXN : 1];
    __shared__ __attribute__((aligned(16))) int8_t qs[MAXN];
    __shared__ __attribute__((aligned(16))) int8_t nqs[GB ? MAXN : 1];  // -q (Gram form)
    __shared__ __attribute__((aligned(16))) int32_t dT[GB ? 32 : 1];    // diagonal of T (Gram form)
    __shared__ uint64_t keys[FLOAT ? MAXN : 1];  // reliability keys (binary32 form)
    __shared__ uint16_t sorted[MAXN];
    __shared__ uint16_t info[MAXK];
    __shared__ uint16_t mrb[MAXK];
    __shared__ uint8_t pivlane[MAXK];  // lane holding the row of pivot t
    __shared__ uint64_t rows[MAXK * W];
    __shared__ uint64_t c0s[W];
    __shared__ uint64_t win[32];
    extern __shared__ uint64_t lists[];  // [L][64]

    // ---- 1. channel values and reliability keys
    for (int j = lane; j < N; j += WAVE) {
        uint32_t mag;
        if (FLOAT) {
            const float v = ((const float*)llr)[f * N + j];
            ys[j] = v;
            qs[j] = v < 0.0f ? -1 : 0;  // hard decision only
            mag = __float_as_uint(fabsf(v));
        } else {
            const int v = mpwsd::read_q1(((const int8_t*)llr)[f * N + j]);
            qs[j] = (int8_t)v;
            if (GB) nqs[j] = (int8_t)-v;
            mag = (uint32_t)(v < 0 ? -(int)v : (int)v);
        }
        if (FLOAT) keys[j] = ((uint64_t)(0xFFFFFFFFu - mag) << 32) | (uint32_t)j;
    }
    if (FLOAT) {
        __syncthreads();
        for (int j = lane; j < N; j += WAVE) {
            const uint64_t kj = keys[j];
            int rank = 0;
            for (int i = 0; i < N; ++i) rank += keys[i] < kj;
            sorted[rank] = (uint16_t)j;
        }
    } else {
        // 16-bit keys (255 - |q|, position), unique: sorted in registers
        // (positions past N take the largest key and sort last)
        uint32_t x[W];
#pragma unroll
        for (int h = 0; h < W; ++h) {
            const int e = lane * W + h;
            uint32_t key = 0xFFFFu;
            if (e < N) {
                const int v = mpwsd::read_q1(((const int8_t*)llr)[f * N + e]);
                key = ((255u - (uint32_t)(v < 0 ? -v : v)) << 8) | (uint32_t)e;
            }
            x[h] = key;
        }
        wave_sort<W>(x, lane);
#pragma unroll
        for (int h = 0; h < W; ++h)
            if (lane * W + h < N) sorted[lane * W + h] = (uint16_t)(x[h] & 0xFFu);
    }
    // information set A = {i : popcount(i) >= m - r}, ascending (compaction by ballot)
    {
        int base = 0;
        for (int h = 0; h * WAVE < N; ++h) {
            const int j = h * WAVE + lane;
            const bool fl = j < N && __popc((unsigned)j) >= m - r;
            const uint64_t bal = __ballot(fl);
            if (fl) info[base + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)j;
            base += __popcll(bal);
        }
    }
    __syncthreads();

    // ---- 2. most reliable basis by Gauss-Jordan elimination, one row per lane
    uint64_t row[W];
    {
        const uint32_t a = lane < K ? info[lane] : 0;
        const uint64_t low = subset_mask64(a & 63u);
#pragma unroll
        for (int w = 0; w < W; ++w)
            row[w] = (lane < K && (((uint32_t)w & ~(a >> 6)) == 0)) ? low : 0;
    }
    // the reliability order in registers (rank 64 h + t in lane t of srt[h]),
    // read with v_readlane; the pivot rows as a scalar lane mask
    uint32_t srt[W];
#pragma unroll
    for (int h = 0; h < W; ++h) srt[h] = 64 * h + lane < N ? sorted[64 * h + lane] : 0u;
    uint64_t piv = 0;
    int count = 0;
#pragma unroll
    for (int h = 0; h < W; ++h) {
        const int nh = N - 64 * h < 64 ? N - 64 * h : 64;
        for (int t = 0; t < nh && count < K; ++t) {
            const int j = __builtin_amdgcn_readlane((int)srt[h], t);
            const int ws = j >> 6, bs = j & 63;
            uint64_t rw = row[0];
#pragma unroll
            for (int w = 1; w < W; ++w)
                if (ws == w) rw = row[w];
            const bool bit = (rw >> bs) & 1ull;
            const uint64_t cand = __ballot(bit) & ~piv;
            if (cand == 0) continue;  // column j depends on the basis so far
            const int p = __builtin_ctzll(cand);
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t pr = readlane_u64(row[w], p);
                if (bit && lane != p) row[w] ^= pr;
            }
            piv |= 1ull << p;
            if (lane == 0) {
                mrb[count] = (uint16_t)j;
                pivlane[count] = (uint8_t)p;
            }
            ++count;
        }
    }
    __syncthreads();
    // pivot t's row (held by lane pivlane[t]) to rows[t]
    {
        const int src = lane < K ? (int)pivlane[lane] : lane;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(row[w] >> 32), src) << 32) |
                               (uint32_t)__shfl((int)(uint32_t)row[w], src);
            if (lane < K) rows[lane * W + w] = v;
        }
    }
    __syncthreads();

    // c0: the codeword with the hard decisions on the basis
    {
        bool hd = false;
        if (lane < K) hd = qs[mrb[lane]] < 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = wave_xor_u64((lane < K && hd) ? rows[lane * W + w] : 0);
            if (lane == 0) c0s[w] = v;
        }
    }
    __syncthreads();
    uint64_t c0[W];
#pragma unroll
    for (int w = 0; w < W; ++w) c0[w] = c0s[w];

    if constexpr (GB > 0) {
        gram_anchors<W, GB>(lane, f, N, K, order, L, qs, nqs, rows, c0, dT, win, anchors, metric_out);
        return;
    }

    // bit planes of q (integer metric)
    uint64_t plane[FLOAT ? 1 : W][8];
    if (!FLOAT) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int j = w * WAVE + lane;
            const uint32_t qb = j < N ? (uint32_t)(uint8_t)qs[j] : 0u;
#pragma unroll
            for (int b = 0; b < 8; ++b) plane[w][b] = __ballot((qb >> b) & 1u);
        }
    }

    // ---- 3. candidates of this lane's range, best L kept in LDS
    uint32_t C = 0;
    for (int s = 0; s <= order; ++s) C += binom_small(K, s);
    const uint32_t lo = (uint32_t)((uint64_t)C * lane / WAVE), hi = (uint32_t)((uint64_t)C * (lane + 1) / WAVE);
    int cnt = 0;
    uint64_t thr = ~0ull;
    if (lo < hi) {
        Pattern p = unrank(lo, K);
        for (uint32_t num = lo; num < hi; ++num) {
            uint64_t c[W];
            build_candidate<W>(c, c0, rows, p);
            uint32_t mk;
            if (FLOAT) {
                float e = 0.0f;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint64_t cw = c[w];
                    const int nb = N - 64 * w < 64 ? N - 64 * w : 64;
                    for (int b = 0; b < nb; ++b) {
                        const float x = ((cw >> b) & 1ull) ? -1.0f : 1.0f;
                        const float d = __fsub_rn(ys[64 * w + b], x);
                        e = __fadd_rn(e, __fmul_rn(d, d));
                    }
                }
                mk = __float_as_uint(e);  // e >= 0: bits are monotone
            } else {
                int M = 0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    int pc = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) pc += __popcll(c[w] & plane[FLOAT ? 0 : w][b]);
                    M += (b == 7 ? -128 : (1 << b)) * pc;
                }
                mk = (uint32_t)M ^ 0x80000000u;  // order-preserving for int32
            }
            const uint64_t key = ((uint64_t)mk << 32) | num;
            if (key < thr) {
                int pos = cnt < L ? cnt : L - 1;
                while (pos > 0 && lists[(pos - 1) * WAVE + lane] > key) {
                    lists[pos * WAVE + lane] = lists[(pos - 1) * WAVE + lane];
                    --pos;
                }
                lists[pos * WAVE + lane] = key;
                if (cnt < L) ++cnt;
                if (cnt == L) thr = lists[(L - 1) * WAVE + lane];
            }
            if (num + 1 < hi) next_pattern(p, K);
        }
    }

    // ---- 4. L rounds of a wave minimum over the lanes' list heads
    int head = 0;
    for (int t = 0; t < L; ++t) {
        const uint64_t mine = head < cnt ? lists[head * WAVE + lane] : ~0ull;
        const uint64_t best = wave_min_u64(mine);
        if (mine == best && best != ~0ull) ++head;
        if (lane == 0) win[t] = best;
    }
    __syncthreads();
    if (lane < L) {
        const uint64_t key = win[lane];
        const Pattern p = unrank((uint32_t)key, K);
        uint64_t c[W];
        build_candidate<W>(c, c0, rows, p);
        uint8_t* dst = anchors + ((size_t)f * L + lane) * NB;
        for (int b = 0; b < NB; ++b) dst[b] = (uint8_t)(c[b >> 3] >> (8 * (b & 7)));
        if (metric_out) {
            const uint32_t mk = (uint32_t)(key >> 32);
            metric_out[f * L + lane] = FLOAT ? (int32_t)mk : (int32_t)(mk ^ 0x80000000u);
        }
    }
}

template <int W>
void launch_w(bool fl, const void* llr, int64_t F, int m, int r, int K, int order, int L, uint8_t* anchors,
              int32_t* metric, hipStream_t s)
{
    const size_t lds = (size_t)L * WAVE * sizeof(uint64_t);
    const dim3 grid((unsigned)F);
    if (fl)
        hipLaunchKernelGGL((osd_kernel<W, true, 0>), grid, dim3(WAVE), lds, s, llr, F, m, r, K, order, L, anchors,
                           metric);
    else if (order <= 2 && K <= 16)
        hipLaunchKernelGGL((osd_kernel<W, false, 1>), grid, dim3(WAVE), 0, s, llr, F, m, r, K, order, L, anchors,
                           metric);
    else if (order <= 2 && K <= 32)
        hipLaunchKernelGGL((osd_kernel<W, false, 2>), grid, dim3(WAVE), 0, s, llr, F, m, r, K, order, L, anchors,
                           metric);
    else
        hipLaunchKernelGGL((osd_kernel<W, false, 0>), grid, dim3(WAVE), lds, s, llr, F, m, r, K, order, L, anchors,
                           metric);
}

}  // namespace

extern "C" int mpwsd_stage1_osd(int r, int m, int order, int L, const void* llr, int dtype, int64_t F,
                                uint8_t* anchors, int32_t* metric, hipStream_t stream)
{
    using mpwsd::fail;
    mpwsd::clear_error();
    if (m < 5 || m > 8 || r < 1 || r >= m)
        return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_stage1_osd: need 1 <= r < m, 5 <= m <= 8 (r=%d m=%d)", r, m);
    const int K = mpwsd::rm_dimension(r, m);
    if (K > MAXK) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_stage1_osd: K=%d exceeds %d", K, MAXK);
    if (order < 0 || order > MAX_ORDER)
        return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_stage1_osd: order must be in [0, %d] (got %d)", MAX_ORDER, order);
    if (L < 1 || L > 32) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_stage1_osd: need 1 <= L <= 32 (L=%d)", L);
    uint32_t C = 0;
    for (int s = 0; s <= order; ++s) C += binom_small(K, s);
    if ((uint32_t)L > C)
        return fail(MPWSD_ERR_ARG, "mpwsd_stage1_osd: L=%d exceeds the %u candidates of order %d", L, C, order);
    if (dtype != MPWSD_I8 && dtype != MPWSD_F32) return fail(MPWSD_ERR_ARG, "mpwsd_stage1_osd: bad dtype %d", dtype);
    if (F < 0 || F > INT_MAX) return fail(MPWSD_ERR_ARG, "mpwsd_stage1_osd: F=%lld out of range", (long long)F);
    if (F == 0) return MPWSD_OK;
    if (!llr || !anchors) return fail(MPWSD_ERR_ARG, "mpwsd_stage1_osd: null pointer");
    const bool fl = dtype == MPWSD_F32;
    switch (m) {
    case 5:
    case 6: launch_w<1>(fl, llr, F, m, r, K, order, L, anchors, metric, stream); break;
    case 7: launch_w<2>(fl, llr, F, m, r, K, order, L, anchors, metric, stream); break;
    default: launch_w<4>(fl, llr, F, m, r, K, order, L, anchors, metric, stream); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MPWSD_ERR_DEVICE, "mpwsd_stage1_osd: %s", hipGetErrorString(e));
    return MPWSD_OK;
}
