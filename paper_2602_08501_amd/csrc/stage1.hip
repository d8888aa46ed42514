// Stage 1 (Sec. III-A): LLR quantizer and min-sum successive-cancellation
// list decoding with a CRC on the most reliable candidate.
//
// Mapping on CDNA4: one lane per list path and L consecutive lanes per frame,
// so a 64-wide wavefront decodes 64/L frames in lock step; all lanes of a
// wave visit the same leaf at the same time, which keeps control flow
// uniform.  Each path owns one LLR buffer per tree level in LDS (level l has
// 2^l values, stored element-major so that the 64 lanes of a wave hit 64
// consecutive slots).  A path reads its parent level through a per-level
// owner index instead of copying buffers when paths are cloned: at a given
// leaf every path rewrites the same levels, each into its own buffer, so a
// buffer another path still refers to is never overwritten while needed.
// Cloning therefore copies only the owner indices, the decided bits and the
// metric.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "apply.h"
#include "common.h"

namespace {

constexpr int WAVE = 64;

template <bool FLOAT> struct Arith;
template <> struct Arith<false> {
    using V = int32_t;        // LLR arithmetic
    using S = int16_t;        // LDS storage: |l| <= 127 * 2^(m - level) <= 32512 (q read in [-127, 127])
    __device__ static V load_ch(const void* p, int64_t i) { return (V)mpwsd::read_q1(((const int8_t*)p)[i]); }
    __device__ static uint32_t key_bits(V pm) { return (uint32_t)pm; }
};
template <> struct Arith<true> {
    using V = float;
    using S = float;
    __device__ static V load_ch(const void* p, int64_t i) { return ((const float*)p)[i]; }
    __device__ static uint32_t key_bits(V pm) { return __float_as_uint(pm); }
};

template <typename V> __device__ inline V f_minsum(V a, V b)
{
    V ma = a < 0 ? -a : a, mb = b < 0 ? -b : b;
    V m = ma < mb ? ma : mb;
    return ((a < 0) != (b < 0)) ? -m : m;
}

// Packed int16 helpers (two 16-bit lanes per 32-bit register; integer ops,
// no floating point involved).
typedef short short2_t __attribute__((ext_vector_type(2)));
__device__ inline short2_t as_s2(uint32_t x) { return __builtin_bit_cast(short2_t, x); }
__device__ inline uint32_t as_u(short2_t x) { return __builtin_bit_cast(uint32_t, x); }
__device__ inline uint32_t pk_add_u16(uint32_t a, uint32_t b) { return as_u(as_s2(a) + as_s2(b)); }
__device__ inline uint32_t pk_sub_u16(uint32_t a, uint32_t b) { return as_u(as_s2(a) - as_s2(b)); }
__device__ inline uint32_t pk_ashr15(uint32_t a) { return as_u(as_s2(a) >> (short2_t){15, 15}); }
__device__ inline uint32_t pk_min_i16(uint32_t a, uint32_t b)
{
    const short2_t x = as_s2(a), y = as_s2(b);
    return as_u(x < y ? x : y);
}
__device__ inline uint32_t pk_max_i16(uint32_t a, uint32_t b)
{
    const short2_t x = as_s2(a), y = as_s2(b);
    return as_u(x > y ? x : y);
}
__device__ inline uint32_t pk_abs_i16(uint32_t a) { return pk_max_i16(a, pk_sub_u16(0u, a)); }
// min-sum f on both halves: sgn(a) sgn(b) min(|a|, |b|), which for integers
// equals max(min(a, b), -max(a, b)) (same signs: the smaller magnitude with
// their sign; opposite signs: minus the smaller magnitude; 0 when a or b is 0)
__device__ inline uint32_t f_pk(uint32_t a, uint32_t b)
{
    return pk_max_i16(pk_min_i16(a, b), pk_sub_u16(0u, pk_max_i16(a, b)));
}
// g on both halves: b + (1 - 2 v) a, v = bit sh of w (low half) and bit
// sh + 1 (high half), sh even.  Each bit is sign-extended to 0 or all ones and
// ored with 1, giving the packed factors +1 / -1 of one multiply-add.
__device__ inline uint32_t g_pk(uint32_t a, uint32_t b, uint32_t w, int sh)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_sbfe((int)w, sh, 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_sbfe((int)w, sh + 1, 1);
    const uint32_t sg = (lo & 0x0000FFFFu) | (hi & 0xFFFF0000u) | 0x00010001u;
    return as_u(as_s2(a) * as_s2(sg) + as_s2(b));
}

// Polar transform x -> x F^{(x)lev} of the n = 2^lev bits held in w[]
// (bit k of position k, 32 per word): within-word butterflies for the first
// five factors, whole-word xors for the rest.
template <int NW> __device__ inline void polar_bits(uint32_t (&w)[NW], int lev)
{
    const uint32_t MK[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu, 0x0000FFFFu};
    const int sw = lev < 5 ? lev : 5;
    for (int s = 0; s < sw; ++s)
#pragma unroll
        for (int i = 0; i < NW; ++i) w[i] ^= (w[i] >> (1 << s)) & MK[s];
    for (int s = 5; s < lev; ++s) {
        const int h = 1 << (s - 5);
#pragma unroll
        for (int i = 0; i < NW; ++i)
            if ((i & h) == 0 && i + h < NW) w[i] ^= w[i + h];
    }
}

// Schedule of the successive-cancellation tree: entry i (a leaf index) is 0
// for an ordinary leaf, or (kind << 4 | level) when a special subtree of
// 2^level leaves starts at leaf i: kind 1 = all frozen (rate 0), kind 2 = all
// frozen but the last leaf (repetition).  With min-sum updates the path
// metric a subtree adds for a decided sub-codeword equals that codeword's
// discrepancy against the subtree's LLRs, so such a subtree is settled from
// its LLRs alone: rate 0 adds D0 = sum_{l<0} |l|, a repetition node offers
// the children PM + D0 (bit 0) and PM + D1, D1 = sum_{l>0} l.  In integer
// arithmetic this is exactly the leaf-by-leaf result; the float form keeps
// the leaf-by-leaf order of additions (all entries 0).
struct Sched {
    uint8_t v[256];
};
// The CRC test as a linear map: with the register starting at 0, its final
// value is the xor of one fixed word per set information bit.  Row b holds,
// over the N decided bits (32 per word), the positions whose word has bit b
// set, so register bit b is the parity of (u & row b).
struct CrcRows {
    uint32_t w[16][8];
};
constexpr int KIND_R0 = 1, KIND_REP = 2;

// Value of lane `lane ^ X` (X < 32): DPP quad permutes for X = 1, 2, else a
// bit-mask swizzle (no memory access).
template <int X>
__device__ inline uint32_t xor_lane(uint32_t v)
{
    // (every lane reads a lane of its own 16-lane row, so no old value is kept)
    if constexpr (X == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (X == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (X == 4) {
        // lanes with bit 2 clear read 4 lanes up (row_shl:4), the others 4 down (row_shr:4)
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x104, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x114, 0xF, 0xF, false);
        return (threadIdx.x & 4) ? dn : up;
    } else if constexpr (X == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else {
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (X << 10));
    }
}
template <int X> __device__ inline uint32_t xor_key(uint32_t v) { return xor_lane<X>(v); }
template <int X> __device__ inline uint64_t xor_key(uint64_t v)
{
    return ((uint64_t)xor_lane<X>((uint32_t)(v >> 32)) << 32) | xor_lane<X>((uint32_t)v);
}
__device__ inline uint32_t shfl_key(uint32_t v, int src) { return (uint32_t)__shfl((int)v, src); }
__device__ inline uint64_t shfl_u64(uint64_t v, int src)
{
    return ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(v >> 32), src) << 32) | (uint32_t)__shfl((int)(uint32_t)v, src);
}
__device__ inline uint64_t shfl_key(uint64_t v, int src) { return shfl_u64(v, src); }

template <int M, int L, bool FLOAT> struct Scl {
    using A = Arith<FLOAT>;
    using V = typename A::V;
    using S = typename A::S;
    static constexpr int N = 1 << M;
    static constexpr int NW = N / 32;    // words of decided bits per path
    static constexpr int TW = (N / 2 + 31) / 32;  // words of the first-half bits
    static constexpr int G = WAVE / L;   // frames per wave
    static constexpr int CHS = N;  // channel row stride
    using Key = typename std::conditional<FLOAT, uint64_t, uint32_t>::type;

    struct Smem {
        // level l of lane x.  Float: rows [2^l - 1, 2^(l+1) - 1), one value
        // per row, row-major [row][lane].  Integer: rows [2^l, 2^(l+1)), two
        // consecutive rows per 32-bit word ([row / 2][lane], low half first),
        // so levels >= 1 are processed as int16 pairs; the top level M - 1 is
        // not stored but recomputed from the channel where level M - 2 needs it.
        S buf[(FLOAT ? N : N / 2) * WAVE];
        S ch[G * CHS];          // channel LLRs of the wave's frames
    };

    // Recompute level LEV of this lane's path from level LEV + 1 (the
    // channel when LEV = M - 1): f for a left child, g for a right child with
    // the left sibling's bits re-encoded.  When sums is set, also returns
    // D0 = sum of |l| over negative outputs and D1 = sum of positive outputs.
    template <int LEV>
    __device__ static V level(Smem& sm, int lane, int gbase, int i, bool use_g, bool sums, uint64_t ptrs,
                              const uint32_t (&ub)[NW], V& d0, V& d1)
    {
        constexpr int n = 1 << LEV;
        constexpr int PW = (n + 31) / 32;
        uint32_t ps[PW];
        if (use_g) {
            const int st = i - n;
            if (n < 32) {
                ps[0] = (ub[st >> 5] >> (st & 31)) & ((1u << (n & 31)) - 1u);
            } else {
#pragma unroll
                for (int w = 0; w < PW; ++w) ps[w] = ub[(st >> 5) + w];
            }
            polar_bits(ps, LEV);
        }
        const S* par;
        int stride;
        if (LEV + 1 == M) {
            par = sm.ch + (lane / L) * CHS;
            stride = 1;
        } else {
            const int owner = gbase + (int)((ptrs >> (8 * (LEV + 1))) & 0xFF);
            par = sm.buf + (2 * n - 1) * WAVE + owner;
            stride = WAVE;
        }
        S* out = sm.buf + (n - 1) * WAVE + lane;
        V o = 0, s0 = 0, s1 = 0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            const V a = (V)par[k * stride];
            const V b = (V)par[(k + n) * stride];
            if (use_g) o = ((ps[k >> 5] >> (k & 31)) & 1u) ? (V)(b - a) : (V)(b + a);
            else o = f_minsum(a, b);
            out[k * WAVE] = (S)o;
            if (!FLOAT && sums) {
                s0 += o < 0 ? (V)-o : (V)0;
                s1 += o > 0 ? o : (V)0;
            }
        }
        d0 = s0;
        d1 = s1;
        return o;
    }

    // Integer form of level(): values two at a time as int16 pairs (v_pk_*
    // integer ops), exact because every value and partial sum stays within
    // +-127 * 2^m <= 32512.  Same results as level() value for value.
    template <int LEV>
    __device__ static V level_pk(Smem& sm, int lane, int gbase, int i, bool use_g, bool sums, uint64_t ptrs,
                                 const uint32_t (&ub)[NW], V& d0, V& d1)
    {
        constexpr int n = 1 << LEV;
        constexpr int PW = (n + 31) / 32;
        uint32_t ps[PW];
        if (use_g) {
            const int st = i - n;
            if (n < 32) {
                ps[0] = (ub[st >> 5] >> (st & 31)) & ((1u << (n & 31)) - 1u);
            } else {
#pragma unroll
                for (int w = 0; w < PW; ++w) ps[w] = ub[(st >> 5) + w];
            }
            polar_bits(ps, LEV);
        }
        uint32_t* bw = reinterpret_cast<uint32_t*>(sm.buf);
        const uint32_t* cw = reinterpret_cast<const uint32_t*>(sm.ch + (lane / L) * CHS);
        if constexpr (LEV + 1 == M) {
            // The top level is recomputed where needed (top_pair), never
            // stored; only a repetition / rate-0 node spanning it needs its sums.
            d0 = d1 = 0;
            if (sums) {
                uint32_t s0 = 0, s1 = 0;
                for (int k = 0; k < n; k += 2) {
                    const uint32_t o = use_g ? g_pk(cw[k / 2], cw[(k + n) / 2], ps[k >> 5], k & 31)
                                             : f_pk(cw[k / 2], cw[(k + n) / 2]);
                    s0 = pk_add_u16(s0, pk_max_i16(pk_sub_u16(0u, o), 0u));
                    s1 = pk_add_u16(s1, pk_max_i16(o, 0u));
                }
                d0 = (V)((s0 & 0xFFFFu) + (s0 >> 16));
                d1 = (V)((s1 & 0xFFFFu) + (s1 >> 16));
            }
            return 0;
        } else if constexpr (LEV == 0) {
            // parent rows 2, 3 in word 1; output row 1 (high half of word 0)
            int32_t a, b;
            if (LEV + 2 == M) {
                const uint32_t w = top_pair(cw, 0, i, ub);
                a = (int16_t)(w & 0xFFFFu);
                b = (int16_t)(w >> 16);
            } else {
                const int owner = gbase + (int)((ptrs >> 8) & 0xFF);
                const uint32_t w = bw[1 * WAVE + owner];
                a = (int16_t)(w & 0xFFFFu);
                b = (int16_t)(w >> 16);
            }
            const int32_t o = use_g ? ((ps[0] & 1u) ? b - a : b + a) : f_minsum(a, b);
            reinterpret_cast<int16_t*>(bw + lane)[1] = (int16_t)o;
            d0 = o < 0 ? -o : 0;
            d1 = o > 0 ? o : 0;
            return o;
        } else {
            const int owner = gbase + (int)((ptrs >> (8 * (LEV + 1))) & 0xFF);
            const uint32_t* pa = bw + n * WAVE + owner;  // parent rows 2n .. 4n-1: words n .. 2n-1
            uint32_t* out = bw + (n / 2) * WAVE + lane;  // rows n .. 2n-1: words n/2 .. n-1
            uint32_t vt[TW];
            if (LEV + 2 == M) top_bits(vt, i, ub);
            const bool topg = LEV + 2 == M && i >= N / 2;
            // the uniform choices are taken once, outside the value loop
            uint32_t r;
            if (use_g) {
                if (topg) r = pairs<LEV, true, true>(pa, cw, vt, ps, out, sums, d0, d1);
                else r = pairs<LEV, true, false>(pa, cw, vt, ps, out, sums, d0, d1);
            } else {
                if (topg) r = pairs<LEV, false, true>(pa, cw, vt, ps, out, sums, d0, d1);
                else r = pairs<LEV, false, false>(pa, cw, vt, ps, out, sums, d0, d1);
            }
            return (V)(int16_t)(r >> 16);  // the last value (row 2n - 1)
        }
    }

    // Values of level LEV two at a time.  USEG: g (else f); TOPG: the parent
    // is the top level in its g form (recomputed from the channel).  The
    // parent rows, the output rows and the channel never overlap (distinct
    // levels), which lets the parent reads be issued ahead of the stores.
    template <int LEV, bool USEG, bool TOPG, int PW>
    __device__ static uint32_t pairs(const uint32_t* __restrict__ pa, const uint32_t* __restrict__ cw,
                                     const uint32_t (&vt)[TW], const uint32_t (&ps)[PW], uint32_t* __restrict__ out,
                                     bool sums, V& d0, V& d1)
    {
        constexpr int n = 1 << LEV;
        uint32_t s0 = 0, s1 = 0, o = 0;
        if (sums) {
#pragma unroll 8
            for (int k = 0; k < n; k += 2) {
                o = pair_value<LEV, USEG, TOPG>(pa, cw, vt, ps, k);
                out[(k / 2) * WAVE] = o;
                s0 = pk_add_u16(s0, pk_max_i16(pk_sub_u16(0u, o), 0u));
                s1 = pk_add_u16(s1, pk_max_i16(o, 0u));
            }
        } else {
#pragma unroll 8
            for (int k = 0; k < n; k += 2) {
                o = pair_value<LEV, USEG, TOPG>(pa, cw, vt, ps, k);
                out[(k / 2) * WAVE] = o;
            }
        }
        d0 = (V)((s0 & 0xFFFFu) + (s0 >> 16));
        d1 = (V)((s1 & 0xFFFFu) + (s1 >> 16));
        return o;
    }

    template <int LEV, bool USEG, bool TOPG, int PW>
    __device__ static uint32_t pair_value(const uint32_t* pa, const uint32_t* cw, const uint32_t (&vt)[TW],
                                          const uint32_t (&ps)[PW], int k)
    {
        constexpr int n = 1 << LEV;
        uint32_t a, b;
        if constexpr (LEV + 2 == M) {
            a = top_pair_t<TOPG>(cw, k, vt);
            b = top_pair_t<TOPG>(cw, k + n, vt);
        } else {
            a = pa[(k / 2) * WAVE];
            b = pa[((k + n) / 2) * WAVE];
        }
        if constexpr (USEG) return g_pk(a, b, ps[k >> 5], k & 31);
        else return f_pk(a, b);
    }

    template <bool TOPG>
    __device__ static uint32_t top_pair_t(const uint32_t* cw, int k, const uint32_t (&vt)[TW])
    {
        const uint32_t a = cw[k / 2], b = cw[(k + N / 2) / 2];
        if constexpr (TOPG) return g_pk(a, b, vt[k >> 5], k & 31);
        else return f_pk(a, b);
    }

    // The top level (M - 1) of the current path for leaf range [i, ...):
    // f of the channel halves while i < N/2, else g with the re-encoded
    // first-half decisions u[0, N/2) (shared by every path descending from
    // the one that computed it, so this path's own bits give the same values).
    __device__ static void top_bits(uint32_t (&vt)[TW], int i, const uint32_t (&ub)[NW])
    {
        if (i < N / 2) return;
        if (N / 2 < 32) {
            vt[0] = ub[0] & ((1u << ((N / 2) & 31)) - 1u);
        } else {
#pragma unroll
            for (int w = 0; w < TW; ++w) vt[w] = ub[w];
        }
        polar_bits(vt, M - 1);
    }
    __device__ static uint32_t top_pair_v(const uint32_t* cw, int k, int i, const uint32_t (&vt)[TW])
    {
        const uint32_t a = cw[k / 2], b = cw[(k + N / 2) / 2];
        return i < N / 2 ? f_pk(a, b) : g_pk(a, b, vt[k >> 5], k & 31);
    }
    __device__ static uint32_t top_pair(const uint32_t* cw, int k, int i, const uint32_t (&ub)[NW])
    {
        uint32_t vt[TW];
        top_bits(vt, i, ub);
        return top_pair_v(cw, k, i, vt);
    }

    // Levels D, D-1, ..., stop for the node starting at leaf i: level D is a
    // right child (g) unless i = 0; the levels below are left children (f).
    template <int D>
    __device__ static V run(Smem& sm, int lane, int gbase, int i, int stop, int slot, uint64_t& ptrs,
                            const uint32_t (&ub)[NW], bool first, V& d0, V& d1)
    {
        V lam;
        if constexpr (FLOAT)
            lam = level<D>(sm, lane, gbase, i, first && i > 0, D == stop, ptrs, ub, d0, d1);
        else
            lam = level_pk<D>(sm, lane, gbase, i, first && i > 0, D == stop, ptrs, ub, d0, d1);
        ptrs = (ptrs & ~(0xFFull << (8 * D))) | ((uint64_t)slot << (8 * D));
        __builtin_amdgcn_wave_barrier();
        if constexpr (D > 0) {
            if (D > stop) lam = run<D - 1>(sm, lane, gbase, i, stop, slot, ptrs, ub, false, d0, d1);
        }
        return lam;
    }

    __device__ static V node(Smem& sm, int lane, int gbase, int i, int stop, int slot, uint64_t& ptrs,
                             const uint32_t (&ub)[NW], V& d0, V& d1)
    {
        const int d = (i == 0) ? M - 1 : __builtin_ctz(i);
        switch (d) {
        case 0: return run<0>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1);
        case 1: return run<1>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1);
        case 2: return run<2>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1);
        case 3: return run<3>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1);
        case 4: return run<4>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1);
        case 5: if constexpr (M > 5) return run<5>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1); else return 0;
        case 6: if constexpr (M > 6) return run<6>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1); else return 0;
        default: if constexpr (M > 7) return run<7>(sm, lane, gbase, i, stop, slot, ptrs, ub, true, d0, d1); else return 0;
        }
    }

    __device__ static Key make_key(bool valid, V pm, int idx)
    {
        if constexpr (FLOAT) {
            const uint64_t hi = valid ? (uint64_t)A::key_bits(pm) : 0xFFFFFFFFull;
            return (hi << 8) | (uint64_t)idx;
        } else {
            // |PM| <= 127 N < 2^15: (PM, index) in one 32-bit key
            return ((valid ? (uint32_t)pm : 0x7FFFFFu) << 7) | (uint32_t)idx;
        }
    }
    __device__ static int key_index(Key k) { return (int)(k & (FLOAT ? 0xFFu : 0x7Fu)); }
    __device__ static bool key_valid(Key k)
    {
        if constexpr (FLOAT) return (uint32_t)(k >> 8) != 0xFFFFFFFFu;
        else return (k >> 7) != 0x7FFFFFu;
    }
    __device__ static V key_pm(Key k)
    {
        if constexpr (FLOAT) return __uint_as_float((uint32_t)(k >> 8));
        else return (V)(k >> 7);
    }

    // Bitonic sort, ascending, of the 2L keys of a frame: lane slot s holds
    // elements 2s (x0) and 2s + 1 (x1).  Stages of size KS = 2, 4, ..., 2L.
    // Stage KS/J of the network has the number base(KS) + log2(KS/2) - log2(J),
    // base(KS) = number of stages of the smaller sizes.
    static constexpr int lg2(int v) { return v <= 1 ? 0 : 1 + lg2(v / 2); }
    template <int KS, int J>
    static constexpr int stage_no() { return (lg2(KS) - 1) * lg2(KS) / 2 + (lg2(KS) - 1 - lg2(J)); }

    // Per-lane direction bits of every stage (bit set: this lane keeps the
    // larger key, of x0 for the in-lane stages), fixed by the lane's slot.
    template <int KS>
    __device__ static uint32_t bitonic_dirs(int s)
    {
        if constexpr (KS <= 2 * L) return dirs_stage<KS, KS / 2>(s) | bitonic_dirs<KS * 2>(s);
        else return 0u;
    }
    template <int KS, int J>
    __device__ static uint32_t dirs_stage(int s)
    {
        const bool up = ((2 * s) & KS) == 0;
        const bool keep_min = J == 1 ? up : ((((2 * s) & J) == 0) == up);
        const uint32_t bit = keep_min ? 0u : (1u << stage_no<KS, J>());
        if constexpr (J > 1) return bit | dirs_stage<KS, J / 2>(s);
        else return bit;
    }

    // Bitonic sort, ascending, of the 2L keys of a frame: lane slot s holds
    // elements 2s (x0) and 2s + 1 (x1).  Stages of size KS = 2, 4, ..., 2L.
    // 32-bit keys take min or max in one v_med3 against 0 / ~0 chosen by the
    // lane's direction bit.
    template <int KS>
    __device__ static void bitonic(Key& x0, Key& x1, int s, uint32_t dirs)
    {
        if constexpr (KS <= 2 * L) {
            stage<KS, KS / 2>(x0, x1, s, dirs);
            bitonic<KS * 2>(x0, x1, s, dirs);
        }
    }
    __device__ static uint32_t med3u(uint32_t a, uint32_t b, uint32_t c) { return max(min(a, b), min(max(a, b), c)); }

    // One 32-bit key per lane over the frame's L lanes: a bitonic sort into
    // descending order (stages numbered 0 .. NSORT1 - 1), then the ascending
    // bitonic merge of a bitonic sequence (stages NSORT1 ...).  Bit P of fd
    // set: stage P keeps the larger key in this lane.
    static constexpr int NSORT1 = lg2(L) * (lg2(L) + 1) / 2;
    template <int KS, int J, int P>
    __device__ static uint32_t sort1_dirs(int s)
    {
        if constexpr (KS <= L) {
            const uint32_t bit = ((((s & J) == 0) == ((s & KS) == 0)) ? 1u : 0u) << P;
            if constexpr (J > 1) return bit | sort1_dirs<KS, J / 2, P + 1>(s);
            else return bit | sort1_dirs<KS * 2, KS, P + 1>(s);
        } else {
            return 0u;
        }
    }
    template <int J, int P>
    __device__ static uint32_t merge1_dirs(int s)
    {
        if constexpr (J >= 1) return ((((s & J) != 0) ? 1u : 0u) << P) | merge1_dirs<J / 2, P + 1>(s);
        else return 0u;
    }
    __device__ static uint32_t one_key_dirs(int s) { return sort1_dirs<2, 1, 0>(s) | merge1_dirs<L / 2, NSORT1>(s); }
    template <int KS, int J, int P>
    __device__ static uint32_t sort1(uint32_t x, uint32_t fd)
    {
        if constexpr (KS <= L) {
            x = med3u(x, xor_lane<J>(x), (uint32_t)(-(int32_t)((fd >> P) & 1u)));
            if constexpr (J > 1) return sort1<KS, J / 2, P + 1>(x, fd);
            else return sort1<KS * 2, KS, P + 1>(x, fd);
        } else {
            return x;
        }
    }
    template <int J, int P>
    __device__ static uint32_t merge1(uint32_t x, uint32_t fd)
    {
        if constexpr (J >= 1) {
            x = med3u(x, xor_lane<J>(x), (uint32_t)(-(int32_t)((fd >> P) & 1u)));
            return merge1<J / 2, P + 1>(x, fd);
        } else {
            return x;
        }
    }
    template <int KS, int J>
    __device__ static void stage(Key& x0, Key& x1, int s, uint32_t dirs)
    {
        if constexpr (!FLOAT) {
            const uint32_t bound = (uint32_t)(-(int32_t)((dirs >> stage_no<KS, J>()) & 1u));  // 0: min, ~0: max
            if constexpr (J == 1) {
                const Key a = x0, b = x1;
                x0 = med3u(a, b, bound);
                x1 = med3u(a, b, ~bound);
            } else {
                const Key y0 = xor_key<J / 2>(x0), y1 = xor_key<J / 2>(x1);
                x0 = med3u(x0, y0, bound);
                x1 = med3u(x1, y1, bound);
                stage<KS, J / 2>(x0, x1, s, dirs);
            }
        } else {
            const bool up = ((2 * s) & KS) == 0;
            if constexpr (J == 1) {
                const Key lo = x0 < x1 ? x0 : x1, hi = x0 < x1 ? x1 : x0;
                x0 = up ? lo : hi;
                x1 = up ? hi : lo;
            } else {
                const Key y0 = xor_key<J / 2>(x0), y1 = xor_key<J / 2>(x1);
                const bool keep_min = (((2 * s) & J) == 0) == up;
                x0 = keep_min ? (y0 < x0 ? y0 : x0) : (y0 < x0 ? x0 : y0);
                x1 = keep_min ? (y1 < x1 ? y1 : x1) : (y1 < x1 ? x1 : y1);
                stage<KS, J / 2>(x0, x1, s, dirs);
            }
        }
    }
};

// q = clamp(round_half_even(fl32(v s)), -127, 127); a non-finite v gives 0
// and is counted in *bad.
__device__ inline uint32_t quantize1(float v, float s, int32_t* __restrict__ bad)
{
    if (!isfinite(v)) {
        if (bad) atomicAdd(bad, 1);
        return 0u;
    }
    float t = rintf(__fmul_rn(v, s));  // a product overflowing to +-inf clamps below
    t = fminf(fmaxf(t, -127.0f), 127.0f);
    return (uint32_t)(uint8_t)(int8_t)t;
}

// The quantizer inside the SCL launch (QUANT): llr is float y, 16-byte
// aligned; q receives the int8 values (4-byte aligned), bad counts non-finite
// inputs.
struct QuantArgs {
    float scale;
    int8_t* q;
    int32_t* bad;
};

template <int M, int L, bool FLOAT, bool QUANT = false>
__global__ __launch_bounds__(WAVE) void scl_kernel(const void* __restrict__ llr, int64_t F,
                                                   uint64_t info0, uint64_t info1, uint64_t info2, uint64_t info3,
                                                   int crc_len, CrcRows crc, Sched sched,
                                                   uint8_t* __restrict__ anchors, uint8_t* __restrict__ crc_ok,
                                                   int32_t* __restrict__ pm_out, QuantArgs qa)
{
    static_assert(!(QUANT && FLOAT), "the quantizer feeds the int8 form");
    using K = Scl<M, L, FLOAT>;
    using A = typename K::A;
    using V = typename K::V;
    using S = typename K::S;
    using Key = typename K::Key;
    constexpr int N = K::N, NW = K::NW, G = K::G;
    __shared__ __attribute__((aligned(16))) typename K::Smem sm;

    const int lane = threadIdx.x;
    const int slot = lane % L;
    const int gbase = lane - slot;  // first lane of this frame group
    const int64_t frame = (int64_t)blockIdx.x * G + lane / L;
    const bool live = frame < F;
    const uint64_t info[4] = {info0, info1, info2, info3};

    // stage the channel values of the wave's frames (coalesced); int8 q four
    // values per lane and load when it is 4-byte aligned, widened to two
    // int16 pairs (a frame's N values never share a word with another frame)
    if constexpr (QUANT) {
        // four values per lane: one 16-byte load of y, one 4-byte store of q
        for (int e = 4 * lane; e < G * N; e += 4 * WAVE) {
            const int64_t fr = (int64_t)blockIdx.x * G + e / N;
            uint32_t w = 0u;
            if (fr < F) {
                const float4 v = *reinterpret_cast<const float4*>((const float*)llr + fr * N + e % N);
                w = quantize1(v.x, qa.scale, qa.bad) | (quantize1(v.y, qa.scale, qa.bad) << 8) |
                    (quantize1(v.z, qa.scale, qa.bad) << 16) | (quantize1(v.w, qa.scale, qa.bad) << 24);
                *reinterpret_cast<uint32_t*>(qa.q + fr * N + e % N) = w;
            }
            auto wide = [](uint32_t b) { return (uint32_t)(uint16_t)(int16_t)(int8_t)(uint8_t)b; };
            uint32_t* d = reinterpret_cast<uint32_t*>(sm.ch + (e / N) * K::CHS + e % N);
            d[0] = wide(w) | (wide(w >> 8) << 16);
            d[1] = wide(w >> 16) | (wide(w >> 24) << 16);
        }
    } else if (!FLOAT && (reinterpret_cast<uintptr_t>(llr) & 3u) == 0) {
        for (int e = 4 * lane; e < G * N; e += 4 * WAVE) {
            const int64_t fr = (int64_t)blockIdx.x * G + e / N;
            const uint32_t w =
                fr < F ? mpwsd::read_q4(*reinterpret_cast<const uint32_t*>((const int8_t*)llr + fr * N + e % N)) : 0u;
            auto wide = [](uint32_t b) { return (uint32_t)(uint16_t)(int16_t)(int8_t)(uint8_t)b; };
            uint32_t* d = reinterpret_cast<uint32_t*>(sm.ch + (e / N) * K::CHS + e % N);
            d[0] = wide(w) | (wide(w >> 8) << 16);
            d[1] = wide(w >> 16) | (wide(w >> 24) << 16);
        }
    } else {
        for (int e = lane; e < G * N; e += WAVE) {
            const int64_t fr = (int64_t)blockIdx.x * G + e / N;
            sm.ch[(e / N) * K::CHS + e % N] = (S)(fr < F ? A::load_ch(llr, fr * N + e % N) : (V)0);
        }
    }
    __syncthreads();

    V pm = 0;
    bool valid = (slot == 0);
    uint64_t ptrs = 0;  // byte l: group slot owning this path's level-l buffer
    const uint32_t dirs = FLOAT ? K::template bitonic_dirs<2>(slot) : 0u;  // sorting-network directions of this lane
    const uint32_t fdirs = FLOAT ? 0u : K::one_key_dirs(slot);
    // the slots hold the paths in ascending (PM, index) order; a frozen leaf
    // adds penalties path by path and breaks that order until the next sort
    bool sorted = true;
    uint32_t ub[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) ub[i] = 0;
#pragma unroll
    for (int l = 0; l < M; ++l) ptrs |= (uint64_t)slot << (8 * l);

    // the schedule is read with scalar loads from the kernel arguments, each
    // entry one node ahead of its use
    const __attribute__((address_space(4))) uint32_t* sw =
        (const __attribute__((address_space(4))) uint32_t*)(const void*)sched.v;
    auto sched_at = [&](int j) { return (int)((sw[j >> 2] >> (8 * (j & 3))) & 0xFFu); };
    int e_next = FLOAT ? 0 : sched_at(0);
    for (int i = 0; i < N;) {
        const int e = e_next;
        const int lev = e & 15, kind = e >> 4;
        if (!FLOAT && i + (1 << lev) < N) e_next = sched_at(i + (1 << lev));
        V d0, d1;
        const V lam = K::node(sm, lane, gbase, i, lev, slot, ptrs, ub, d0, d1);
        const int last = i + (1 << lev) - 1;  // the leaf a decision is taken at
        i += 1 << lev;
        if (kind == 0) {
            d0 = lam < 0 ? (V)-lam : (V)0;
            d1 = lam > 0 ? lam : (V)0;
        }
        const bool frozen = kind == KIND_R0 || (kind == 0 && ((info[last >> 6] >> (last & 63)) & 1ull) == 0);
        if (frozen) {
            if (valid) pm = pm + d0;
            sorted = false;
            continue;  // u = 0 already
        }
        // information bit: slot s takes the s-th smallest of the 2L children's
        // keys (PM, parent slot, bit), which also names its parent and bit
        Key mine;
        bool fast = false;
        if constexpr (!FLOAT) fast = kind == 0 && sorted;
        if (fast) {
            // ordinary leaf: one child of each path adds nothing to its PM, so
            // those L keys are already ascending by slot; the other L (the
            // penalised children) are sorted descending, the lane-wise minimum
            // of the two holds the L smallest as a bitonic sequence, and one
            // bitonic merge puts the s-th smallest on slot s
            const int zb = lam < 0 ? 1 : 0;
            const Key a = K::make_key(valid, pm, 2 * slot + zb);
            const Key b = K::make_key(valid, (V)(pm + (lam < 0 ? -lam : lam)), 2 * slot + 1 - zb);
            const Key bd = (Key)K::template sort1<2, 1, 0>((uint32_t)b, fdirs);
            mine = (Key)K::template merge1<L / 2, K::NSORT1>((uint32_t)(a < bd ? a : bd), fdirs);
        } else if constexpr (!FLOAT) {
            // both children may be penalised (a repetition node, or a leaf
            // after a frozen one reordered the PMs): the bit-0 keys are sorted
            // descending and the bit-1 keys ascending by the same networks with
            // opposite directions, then the lane-wise minimum and one bitonic
            // merge as above
            const Key x0 = K::make_key(valid, (V)(pm + d0), 2 * slot);
            const Key x1 = K::make_key(valid, (V)(pm + d1), 2 * slot + 1);
            const Key xd = (Key)K::template sort1<2, 1, 0>((uint32_t)x0, fdirs);
            const Key xa = (Key)K::template sort1<2, 1, 0>((uint32_t)x1, fdirs ^ ((1u << K::NSORT1) - 1u));
            mine = (Key)K::template merge1<L / 2, K::NSORT1>((uint32_t)(xa < xd ? xa : xd), fdirs);
        } else {
            // all 2L children (two keys per lane) through a bitonic sort
            Key x0 = K::make_key(valid, (V)(pm + d0), 2 * slot);
            Key x1 = K::make_key(valid, (V)(pm + d1), 2 * slot + 1);
            K::template bitonic<2>(x0, x1, slot, dirs);
            const int src = gbase + (slot >> 1);
            const Key y0 = shfl_key(x0, src), y1 = shfl_key(x1, src);
            mine = (slot & 1) ? y1 : y0;
        }
        sorted = true;
        const int c = K::key_index(mine);
        valid = K::key_valid(mine);
        pm = K::key_pm(mine);
        const int par = gbase + (c >> 1);
        ptrs = shfl_u64(ptrs, par);
#pragma unroll
        for (int w = 0; w < NW; ++w) ub[w] = (uint32_t)__shfl((int)ub[w], par);
        ub[last >> 5] |= (uint32_t)(c & 1) << (last & 31);
    }

    // final order: (PM, slot) ascending
    const uint64_t fkey = ((uint64_t)(valid ? A::key_bits(pm) : 0xFFFFFFFFu) << 8) | (uint64_t)slot;
    int rank = 0;
#pragma unroll
    for (int c = 0; c < L; ++c) rank += shfl_u64(fkey, gbase + c) < fkey;
    uint32_t cw[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) cw[w] = ub[w];
    polar_bits(cw, M);
    if (live) {
        uint32_t* dst = (uint32_t*)(anchors + ((size_t)frame * L + rank) * (N / 8));
#pragma unroll
        for (int w = 0; w < NW; ++w) dst[w] = cw[w];
        if (pm_out) pm_out[frame * L + rank] = (int32_t)A::key_bits(pm);
        if (rank == 0) {
            int ok = 0;
            if (crc_len > 0) {
                uint32_t reg = 0;
                for (int b = 0; b < crc_len; ++b) {
                    uint32_t x = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) x ^= ub[w] & crc.w[b][w];
                    reg |= (uint32_t)(__popc(x) & 1) << b;
                }
                ok = reg == 0;
            }
            crc_ok[frame] = (uint8_t)ok;
        }
    }
}


__global__ void quantize_kernel(const float* __restrict__ y, int64_t n, float s, int8_t* __restrict__ q,
                                int32_t* __restrict__ bad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        q[i] = (int8_t)quantize1(y[i], s, bad);
}

// four values per thread: one 16-byte load, one 4-byte store (y 16-byte and
// q 4-byte aligned; n4 = number of quadruples)
__global__ void quantize4_kernel(const float4* __restrict__ y, int64_t n4, float s, uint32_t* __restrict__ q,
                                 int32_t* __restrict__ bad)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = y[i];
        q[i] = quantize1(v.x, s, bad) | (quantize1(v.y, s, bad) << 8) | (quantize1(v.z, s, bad) << 16) |
               (quantize1(v.w, s, bad) << 24);
    }
}

// Maximal rate-0 and repetition subtrees of the frozen pattern, in SC order.
Sched make_sched(int m, const uint64_t* info)
{
    Sched sc{};
    const int n = 1 << m;
    auto is_info = [&](int j) { return ((info[j >> 6] >> (j & 63)) & 1ull) != 0; };
    struct Rec {
        static void visit(Sched& sc, const decltype(is_info)& inf, int lev, int a)
        {
            const int n = 1 << lev;
            if (lev > 0) {
                int cnt = 0;
                for (int j = a; j < a + n; ++j) cnt += inf(j);
                if (cnt == 0) { sc.v[a] = (uint8_t)((KIND_R0 << 4) | lev); return; }
                if (cnt == 1 && inf(a + n - 1)) { sc.v[a] = (uint8_t)((KIND_REP << 4) | lev); return; }
                visit(sc, inf, lev - 1, a);
                visit(sc, inf, lev - 1, a + n / 2);
                return;
            }
            sc.v[a] = 0;
        }
    };
    Rec::visit(sc, is_info, m, 0);
    (void)n;
    return sc;
}

// Rows of the CRC test (CrcRows).  The register is fed the information bits
// in ascending position: fb = (top bit) xor bit, shift left, xor the
// polynomial when fb is set.  A single 1 followed by t zeros leaves
// step0^t(poly), step0 being a step with input 0; walking the information
// positions from the last one down, t grows by one per position.
CrcRows make_crc_rows(int m, const uint64_t* info, int crc_len, uint32_t poly)
{
    CrcRows cr{};
    if (crc_len <= 0) return cr;
    const uint32_t top = 1u << (crc_len - 1), mask = (crc_len == 32) ? ~0u : (1u << crc_len) - 1u;
    uint32_t cur = poly & mask;
    for (int j = (1 << m) - 1; j >= 0; --j) {
        if (((info[j >> 6] >> (j & 63)) & 1ull) == 0) continue;
        for (int b = 0; b < crc_len; ++b)
            if ((cur >> b) & 1u) cr.w[b][j >> 5] |= 1u << (j & 31);
        const bool fb = (cur & top) != 0;
        cur = (cur << 1) & mask;
        if (fb) cur ^= poly & mask;
    }
    return cr;
}

template <int M, int L, bool FL>
void launch_scl3(const void* llr, int64_t F, const uint64_t* info, int crc_len, uint32_t poly, uint8_t* anchors,
                 uint8_t* crc_ok, int32_t* pm, const QuantArgs* qa, hipStream_t s)
{
    constexpr int64_t per = WAVE / L;
    const int64_t blocks = (F + per - 1) / per;
    if constexpr (!FL) {
        if (qa) {
            hipLaunchKernelGGL((scl_kernel<M, L, false, true>), dim3((unsigned)blocks), dim3(WAVE), 0, s, llr, F,
                               info[0], info[1], info[2], info[3], crc_len, make_crc_rows(M, info, crc_len, poly),
                               make_sched(M, info), anchors, crc_ok, pm, *qa);
            return;
        }
    }
    hipLaunchKernelGGL((scl_kernel<M, L, FL>), dim3((unsigned)blocks), dim3(WAVE), 0, s, llr, F, info[0], info[1],
                       info[2], info[3], crc_len, make_crc_rows(M, info, crc_len, poly), make_sched(M, info), anchors,
                       crc_ok, pm, QuantArgs{0.0f, nullptr, nullptr});
}

template <int M, bool FL>
void launch_scl(const void* llr, int64_t F, int L, const uint64_t* info, int crc_len, uint32_t poly,
                uint8_t* anchors, uint8_t* crc_ok, int32_t* pm, const QuantArgs* qa, hipStream_t s)
{
    switch (L) {
    case 1: launch_scl3<M, 1, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    case 2: launch_scl3<M, 2, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    case 4: launch_scl3<M, 4, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    case 8: launch_scl3<M, 8, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    case 16: launch_scl3<M, 16, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    default: launch_scl3<M, 32, FL>(llr, F, info, crc_len, poly, anchors, crc_ok, pm, qa, s); break;
    }
}

}  // namespace

extern "C" int mpwsd_quantize_llr(const float* y, int64_t n, float scale, int8_t* q, int32_t* bad,
                                  hipStream_t stream)
{
    mpwsd::clear_error();
    if (n < 0 || (n > 0 && (!y || !q))) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_quantize_llr: bad arguments");
    if (!std::isfinite(scale)) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_quantize_llr: scale must be finite");
    if (n == 0) return MPWSD_OK;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(y) & 15u) == 0 && (reinterpret_cast<uintptr_t>(q) & 3u) == 0 && n >= 4) {
        const int64_t n4 = n / 4;
        const int64_t want4 = (n4 + 255) / 256;
        hipLaunchKernelGGL(quantize4_kernel, dim3((unsigned)(want4 < 8192 ? want4 : 8192)), dim3(256), 0, stream,
                           reinterpret_cast<const float4*>(y), n4, scale, reinterpret_cast<uint32_t*>(q), bad);
        done = 4 * n4;
    }
    if (done < n) {
        const int64_t rest = n - done;
        const int64_t want = (rest + 255) / 256;
        hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)(want < 8192 ? want : 8192)), dim3(256), 0, stream,
                           y + done, rest, scale, q + done, bad);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_quantize_llr: %s", hipGetErrorString(e));
    return MPWSD_OK;
}

namespace {
// Argument checks shared by the SCL entry points (nothing enqueued on error).
int scl_check(const char* fn, int r, int m, int crc_len, uint32_t crc_poly, int L, int64_t F)
{
    using namespace mpwsd;
    if (m < 5 || m > 8 || r < 1 || r >= m)
        return fail(MPWSD_ERR_UNSUPPORTED, "%s: need 1 <= r < m, 5 <= m <= 8 (r=%d m=%d)", fn, r, m);
    const int K = rm_dimension(r, m);
    if (L < 1 || L > 32 || (L & (L - 1)) != 0)
        return fail(MPWSD_ERR_UNSUPPORTED, "%s: L must be a power of two <= 32 (L=%d)", fn, L);
    if (K < 6 && L > (1 << K))
        return fail(MPWSD_ERR_UNSUPPORTED, "%s: L=%d exceeds the code size 2^%d", fn, L, K);
    if (crc_len < 0 || crc_len > 16 || crc_len > K)
        return fail(MPWSD_ERR_UNSUPPORTED, "%s: crc_len must be in [0, min(16, K)] (got %d)", fn, crc_len);
    if (crc_len > 0 && ((crc_poly >> crc_len) & 1u) == 0)
        return fail(MPWSD_ERR_ARG, "%s: crc_poly must include the x^%d term", fn, crc_len);
    if (F < 0) return fail(MPWSD_ERR_ARG, "%s: F < 0", fn);
    return MPWSD_OK;
}

int scl_launch(const char* fn, int r, int m, int crc_len, uint32_t crc_poly, int L, const void* llr, bool fl,
               int64_t F, uint8_t* anchors, uint8_t* crc_ok, int32_t* pm, const QuantArgs* qa, hipStream_t stream)
{
    using namespace mpwsd;
    uint64_t info[4] = {0, 0, 0, 0};
    for (int i = 0; i < (1 << m); ++i)
        if (__builtin_popcount((unsigned)i) >= m - r) info[i >> 6] |= 1ull << (i & 63);
    switch (m) {
    case 5: fl ? launch_scl<5, true>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream)
               : launch_scl<5, false>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream); break;
    case 6: fl ? launch_scl<6, true>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream)
               : launch_scl<6, false>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream); break;
    case 7: fl ? launch_scl<7, true>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream)
               : launch_scl<7, false>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream); break;
    default: fl ? launch_scl<8, true>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream)
                : launch_scl<8, false>(llr, F, L, info, crc_len, crc_poly, anchors, crc_ok, pm, qa, stream); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MPWSD_ERR_DEVICE, "%s: %s", fn, hipGetErrorString(e));
    return MPWSD_OK;
}
}  // namespace

extern "C" int mpwsd_stage1_scl(int r, int m, int crc_len, uint32_t crc_poly, int L, const void* llr, int dtype,
                                int64_t F, uint8_t* anchors, uint8_t* crc_ok, int32_t* pm, hipStream_t stream)
{
    using namespace mpwsd;
    clear_error();
    const char* fn = "mpwsd_stage1_scl";
    int rc = scl_check(fn, r, m, crc_len, crc_poly, L, F);
    if (rc != MPWSD_OK) return rc;
    if (dtype != MPWSD_I8 && dtype != MPWSD_F32) return fail(MPWSD_ERR_ARG, "mpwsd_stage1_scl: bad dtype %d", dtype);
    if (F == 0) return MPWSD_OK;
    if (!llr || !anchors || !crc_ok) return fail(MPWSD_ERR_ARG, "mpwsd_stage1_scl: null pointer");
    if ((reinterpret_cast<uintptr_t>(anchors) & 3u) != 0)
        return fail(MPWSD_ERR_ARG, "mpwsd_stage1_scl: anchors must be 4-byte aligned");
    return scl_launch(fn, r, m, crc_len, crc_poly, L, llr, dtype == MPWSD_F32, F, anchors, crc_ok, pm, nullptr,
                      stream);
}

extern "C" int mpwsd_stage1_scl_quantized(int r, int m, int crc_len, uint32_t crc_poly, int L, const float* y,
                                          float scale, int64_t F, int8_t* q, int32_t* bad, uint8_t* anchors,
                                          uint8_t* crc_ok, int32_t* pm, hipStream_t stream)
{
    using namespace mpwsd;
    clear_error();
    const char* fn = "mpwsd_stage1_scl_quantized";
    int rc = scl_check(fn, r, m, crc_len, crc_poly, L, F);
    if (rc != MPWSD_OK) return rc;
    if (!std::isfinite(scale)) return fail(MPWSD_ERR_ARG, "%s: scale must be finite", fn);
    if (F == 0) return MPWSD_OK;
    if (!y || !q || !anchors || !crc_ok) return fail(MPWSD_ERR_ARG, "%s: null pointer", fn);
    if ((reinterpret_cast<uintptr_t>(anchors) & 3u) != 0) return fail(MPWSD_ERR_ARG, "%s: anchors must be 4-byte aligned", fn);
    if ((reinterpret_cast<uintptr_t>(y) & 15u) != 0 || (reinterpret_cast<uintptr_t>(q) & 3u) != 0) {
        // the fused launch reads y 16 bytes and writes q 4 bytes at a time: the
        // same two steps as separate launches otherwise
        rc = mpwsd_quantize_llr(y, F << m, scale, q, bad, stream);
        if (rc != MPWSD_OK) return rc;
        clear_error();
        return scl_launch(fn, r, m, crc_len, crc_poly, L, q, false, F, anchors, crc_ok, pm, nullptr, stream);
    }
    const QuantArgs qa{scale, q, bad};
    return scl_launch(fn, r, m, crc_len, crc_poly, L, y, false, F, anchors, crc_ok, pm, &qa, stream);
}
