// Stage 2 (Sec. III-B, Eq. (4)-(5), Alg. 1): multipoint code-weight sphere
// decoding of the frames whose stage-1 CRC failed.
//
// A "column" is one (failing frame, path) pair.  Per column the workspace
// holds the centre c (packed bits), z = llr * (1 - 2c) and the metric.  The
// move search of one iteration is the contraction S = W Z of the move matrix
// W (P x N, 0/1) with the z columns, followed by an argmin over P:
//   * int8 form: chunks of 128 moves are staged in LDS and fed to
//     v_mfma_i32_16x16x64_i8 against -z fragments that stay in VGPRs for the
//     whole sweep.  The accumulator is seeded so that each result reads
//     128 S + (row within the chunk), a running v_min3 keeps the smallest,
//     and per chunk the exact key (S << 32 | p) is formed from the row
//     index, so the smallest p attaining the minimum wins.  Two move tables:
//     the bit-packed one (unpacked into LDS per chunk), and the paired-half
//     one of mpwsd_group_moves (rows of N/2 bytes, each scoring a move and
//     its translate against the two halves of z; copied verbatim into LDS).
//   * float form: the same contraction summed sequentially in binary32 in
//     ascending position order on the vector ALUs, with the exact move index
//     carried in a 64-bit key.
// Work is split over (column tile x move chunk) units spread evenly over a
// fixed, device-filling grid; split results meet in an atomicMin per column,
// which is order independent, so the result does not depend on the split.
// After each search a resolve pass applies the moves, logs them and builds
// the next iteration's active list (a column that did not move can never
// move again); with merging it also drops the columns whose centre another
// column of the frame already holds.  All counts live in device memory, so T
// iterations enqueue without any host round trip and can be captured in a
// HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>

#include "apply.h"
#include "common.h"
#include "group.h"

namespace {

constexpr int WAVE = 64;
constexpr int RC = 128;  // moves per chunk
typedef int v4i __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- workspace
struct SegWs {
    int32_t* hdr;     // [0]=F2 [1]=err, then per iteration t <= T the pair
                      // [ncol(t)] columns to search, [ncol(t)+1] frames
                      // holding them (kept with merging), 8-byte aligned
    int32_t* fid;     // [F] compacted failing frames
    int32_t* slot;    // [F] frame -> compacted slot (-1 when decided)
    int32_t* act[2];  // [F*L] active column lists (ping-pong)
    int32_t* fl[2];   // [F] frames with an active column (merging; ping-pong)
    uint64_t* key64;  // [F*L] per-column minimum: int8 (S << 32 | p) as int64,
                      // float (orderable(S) << 32 | p) as uint64
    int32_t* metric;  // [F*L] int8: M; float: unused
    int32_t* tag;     // [F*L] path state for the merging of equal centres
    uint8_t* cw;      // [F*L][N/8] centres
    void* z;          // [F*L][KP] int8 -z (negated) or [F*L][N] float z
    size_t bytes;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int hdr_len(int T) { return 4 + 2 * T; }

// index in hdr of the column count of iteration t (the frame count follows)
__host__ __device__ constexpr int ncol(int t) { return 2 + 2 * t; }

int kpad(int N) { return N < 64 ? 64 : N; }

SegWs carve(const mpwsd_segment& sg, int L, int T, uint8_t* base)
{
    const size_t F = (size_t)sg.F, C = F * (size_t)L;
    const int N = 1 << sg.m;
    SegWs w{};
    size_t off = 0;
    auto take = [&](size_t b) { uint8_t* p = base ? base + off : nullptr; off += align_up(b); return p; };
    w.hdr = (int32_t*)take(sizeof(int32_t) * (size_t)hdr_len(T));
    w.fid = (int32_t*)take(sizeof(int32_t) * F);
    w.slot = (int32_t*)take(sizeof(int32_t) * F);
    w.act[0] = (int32_t*)take(sizeof(int32_t) * C);
    w.act[1] = (int32_t*)take(sizeof(int32_t) * C);
    w.fl[0] = (int32_t*)take(sizeof(int32_t) * F);
    w.fl[1] = (int32_t*)take(sizeof(int32_t) * F);
    w.key64 = (uint64_t*)take(sizeof(uint64_t) * C);
    w.tag = (int32_t*)take(sizeof(int32_t) * C);
    if (sg.dtype == MPWSD_I8) {
        w.metric = (int32_t*)take(sizeof(int32_t) * C);
        w.z = take(C * (size_t)kpad(N));
    } else {
        w.z = take(C * (size_t)N * sizeof(float));
    }
    w.cw = take(C * (size_t)(N / 8));
    w.bytes = off;
    return w;
}

int device_cus()
{
    static std::mutex mu;
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) {
        int cus = 0;
        return hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0
                   ? cus : 256;
    }
    std::lock_guard<std::mutex> g(mu);
    if (!cache[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

// ---------------------------------------------------------------- compaction
// Failing frames are appended to the compacted list with one atomic per
// workgroup (their order in the list is irrelevant: every frame is decoded
// independently and results are written per frame).
// Clears a segment header (and, for the first segment of a call, the
// caller's statistics) before the compaction.
__global__ void hdr_zero_kernel(int32_t* __restrict__ hdr, int n, int32_t* __restrict__ stats, int ns)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) hdr[i] = 0;
    if (stats)
        for (int i = threadIdx.x; i < ns; i += blockDim.x) stats[i] = 0;
}

__global__ __launch_bounds__(256) void compact_kernel(const uint8_t* __restrict__ crc_ok, int64_t F,
                                                      int32_t* __restrict__ hdr, int32_t* __restrict__ fid,
                                                      int32_t* __restrict__ slot)
{
    __shared__ int wsum[4];
    __shared__ int base_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t f = (int64_t)blockIdx.x * 256 + tid;
    const bool in = f < F;
    const bool fail = in && !(crc_ok && crc_ok[f]);
    const uint64_t bal = __ballot(fail);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(bal);
    __syncthreads();
    if (tid == 0) {
        const int tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base_s = tot ? atomicAdd(&hdr[0], tot) : 0;
    }
    __syncthreads();
    int off = base_s + before;
    for (int w = 0; w < wid; ++w) off += wsum[w];
    if (fail) {
        fid[off] = (int32_t)f;
        slot[f] = off;
    } else if (in) {
        slot[f] = -1;
    }
}

__global__ void stats_zero_kernel(int32_t* stats, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) stats[i] = 0;
}

// Per-iteration active counts and the out-of-table count into stats
// (workgroup 0 of the final choice, when every count is final).
__device__ inline void stats_add(const int32_t* __restrict__ hdr, int T, int32_t* __restrict__ stats)
{
    const int t = threadIdx.x;
    if (t < T) atomicAdd(&stats[1 + t], hdr[ncol(t)]);
    if (t == 0) atomicAdd(&stats[1 + T], hdr[1]);
}

// ---------------------------------------------------------------- init
// Two index ranges, PP = KP/16 threads (16 positions each) per item:
//   frames f < F: every frame's move log is filled with -1, and a decided
//     frame takes its first anchor (decision, k = 0, metric);
//   columns c < hdr[0] L of the failing frames (c = list index * L + path):
//     centre bits, -z and the metric M(c) = sum_{c_j = 1} q_j (int8 form).
// Thread 0 also publishes the number of columns for the first search.
template <bool FLOAT>
__global__ __launch_bounds__(256) void init_kernel(
    const void* __restrict__ llr, const uint8_t* __restrict__ anchors, int64_t F, int L, int T, int N, int KP,
    int32_t* __restrict__ hdr, const int32_t* __restrict__ slot, const int32_t* __restrict__ fid,
    int32_t* __restrict__ act0, uint64_t* __restrict__ key64, int32_t* __restrict__ metric,
    int32_t* __restrict__ tag, uint8_t* __restrict__ cw, void* __restrict__ zbuf, uint8_t* __restrict__ out_cw,
    int32_t* __restrict__ out_k,
    int32_t* __restrict__ out_metric, int32_t* __restrict__ out_moves, int32_t* __restrict__ stats)
{
    const int PP = KP / 16;  // pieces per item (4, 8 or 16: an item's pieces share a wave)
    const int pps = __builtin_ctz((unsigned)PP);
    const int NB = N / 8;
    const int64_t nfail = hdr[0];
    const int64_t part1 = F * PP;
    const int64_t total = part1 + nfail * L * PP;
    const bool log16 = (L * T) % 4 == 0 && (reinterpret_cast<uintptr_t>(out_moves) & 15u) == 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[ncol(0)] = (int32_t)(nfail * L);
        if (stats) atomicAdd(&stats[0], (int32_t)nfail);
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ((total + 63) & ~int64_t(63));
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g >= total) continue;  // whole items: total and part1 are multiples of PP
        const int piece = (int)g & (PP - 1);
        const int j0 = 16 * piece;
        const bool inpos = j0 < N;
        if (g < part1) {
            // ---- frame f
            const int64_t f = g >> pps;
            if (out_moves) {
                if (log16) {
                    // 16-byte stores: a frame's pieces write consecutive quads
                    v4i* o = (v4i*)(out_moves + (size_t)f * L * T);
                    for (int e = piece; e < L * T / 4; e += PP) o[e] = v4i{-1, -1, -1, -1};
                } else {
                    for (int e = piece; e < L * T; e += PP) out_moves[(size_t)f * L * T + e] = -1;
                }
            }
            if (slot[f] >= 0) continue;  // failing: its columns are items of the second range
            const uint32_t bits = inpos ? *(const uint16_t*)(anchors + (size_t)f * L * NB + 2 * piece) : 0u;
            int part = 0;
            if (!FLOAT && inpos) {
                const v4i qv = *(const v4i*)((const int8_t*)llr + (size_t)f * N + j0);
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    part = mpwsd::masked_sum4(mpwsd::read_q4((uint32_t)qv[d]), bits >> (4 * d), part);
            }
            for (int o = 1; o < PP; o <<= 1) part += __shfl_xor(part, o);
            if (inpos) *(uint16_t*)(out_cw + (size_t)f * NB + 2 * piece) = (uint16_t)bits;
            if (piece == 0) {
                if (out_k) out_k[f] = 0;
                if (out_metric) {
                    if (FLOAT) {
                        const uint8_t* a = anchors + (size_t)f * L * NB;
                        const float* y = (const float*)llr + (size_t)f * N;
                        float e = 0.0f;
                        for (int j = 0; j < N; ++j) {
                            const float x = ((a[j >> 3] >> (j & 7)) & 1) ? -1.0f : 1.0f;
                            const float dlt = __fsub_rn(y[j], x);
                            e = __fadd_rn(e, __fmul_rn(dlt, dlt));
                        }
                        out_metric[f] = (int32_t)__float_as_uint(e);
                    } else {
                        out_metric[f] = part;
                    }
                }
            }
        } else {
            // ---- column c of the failing frames (c < F L <= 2^30: 32-bit division)
            const uint32_t col = (uint32_t)((g - part1) >> pps);
            const uint32_t s = col / (uint32_t)L;
            const int k = (int)(col - s * (uint32_t)L);
            const int64_t f = fid[s];
            const uint32_t bits = inpos ? *(const uint16_t*)(anchors + ((size_t)f * L + k) * NB + 2 * piece) : 0u;
            int part = 0;
            if (!FLOAT) {
                v4i zv = v4i{0, 0, 0, 0};
                if (inpos) {
                    const v4i qv = *(const v4i*)((const int8_t*)llr + (size_t)f * N + j0);
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const uint32_t wq = mpwsd::read_q4((uint32_t)qv[d]);
                        const uint32_t nib = bits >> (4 * d);
                        part = mpwsd::masked_sum4(wq, nib, part);
                        zv[d] = (int)mpwsd::neg_bytes(wq, ~nib);  // -z: q where the bit is 1, -q where it is 0
                    }
                }
                *(v4i*)((int8_t*)zbuf + (size_t)col * KP + j0) = zv;
            } else if (inpos) {
                const float* y = (const float*)llr + (size_t)f * N + j0;
                float* z = (float*)zbuf + (size_t)col * N + j0;
#pragma unroll
                for (int j = 0; j < 16; ++j) z[j] = ((bits >> j) & 1) ? -y[j] : y[j];
            }
            for (int o = 1; o < PP; o <<= 1) part += __shfl_xor(part, o);
            if (inpos) *(uint16_t*)(cw + (size_t)col * NB + 2 * piece) = (uint16_t)bits;
            if (piece == 0) {
                act0[col] = (int32_t)col;
                tag[col] = 0;
                key64[col] = FLOAT ? ~0ull : (uint64_t)LLONG_MAX;
                if (!FLOAT) metric[col] = part;
            }
        }
    }
}

// ---------------------------------------------------------------- int8 search
// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8),
// and each XCD has its own L2.  The searches number their workgroups so that
// those of one XCD take consecutive work ranges: a column tile's -z, and the
// chunks it sweeps, are then fetched into one L2 instead of into several.
// A bijection of [0, gridDim.x) for any grid size.
__device__ inline int64_t xcd_block()
{
    constexpr int64_t X = 8;
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t per = G / X, rem = G % X, x = b % X;
    return x * per + (x < rem ? x : rem) + b / X;
}

// Unpack 32 bits (LSB first) into 32 bytes: a set bit becomes 0x80 (-128),
// a clear bit 0.  Each nibble, placed at bits 7..10, spreads to bit 7 of four
// bytes with one full-rate 24-bit multiply by 1 + 2^7 + 2^14 + 2^21 (the four
// shifted copies do not overlap).
__device__ inline void unpack32(uint32_t x, uint32_t (&o)[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t t7 = (k < 2 ? (x << (7 - 4 * k)) : (x >> (4 * k - 7))) & 0x780u;
        o[k] = __umul24(t7, 0x204081u) & 0x80808080u;
    }
}

// The sweep of one column tile of one code over move chunks [c0, c1): every
// wave keeps its columns' -z fragments in VGPRs, the workgroup stages the
// chunks through LDS, and each column's lexicographic (S, p) minimum over the
// range is folded into keys[column] with one atomicMin.
// pmap (or NULL): the index in the original table of row p of `moves`
// (ascending in p), rows at or past P map to pmap_pad.
template <int N, int NC, int NWAVES>
__device__ __forceinline__ void sweep_tile(int8_t* __restrict__ lds, const int8_t* __restrict__ z,
                                           const uint8_t* __restrict__ moves, int64_t P,
                                           const int32_t* __restrict__ act, int n, long long* __restrict__ keys,
                                           int tile, int c0, int c1, const int32_t* __restrict__ pmap,
                                           int64_t pmap_pad)
{
    constexpr int KP = N < 64 ? 64 : N;         // K padded to the MFMA depth
    constexpr int RS = KP + 16;                 // LDS row stride: conflict-free 16-byte reads
    constexpr int CT = NWAVES * 16 * NC;        // columns per tile
    constexpr int HK = KP / 64;                 // MFMAs per 16 x 16 output tile
    constexpr int NT = NWAVES * WAVE;
    constexpr int NB = N / 8;                   // packed bytes per move
    constexpr int UW = N / 32;                  // 32-bit units per move
    // chunk buffer b (0 or 1); computed from lds at every use so the compiler
    // keeps the LDS address space (ds_read/ds_write, not flat accesses)
    auto buf = [lds](int b) { return lds + b * (RC * RS); };

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const v4i seed0 = {4 * lg, 4 * lg + 1, 4 * lg + 2, 4 * lg + 3};

    if (N < KP) {  // positions >= N stay zero
        for (int e = tid; e < 2 * RC; e += NT) {
            int8_t* row = buf(e / RC) + (e % RC) * RS;
            for (int j = N; j < KP; j += 16) *(v4i*)(row + j) = v4i{0, 0, 0, 0};
        }
    }

    // this thread's share of a chunk: units of 32 packed bits
    constexpr int UR = (RC * KP / 32 + NT - 1) / NT;
    constexpr int units = RC * UW;
    auto fetch = [&](int chunk, uint32_t (&reg)[UR]) {
#pragma unroll
        for (int r = 0; r < UR; ++r) {
            const int u = tid + r * NT;
            reg[r] = 0;
            if (u < units) {
                const int row = u / UW, wd = u % UW;
                const int64_t p = (int64_t)chunk * RC + row;
                if (p < P) reg[r] = *(const uint32_t*)(moves + (size_t)p * NB + 4 * wd);
            }
        }
    };
    auto store = [&](int b, const uint32_t (&reg)[UR]) {
#pragma unroll
        for (int r = 0; r < UR; ++r) {
            const int u = tid + r * NT;
            if (u < units) {
                const int row = u / UW, wd = u % UW;
                uint32_t o[8];
                unpack32(reg[r], o);
                int8_t* dst = buf(b) + row * RS + 32 * wd;
                *(v4i*)(dst) = v4i{(int)o[0], (int)o[1], (int)o[2], (int)o[3]};
                *(v4i*)(dst + 16) = v4i{(int)o[4], (int)o[5], (int)o[6], (int)o[7]};
            }
        }
    };

    // -z fragments of this wave's columns; they stay in VGPRs for the sweep
    v4i zf[NC][HK];
    int colid[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int pos = tile * CT + wave * 16 * NC + c * 16 + li;
        colid[c] = pos < n ? act[pos] : -1;
#pragma unroll
        for (int h = 0; h < HK; ++h) {
            if (colid[c] >= 0)
                zf[c][h] = *(const v4i*)(z + (size_t)colid[c] * KP + lg * (KP / 4) + 16 * h);
            else
                zf[c][h] = v4i{0, 0, 0, 0};
        }
    }
    // Chunks are swept in decreasing order, so a chunk replaces the running
    // best when its minimum S is <= the best S (ties go to the lower chunk);
    // within a chunk D = 128 S + row orders by (S, row).
    int run[NC], runk[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) { run[c] = INT_MAX; runk[c] = 0; }

    uint32_t reg[UR];
    fetch(c1 - 1, reg);
    store(0, reg);
    __syncthreads();
    for (int k = c1 - 1; k >= c0; --k) {
        const int b = (c1 - 1 - k) & 1;
        if (k > c0) fetch(k - 1, reg);
        int cm[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) cm[c] = INT_MAX;
#pragma unroll 2
        for (int tt = 0; tt < RC / 16; ++tt) {
            v4i af[HK];
            const int8_t* src = buf(b) + (tt * 16 + li) * RS + lg * (KP / 4);
#pragma unroll
            for (int h = 0; h < HK; ++h) af[h] = *(const v4i*)(src + 16 * h);
            // accumulator seed: the row's index within the chunk
            const v4i seed = seed0 + v4i{16 * tt, 16 * tt, 16 * tt, 16 * tt};
            // all column blocks' MFMAs back to back into separate
            // accumulators, so the matrix pipe never waits on the epilogue
            v4i acc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[0], zf[c][0], seed, 0, 0, 0);
#pragma unroll
            for (int h = 1; h < HK; ++h)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[h], zf[c][h], acc[c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {  // two v_min3 per four values
                int t3 = min(min(acc[c][0], acc[c][1]), acc[c][2]);
                // keeps the compiler from rebalancing the two minima into three
                // instructions that each read matrix-core results
                asm volatile("" : "+v"(t3));
                cm[c] = min(min(cm[c], t3), acc[c][3]);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bool take = cm[c] <= (run[c] | 127);  // S(cm) <= S(run)
            run[c] = take ? cm[c] : run[c];
            runk[c] = take ? k : runk[c];
        }
        if (k > c0) store(b ^ 1, reg);
        __syncthreads();
    }
    // lanes li, li+16, li+32, li+48 hold the same column
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        int64_t p = (int64_t)((runk[c] << 7) | (run[c] & 127));
        if (pmap) p = p < P ? (int64_t)pmap[p] : pmap_pad;
        long long v = ((long long)(run[c] >> 7) << 32) | (long long)(uint32_t)p;
        long long o = __shfl_xor(v, 16);
        v = o < v ? o : v;
        o = __shfl_xor(v, 32);
        v = o < v ? o : v;
        if (lg == 0 && colid[c] >= 0) atomicMin(&keys[colid[c]], v);
    }
}

// ---------------------------------------------------------------- paired-half int8 search
// Tables of mpwsd_group_moves (layout in group.h): each 128-row chunk has one
// normal u, and each row of N/2 bits is scored against both halves of every
// column's z, {u.x = 0} and {u.x = 1}.  A lane group holds N/8 positions of
// each half among its own N/4 positions, so the two half fragments are
// gathered from the lane's canonical -z with one v_perm_b32 per output dword
// whenever the normal changes.  Rows are sorted by canonical index for both
// halves, so D = 128 S + row still picks the smallest index inside a
// (chunk, half); across chunks and halves, equal minima are settled by the
// canonical indices themselves.
struct PwTable {
    const int32_t* u;       // [chunks]
    const uint8_t* rows;    // [chunks][128][N/2]
    const int32_t* canon;   // [chunks][2][128]
    const int32_t* sel;     // [N/4][N/4] byte selectors per normal
    int chunks;
    const uint8_t* xrows;   // [extras][N/8] moves kept apart (plain rows)
    const int32_t* xcanon;  // [extras] their indices in the original table
    int extras;
};

PwTable pw_table(const uint8_t* grouped, int m, int64_t chunks, int64_t extras)
{
    const mpwsd::GroupLayout g = mpwsd::group_layout(m, chunks, extras);
    return PwTable{(const int32_t*)(grouped + g.u_off), grouped + g.rows_off, (const int32_t*)(grouped + g.canon_off),
                   (const int32_t*)(grouped + g.sel_off), (int)chunks, grouped + g.xrows_off,
                   (const int32_t*)(grouped + g.xcanon_off), (int)extras};
}

template <int WDW, int S>
__device__ __forceinline__ void pw_gather(const uint32_t* zc, const uint32_t (&f0)[WDW], const uint32_t (&f1)[WDW],
                                          v4i* zw0, v4i* zw1)
{
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
        const int lo = ((k >> S) << (S + 1)) | (k & ((1 << S) - 1));
        const int hi = lo + (1 << S);
        zw0[k >> 2][k & 3] = (int)__builtin_amdgcn_perm(zc[hi], zc[lo], f0[k]);
        zw1[k >> 2][k & 3] = (int)__builtin_amdgcn_perm(zc[hi], zc[lo], f1[k]);
    }
}

template <int WDW, int S>
__device__ __forceinline__ void pw_scatter(const v4i* zw0, const v4i* zw1, const uint32_t (&inv)[2 * WDW],
                                           uint32_t* zc)
{
#pragma unroll
    for (int k = 0; k < WDW; ++k) {
        const int lo = ((k >> S) << (S + 1)) | (k & ((1 << S) - 1));
        const int hi = lo + (1 << S);
        zc[lo] = __builtin_amdgcn_perm((uint32_t)zw1[k >> 2][k & 3], (uint32_t)zw0[k >> 2][k & 3], inv[lo]);
        zc[hi] = __builtin_amdgcn_perm((uint32_t)zw1[k >> 2][k & 3], (uint32_t)zw0[k >> 2][k & 3], inv[hi]);
    }
}

// Re-gathers the half fragments of every column block for a new normal:
// back to the canonical -z with the old normal's inverse selectors, then the
// new halves (first == true: the canonical -z is loaded from z instead).
// The selectors come from the table (scalar loads, wave-uniform).
template <int N, int NC, int HW>
__device__ __forceinline__ void pw_renormal(v4i (&zw)[2][NC][HW], const int32_t* __restrict__ sel, int old_u, int u,
                                            bool first, int lg, const int8_t* __restrict__ z, const int (&colid)[NC])
{
    constexpr int LB = N / 4, LDW = LB / 4, WDW = LDW / 2, SELW = N / 4;
    typedef const __attribute__((address_space(4))) int32_t* const_i32;
    const const_i32 sn = (const_i32)sel + u * SELW;
    const int Sn = sn[0];
    uint32_t f0[WDW], f1[WDW];
#pragma unroll
    for (int q = 0; q < WDW; ++q) {
        f0[q] = (uint32_t)sn[1 + q];
        f1[q] = (uint32_t)sn[1 + WDW + q];
    }
    if (first) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            uint32_t zc[LDW];
#pragma unroll
            for (int d = 0; d < LDW / 4; ++d) {
                v4i v = v4i{0, 0, 0, 0};
                if (colid[c] >= 0) v = *(const v4i*)(z + (size_t)colid[c] * N + lg * LB + 16 * d);
#pragma unroll
                for (int e = 0; e < 4; ++e) zc[4 * d + e] = (uint32_t)v[e];
            }
            switch (Sn) {
            case 0: pw_gather<WDW, 0>(zc, f0, f1, zw[0][c], zw[1][c]); break;
            case 1: pw_gather<WDW, 1>(zc, f0, f1, zw[0][c], zw[1][c]); break;
            case 2: pw_gather<WDW, 2>(zc, f0, f1, zw[0][c], zw[1][c]); break;
            default:
                if constexpr (WDW >= 8) pw_gather<WDW, 3>(zc, f0, f1, zw[0][c], zw[1][c]);
                break;
            }
        }
        return;
    }
    const const_i32 so = (const_i32)sel + old_u * SELW;
    const int So = so[0];
    uint32_t inv[LDW];
#pragma unroll
    for (int q = 0; q < LDW; ++q) inv[q] = (uint32_t)so[1 + 2 * WDW + q];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        uint32_t zc[LDW];
        switch (So) {
        case 0: pw_scatter<WDW, 0>(zw[0][c], zw[1][c], inv, zc); break;
        case 1: pw_scatter<WDW, 1>(zw[0][c], zw[1][c], inv, zc); break;
        case 2: pw_scatter<WDW, 2>(zw[0][c], zw[1][c], inv, zc); break;
        default:
            if constexpr (WDW >= 8) pw_scatter<WDW, 3>(zw[0][c], zw[1][c], inv, zc);
            break;
        }
        switch (Sn) {
        case 0: pw_gather<WDW, 0>(zc, f0, f1, zw[0][c], zw[1][c]); break;
        case 1: pw_gather<WDW, 1>(zc, f0, f1, zw[0][c], zw[1][c]); break;
        case 2: pw_gather<WDW, 2>(zc, f0, f1, zw[0][c], zw[1][c]); break;
        default:
            if constexpr (WDW >= 8) pw_gather<WDW, 3>(zc, f0, f1, zw[0][c], zw[1][c]);
            break;
        }
    }
}

// Chunks are swept in increasing order in groups of up to PW_GROUP chunks of
// one normal.  A lane sees rows 16 tt + 4 lg + j (tt < 8, j < 4) of a chunk,
// so its accumulator seed 32 q + 4 tt + j (q: the chunk's place in the group)
// orders its rows of the group by chunk and row, i.e. canonically for both
// halves; a group's minima are folded into the running best, with the
// canonical indices from LDS, once per group.
constexpr int PW_GROUP = 4;
constexpr int PW_CSLOTS = 8;  // chunks whose canonical indices stay in LDS
constexpr int PW_NBUF = 3;    // row buffers: two chunks are loaded ahead

template <int N, int NC, int NWAVES>
__device__ __forceinline__ void sweep_tile_pw(int8_t* __restrict__ lds, const int8_t* __restrict__ z, const PwTable& g,
                                              const int32_t* __restrict__ act, int n, long long* __restrict__ keys,
                                              int tile, int c0, int c1)
{
    constexpr int KW = N / 2;      // positions per half = bytes per row
    constexpr int HW = KW / 64;    // MFMAs per 16 x 16 output tile and half
    constexpr int CT = NWAVES * 16 * NC;
    constexpr int NI = RC * KW / 1024;  // 1 KB direct-to-LDS loads per chunk of rows
    static_assert(NI % NWAVES == 0 && 64 % NWAVES == 0, "loads per wave");
    // vector-memory operations of one wave per chunk: its rows and its share
    // of the canonical indices
    constexpr int VM_PER_CHUNK = NI / NWAVES + 1;
    // row buffer b (0 .. PW_NBUF-1), rows stored as in the table (swizzled
    // segments); canonical indices of chunk k in slot k % PW_CSLOTS
    auto buf = [lds](int b) { return lds + b * (RC * KW); };
    auto cbuf = [lds](int slot) { return (int32_t*)(lds + PW_NBUF * (RC * KW)) + slot * (2 * RC); };
    typedef __attribute__((address_space(3))) void* lds_ptr;
    typedef const __attribute__((address_space(4))) int32_t* const_i32;
    const const_i32 ut = (const_i32)g.u;  // normals: read-only, scalar loads

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    // LDS offset of this lane's A fragment hh of a 16-row tile (row li of the
    // tile; the swizzle depends on li only, as tiles start at multiples of 16)
    const int swz = (li / (256 / KW)) % (KW / 16);
    int aoff[HW];
#pragma unroll
    for (int hh = 0; hh < HW; ++hh) aoff[hh] = li * KW + 16 * ((lg * (KW / 64) + hh) ^ swz);

    // rows and canonical indices of a chunk are copied into LDS by the
    // direct-to-LDS loads, PW_NBUF - 1 chunks ahead: the copy's latency is
    // longer than one chunk's arithmetic
    auto fetch = [&](int chunk, int b, int slot) {
        for (int i = wave; i < NI; i += NWAVES)
            __builtin_amdgcn_global_load_lds(g.rows + (size_t)chunk * RC * KW + i * 1024 + lane * 16,
                                             (lds_ptr)(buf(b) + i * 1024), 16, 0, 0);
        constexpr int CL = 64 / NWAVES;  // lanes per wave for the 1 KB of indices
        if (lane < CL)
            __builtin_amdgcn_global_load_lds(g.canon + (size_t)chunk * 2 * RC + wave * CL * 4 + lane * 4,
                                             (lds_ptr)(cbuf(slot) + wave * CL * 4), 16, 0, 0);
    };
    // wait until at most n chunks' loads of this wave are in flight
    auto wait_chunks = [](int n) {
        constexpr int e = 0x7 << 4, l = 0xF << 8;  // no wait on export / LDS counters
        if (n >= 1) {
            constexpr int v = VM_PER_CHUNK;
            __builtin_amdgcn_s_waitcnt((v & 0xF) | ((v >> 4) << 14) | e | l);
        } else {
            __builtin_amdgcn_s_waitcnt(e | l);
        }
    };

    int colid[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int pos = tile * CT + wave * 16 * NC + c * 16 + li;
        colid[c] = pos < n ? act[pos] : -1;
    }

    // the two half fragments of this wave's columns (the canonical -z: lane
    // group lg holds positions [lg N/4, (lg + 1) N/4))
    v4i zw[2][NC][HW];
    // running best per column block: (S << 32 | canonical index)
    long long run[NC];
    // group minima per half and column block: 128 S + seed
    int cm[2][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        run[c] = LLONG_MAX;
        cm[0][c] = cm[1][c] = INT_MAX;
    }
    int gs = c0, gq = 0;  // first chunk and size of the open group
    auto flush = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int seed = cm[h][c] & 127;
                const int row = ((seed << 2) & 0x70) | (lg << 2) | (seed & 3);
                const int slot = (gs + (seed >> 5)) & (PW_CSLOTS - 1);
                const int cn = cbuf(slot)[h * RC + row];
                const long long key = ((long long)(cm[h][c] >> 7) << 32) | (long long)(uint32_t)cn;
                run[c] = key < run[c] ? key : run[c];
                cm[h][c] = INT_MAX;
            }
    };

    static_assert(PW_NBUF == 3, "two chunks in flight");
    fetch(c0, 0, c0 & (PW_CSLOTS - 1));
    if (c0 + 1 < c1) fetch(c0 + 1, 1, (c0 + 1) & (PW_CSLOTS - 1));
    wait_chunks(c0 + 1 < c1 ? 1 : 0);
    int u_k = ut[c0];
    int u_n1 = c0 + 1 < c1 ? ut[c0 + 1] : 0;
    int cur_u = u_k;
    pw_renormal<N, NC, HW>(zw, g.sel, 0, u_k, true, lg, z, colid);
    __syncthreads();
    int b = 0;  // buffer of chunk k
    for (int k = c0; k < c1; ++k) {
        const int u = u_k;
        int u_n2 = 0;
        if (k + 2 < c1) {
            const int b2 = b >= 1 ? b - 1 : 2;  // (b + 2) % 3
            fetch(k + 2, b2, (k + 2) & (PW_CSLOTS - 1));
            u_n2 = ut[k + 2];
        }
        if (u != cur_u || gq == PW_GROUP) {
            if (gq > 0) flush();
            gs = k;
            gq = 0;
        }
        if (u != cur_u) {
            pw_renormal<N, NC, HW>(zw, g.sel, cur_u, u, false, lg, z, colid);
            cur_u = u;
        }
        // seeds 32 gq + 4 tt + j, advanced by 64-bit adds
        unsigned long long s01 = ((unsigned long long)(32 * gq + 1) << 32) | (unsigned)(32 * gq);
        unsigned long long s23 = ((unsigned long long)(32 * gq + 3) << 32) | (unsigned)(32 * gq + 2);
        // two 16-row steps at a time: their 8 values per column and half are
        // folded with 3 v_min3 that read matrix-core results and 1 that does
        // not (the reading ones cost matrix-pipe time); the A fragments of
        // the next pair of steps are read while this pair computes, into
        // alternating registers
        auto pair = [&](const v4i (&af)[2][HW]) {
            v4i acc[2][2][NC];  // [step][half][column block]
#pragma unroll
            for (int st = 0; st < 2; ++st) {
                const v4i seed = {(int)(uint32_t)s01, (int)(uint32_t)(s01 >> 32), (int)(uint32_t)s23,
                                  (int)(uint32_t)(s23 >> 32)};
                s01 += 0x0000000400000004ull;
                s23 += 0x0000000400000004ull;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        acc[st][h][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[st][0], zw[h][c][0], seed, 0, 0, 0);
#pragma unroll
                for (int hh = 1; hh < HW; ++hh)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            acc[st][h][c] =
                                __builtin_amdgcn_mfma_i32_16x16x64_i8(af[st][hh], zw[h][c][hh], acc[st][h][c], 0, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const v4i& x = acc[0][h][c];
                    const v4i& y = acc[1][h][c];
                    int t1 = min(min(x[0], x[1]), x[2]);
                    int t2 = min(min(x[3], y[0]), y[1]);
                    asm volatile("" : "+v"(t1), "+v"(t2));
                    int t3 = min(min(cm[h][c], y[2]), y[3]);
                    asm volatile("" : "+v"(t3));
                    cm[h][c] = min(min(t3, t1), t2);
                }
        };
        auto load_pair = [&](int tp, v4i (&a)[2][HW]) {
#pragma unroll
            for (int st = 0; st < 2; ++st)
#pragma unroll
                for (int hh = 0; hh < HW; ++hh) a[st][hh] = *(const v4i*)(buf(b) + (2 * tp + st) * 16 * KW + aoff[hh]);
        };
        static_assert(RC / 32 == 4, "four pairs of steps per chunk");
        v4i a0[2][HW], a1[2][HW];
        load_pair(0, a0);
        load_pair(1, a1);
        pair(a0);
        load_pair(2, a0);
        pair(a1);
        load_pair(3, a1);
        pair(a0);
        pair(a1);
        ++gq;
        // chunk k + 1 has landed in LDS (the direct loads count as vector
        // memory operations) before any wave goes on; chunk k + 2 may not
        wait_chunks(k + 2 < c1 ? 1 : 0);
        u_k = u_n1;
        u_n1 = u_n2;
        b = b == 2 ? 0 : b + 1;
        // every wave's LDS reads of this chunk are done (its buffer is the
        // next one to be refilled) and the loads above have landed; a plain
        // barrier, as a workgroup fence would also wait for chunk k + 2
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
    }
    flush();
    // lanes li, li+16, li+32, li+48 hold the same column
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        long long v = run[c];
        long long o = __shfl_xor(v, 16);
        v = o < v ? o : v;
        o = __shfl_xor(v, 32);
        v = o < v ? o : v;
        if (lg == 0 && colid[c] >= 0) atomicMin(&keys[colid[c]], v);
    }
}

// occupancy hint (minimum waves per SIMD) of the paired-half kernels: the two
// halves double the accumulators, so at most 3 (170 VGPRs), 2 for 8 column
// blocks or N = 256
template <int N, int NC, int BPC>
constexpr int pw_waves_per_simd() { return (NC >= 8 || N >= 256) ? 2 : (BPC > 3 ? 3 : BPC); }

template <int N, int NC, int NWAVES, int BPC>
__global__ __launch_bounds__(NWAVES * WAVE, (pw_waves_per_simd<N, NC, BPC>())) void search_pw_kernel(
    const int8_t* __restrict__ z, PwTable g, const int32_t* __restrict__ act, const int32_t* __restrict__ count,
    long long* __restrict__ keys)
{
    constexpr int CT = NWAVES * 16 * NC;
    __shared__ __attribute__((aligned(16))) int8_t lds[PW_NBUF * RC * (N / 2) + PW_CSLOTS * 2 * RC * 4];
    const int n = *count;
    if (n <= 0) return;
    const int tiles = (n + CT - 1) / CT;
    const int C = g.chunks;
    const int64_t U = (int64_t)tiles * C;
    const int64_t wg = xcd_block();
    int64_t u0 = U * wg / gridDim.x;
    const int64_t u1 = U * (wg + 1) / gridDim.x;
    while (u0 < u1) {
        const int tile = (int)(u0 / C);
        const int c0 = (int)(u0 % C);
        const int c1 = (int)std::min<int64_t>(C, c0 + (u1 - u0));
        u0 += c1 - c0;
        sweep_tile_pw<N, NC, NWAVES>(lds, z, g, act, n, keys, tile, c0, c1);
    }
}

// One code: (column tile x move chunk) units spread evenly over the grid.
template <int N, int NC, int NWAVES, int BPC>
__global__ __launch_bounds__(NWAVES * WAVE, BPC) void search_i8_kernel(
    const int8_t* __restrict__ z, const uint8_t* __restrict__ moves, int64_t P,
    const int32_t* __restrict__ act, const int32_t* __restrict__ count, long long* __restrict__ keys,
    const int32_t* __restrict__ pmap, int64_t pmap_pad)
{
    constexpr int KP = N < 64 ? 64 : N;
    constexpr int CT = NWAVES * 16 * NC;
    __shared__ __attribute__((aligned(16))) int8_t lds[2 * RC * (KP + 16)];
    const int n = *count;
    if (n <= 0) return;
    const int tiles = (n + CT - 1) / CT;
    const int C = (int)((P + RC - 1) / RC);
    const int64_t U = (int64_t)tiles * C;
    const int64_t wg = xcd_block();
    int64_t u0 = U * wg / gridDim.x;
    const int64_t u1 = U * (wg + 1) / gridDim.x;
    while (u0 < u1) {
        const int tile = (int)(u0 / C);
        const int c0 = (int)(u0 % C);
        const int c1 = (int)std::min<int64_t>(C, c0 + (u1 - u0));
        u0 += c1 - c0;
        sweep_tile<N, NC, NWAVES>(lds, z, moves, P, act, n, keys, tile, c0, c1, pmap, pmap_pad);
    }
}

// Several codes in one launch: the units of all segments are concatenated
// and spread over one persistent grid; a workgroup's range may cross from one
// code into the next.
struct SegSearch {
    const int8_t* z;
    const uint8_t* moves;
    int64_t P;
    const int32_t* act;
    const int32_t* count;
    long long* keys;
    int N;
    int grouped;  // 1: pw holds the paired-half table (N = 128 or 256)
    PwTable pw;
    const int32_t* pmap;  // plain rows only: indices of the rows, or NULL
    int64_t pmap_pad;
};
constexpr int kMaxSeg = 4;
struct MultiSearch {
    SegSearch s[kMaxSeg];
    int nseg;
};

template <int KPMAX, int NC, int NWAVES, int BPC>
__global__ __launch_bounds__(NWAVES * WAVE, BPC) void search_i8_multi_kernel(MultiSearch ms)
{
    constexpr int CT = NWAVES * 16 * NC;
    // the plain layout of KPMAX is larger than the paired-half one of KPMAX
    // with its chunk indices
    static_assert(2 * RC * (KPMAX + 16) >= PW_NBUF * RC * (KPMAX / 2) + PW_CSLOTS * 2 * RC * 4, "LDS");
    __shared__ __attribute__((aligned(16))) int8_t lds[2 * RC * (KPMAX + 16)];
    int64_t ustart[kMaxSeg + 1];
    int nn[kMaxSeg], cc[kMaxSeg];
    ustart[0] = 0;
#pragma unroll
    for (int i = 0; i < kMaxSeg; ++i) {
        const bool on = i < ms.nseg;
        nn[i] = on ? *ms.s[i].count : 0;
        cc[i] = on ? (ms.s[i].grouped ? ms.s[i].pw.chunks : (int)((ms.s[i].P + RC - 1) / RC)) : 1;
        const int tiles = (nn[i] + CT - 1) / CT;
        ustart[i + 1] = ustart[i] + (int64_t)tiles * cc[i];
    }
    const int64_t U = ustart[kMaxSeg];
    const int64_t wg = xcd_block();
    int64_t u0 = U * wg / gridDim.x;
    const int64_t u1 = U * (wg + 1) / gridDim.x;
    while (u0 < u1) {
        int si = 0;
#pragma unroll
        for (int i = 1; i < kMaxSeg; ++i) si = u0 >= ustart[i] ? i : si;
        const SegSearch& sg = ms.s[si];
        const int64_t local = u0 - ustart[si];
        const int C = cc[si];
        const int tile = (int)(local / C);
        const int c0 = (int)(local % C);
        const int c1 = (int)std::min<int64_t>(C, c0 + (u1 - u0));
        u0 += c1 - c0;
        if (sg.grouped) {
            if (sg.N == 128)
                sweep_tile_pw<128, NC, NWAVES>(lds, sg.z, sg.pw, sg.act, nn[si], sg.keys, tile, c0, c1);
            else if constexpr (KPMAX >= 256)
                sweep_tile_pw<256, (NC > 4 ? 4 : NC), NWAVES>(lds, sg.z, sg.pw, sg.act, nn[si], sg.keys, tile, c0,
                                                              c1);
            continue;
        }
        switch (sg.N) {
        case 32: sweep_tile<32, NC, NWAVES>(lds, sg.z, sg.moves, sg.P, sg.act, nn[si], sg.keys, tile, c0, c1, sg.pmap, sg.pmap_pad); break;
        case 64: sweep_tile<64, NC, NWAVES>(lds, sg.z, sg.moves, sg.P, sg.act, nn[si], sg.keys, tile, c0, c1, sg.pmap, sg.pmap_pad); break;
        case 128: sweep_tile<128, NC, NWAVES>(lds, sg.z, sg.moves, sg.P, sg.act, nn[si], sg.keys, tile, c0, c1, sg.pmap, sg.pmap_pad); break;
        default:
            if constexpr (KPMAX >= 256)
                sweep_tile<256, NC, NWAVES>(lds, sg.z, sg.moves, sg.P, sg.act, nn[si], sg.keys, tile, c0, c1,
                                            sg.pmap, sg.pmap_pad);
            break;
        }
    }
}

// ---------------------------------------------------------------- int8 resolve
// Thread per active column: the search left the exact (S_min, p*) in the
// key; when S_min < 0 the move is applied (centre bits flip, the stored -z
// changes sign on the move's support, M += S, p* logged), the -z column being
// read and written in independent 16-byte pieces, and the column is appended
// to the next active list with one atomic per wave.  (This is the form that
// searches every path; resolve_merge_kernel is the one that merges.)
__global__ __launch_bounds__(256) void resolve_i8_kernel(
    int8_t* __restrict__ z, uint8_t* __restrict__ cw, int32_t* __restrict__ metric, const uint8_t* __restrict__ moves,
    int N, int KP, int64_t P, const int32_t* __restrict__ act_in, int32_t* __restrict__ act_out,
    int32_t* __restrict__ hdr, int t, int T, long long* __restrict__ keys, const int32_t* __restrict__ fid, int L,
    int32_t* __restrict__ out_moves)
{
    const int lane = threadIdx.x & 63;
    const int n = hdr[ncol(t)];
    const int NB = N / 8;
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int pos = base + lane;
        bool moved = false;
        int col = 0;
        if (pos < n) {
            col = act_in[pos];
            const long long key = keys[col];
            keys[col] = LLONG_MAX;  // ready for the next iteration
            const int S = (int)(key >> 32);
            const int64_t p = (int64_t)(uint32_t)key;
            if (key != LLONG_MAX && S < 0) {
                if (p >= P) {
                    atomicAdd(&hdr[1], 1);
                } else {
                    mpwsd::apply_move_i8(moves + (size_t)p * NB, cw + (size_t)col * NB, z + (size_t)col * KP, N);
                    metric[col] += S;
                    if (out_moves) {
                        const int s = col / L, k = col % L;
                        out_moves[((size_t)fid[s] * L + k) * T + t] = (int32_t)p;
                    }
                    moved = true;
                }
            }
        }
        const uint64_t bal = __ballot(moved);
        int wbase = 0;
        if (lane == 0 && bal) wbase = atomicAdd(&hdr[ncol(t + 1)], __popcll(bal));
        wbase = __shfl(wbase, 0);
        if (moved) act_out[wbase + __popcll(bal & ((1ull << lane) - 1ull))] = col;
    }
}

// ---------------------------------------------------------------- float search
// Sequential binary32 sums in ascending position order, on the vector ALUs.
// Lanes map to columns (64 columns per wave, z columns in LDS as [pos][col]);
// the supports of a chunk of moves are staged in LDS and read by broadcast.
__device__ inline uint32_t orderable(float v)
{
    const uint32_t u = __float_as_uint(v + 0.0f);  // -0 -> +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One wave per workgroup: 64 columns, z held in LDS as [position][column]
// (N <= 256 floats per column), supports and weights of 64 moves staged per
// step (moves of any weight: tables of larger spheres mix weights).
template <int N>
__global__ __launch_bounds__(WAVE) void search_f32_kernel(const float* __restrict__ z, const uint8_t* __restrict__ moves,
                                                          int64_t P, const int32_t* __restrict__ act,
                                                          const int32_t* __restrict__ hdr, int t,
                                                          unsigned long long* __restrict__ keys)
{
    constexpr int CT = WAVE;  // columns per tile (one per lane)
    constexpr int MC = 64;    // moves per staged step
    constexpr int NB = N / 8;
    __shared__ float zs[N * CT];
    __shared__ uint8_t sup[MC * N];  // ascending supports
    __shared__ int wts[MC];           // their weights
    const int n = hdr[ncol(t)];
    if (n <= 0) return;
    const int lane = threadIdx.x;
    const int tiles = (n + CT - 1) / CT;
    const int C = (int)((P + MC - 1) / MC);
    const int64_t U = (int64_t)tiles * C;
    const int64_t wg = xcd_block();
    int64_t u0 = U * wg / gridDim.x;
    const int64_t u1 = U * (wg + 1) / gridDim.x;
    while (u0 < u1) {
        const int tile = (int)(u0 / C);
        const int c0 = (int)(u0 % C);
        const int c1 = (int)std::min<int64_t>(C, c0 + (u1 - u0));
        u0 += c1 - c0;
        const int pos = tile * CT + lane;
        const int col = pos < n ? act[pos] : -1;
        __syncthreads();
        for (int j = 0; j < N; ++j) zs[j * CT + lane] = col >= 0 ? z[(size_t)col * N + j] : 0.0f;
        unsigned long long best = ~0ull;
        for (int k = c0; k < c1; ++k) {
            __syncthreads();
            {   // lane q extracts the support of move k * MC + q in ascending order
                const int64_t p = (int64_t)k * MC + lane;
                if (p < P) {
                    const uint8_t* row = moves + (size_t)p * NB;
                    int cnt = 0;
                    for (int wd = 0; wd < N / 32; ++wd) {
                        uint32_t bits = *(const uint32_t*)(row + 4 * wd);
                        while (bits) {
                            sup[lane * N + cnt++] = (uint8_t)(32 * wd + __builtin_ctz(bits));
                            bits &= bits - 1;
                        }
                    }
                    wts[lane] = cnt;
                }
            }
            __syncthreads();
            const int pm = (int)std::min<int64_t>(MC, P - (int64_t)k * MC);
            for (int q = 0; q < pm; ++q) {
                const uint8_t* sp = sup + q * N;
                const int wq = wts[q];
                float s = zs[sp[0] * CT + lane];
                for (int i = 1; i < wq; ++i) s = __fadd_rn(s, zs[sp[i] * CT + lane]);
                const unsigned long long kk =
                    ((unsigned long long)orderable(s) << 32) | (unsigned long long)((int64_t)k * MC + q);
                best = kk < best ? kk : best;
            }
        }
        if (col >= 0) atomicMin(&keys[col], best);
    }
}

__global__ __launch_bounds__(256) void resolve_f32_kernel(
    float* __restrict__ z, uint8_t* __restrict__ cw, const uint8_t* __restrict__ moves, int N, int64_t P,
    const int32_t* __restrict__ act_in, int32_t* __restrict__ act_out, int32_t* __restrict__ hdr, int t, int T,
    unsigned long long* __restrict__ keys, const int32_t* __restrict__ fid, int L, int32_t* __restrict__ out_moves)
{
    const int lane = threadIdx.x & 63;
    const int NB = N / 8, NWD = N / 32;
    const int n = hdr[ncol(t)];
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int pos = base + lane;
        bool moved = false;
        int col = 0;
        if (pos < n) {
            col = act_in[pos];
            const unsigned long long key = keys[col];
            keys[col] = ~0ull;
            const uint32_t ob = (uint32_t)(key >> 32);
            // orderable(S) < orderable(+0) = 0x80000000 <=> S < 0
            if (key != ~0ull && ob < 0x80000000u) {
                const int64_t p = (int64_t)(key & 0xFFFFFFFFull);
                if (p >= P) {
                    atomicAdd(&hdr[1], 1);
                } else {
                    const uint32_t* mv = (const uint32_t*)(moves + (size_t)p * NB);
                    uint32_t* c32 = (uint32_t*)(cw + (size_t)col * NB);
                    float* zc = z + (size_t)col * N;
                    for (int wd = 0; wd < NWD; ++wd) {
                        uint32_t bits = mv[wd];
                        c32[wd] ^= bits;
                        while (bits) {
                            const int j = 32 * wd + __builtin_ctz(bits);
                            zc[j] = -zc[j];
                            bits &= bits - 1;
                        }
                    }
                    if (out_moves) {
                        const int s = col / L, k = col % L;
                        out_moves[((size_t)fid[s] * L + k) * T + t] = (int32_t)p;
                    }
                    moved = true;
                }
            }
        }
        const uint64_t bal = __ballot(moved);
        int wbase = 0;
        if (lane == 0 && bal) wbase = atomicAdd(&hdr[ncol(t + 1)], __popcll(bal));
        wbase = __shfl(wbase, 0);
        if (moved) act_out[wbase + __popcll(bal & ((1ull << lane) - 1ull))] = col;
    }
}

// ---------------------------------------------------------------- resolve with merging
// Paths of one frame that reach the same centre have the same future: the
// search of an iteration, the move it picks and whether the path stops are
// functions of the centre alone (z and M are).  This resolve applies the
// moves of iteration t frame by frame and, for t < T - 1, compares each path
// that moved with the other paths of its frame:
//   * at the centre of a path that did not move (it searched there, or at an
//     equal centre, and found no improving move) it would stop at t + 1: it
//     is not searched again, and its state is already final;
//   * at the centre of a moved path of smaller index ("leader") it follows
//     that path: it is not searched again, and select gives it the leader's
//     later moves;
//   * otherwise it goes on to iteration t + 1.
// Decisions, metrics and move logs are those of searching every path (ties
// go to the smaller path index, and a leader always has a smaller index than
// its followers); only the searched paths per iteration drop.
//
// tag[column]: >= 0 the last iteration the column was (or, equal to t + 1,
// will be) searched in; < 0 a follower, -1 - (first skipped iteration << 5 |
// leader).  A column is searched in iteration t iff its tag is t.
//
// Lanes are paths: LP = L rounded up to a power of two lanes per frame,
// 64 / LP frames per wave; the new centres stay in registers and are compared
// word by word across the frame's lanes.  The frames with a column left to
// search form the next frame list (all failing frames in iteration 0).
// Kept columns and frames are gathered in LDS and appended to the next lists
// with one global atomic per flush: a wave adds at most 64 of each per pass, a
// workgroup 256.
struct ResolveLds {
    static constexpr int KBUF = 1024;
    int32_t kcol[KBUF], kfrm[KBUF];
    int kcnt[2];
    unsigned long long kbase;
};

// The resolve of one segment by the workgroups bid = 0 .. nbid - 1 of a launch.
template <bool FLOAT, int NW>
__device__ __forceinline__ void resolve_merge_body(
    ResolveLds& sh, int bid, int nbid, void* __restrict__ zbuf, uint32_t* __restrict__ cw,
    int32_t* __restrict__ metric, const uint8_t* __restrict__ moves, int KP, int64_t P, int32_t* __restrict__ hdr,
    int t, int T, unsigned long long* __restrict__ keys, const int32_t* __restrict__ fid, int L, int LP,
    int32_t* __restrict__ out_moves, int32_t* __restrict__ tag, const int32_t* __restrict__ fl_in,
    int32_t* __restrict__ fl_out, int32_t* __restrict__ act_out, int fcap)
{
    constexpr int N = 32 * NW;
    typedef int v4i_t __attribute__((ext_vector_type(4)));
    constexpr int KBUF = ResolveLds::KBUF;
    int32_t* kcol = sh.kcol;
    int32_t* kfrm = sh.kfrm;
    int* kcnt = sh.kcnt;
    unsigned long long& kbase = sh.kbase;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per_wave = WAVE / LP;
    const int g = lane / LP, k = lane % LP, gbase = g * LP;
    const uint64_t gmask = ((1ull << LP) - 1ull) << gbase;
    const bool merge = t + 1 < T;
    const int fpb = (blockDim.x / WAVE) * per_wave;  // frames per workgroup pass
    // the first pass's list entry is read before the list length is known
    // (the two loads are in flight together); an entry past the length is
    // stale and unused.  fcap is the list's capacity.
    const int i0 = bid * fpb + wave * per_wave + g;
    int s_first = fl_in && i0 < fcap ? fl_in[i0] : i0;
    const int nfr = fl_in ? hdr[ncol(t) + 1] : hdr[0];
    if (threadIdx.x == 0) kcnt[0] = kcnt[1] = 0;
    __syncthreads();
    auto flush = [&]() {  // every thread of the workgroup, after a barrier
        const int nc = kcnt[0], nf = kcnt[1];
        if (threadIdx.x == 0)
            kbase = (nc | nf) ? atomicAdd(reinterpret_cast<unsigned long long*>(hdr + ncol(t + 1)),
                                          ((unsigned long long)nf << 32) | (unsigned long long)nc)
                              : 0ull;
        __syncthreads();
        const unsigned long long base = kbase;
        for (int x = threadIdx.x; x < nc; x += blockDim.x) act_out[(int)(uint32_t)base + x] = kcol[x];
        for (int x = threadIdx.x; x < nf; x += blockDim.x) fl_out[(int)(base >> 32) + x] = kfrm[x];
        __syncthreads();
        if (threadIdx.x == 0) kcnt[0] = kcnt[1] = 0;
        __syncthreads();
    };
    for (int b0 = bid * fpb; b0 < nfr; b0 += nbid * fpb) {  // the same passes for the whole workgroup
        const int i = b0 + wave * per_wave + g;
        const bool ok = i < nfr && k < L;
        const int s = !ok ? 0 : i == i0 ? s_first : fl_in ? fl_in[i] : i;
        const int64_t col = (int64_t)s * L + k;
        // every load that does not need the key is issued at once
        int tg = -1, M = 0, f = 0;
        unsigned long long key = 0;
        uint32_t c[NW] = {};
        v4i_t zv[2 * NW];
        if (ok) {
            tg = tag[col];
            key = keys[col];
#pragma unroll
            for (int w = 0; w < NW; ++w) c[w] = cw[(size_t)col * NW + w];
            if (!FLOAT) {
                M = metric[col];
                const v4i_t* zp = reinterpret_cast<const v4i_t*>((const int8_t*)zbuf + (size_t)col * KP);
#pragma unroll
                for (int q = 0; q < 2 * NW; ++q) zv[q] = zp[q];
            }
            if (out_moves) f = fid[s];
        }
        bool moved = false;
        int64_t p = 0;
        int S = 0;
        if (tg == t) {
            if (FLOAT) {
                keys[col] = ~0ull;
                // orderable(S) < orderable(+0) = 0x80000000 <=> S < 0
                moved = key != ~0ull && (uint32_t)(key >> 32) < 0x80000000u;
            } else {
                keys[col] = (unsigned long long)LLONG_MAX;
                S = (int)((long long)key >> 32);
                moved = (long long)key != LLONG_MAX && S < 0;
            }
            p = (int64_t)(key & 0xFFFFFFFFull);
            if (moved && p >= P) {
                atomicAdd(&hdr[1], 1);
                moved = false;
            }
        }
        if (moved) {
            const uint32_t* mv = reinterpret_cast<const uint32_t*>(moves + (size_t)p * (N / 8));
            uint32_t mb[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) mb[w] = mv[w];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                c[w] ^= mb[w];
                cw[(size_t)col * NW + w] = c[w];
            }
            if (FLOAT) {
                float* zc = (float*)zbuf + (size_t)col * N;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    for (uint32_t bits = mb[w]; bits; bits &= bits - 1) {
                        const int j = 32 * w + __builtin_ctz(bits);
                        zc[j] = -zc[j];
                    }
            } else {
                v4i_t* zp = reinterpret_cast<v4i_t*>((int8_t*)zbuf + (size_t)col * KP);
#pragma unroll
                for (int q = 0; q < 2 * NW; ++q) {
                    const uint32_t bits = mb[q >> 1] >> (16 * (q & 1));
#pragma unroll
                    for (int d = 0; d < 4; ++d) zv[q][d] = (int)mpwsd::neg_bytes((uint32_t)zv[q][d], bits >> (4 * d));
                    zp[q] = zv[q];
                }
                metric[col] = M + S;
            }
            if (out_moves) out_moves[((size_t)f * L + k) * T + t] = (int32_t)p;
        }
        if (merge) {
            const uint64_t mvb = __ballot(moved);
            bool keep = false;
            if (mvb) {
                const uint64_t stb = __ballot(tg >= 0 && !moved);
                bool stop = false;
                int lead = -1;
                for (int j = 0; j < L; ++j) {
                    bool eq = true;
#pragma unroll
                    for (int w = 0; w < NW; ++w) eq = (__shfl(c[w], gbase + j) == c[w]) && eq;
                    if (moved && eq && j != k) {
                        if ((stb >> (gbase + j)) & 1) stop = true;
                        else if (((mvb >> (gbase + j)) & 1) && j < k && lead < 0) lead = j;
                    }
                }
                keep = moved && !stop && lead < 0;
                if (keep) tag[col] = t + 1;
                else if (moved && !stop) tag[col] = -1 - (((t + 1) << 5) | lead);
            }
            // into the workgroup's buffers: one LDS atomic per wave and list
            const uint64_t kb = __ballot(keep);
            const uint64_t fb = __ballot(k == 0 && (kb & gmask) != 0);
            int cb = 0, fbs = 0;
            if (lane == 0 && kb) cb = atomicAdd(&kcnt[0], __popcll(kb));
            if (lane == 0 && fb) fbs = atomicAdd(&kcnt[1], __popcll(fb));
            cb = __shfl(cb, 0);
            fbs = __shfl(fbs, 0);
            if (keep) kcol[cb + __popcll(kb & ((1ull << lane) - 1ull))] = (int32_t)col;
            if ((fb >> lane) & 1) kfrm[fbs + __popcll(fb & ((1ull << lane) - 1ull))] = s;
        }
        __syncthreads();
        // every wave reads the counts between this barrier and the next one
        // (flush's first, or the one below), before any wave of the next pass
        // adds to them, so all waves take the same branch
        if (merge) {
            if (kcnt[0] > KBUF - 256 || kcnt[1] > KBUF - 256) flush();
            else __syncthreads();
        }
    }
    if (merge) flush();
}

template <bool FLOAT, int NW>
__global__ __launch_bounds__(256) void resolve_merge_kernel(
    void* __restrict__ zbuf, uint32_t* __restrict__ cw, int32_t* __restrict__ metric,
    const uint8_t* __restrict__ moves, int KP, int64_t P, int32_t* __restrict__ hdr, int t, int T,
    unsigned long long* __restrict__ keys, const int32_t* __restrict__ fid, int L, int LP,
    int32_t* __restrict__ out_moves, int32_t* __restrict__ tag, const int32_t* __restrict__ fl_in,
    int32_t* __restrict__ fl_out, int32_t* __restrict__ act_out, int fcap)
{
    __shared__ ResolveLds sh;
    resolve_merge_body<FLOAT, NW>(sh, blockIdx.x, gridDim.x, zbuf, cw, metric, moves, KP, P, hdr, t, T, keys, fid, L,
                                  LP, out_moves, tag, fl_in, fl_out, act_out, fcap);
}

// One resolve launch for the segments of a multi-code call: segment i takes
// the workgroups [b_end of segment i - 1, b_end of segment i).
struct SegResolve {
    void* z;
    uint32_t* cw;
    int32_t* metric;
    const uint8_t* moves;
    int64_t P;
    int32_t* hdr;
    unsigned long long* keys;
    const int32_t* fid;
    int32_t* out_moves;
    int32_t* tag;
    const int32_t* fl_in;
    int32_t* fl_out;
    int32_t* act_out;
    int KP, NW, fcap, b_end;
};
struct MultiResolve {
    SegResolve s[kMaxSeg];
    int nseg;
};

template <bool FLOAT>
__global__ __launch_bounds__(256) void resolve_merge_multi_kernel(MultiResolve mr, int t, int T, int L, int LP)
{
    __shared__ ResolveLds sh;
    int i = 0;
    while (i + 1 < mr.nseg && (int)blockIdx.x >= mr.s[i].b_end) ++i;
    const SegResolve& g = mr.s[i];
    const int b0 = i == 0 ? 0 : mr.s[i - 1].b_end;
    const int bid = (int)blockIdx.x - b0, nbid = g.b_end - b0;
#define MPWSD_RESOLVE_BODY(NW)                                                                                        resolve_merge_body<FLOAT, NW>(sh, bid, nbid, g.z, g.cw, g.metric, g.moves, g.KP, g.P, g.hdr, t, T, g.keys,                                       g.fid, L, LP, g.out_moves, g.tag, g.fl_in, g.fl_out, g.act_out, g.fcap)
    switch (g.NW) {  // uniform over the workgroup
    case 1: MPWSD_RESOLVE_BODY(1); break;
    case 2: MPWSD_RESOLVE_BODY(2); break;
    case 4: MPWSD_RESOLVE_BODY(4); break;
    default: MPWSD_RESOLVE_BODY(8); break;
    }
#undef MPWSD_RESOLVE_BODY
}

// ---------------------------------------------------------------- select
// Alg. 1 return step: per failing frame, the path of smallest metric, ties
// to the smallest path index.  With merging (tag != NULL) a follower ends
// where its chain of leaders ends, at the same metric and a larger index, so
// it is never the choice and is skipped; its move log takes the leaders'
// moves from the iteration it stopped being searched (entries that no
// follower's fix-up writes).
template <bool FLOAT>
__global__ void select_kernel(const void* __restrict__ llr, const int32_t* __restrict__ hdr,
                              const int32_t* __restrict__ fid, int L, int N, const int32_t* __restrict__ metric,
                              const uint8_t* __restrict__ cw, uint8_t* __restrict__ out_cw, int32_t* __restrict__ out_k,
                              int32_t* __restrict__ out_metric, int T, int32_t* __restrict__ stats,
                              const int32_t* __restrict__ tag, int32_t* __restrict__ out_moves)
{
    if (stats && blockIdx.x == 0) stats_add(hdr, T, stats);
    const int f2 = hdr[0];
    const int NB = N / 8;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < f2; s += gridDim.x * blockDim.x) {
        const int f = fid[s];
        uint32_t follower = 0;
        if (tag)
            for (int k = 0; k < L; ++k) {
                const int tg = tag[(size_t)s * L + k];
                if (tg >= 0) continue;
                follower |= 1u << k;
                if (!out_moves) continue;
                int from = (-1 - tg) >> 5, cur = (-1 - tg) & 31;
                for (int hop = 0; hop < L; ++hop) {
                    const int ct = tag[(size_t)s * L + cur];
                    const int upto = ct < 0 ? ((-1 - ct) >> 5) : T;
                    for (int u = from; u < upto; ++u)
                        out_moves[((size_t)f * L + k) * T + u] = out_moves[((size_t)f * L + cur) * T + u];
                    if (ct >= 0) break;
                    from = upto;
                    cur = (-1 - ct) & 31;
                }
            }
        int kb = 0;
        int32_t mb = 0;
        if (FLOAT) {
            const float* y = (const float*)llr + (size_t)f * N;
            float best = 0.0f;
            for (int k = 0; k < L; ++k) {
                if ((follower >> k) & 1) continue;
                const uint8_t* c = cw + ((size_t)s * L + k) * NB;
                float e = 0.0f;
                for (int j = 0; j < N; ++j) {
                    const float x = ((c[j >> 3] >> (j & 7)) & 1) ? -1.0f : 1.0f;
                    const float d = __fsub_rn(y[j], x);
                    e = __fadd_rn(e, __fmul_rn(d, d));
                }
                if (k == 0 || e < best) { best = e; kb = k; }
            }
            mb = (int32_t)__float_as_uint(best);
        } else {
            mb = metric[(size_t)s * L];
            for (int k = 1; k < L; ++k) {
                if ((follower >> k) & 1) continue;
                const int32_t v = metric[(size_t)s * L + k];
                if (v < mb) { mb = v; kb = k; }
            }
        }
        // NB is a multiple of 4; both rows are 4-byte aligned
        const uint32_t* c = reinterpret_cast<const uint32_t*>(cw + ((size_t)s * L + kb) * NB);
        uint32_t* o = reinterpret_cast<uint32_t*>(out_cw + (size_t)f * NB);
        for (int b = 0; b < NB / 4; ++b) o[b] = c[b];
        if (out_k) out_k[f] = kb;
        if (out_metric) out_metric[f] = mb;
    }
}

// ---------------------------------------------------------------- launches
// Tile shapes of the int8 search (column blocks per wave, waves per
// workgroup, default workgroups per CU).
struct Variant {
    int nc, nw, bpc;
};
constexpr Variant kVariants[] = {{8, 4, 2}, {4, 4, 4}, {4, 8, 2}, {8, 2, 4}, {2, 4, 4}, {3, 4, 4}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int default_variant(int N) { return N >= 256 ? 1 : 0; }

template <int N, int V>
void launch_search_i8_v(const int8_t* zneg, const uint8_t* moves, int64_t P, const int32_t* act,
                        const int32_t* count, long long* keys, hipStream_t s, int grid, const int32_t* pmap,
                        int64_t pmap_pad)
{
    constexpr Variant v = kVariants[V];
    hipLaunchKernelGGL((search_i8_kernel<N, v.nc, v.nw, v.bpc>), dim3(grid), dim3(v.nw * WAVE), 0, s, zneg, moves, P,
                       act, count, keys, pmap, pmap_pad);
}

// paired-half search: column blocks per wave capped at 4 for N = 256 (VGPRs)
template <int N, int V>
void launch_search_pw_v(const int8_t* zneg, const PwTable& g, const int32_t* act, const int32_t* count,
                        long long* keys, hipStream_t s, int grid)
{
    constexpr Variant v = kVariants[V];
    constexpr int nc = (N >= 256 && v.nc > 4) ? 4 : v.nc;
    hipLaunchKernelGGL((search_pw_kernel<N, nc, v.nw, v.bpc>), dim3(grid), dim3(v.nw * WAVE), 0, s, zneg, g, act,
                       count, keys);
}

template <int N>
void launch_search_pw_n(const int8_t* zneg, const PwTable& g, const int32_t* act, const int32_t* count,
                        long long* keys, hipStream_t s, int variant, int grid)
{
    switch (variant) {
    case 0: launch_search_pw_v<N, 0>(zneg, g, act, count, keys, s, grid); break;
    case 1: launch_search_pw_v<N, 1>(zneg, g, act, count, keys, s, grid); break;
    case 2: launch_search_pw_v<N, 2>(zneg, g, act, count, keys, s, grid); break;
    case 3: launch_search_pw_v<N, 3>(zneg, g, act, count, keys, s, grid); break;
    case 4: launch_search_pw_v<N, 4>(zneg, g, act, count, keys, s, grid); break;
    default: launch_search_pw_v<N, 5>(zneg, g, act, count, keys, s, grid); break;
    }
}

template <int N>
void launch_search_i8_n(const int8_t* zneg, const uint8_t* moves, int64_t P, const int32_t* act,
                        const int32_t* count, long long* keys, hipStream_t s, int variant, int grid,
                        const int32_t* pmap = nullptr, int64_t pmap_pad = 0)
{
    switch (variant) {
    case 0: launch_search_i8_v<N, 0>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    case 1: launch_search_i8_v<N, 1>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    case 2: launch_search_i8_v<N, 2>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    case 3: launch_search_i8_v<N, 3>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    case 4: launch_search_i8_v<N, 4>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    default: launch_search_i8_v<N, 5>(zneg, moves, P, act, count, keys, s, grid, pmap, pmap_pad); break;
    }
}

void launch_search_f32(const SegWs& w, const mpwsd_segment& sg, int t, hipStream_t s, int grid)
{
    const float* z = (const float*)w.z;
    unsigned long long* keys = (unsigned long long*)w.key64;
    switch (sg.m) {
    case 5: hipLaunchKernelGGL(search_f32_kernel<32>, dim3(grid), dim3(WAVE), 0, s, z, sg.moves, sg.P, w.act[t & 1], w.hdr, t, keys); break;
    case 6: hipLaunchKernelGGL(search_f32_kernel<64>, dim3(grid), dim3(WAVE), 0, s, z, sg.moves, sg.P, w.act[t & 1], w.hdr, t, keys); break;
    case 7: hipLaunchKernelGGL(search_f32_kernel<128>, dim3(grid), dim3(WAVE), 0, s, z, sg.moves, sg.P, w.act[t & 1], w.hdr, t, keys); break;
    default: hipLaunchKernelGGL(search_f32_kernel<256>, dim3(grid), dim3(WAVE), 0, s, z, sg.moves, sg.P, w.act[t & 1], w.hdr, t, keys); break;
    }
}

// The moves a paired-half layout keeps apart: plain rows, searched into the
// same keys with their original indices (ties meet the paired-half results in
// the same atomicMin).
void launch_extras(int N, const int8_t* zneg, const PwTable& g, int64_t P, const int32_t* act, const int32_t* count,
                   long long* keys, int variant, int blocks_per_cu, hipStream_t s)
{
    if (g.extras <= 0) return;
    const int var = variant >= 0 ? variant : default_variant(N);
    const int pfit = (160 * 1024) / (2 * RC * (kpad(N) + 16));
    const int grid = device_cus() * (blocks_per_cu > 0 ? std::min(blocks_per_cu, pfit) : std::min(kVariants[var].bpc, pfit));
    if (N == 128)
        launch_search_i8_n<128>(zneg, g.xrows, g.extras, act, count, keys, s, var, grid, g.xcanon, P);
    else
        launch_search_i8_n<256>(zneg, g.xrows, g.extras, act, count, keys, s, var, grid, g.xcanon, P);
}

template <int KPMAX, int V>
void launch_multi_v(const MultiSearch& ms, hipStream_t s, int grid)
{
    constexpr Variant v = kVariants[V];
    hipLaunchKernelGGL((search_i8_multi_kernel<KPMAX, v.nc, v.nw, v.bpc>), dim3(grid), dim3(v.nw * WAVE), 0, s, ms);
}

// variants 0..2 have a multi-code form; others fall back to the default
void launch_search_multi(const MultiSearch& ms, int maxN, int variant, int blocks_per_cu, hipStream_t s)
{
    const int cus = device_cus();
    const int kp = maxN <= 128 ? 128 : 256;
    int var = (variant >= 0 && variant <= 2) ? variant : default_variant(maxN);
    const int lds_fit = (160 * 1024) / (2 * RC * (kp + 16));
    const int grid = cus * (blocks_per_cu > 0 ? blocks_per_cu : std::min(kVariants[var].bpc, lds_fit));
    if (kp == 128) {
        switch (var) {
        case 0: launch_multi_v<128, 0>(ms, s, grid); break;
        case 1: launch_multi_v<128, 1>(ms, s, grid); break;
        default: launch_multi_v<128, 2>(ms, s, grid); break;
        }
    } else {
        switch (var) {
        case 0: launch_multi_v<256, 1>(ms, s, grid); break;  // NC = 8 does not fit N = 256 registers
        case 1: launch_multi_v<256, 1>(ms, s, grid); break;
        default: launch_multi_v<256, 2>(ms, s, grid); break;
        }
    }
}

// Phases of stage 2 for one segment.
// zero_stats: this is the first segment of the call, whose first kernel also
// clears the caller's statistics.
void seg_prologue(const mpwsd_segment& sg, int L, int T, const SegWs& w, int32_t* stats, bool zero_stats,
                  hipStream_t s)
{
    const int N = 1 << sg.m, KP = kpad(N);
    const bool fl = sg.dtype == MPWSD_F32;
    hipLaunchKernelGGL(hdr_zero_kernel, dim3(1), dim3(128), 0, s, w.hdr, hdr_len(T), zero_stats ? stats : nullptr,
                       2 + T);
    hipLaunchKernelGGL(compact_kernel, dim3((unsigned)((sg.F + 255) / 256)), dim3(256), 0, s, sg.crc_ok, sg.F, w.hdr,
                       w.fid, w.slot);
    const int64_t work = sg.F * (int64_t)(L + 1) * (KP / 16);  // upper bound on the items' threads
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 16 * device_cus()));
    if (fl)
        hipLaunchKernelGGL(init_kernel<true>, dim3(blocks), dim3(256), 0, s, sg.llr, sg.anchors, sg.F, L, T, N, KP,
                           w.hdr, w.slot, w.fid, w.act[0], w.key64, w.metric, w.tag, w.cw, w.z, sg.out_cw, sg.out_k,
                           sg.out_metric, sg.out_moves, stats);
    else
        hipLaunchKernelGGL(init_kernel<false>, dim3(blocks), dim3(256), 0, s, sg.llr, sg.anchors, sg.F, L, T, N, KP,
                           w.hdr, w.slot, w.fid, w.act[0], w.key64, w.metric, w.tag, w.cw, w.z, sg.out_cw, sg.out_k,
                           sg.out_metric, sg.out_moves, stats);
}

int lanes_per_frame(int L)
{
    int lp = 1;
    while (lp < L) lp <<= 1;
    return lp;
}

// Resolve of iteration t: with merging, frame by frame (resolve_merge_kernel),
// else column by column.
template <bool FLOAT>
void launch_resolve_merge(const mpwsd_segment& sg, int L, int T, const SegWs& w, int t, hipStream_t s)
{
    const int N = 1 << sg.m, KP = kpad(N);
    const int lp = lanes_per_frame(L);
    const int64_t frames_per_block = 4 * (WAVE / lp);
    const unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((sg.F + frames_per_block - 1) / frames_per_block, 4 * device_cus()));
    const int32_t* fl_in = t == 0 ? nullptr : w.fl[t & 1];
    int32_t* fl_out = w.fl[(t + 1) & 1];
    int32_t* act_out = w.act[(t + 1) & 1];
    unsigned long long* keys = (unsigned long long*)w.key64;
    uint32_t* cw = (uint32_t*)w.cw;
#define MPWSD_RESOLVE_MERGE(NW)                                                                                    \
    hipLaunchKernelGGL((resolve_merge_kernel<FLOAT, NW>), dim3(blocks), dim3(256), 0, s, w.z, cw, w.metric,       \
                       sg.moves, KP, sg.P, w.hdr, t, T, keys, w.fid, L, lp, sg.out_moves, w.tag, fl_in, fl_out,   \
                       act_out, (int)sg.F)
    switch (N) {
    case 32: MPWSD_RESOLVE_MERGE(1); break;
    case 64: MPWSD_RESOLVE_MERGE(2); break;
    case 128: MPWSD_RESOLVE_MERGE(4); break;
    default: MPWSD_RESOLVE_MERGE(8); break;
    }
#undef MPWSD_RESOLVE_MERGE
}

// The resolves of iteration t of every segment of a multi-code call in one
// launch (merging on), each segment with the grid its own launch would have.
template <bool FLOAT>
void launch_resolve_multi(const mpwsd_segment* segs, int nseg, int L, int T, const SegWs* w, int t, hipStream_t s)
{
    MultiResolve mr{};
    const int lp = lanes_per_frame(L);
    const int64_t frames_per_block = 4 * (WAVE / lp);
    int blocks = 0;
    for (int i = 0; i < nseg; ++i) {
        const mpwsd_segment& sg = segs[i];
        if (sg.F == 0) continue;
        const int N = 1 << sg.m;
        SegResolve& g = mr.s[mr.nseg++];
        g.z = w[i].z;
        g.cw = (uint32_t*)w[i].cw;
        g.metric = w[i].metric;
        g.moves = sg.moves;
        g.P = sg.P;
        g.hdr = w[i].hdr;
        g.keys = (unsigned long long*)w[i].key64;
        g.fid = w[i].fid;
        g.out_moves = sg.out_moves;
        g.tag = w[i].tag;
        g.fl_in = t == 0 ? nullptr : w[i].fl[t & 1];
        g.fl_out = w[i].fl[(t + 1) & 1];
        g.act_out = w[i].act[(t + 1) & 1];
        g.KP = kpad(N);
        g.NW = N / 32;
        g.fcap = (int)sg.F;
        blocks += (int)std::max<int64_t>(
            1, std::min<int64_t>((sg.F + frames_per_block - 1) / frames_per_block, 4 * device_cus()));
        g.b_end = blocks;
    }
    if (mr.nseg > 0)
        hipLaunchKernelGGL(resolve_merge_multi_kernel<FLOAT>, dim3((unsigned)blocks), dim3(256), 0, s, mr, t, T, L,
                           lp);
}

void seg_resolve(const mpwsd_segment& sg, int L, int T, const SegWs& w, int t, bool merge, hipStream_t s)
{
    if (merge) {
        if (sg.dtype == MPWSD_F32)
            launch_resolve_merge<true>(sg, L, T, w, t, s);
        else
            launch_resolve_merge<false>(sg, L, T, w, t, s);
        return;
    }
    const int N = 1 << sg.m, KP = kpad(N);
    const int resolve_blocks = device_cus() * 4;
    if (sg.dtype == MPWSD_F32)
        hipLaunchKernelGGL(resolve_f32_kernel, dim3(resolve_blocks), dim3(256), 0, s, (float*)w.z, w.cw, sg.moves, N,
                           sg.P, w.act[t & 1], w.act[(t + 1) & 1], w.hdr, t, T, (unsigned long long*)w.key64, w.fid,
                           L, sg.out_moves);
    else
        hipLaunchKernelGGL(resolve_i8_kernel, dim3(resolve_blocks), dim3(256), 0, s, (int8_t*)w.z, w.cw, w.metric,
                           sg.moves, N, KP, sg.P, w.act[t & 1], w.act[(t + 1) & 1], w.hdr, t, T,
                           (long long*)w.key64, w.fid, L, sg.out_moves);
}

void seg_epilogue(const mpwsd_segment& sg, int L, int T, const SegWs& w, bool merge, int32_t* stats, hipStream_t s)
{
    const int N = 1 << sg.m;
    const int32_t* tag = merge ? w.tag : nullptr;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((sg.F + 255) / 256, 4096));
    if (sg.dtype == MPWSD_F32)
        hipLaunchKernelGGL(select_kernel<true>, dim3(blocks), dim3(256), 0, s, sg.llr, w.hdr, w.fid, L, N, w.metric,
                           w.cw, sg.out_cw, sg.out_k, sg.out_metric, T, stats, tag, sg.out_moves);
    else
        hipLaunchKernelGGL(select_kernel<false>, dim3(blocks), dim3(256), 0, s, sg.llr, w.hdr, w.fid, L, N,
                           w.metric, w.cw, sg.out_cw, sg.out_k, sg.out_metric, T, stats, tag, sg.out_moves);
}

int run_segment(const mpwsd_segment& sg, int L, int T, const SegWs& w, int32_t* stats, bool zero_stats,
                hipEvent_t* ev, const int* variant, const int* blocks_per_cu, bool merge, hipStream_t s)
{
    const int N = 1 << sg.m;
    seg_prologue(sg, L, T, w, stats, zero_stats, s);
    for (int t = 0; t < T; ++t) {
        if (ev) (void)hipEventRecord(ev[2 * t], s);
        if (sg.dtype == MPWSD_F32)
            launch_search_f32(w, sg, t, s, device_cus() * 4);
        else
            mpwsd::launch_search_i8(N, (const int8_t*)w.z, sg.moves, sg.P, sg.grouped, sg.grouped_chunks,
                                    sg.grouped_extras, w.act[t & 1], w.hdr + ncol(t), (long long*)w.key64, variant[t],
                                    blocks_per_cu[t], s);
        if (ev) (void)hipEventRecord(ev[2 * t + 1], s);
        seg_resolve(sg, L, T, w, t, merge, s);
    }
    seg_epilogue(sg, L, T, w, merge, stats, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_decode_batch: %s", hipGetErrorString(e));
    return MPWSD_OK;
}

// Several int8 segments: every iteration's search of all codes is ONE launch,
// and so is its resolve (with merging).
int run_multi(const mpwsd_segment* segs, int nseg, int L, int T, const SegWs* w, int32_t* stats, hipEvent_t* ev,
              const int* variant, const int* blocks_per_cu, bool merge, hipStream_t s)
{
    MultiSearch base{};
    int owner[kMaxSeg];       // segment of each entry of the launch
    int apart[kMaxSeg];       // segments whose extra moves get launches of their own
    int napart = 0;
    int maxN = 0;
    for (int i = 0; i < nseg; ++i) {
        if (segs[i].F == 0) continue;
        seg_prologue(segs[i], L, T, w[i], stats, base.nseg == 0, s);
        owner[base.nseg] = i;
        SegSearch& g = base.s[base.nseg++];
        g.z = (const int8_t*)w[i].z;
        g.moves = segs[i].moves;
        g.P = segs[i].P;
        g.keys = (long long*)w[i].key64;
        g.N = 1 << segs[i].m;
        g.grouped = segs[i].grouped && (g.N == 128 || g.N == 256);
        g.pmap = nullptr;
        g.pmap_pad = 0;
        if (g.grouped)
            g.pw = pw_table(segs[i].grouped, segs[i].m, segs[i].grouped_chunks, segs[i].grouped_extras);
        maxN = std::max(maxN, g.N);
    }
    // extra moves of paired-half segments: entries of the same launch while
    // they fit, else a launch of their own
    for (int e = 0, ne = base.nseg; e < ne; ++e) {
        const SegSearch& g = base.s[e];
        if (!g.grouped || g.pw.extras <= 0) continue;
        if (base.nseg == kMaxSeg) {
            apart[napart++] = owner[e];
            continue;
        }
        owner[base.nseg] = owner[e];
        SegSearch& x = base.s[base.nseg++];
        x = g;
        x.grouped = 0;
        x.moves = g.pw.xrows;
        x.P = g.pw.extras;
        x.pmap = g.pw.xcanon;
        x.pmap_pad = g.P;
    }
    for (int t = 0; t < T; ++t) {
        MultiSearch ms = base;
        for (int e = 0; e < ms.nseg; ++e) {
            ms.s[e].act = w[owner[e]].act[t & 1];
            ms.s[e].count = w[owner[e]].hdr + ncol(t);
        }
        if (ev) (void)hipEventRecord(ev[2 * t], s);
        if (ms.nseg > 0) launch_search_multi(ms, maxN, variant[t], blocks_per_cu[t], s);
        for (int a = 0; a < napart; ++a) {
            const int i = apart[a];
            const int N = 1 << segs[i].m;
            launch_extras(N, (const int8_t*)w[i].z,
                          pw_table(segs[i].grouped, segs[i].m, segs[i].grouped_chunks, segs[i].grouped_extras),
                          segs[i].P, w[i].act[t & 1], w[i].hdr + ncol(t), (long long*)w[i].key64, -1, 0, s);
        }
        if (ev) (void)hipEventRecord(ev[2 * t + 1], s);
        if (merge) {
            launch_resolve_multi<false>(segs, nseg, L, T, w, t, s);  // int8: the only form of a multi-code call
        } else {
            for (int i = 0; i < nseg; ++i)
                if (segs[i].F > 0) seg_resolve(segs[i], L, T, w[i], t, merge, s);
        }
    }
    for (int i = 0; i < nseg; ++i)
        if (segs[i].F > 0) seg_epilogue(segs[i], L, T, w[i], merge, stats, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_decode_batch: %s", hipGetErrorString(e));
    return MPWSD_OK;
}

int validate(const mpwsd_segment* segs, int nseg, int L, int T, bool check_ptrs)
{
    using mpwsd::fail;
    if (!segs || nseg < 1) return fail(MPWSD_ERR_ARG, "mpwsd_decode_batch: need at least one segment");
    if (L < 1 || L > 32) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_decode_batch: need 1 <= L <= 32 (L=%d)", L);
    if (T < 1 || T > 64) return fail(MPWSD_ERR_UNSUPPORTED, "mpwsd_decode_batch: need 1 <= T <= 64 (T=%d)", T);
    for (int i = 0; i < nseg; ++i) {
        const mpwsd_segment& s = segs[i];
        if (s.m < 5 || s.m > 8 || s.r < 1 || s.r >= s.m)
            return fail(MPWSD_ERR_UNSUPPORTED, "segment %d: need 1 <= r < m, 5 <= m <= 8", i);
        if (s.dtype != MPWSD_I8 && s.dtype != MPWSD_F32) return fail(MPWSD_ERR_ARG, "segment %d: bad dtype", i);
        if (s.dtype != segs[0].dtype) return fail(MPWSD_ERR_ARG, "segment %d: all segments need the same dtype", i);
        if (s.F < 0) return fail(MPWSD_ERR_ARG, "segment %d: F < 0", i);
        if (s.P > mpwsd::kMaxMoves || !mpwsd::valid_move_count(s.r, s.m, s.P))
            return fail(MPWSD_ERR_ARG,
                        "segment %d: P=%lld is not the size of a move table of RM(%d,%d) (minimum-weight words: %lld)",
                        i, (long long)s.P, s.r, s.m, (long long)mpwsd::rm_min_weight_count(s.r, s.m));
        if (s.F * (int64_t)L > INT_MAX / 2) return fail(MPWSD_ERR_UNSUPPORTED, "segment %d: F * L too large", i);
        if (check_ptrs && s.F > 0 && (!s.moves || !s.llr || !s.anchors || !s.out_cw))
            return fail(MPWSD_ERR_ARG, "segment %d: null pointer", i);
        if (check_ptrs && (reinterpret_cast<uintptr_t>(s.moves) & 3u) != 0)
            return fail(MPWSD_ERR_ARG, "segment %d: moves must be 4-byte aligned", i);
        // int8 q is read 16 positions at a time, anchors and decisions in 2- and 4-byte words
        if (check_ptrs && (reinterpret_cast<uintptr_t>(s.llr) & (s.dtype == MPWSD_I8 ? 15u : 3u)) != 0)
            return fail(MPWSD_ERR_ARG, "segment %d: llr must be %d-byte aligned", i, s.dtype == MPWSD_I8 ? 16 : 4);
        if (check_ptrs && ((reinterpret_cast<uintptr_t>(s.anchors) | reinterpret_cast<uintptr_t>(s.out_cw)) & 3u) != 0)
            return fail(MPWSD_ERR_ARG, "segment %d: anchors and out_cw must be 4-byte aligned", i);
        if (s.grouped) {
            if (s.m < 7)
                return fail(MPWSD_ERR_ARG, "segment %d: a paired-half table needs m = 7 or 8", i);
            if (s.grouped_extras < 0 || s.grouped_extras > s.P)
                return fail(MPWSD_ERR_ARG, "segment %d: grouped_extras %lld out of range", i,
                            (long long)s.grouped_extras);
            if (s.grouped_chunks < mpwsd::group_min_chunks(s.P, s.grouped_extras) ||
                s.grouped_chunks > mpwsd::group_max_chunks(s.m, s.P))
                return fail(MPWSD_ERR_ARG, "segment %d: grouped_chunks %lld does not fit P = %lld", i,
                            (long long)s.grouped_chunks, (long long)s.P);
            if ((reinterpret_cast<uintptr_t>(s.grouped) & 255u) != 0)
                return fail(MPWSD_ERR_ARG, "segment %d: grouped must be 256-byte aligned", i);
        }
    }
    return MPWSD_OK;
}

}  // namespace

namespace mpwsd {
int device_cu_count() { return device_cus(); }

void launch_search_i8(int N, const int8_t* zneg, const uint8_t* moves, int64_t P, const uint8_t* grouped,
                      int64_t grouped_chunks, int64_t grouped_extras, const int32_t* act, const int32_t* count,
                      long long* keys, int variant, int blocks_per_cu, hipStream_t s)
{
    const int cus = device_cus();
    const bool pw = grouped && (N == 128 || N == 256);
    const int var = variant >= 0 ? variant : default_variant(N);
    // workgroups per CU: requested, else the variant's default capped by how
    // many fit in the 160 KB LDS of a CU
    const int lds_ws = pw ? PW_NBUF * RC * (N / 2) + PW_CSLOTS * 2 * RC * 4 : 2 * RC * (kpad(N) + 16);
    const int lds_fit = (160 * 1024) / lds_ws;
    const int grid = cus * (blocks_per_cu > 0 ? blocks_per_cu : std::min(kVariants[var].bpc, lds_fit));
    if (pw) {
        const PwTable g = pw_table(grouped, N == 128 ? 7 : 8, grouped_chunks, grouped_extras);
        if (g.chunks > 0) {
            if (N == 128)
                launch_search_pw_n<128>(zneg, g, act, count, keys, s, var, grid);
            else
                launch_search_pw_n<256>(zneg, g, act, count, keys, s, var, grid);
        }
        launch_extras(N, zneg, g, P, act, count, keys, variant, blocks_per_cu, s);
        return;
    }
    switch (N) {
    case 32: launch_search_i8_n<32>(zneg, moves, P, act, count, keys, s, var, grid); break;
    case 64: launch_search_i8_n<64>(zneg, moves, P, act, count, keys, s, var, grid); break;
    case 128: launch_search_i8_n<128>(zneg, moves, P, act, count, keys, s, var, grid); break;
    default: launch_search_i8_n<256>(zneg, moves, P, act, count, keys, s, var, grid); break;
    }
}
}  // namespace mpwsd

extern "C" size_t mpwsd_workspace_bytes(const mpwsd_segment* segs, int nseg, int L, int T)
{
    mpwsd::clear_error();
    if (validate(segs, nseg, L, T, false) != MPWSD_OK) return 0;
    size_t tot = 0;
    for (int i = 0; i < nseg; ++i) tot += carve(segs[i], L, T, nullptr).bytes;
    return tot;
}

namespace {
int decode(const mpwsd_segment* segs, int nseg, int L, int T, void* ws, size_t ws_bytes, int32_t* stats,
           const mpwsd_options* opt, hipStream_t stream)
{
    int rc = validate(segs, nseg, L, T, true);
    if (rc != MPWSD_OK) return rc;
    // search tiles of every iteration (T <= 64)
    int variant[64], bpc[64];
    for (int t = 0; t < T; ++t) {
        variant[t] = opt ? opt->search_variant : -1;
        bpc[t] = opt ? opt->blocks_per_cu : 0;
        if (opt && opt->iter_variant) variant[t] = opt->iter_variant[t];
        if (opt && opt->iter_blocks_per_cu) bpc[t] = opt->iter_blocks_per_cu[t];
        if (variant[t] < -1 || variant[t] >= kNumVariants)
            return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_decode_batch: search variant %d (iteration %d) out of range",
                               variant[t], t);
        if (bpc[t] < 0 || bpc[t] > 16)
            return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_decode_batch: blocks_per_cu %d (iteration %d) out of range",
                               bpc[t], t);
    }
    const bool merge = !(opt && opt->no_merge);
    size_t need = 0;
    for (int i = 0; i < nseg; ++i) need += carve(segs[i], L, T, nullptr).bytes;
    if (!ws || ws_bytes < need)
        return mpwsd::fail(MPWSD_ERR_SIZE, "mpwsd_decode_batch: workspace needs %zu bytes, got %zu", need, ws_bytes);
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
        return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_decode_batch: workspace must be 256-byte aligned");
    // the first non-empty segment's first kernel clears stats; with none, a
    // kernel of its own does
    bool any = false;
    for (int i = 0; i < nseg; ++i) any = any || segs[i].F > 0;
    if (stats && !any) hipLaunchKernelGGL(stats_zero_kernel, dim3(1), dim3(128), 0, stream, stats, 2 + T);
    uint8_t* base = (uint8_t*)ws;
    if (nseg > 1 && nseg <= kMaxSeg && segs[0].dtype == MPWSD_I8) {
        SegWs w[kMaxSeg];
        for (int i = 0; i < nseg; ++i) {
            w[i] = carve(segs[i], L, T, base);
            base += w[i].bytes;
        }
        return run_multi(segs, nseg, L, T, w, stats, (opt && opt->events) ? opt->events : nullptr, variant, bpc,
                         merge, stream);
    }
    bool first = true;
    for (int i = 0; i < nseg; ++i) {
        const SegWs w = carve(segs[i], L, T, base);
        base += w.bytes;
        if (segs[i].F == 0) continue;
        hipEvent_t* ev = (opt && opt->events) ? opt->events + (size_t)2 * T * i : nullptr;
        rc = run_segment(segs[i], L, T, w, stats, first, ev, variant, bpc, merge, stream);
        first = false;
        if (rc != MPWSD_OK) return rc;
    }
    return MPWSD_OK;
}
}  // namespace

extern "C" int mpwsd_decode_batch(const mpwsd_segment* segs, int nseg, int L, int T, void* ws, size_t ws_bytes,
                                  int32_t* stats, hipStream_t stream)
{
    mpwsd::clear_error();
    return decode(segs, nseg, L, T, ws, ws_bytes, stats, nullptr, stream);
}

// ---------------------------------------------------------------- no-alloc form
// The workspace of mpwsd_decode_batch_noalloc: a fixed device array of the
// library, one copy per GPU, held until the process ends.  Host code never
// passes its name to a kernel or a copy: the name is a host-side stand-in,
// and the device address of each GPU's copy is looked up once per device.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static_assert(kNoallocScratchBytes == MPWSD_NOALLOC_SCRATCH_BYTES, "scratch size as declared in mpwsd.h");
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (looked up on the
// first call on each device), or nullptr with the error recorded.
void* scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_decode_batch_noalloc: no current device (or device id >= %d)",
                    kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_decode_batch_noalloc: scratch address on device %d: %s", dev,
                        hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int mpwsd_decode_batch_noalloc(const mpwsd_segment* segs, int nseg, int L, int T, int32_t* stats,
                                          hipStream_t stream)
{
    mpwsd::clear_error();
    int rc = validate(segs, nseg, L, T, true);
    if (rc != MPWSD_OK) return rc;
    size_t need = 0;
    for (int i = 0; i < nseg; ++i) need += carve(segs[i], L, T, nullptr).bytes;
    if (need > kNoallocScratchBytes)
        return mpwsd::fail(MPWSD_ERR_SIZE,
                           "mpwsd_decode_batch_noalloc: these segments need %zu bytes of workspace, above the fixed "
                           "%zu (use mpwsd_decode_batch with a workspace of its size)",
                           need, kNoallocScratchBytes);
    void* ws = scratch_ptr();
    if (!ws) return MPWSD_ERR_DEVICE;
    return decode(segs, nseg, L, T, ws, kNoallocScratchBytes, stats, nullptr, stream);
}

extern "C" int mpwsd_decode_batch_ex(const mpwsd_segment* segs, int nseg, int L, int T, void* ws, size_t ws_bytes,
                                     int32_t* stats, const mpwsd_options* options, hipStream_t stream)
{
    mpwsd::clear_error();
    return decode(segs, nseg, L, T, ws, ws_bytes, stats, options, stream);
}

extern "C" int mpwsd_search_variants(mpwsd_variant_info* info, int cap)
{
    for (int i = 0; i < kNumVariants && info && i < cap; ++i)
        info[i] = mpwsd_variant_info{kVariants[i].nc, kVariants[i].nw, 16 * kVariants[i].nc * kVariants[i].nw,
                                     kVariants[i].bpc};
    return kNumVariants;
}
