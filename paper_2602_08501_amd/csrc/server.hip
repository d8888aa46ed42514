// Serving: continuous batching of arriving frames over persistent per-code
// state in a caller-provided device arena (see mpwsd.h).
//
// Per code the arena holds a pool of `capacity` frame slots; a frame's L
// paths are the columns slot * L + k.  Every tick enqueues, on the server's
// stream:
//   H2D of the newly admitted frames  -> quantize (per-frame scale)
//   -> stage 1 (mpwsd_stage1_scl on the contiguous new frames)
//   -> enter: decided frames emit a result record, the others' paths join
//      the active list that already holds older paths
//   -> one search over the whole active list -> resolve, frame by frame:
//      apply moves; a path that moved onto the centre of a path of its frame
//      that does not go on stops, one that moved onto the centre of a moving
//      path of smaller index follows it (equal centres have the same future,
//      and the follower can never be the frame's choice); when no path of a
//      frame goes on, the frame's decision is chosen and a record emitted
//   -> D2H of the result records.
// Paths that move, have iterations left and were not merged form the next
// tick's list, and their frames the next frame list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "apply.h"
#include "common.h"
#include "group.h"

namespace {


struct Record {
    int32_t slot, stage, k, metric;
    uint8_t cw[32];
};

// header words: records, errors, and per active list (two, ping-pong) the
// pair (columns, frames), 8-byte aligned so that one 64-bit atomic appends
// columns and frames together
enum { H_CCOUNT = 2, H_ERR = 3, H_LIST0 = 4, H_LIST1 = 6, H_WORDS = 64 };
__host__ __device__ inline int list_words(int which) { return which ? H_LIST1 : H_LIST0; }

// Position of this lane's item in a list appended to by the whole wave (one
// atomic per wave).  Every lane of the wave must call it.
__device__ inline int wave_append(bool flag, int32_t* counter)
{
    const uint64_t bal = __ballot(flag);
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(counter, __popcll(bal));
    base = __shfl(base, 0);
    return base + __popcll(bal & ((1ull << lane) - 1ull));
}

__global__ void srv_prep_kernel(int32_t* hdr, int nxt)
{
    if (threadIdx.x == 0) {
        hdr[list_words(nxt)] = 0;
        hdr[list_words(nxt) + 1] = 0;
        hdr[H_CCOUNT] = 0;
    }
}

__device__ inline uint32_t srv_quantize1(float v, float s, int32_t* __restrict__ hdr)
{
    if (!isfinite(v)) {
        atomicAdd(&hdr[H_ERR], 1);
        return 0u;
    }
    float t = rintf(__fmul_rn(v, s));
    t = fminf(fmaxf(t, -127.0f), 127.0f);
    return (uint32_t)(uint8_t)(int8_t)t;
}

// four values per thread (N is a multiple of 4, so a quadruple lies in one
// frame and shares its scale); staging buffers are 256-byte aligned
__global__ void srv_quantize_kernel(const float* __restrict__ y, const float* __restrict__ scale, int n, int N,
                                    int8_t* __restrict__ q, int32_t* __restrict__ hdr)
{
    const int64_t total4 = (int64_t)n * N / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = reinterpret_cast<const float4*>(y)[i];
        const float s = scale[(4 * i) / N];
        reinterpret_cast<uint32_t*>(q)[i] = srv_quantize1(v.x, s, hdr) | (srv_quantize1(v.y, s, hdr) << 8) |
                                            (srv_quantize1(v.z, s, hdr) << 16) | (srv_quantize1(v.w, s, hdr) << 24);
    }
}

// thread per (new frame, path); a frame's L threads are consecutive lanes
__global__ __launch_bounds__(256) void srv_enter_kernel(
    int n, int L, int N, int KP, const int8_t* __restrict__ q, const uint8_t* __restrict__ anc,
    const uint8_t* __restrict__ ok, const int32_t* __restrict__ newslot, uint8_t* __restrict__ cw,
    int8_t* __restrict__ zneg, int32_t* __restrict__ metric, int32_t* __restrict__ citer, long long* __restrict__ key,
    int32_t* __restrict__ tag, int32_t* __restrict__ act, int32_t* __restrict__ fl, int32_t* __restrict__ hdr, int cur,
    Record* __restrict__ rec)
{
    const int NB = N / 8;
    const int total = n * L;
    for (int base = blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total; base += gridDim.x * blockDim.x) {
        const int idx = base + (threadIdx.x & 63);
        const bool live = idx < total;
        const int i = live ? idx / L : 0, k = live ? idx % L : 0;
        const bool decided = live && ok[i];
        const uint8_t* a = anc + ((size_t)i * L + k) * NB;
        const int8_t* qi = q + (size_t)i * N;
        const int slot = live ? newslot[i] : 0;
        // the paths of the other new frames become active columns: centre
        // bits, -z and the metric, 16 positions (one 16-byte piece) at a time
        const bool join = live && !decided;
        const int col = slot * L + k;
        int m = 0;
        if (live && (!decided || k == 0)) {
            typedef int v4i_t __attribute__((ext_vector_type(4)));
            for (int j0 = 0; j0 < KP; j0 += 16) {
                const bool inpos = j0 < N;
                const uint32_t bits = inpos ? *(const uint16_t*)(a + j0 / 8) : 0u;
                const v4i_t qv = inpos ? *(const v4i_t*)(qi + j0) : v4i_t{0, 0, 0, 0};
                v4i_t zv;
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const uint32_t nib = bits >> (4 * d);
                    m = mpwsd::masked_sum4((uint32_t)qv[d], nib, m);
                    zv[d] = (int)mpwsd::neg_bytes((uint32_t)qv[d], ~nib);  // -z: q where the bit is 1, else -q
                }
                if (join) {
                    *(v4i_t*)(zneg + (size_t)col * KP + j0) = zv;
                    if (inpos) *(uint16_t*)(cw + (size_t)col * NB + j0 / 8) = (uint16_t)bits;
                }
            }
        }
        // a decided frame emits its result record
        const bool emit = decided && k == 0;
        const int rpos = wave_append(emit, &hdr[H_CCOUNT]);
        if (emit) {
            Record& r = rec[rpos];
            r.slot = slot;
            r.stage = 1;
            r.k = 0;
            r.metric = m;
            for (int b = 0; b < 32; ++b) r.cw[b] = b < NB ? a[b] : 0;
        }
        if (join) {
            metric[col] = m;
            citer[col] = 0;
            key[col] = LLONG_MAX;
            tag[col] = 1;
        }
        const int apos = wave_append(join, &hdr[list_words(cur)]);
        if (join) act[apos] = col;
        const int fpos = wave_append(join && k == 0, &hdr[list_words(cur) + 1]);
        if (join && k == 0) fl[fpos] = slot;
    }
}

// Frame by frame (L lanes per frame, L a power of two <= 32), over the
// frames that hold a searched path.  tag[column]: 1 searched this tick, 0
// stopped (final state), < 0 following another path of the frame.
__global__ __launch_bounds__(256) void srv_resolve_kernel(
    int L, int T, int N, int KP, int64_t P, const uint8_t* __restrict__ moves, uint8_t* __restrict__ cw,
    int8_t* __restrict__ zneg, int32_t* __restrict__ metric, int32_t* __restrict__ citer, long long* __restrict__ key,
    int32_t* __restrict__ tag, const int32_t* __restrict__ fl_in, int32_t* __restrict__ fl_out,
    int32_t* __restrict__ act_out, int32_t* __restrict__ hdr, int cur, Record* __restrict__ rec)
{
    const int NB = N / 8, NW = N / 32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per_wave = 64 / L;
    const int g = lane / L, k = lane % L, gbase = g * L;
    const uint64_t gmask = (L == 64 ? ~0ull : ((1ull << L) - 1ull)) << gbase;
    const int nfr = hdr[list_words(cur) + 1];
    const int step = gridDim.x * (blockDim.x / 64) * per_wave;
    for (int i0 = (blockIdx.x * (blockDim.x / 64) + wave) * per_wave; i0 < nfr; i0 += step) {
        const int i = i0 + g;
        const bool ok = i < nfr;
        const int slot = ok ? fl_in[i] : 0;
        const int col = slot * L + k;
        const int tg = ok ? tag[col] : -1;
        bool moved = false, cont = false;
        if (tg == 1) {
            const long long kv = key[col];
            key[col] = LLONG_MAX;
            const int S = (int)(kv >> 32);
            const int64_t p = (int64_t)(uint32_t)kv;
            moved = kv != LLONG_MAX && S < 0 && p < P;
            if (moved) {
                mpwsd::apply_move_i8(moves + (size_t)p * NB, cw + (size_t)col * NB, zneg + (size_t)col * KP, N);
                metric[col] += S;
                citer[col] += 1;
            }
            cont = moved && citer[col] < T;
        }
        // this lane's centre and metric (its own writes above)
        uint32_t c[8] = {};
        if (tg >= 0)
            for (int w = 0; w < NW; ++w) c[w] = reinterpret_cast<const uint32_t*>(cw)[(size_t)col * NW + w];
        const int mv = tg >= 0 ? metric[col] : INT_MAX;
        // merging: paths of the same frame share every tick, so a path that
        // goes on is compared with the paths that do not (their centres have
        // no improving move) and with the other paths that go on
        const uint64_t cb = __ballot(cont);
        bool stop = false;
        int lead = -1;
        if (cb) {
            const uint64_t sb = __ballot(tg >= 0 && !cont);
            for (int j = 0; j < L; ++j) {
                bool eq = true;
                for (int w = 0; w < 8; ++w)
                    if (w < NW) eq = (__shfl(c[w], gbase + j) == c[w]) && eq;
                if (cont && eq && j != k) {
                    if ((sb >> (gbase + j)) & 1) stop = true;
                    else if (((cb >> (gbase + j)) & 1) && j < k && lead < 0) lead = j;
                }
            }
        }
        const bool keep = cont && !stop && lead < 0;
        if (tg == 1) tag[col] = keep ? 1 : ((cont && !stop) ? -1 - lead : 0);
        // next column and frame lists: one 64-bit atomic per wave
        const uint64_t kb = __ballot(keep);
        const uint64_t fb = __ballot(k == 0 && ok && ((kb & gmask) != 0));
        unsigned long long base = 0;
        if (lane == 0 && kb)
            base = atomicAdd(reinterpret_cast<unsigned long long*>(hdr + list_words(cur ^ 1)),
                             ((unsigned long long)__popcll(fb) << 32) | (unsigned long long)__popcll(kb));
        base = __shfl(base, 0);
        if (keep) act_out[(int)(uint32_t)base + __popcll(kb & ((1ull << lane) - 1ull))] = col;
        if ((fb >> lane) & 1) fl_out[(int)(base >> 32) + __popcll(fb & ((1ull << lane) - 1ull))] = slot;
        // a frame with no path left to search takes the smallest metric among
        // its non-following paths, ties to the smallest index (Alg. 1)
        const bool done = ok && (kb & gmask) == 0;
        int kbst = 0, mb = INT_MAX;
        for (int j = 0; j < L; ++j) {
            const int v = __shfl(mv, gbase + j);
            if (v < mb) { mb = v; kbst = j; }
        }
        uint32_t cc[8] = {};
        for (int w = 0; w < 8; ++w)
            if (w < NW) cc[w] = __shfl(c[w], gbase + kbst);
        const bool emit = done && k == 0;
        const int rpos = wave_append(emit, &hdr[H_CCOUNT]);
        if (emit) {
            Record& r = rec[rpos];
            r.slot = slot;
            r.stage = 2;
            r.k = kbst;
            r.metric = mb;
            for (int b = 0; b < 32; ++b) r.cw[b] = b < NB ? (uint8_t)(cc[b >> 2] >> (8 * (b & 3))) : 0;
        }
    }
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct CodeLayout {
    size_t yst, sst, qst, ancst, okst, newslot, cw, zneg, metric, citer, key, tag, fl0, fl1, act0, act1, hdr, rec,
        bytes;
};

CodeLayout layout(const mpwsd_server_code& c)
{
    const size_t C = (size_t)c.capacity, N = (size_t)1 << c.m, KP = N < 64 ? 64 : N, L = (size_t)c.L;
    CodeLayout l{};
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += al(b); return o; };
    l.yst = take(C * N * 4);
    l.sst = take(C * 4);
    l.qst = take(C * N);
    l.ancst = take(C * L * N / 8);
    l.okst = take(C);
    l.newslot = take(C * 4);
    l.cw = take(C * L * N / 8);
    l.zneg = take(C * L * KP);
    l.metric = take(C * L * 4);
    l.citer = take(C * L * 4);
    l.key = take(C * L * 8);
    l.tag = take(C * L * 4);
    l.fl0 = take(C * 4);
    l.fl1 = take(C * 4);
    l.act0 = take(C * L * 4);
    l.act1 = take(C * L * 4);
    l.hdr = take(H_WORDS * 4);
    l.rec = take(C * sizeof(Record));
    l.bytes = off;
    return l;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Submitted frames not yet admitted, first in first out: blocks of B rows of
// N values, recycled through a short spare list, so that a growing backlog
// neither allocates per frame nor copies what is queued.
struct Waiting {
    static constexpr size_t B = 4096;  // rows per block
    static constexpr size_t kSpare = 16;
    struct Block {
        std::unique_ptr<float[]> y;  // [B][N]
        float scale[B];
        uint64_t tag[B];
        double t[B];
    };
    Waiting() = default;
    Waiting(const Waiting&) = delete;  // move-only (so is the code state that holds it)
    Waiting& operator=(const Waiting&) = delete;
    Waiting(Waiting&&) = default;
    Waiting& operator=(Waiting&&) = default;
    int N = 0;
    std::deque<std::unique_ptr<Block>> blocks;  // front: the oldest rows
    std::vector<std::unique_ptr<Block>> spare;
    size_t head = 0;   // first queued row in the front block
    size_t count = 0;  // queued rows
    size_t size() const { return count; }
    bool empty() const { return count == 0; }
    void push(const float* row, float sc, uint64_t tg, double ts)
    {
        const size_t pos = head + count;
        if (pos / B == blocks.size()) blocks.push_back(take());
        Block& b = *blocks[pos / B];
        const size_t k = pos % B;
        std::memcpy(&b.y[k * N], row, sizeof(float) * N);
        b.scale[k] = sc;
        b.tag[k] = tg;
        b.t[k] = ts;
        ++count;
    }
    // The blocks that hold the first n rows, and the first row's index in
    // the first of them.  Pushes only append (rows past the last queued one,
    // new blocks at the back), so these rows and blocks stay as they are
    // until pop: a reader may use them without the lock.
    size_t front_blocks(size_t n, std::vector<const Block*>* out) const
    {
        out->clear();
        for (size_t b = 0; n > 0 && b <= (head + n - 1) / B; ++b) out->push_back(blocks[b].get());
        return head;
    }
    void pop(size_t n)
    {
        head += n;
        count -= n;
        while (head >= B) {
            give(std::move(blocks.front()));
            blocks.pop_front();
            head -= B;
        }
        if (count == 0) {
            while (!blocks.empty()) {
                give(std::move(blocks.front()));
                blocks.pop_front();
            }
            head = 0;
        }
    }

private:
    std::unique_ptr<Block> take()
    {
        if (!spare.empty()) {
            std::unique_ptr<Block> b = std::move(spare.back());
            spare.pop_back();
            return b;
        }
        std::unique_ptr<Block> b(new Block);
        b->y.reset(new float[B * (size_t)N]);
        return b;
    }
    void give(std::unique_ptr<Block> b)
    {
        if (spare.size() < kSpare) spare.push_back(std::move(b));
    }
};

struct Code {
    mpwsd_server_code c;
    int N, KP, NB;
    CodeLayout lay;
    uint8_t* base;
    std::vector<int> free_slots;
    std::vector<uint64_t> slot_tag;
    std::vector<double> slot_t;
    // submissions may come from another thread than the ticks: the waiting
    // queue is the only state they share, under this lock
    std::unique_ptr<std::mutex> mu = std::make_unique<std::mutex>();
    Waiting waiting;
    std::vector<const Waiting::Block*> front;  // the ticking thread's view of the queue's front
    int in_slots = 0;  // admitted, not yet harvested
    int cur = 0;       // active list the next tick searches
    template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

struct TickBuf {
    hipEvent_t ev = nullptr;
    bool busy = false;
    struct PerCode {
        float* y = nullptr;       // pinned [capacity][N]
        float* scale = nullptr;   // pinned [capacity]
        int32_t* slot = nullptr;  // pinned [capacity]
        int32_t* hdr = nullptr;   // pinned [H_WORDS]
        Record* rec = nullptr;    // pinned [capacity]
        int maxrec = 0;
    };
    std::vector<PerCode> pc;
};

}  // namespace

struct mpwsd_server {
    std::vector<Code> codes;
    hipStream_t stream = nullptr;
    TickBuf ticks[2];
    int next_tick = 0;
    std::deque<mpwsd_result> done;
    std::atomic<int64_t> submitted{0};
    int64_t returned = 0;
};

namespace {

int check_codes(const mpwsd_server_code* codes, int ncodes)
{
    using mpwsd::fail;
    if (!codes || ncodes < 1 || ncodes > 16) return fail(MPWSD_ERR_ARG, "server: need 1..16 codes");
    for (int i = 0; i < ncodes; ++i) {
        const auto& c = codes[i];
        if (c.m < 5 || c.m > 8 || c.r < 1 || c.r >= c.m)
            return fail(MPWSD_ERR_UNSUPPORTED, "server code %d: need 1 <= r < m, 5 <= m <= 8", i);
        if (c.P > mpwsd::kMaxMoves || !mpwsd::valid_move_count(c.r, c.m, c.P))
            return fail(MPWSD_ERR_ARG, "server code %d: P=%lld is not the size of a move table of RM(%d,%d)", i,
                        (long long)c.P, c.r, c.m);
        if (c.L < 1 || c.L > 32 || (c.L & (c.L - 1)) || c.T < 1 || c.T > 64)
            return fail(MPWSD_ERR_UNSUPPORTED, "server code %d: L must be a power of two <= 32, 1 <= T <= 64", i);
        if (c.capacity < 1 || (int64_t)c.capacity * c.L > (1 << 26))
            return fail(MPWSD_ERR_ARG, "server code %d: bad capacity %d", i, c.capacity);
        if (!c.moves) return fail(MPWSD_ERR_ARG, "server code %d: moves is NULL", i);
        if (c.grouped) {
            if (c.m < 7) return fail(MPWSD_ERR_ARG, "server code %d: a paired-half table needs m = 7 or 8", i);
            if (c.grouped_extras < 0 || c.grouped_extras > c.P)
                return fail(MPWSD_ERR_ARG, "server code %d: grouped_extras %lld out of range", i,
                            (long long)c.grouped_extras);
            if (c.grouped_chunks < mpwsd::group_min_chunks(c.P, c.grouped_extras) ||
                c.grouped_chunks > mpwsd::group_max_chunks(c.m, c.P))
                return fail(MPWSD_ERR_ARG, "server code %d: grouped_chunks %lld does not fit P = %lld", i,
                            (long long)c.grouped_chunks, (long long)c.P);
            if ((reinterpret_cast<uintptr_t>(c.grouped) & 255u) != 0)
                return fail(MPWSD_ERR_ARG, "server code %d: grouped must be 256-byte aligned", i);
        }
    }
    return MPWSD_OK;
}

void harvest(mpwsd_server* s, TickBuf& tb)
{
    const double t = now_s();
    for (size_t ci = 0; ci < s->codes.size(); ++ci) {
        Code& c = s->codes[ci];
        TickBuf::PerCode& p = tb.pc[ci];
        const int nrec = std::min(p.hdr[H_CCOUNT], p.maxrec);
        for (int i = 0; i < nrec; ++i) {
            const Record& r = p.rec[i];
            mpwsd_result res{};
            res.tag = c.slot_tag[r.slot];
            res.code = (int32_t)ci;
            res.stage = r.stage;
            res.k = r.k;
            res.metric = r.metric;
            std::memcpy(res.cw, r.cw, sizeof res.cw);
            res.t_submit = c.slot_t[r.slot];
            res.t_done = t;
            s->done.push_back(res);
            c.free_slots.push_back(r.slot);
            --c.in_slots;
        }
    }
    tb.busy = false;
}

int enqueue_tick(mpwsd_server* s, TickBuf& tb)
{
    hipStream_t st = s->stream;
    for (size_t ci = 0; ci < s->codes.size(); ++ci) {
        Code& c = s->codes[ci];
        TickBuf::PerCode& p = tb.pc[ci];
        // the lock covers reading the queue's front, not the copies: a
        // submitting thread only appends meanwhile
        int n_new;
        size_t h;
        {
            std::lock_guard<std::mutex> lock(*c.mu);
            n_new = (int)std::min(c.waiting.size(), c.free_slots.size());
            h = c.waiting.front_blocks((size_t)n_new, &c.front);
        }
        for (int i = 0; i < n_new; ++i) {
            const size_t pos = h + (size_t)i, w = pos % Waiting::B;
            const Waiting::Block& b = *c.front[pos / Waiting::B];
            const int slot = c.free_slots.back();
            c.free_slots.pop_back();
            std::memcpy(p.y + (size_t)i * c.N, &b.y[w * c.N], sizeof(float) * c.N);
            p.scale[i] = b.scale[w];
            p.slot[i] = slot;
            c.slot_tag[slot] = b.tag[w];
            c.slot_t[slot] = b.t[w];
        }
        if (n_new > 0) {
            std::lock_guard<std::mutex> lock(*c.mu);
            c.waiting.pop((size_t)n_new);
        }
        c.in_slots += n_new;
        p.maxrec = c.in_slots;
        if (c.in_slots == 0) {
            p.hdr[H_CCOUNT] = 0;
            continue;
        }
        const int L = c.c.L, nxt = c.cur ^ 1;
        int32_t* hdr = c.at<int32_t>(c.lay.hdr);
        int32_t* act[2] = {c.at<int32_t>(c.lay.act0), c.at<int32_t>(c.lay.act1)};
        int32_t* fl[2] = {c.at<int32_t>(c.lay.fl0), c.at<int32_t>(c.lay.fl1)};
        hipLaunchKernelGGL(srv_prep_kernel, dim3(1), dim3(64), 0, st, hdr, nxt);
        if (n_new > 0) {
            (void)hipMemcpyAsync(c.at<float>(c.lay.yst), p.y, sizeof(float) * c.N * n_new, hipMemcpyHostToDevice, st);
            (void)hipMemcpyAsync(c.at<float>(c.lay.sst), p.scale, sizeof(float) * n_new, hipMemcpyHostToDevice, st);
            (void)hipMemcpyAsync(c.at<int32_t>(c.lay.newslot), p.slot, sizeof(int32_t) * n_new, hipMemcpyHostToDevice,
                                 st);
            const int64_t tot = (int64_t)n_new * c.N / 4;
            hipLaunchKernelGGL(srv_quantize_kernel, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 4096)),
                               dim3(256), 0, st, c.at<float>(c.lay.yst), c.at<float>(c.lay.sst), n_new, c.N,
                               c.at<int8_t>(c.lay.qst), hdr);
            int rc = mpwsd_stage1_scl(c.c.r, c.c.m, c.c.crc_len, c.c.crc_poly, L, c.at<int8_t>(c.lay.qst), MPWSD_I8,
                                      n_new, c.at<uint8_t>(c.lay.ancst), c.at<uint8_t>(c.lay.okst), nullptr, st);
            if (rc != MPWSD_OK) return rc;
            const int64_t work = (int64_t)n_new * L;
            hipLaunchKernelGGL(srv_enter_kernel, dim3((unsigned)std::min<int64_t>((work + 255) / 256, 4096)),
                               dim3(256), 0, st, n_new, L, c.N, c.KP, c.at<int8_t>(c.lay.qst),
                               c.at<uint8_t>(c.lay.ancst), c.at<uint8_t>(c.lay.okst), c.at<int32_t>(c.lay.newslot),
                               c.at<uint8_t>(c.lay.cw), c.at<int8_t>(c.lay.zneg), c.at<int32_t>(c.lay.metric),
                               c.at<int32_t>(c.lay.citer), c.at<long long>(c.lay.key), c.at<int32_t>(c.lay.tag),
                               act[c.cur], fl[c.cur], hdr, c.cur, c.at<Record>(c.lay.rec));
        }
        // one stage-2 iteration over every active path of this code
        mpwsd::launch_search_i8(c.N, c.at<int8_t>(c.lay.zneg), c.c.moves, c.c.P, c.c.grouped, c.c.grouped_chunks,
                                c.c.grouped_extras,
                                act[c.cur], hdr + list_words(c.cur), c.at<long long>(c.lay.key), -1, 0, st);
        const int frames_per_block = 4 * (64 / L);
        hipLaunchKernelGGL(srv_resolve_kernel,
                           dim3((unsigned)std::min((c.c.capacity + frames_per_block - 1) / frames_per_block, 2048)),
                           dim3(256), 0, st, L, c.c.T, c.N, c.KP, c.c.P, c.c.moves, c.at<uint8_t>(c.lay.cw),
                           c.at<int8_t>(c.lay.zneg), c.at<int32_t>(c.lay.metric), c.at<int32_t>(c.lay.citer),
                           c.at<long long>(c.lay.key), c.at<int32_t>(c.lay.tag), fl[c.cur], fl[nxt], act[nxt], hdr,
                           c.cur, c.at<Record>(c.lay.rec));
        (void)hipMemcpyAsync(p.hdr, hdr, sizeof(int32_t) * H_WORDS, hipMemcpyDeviceToHost, st);
        (void)hipMemcpyAsync(p.rec, c.at<Record>(c.lay.rec), sizeof(Record) * p.maxrec, hipMemcpyDeviceToHost, st);
        c.cur = nxt;
    }
    hipError_t e = hipEventRecord(tb.ev, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return mpwsd::fail(MPWSD_ERR_DEVICE, "mpwsd_server_tick: %s", hipGetErrorString(e));
    tb.busy = true;
    return MPWSD_OK;
}

}  // namespace

extern "C" size_t mpwsd_server_arena_bytes(const mpwsd_server_code* codes, int ncodes)
{
    mpwsd::clear_error();
    if (check_codes(codes, ncodes) != MPWSD_OK) return 0;
    size_t t = 0;
    for (int i = 0; i < ncodes; ++i) t += layout(codes[i]).bytes;
    return t;
}

extern "C" int mpwsd_server_create(const mpwsd_server_code* codes, int ncodes, void* arena, size_t arena_bytes,
                                   mpwsd_server** out)
{
    using mpwsd::fail;
    mpwsd::clear_error();
    int rc = check_codes(codes, ncodes);
    if (rc != MPWSD_OK) return rc;
    if (!out) return fail(MPWSD_ERR_ARG, "mpwsd_server_create: out is NULL");
    size_t need = 0;
    for (int i = 0; i < ncodes; ++i) need += layout(codes[i]).bytes;
    if (!arena || arena_bytes < need)
        return fail(MPWSD_ERR_SIZE, "mpwsd_server_create: arena needs %zu bytes, got %zu", need, arena_bytes);
    if ((reinterpret_cast<uintptr_t>(arena) & 255u) != 0)
        return fail(MPWSD_ERR_ARG, "mpwsd_server_create: arena must be 256-byte aligned");
    auto* s = new mpwsd_server();
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    uint8_t* base = (uint8_t*)arena;
    for (int i = 0; i < ncodes && e == hipSuccess; ++i) {
        Code c;
        c.c = codes[i];
        c.N = 1 << codes[i].m;
        c.waiting.N = c.N;
        c.KP = c.N < 64 ? 64 : c.N;
        c.NB = c.N / 8;
        c.lay = layout(codes[i]);
        c.base = base;
        base += c.lay.bytes;
        c.free_slots.resize(codes[i].capacity);
        for (int k = 0; k < codes[i].capacity; ++k) c.free_slots[k] = codes[i].capacity - 1 - k;
        c.slot_tag.assign(codes[i].capacity, 0);
        c.slot_t.assign(codes[i].capacity, 0.0);
        s->codes.push_back(std::move(c));
    }
    for (auto& tb : s->ticks) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&tb.ev, hipEventDisableTiming);
        tb.pc.resize(ncodes);
        for (int i = 0; i < ncodes && e == hipSuccess; ++i) {
            const Code& c = s->codes[i];
            const size_t C = (size_t)c.c.capacity;
            auto& p = tb.pc[i];
            e = hipHostMalloc((void**)&p.y, C * c.N * sizeof(float), hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void**)&p.scale, C * sizeof(float), hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void**)&p.slot, C * sizeof(int32_t), hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void**)&p.hdr, H_WORDS * sizeof(int32_t), hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void**)&p.rec, C * sizeof(Record), hipHostMallocDefault);
        }
    }
    // zero the per-code headers (counts) with a kernel, not a memset node
    for (auto& c : s->codes)
        if (e == hipSuccess) {
            hipLaunchKernelGGL(srv_prep_kernel, dim3(1), dim3(64), 0, s->stream, c.at<int32_t>(c.lay.hdr), 0);
            hipLaunchKernelGGL(srv_prep_kernel, dim3(1), dim3(64), 0, s->stream, c.at<int32_t>(c.lay.hdr), 1);
            e = hipGetLastError();
        }
    if (e != hipSuccess) {
        int r = fail(MPWSD_ERR_DEVICE, "mpwsd_server_create: %s", hipGetErrorString(e));
        mpwsd_server_destroy(s);
        return r;
    }
    *out = s;
    return MPWSD_OK;
}

extern "C" int mpwsd_server_submit(mpwsd_server* s, int code, int n, const float* y, const float* scale,
                                   const uint64_t* tags)
{
    using mpwsd::fail;
    mpwsd::clear_error();
    if (!s || code < 0 || code >= (int)s->codes.size() || n < 0 || (n > 0 && (!y || !scale || !tags)))
        return fail(MPWSD_ERR_ARG, "mpwsd_server_submit: bad arguments");
    Code& c = s->codes[code];
    const double t = now_s();
    {
        std::lock_guard<std::mutex> lock(*c.mu);
        for (int i = 0; i < n; ++i) c.waiting.push(y + (size_t)i * c.N, scale[i], tags[i], t);
    }
    s->submitted += n;
    return MPWSD_OK;
}

extern "C" int mpwsd_server_tick(mpwsd_server* s, int64_t* in_flight)
{
    mpwsd::clear_error();
    if (!s) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_server_tick: server is NULL");
    // harvest finished ticks in order
    for (int k = 0; k < 2; ++k) {
        TickBuf& tb = s->ticks[(s->next_tick + k) & 1];
        if (tb.busy && hipEventQuery(tb.ev) == hipSuccess) harvest(s, tb);
    }
    bool work = false;
    for (auto& c : s->codes) {
        if (c.in_slots > 0) {
            work = true;
            break;
        }
        std::lock_guard<std::mutex> lock(*c.mu);
        if (!c.waiting.empty()) {
            work = true;
            break;
        }
    }
    if (work) {
        TickBuf& tb = s->ticks[s->next_tick];
        if (tb.busy) {  // both in flight: wait for the older one
            (void)hipEventSynchronize(tb.ev);
            harvest(s, tb);
        }
        int rc = enqueue_tick(s, tb);
        if (rc != MPWSD_OK) return rc;
        s->next_tick ^= 1;
    }
    if (in_flight) *in_flight = s->submitted - s->returned;
    return MPWSD_OK;
}

extern "C" int mpwsd_server_poll(mpwsd_server* s, mpwsd_result* out, int cap)
{
    mpwsd::clear_error();
    if (!s || cap < 0 || (cap > 0 && !out)) return mpwsd::fail(MPWSD_ERR_ARG, "mpwsd_server_poll: bad arguments");
    int n = 0;
    while (n < cap && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    s->returned += n;
    return n;
}

extern "C" int mpwsd_server_destroy(mpwsd_server* s)
{
    mpwsd::clear_error();
    if (!s) return MPWSD_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& tb : s->ticks) {
        if (tb.ev) (void)hipEventDestroy(tb.ev);
        for (auto& p : tb.pc) {
            if (p.y) (void)hipHostFree(p.y);
            if (p.scale) (void)hipHostFree(p.scale);
            if (p.slot) (void)hipHostFree(p.slot);
            if (p.hdr) (void)hipHostFree(p.hdr);
            if (p.rec) (void)hipHostFree(p.rec);
        }
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return MPWSD_OK;
}

extern "C" int mpwsd_serve_trace(mpwsd_server* s, int64_t n, const int32_t* code, const int64_t* row,
                                 const float* scale, const double* arrival, const float* const* pools,
                                 mpwsd_result* out)
{
    using mpwsd::fail;
    mpwsd::clear_error();
    if (!s || n < 0 || (n > 0 && (!code || !row || !scale || !arrival || !pools || !out)))
        return fail(MPWSD_ERR_ARG, "mpwsd_serve_trace: bad arguments");
    for (int64_t i = 0; i < n; ++i)
        if (code[i] < 0 || code[i] >= (int)s->codes.size() || !pools[code[i]] || row[i] < 0 ||
            !(arrival[i] >= 0.0 && arrival[i] < 1e9))  // also rejects NaN: every arrival must come
            return fail(MPWSD_ERR_ARG, "mpwsd_serve_trace: bad trace entry %lld", (long long)i);
    const double t0 = now_s();
    // a producer thread submits each frame at its arrival time (as requests
    // arriving on their own threads would); this thread ticks and polls
    std::atomic<bool> stop{false};
    std::thread producer([&]() {
        const int nc = (int)s->codes.size();
        int64_t i = 0;
        while (i < n && !stop.load(std::memory_order_relaxed)) {
            const double wait = arrival[i] - (now_s() - t0);
            if (wait > 0.0) {
                if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 1e-4));
                continue;
            }
            // every frame that has arrived by now, one lock per code; each
            // frame carries its scheduled arrival as its submission time
            const double t = now_s() - t0;
            int64_t j = i;
            while (j < n && arrival[j] <= t) ++j;
            for (int c = 0; c < nc; ++c) {
                Code& cd = s->codes[c];
                std::lock_guard<std::mutex> lock(*cd.mu);
                for (int64_t f = i; f < j; ++f)
                    if (code[f] == c) cd.waiting.push(pools[c] + (size_t)row[f] * cd.N, scale[f], (uint64_t)f,
                                                      t0 + arrival[f]);
            }
            s->submitted += j - i;
            i = j;
        }
    });
    int rc = MPWSD_OK;
    int64_t got = 0;
    std::vector<mpwsd_result> buf(4096);
    while (got < n) {
        int64_t inflight = 0;
        rc = mpwsd_server_tick(s, &inflight);
        if (rc != MPWSD_OK) break;
        int k;
        while ((k = mpwsd_server_poll(s, buf.data(), (int)buf.size())) > 0) {
            for (int i = 0; i < k; ++i) {
                const int64_t tag = (int64_t)buf[i].tag;
                if (tag >= 0 && tag < n) out[tag] = buf[i];
            }
            got += k;
        }
        if (inflight == 0 && got < n) std::this_thread::sleep_for(std::chrono::microseconds(20));  // idle
    }
    stop.store(true);
    producer.join();
    return rc;
}
