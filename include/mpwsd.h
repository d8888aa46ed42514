/*
 * mpwsd.h - multipoint code-weight sphere decoding (MP-WSD) on AMD Instinct
 * MI355X (gfx950).
 *
 * The decoder of Jo, Choi, Kim and Lee, "Multipoint Code-Weight Sphere
 * Decoding: Parallel Near-ML Decoding for Short-Blocklength Codes", for
 * Reed-Muller codes RM(r, m) with 5 <= m <= 8 (N = 2^m = 32 ... 256):
 *   stage 1 (Sec. III-A): successive-cancellation list decoding with a CRC,
 *     or ordered-statistics decoding of order k;
 *   stage 2 (Sec. III-B, Alg. 1): for frames whose stage-1 CRC fails (or for
 *     every frame, in the always-on mode), L parallel greedy searches over a
 *     precomputed sphere S_rho(0) (Eq. (2)-(3)), each scoring every move by
 *     its correlation gain (Eq. (5)), followed by the choice of the best path.
 *
 * Conventions shared by every call
 *   - Bit vectors are packed least-significant-bit first: bit j of a vector
 *     of N bits is bit (j % 8) of byte j / 8; a vector occupies N/8 bytes.
 *   - Code RM(r, m) in Kronecker form: u in {0,1}^N, c = u F^{(x)m},
 *     F = [[1,0],[1,1]], natural index order.  Information positions are
 *     A = { i : popcount(i) >= m - r } in ascending order; information bit t
 *     of v = payload || crc is u_{A[t]}.
 *   - CRC (Sec. II-B, K' = K + K_crc): remainder of p(x) x^crc_len modulo
 *     g(x) (crc_poly includes the x^crc_len term; 0x43 is x^6 + x + 1),
 *     first bit = highest degree, no reflection, zero init, no final xor.
 *   - LLR inputs are either int8 q (dtype MPWSD_I8) or float y (MPWSD_F32),
 *     row-major [F][N].  A positive value favours bit 0 (x = 1 - 2c).
 *     int8 values are read in the symmetric range [-127, 127]: every call
 *     reads a q of -128 as -127 (mpwsd_quantize_llr never writes -128).  The
 *     symmetric range keeps the negation z = q (1 - 2c) exact in int8 and
 *     bounds every stage-1 value by 127 N.
 *   - Device pointers are plain device addresses (hipMalloc or a framework
 *     tensor); the caller owns every buffer.  The library allocates no device
 *     memory; all work is enqueued on the caller's stream and nothing
 *     synchronises it.  Its only process-wide host state is a set of memo
 *     tables filled once under a lock and never changed after: the weight
 *     distribution of each code whose sphere sizes were needed, and the
 *     compute-unit count of each device.  They affect no result.
 *   - Every call returns MPWSD_OK (0) or a negative error code; arguments are
 *     validated before anything is enqueued, and on error nothing is written.
 *     mpwsd_last_error() describes the last failure of the calling thread.
 *     Faults of enqueued kernels surface at the caller's stream sync.
 */
#ifndef MPWSD_H
#define MPWSD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MPWSD_OK = 0,
    MPWSD_ERR_ARG = -1,         /* null pointer, negative size, bad enum */
    MPWSD_ERR_SIZE = -2,        /* caller buffer or workspace too small */
    MPWSD_ERR_DEVICE = -3,      /* a HIP call failed while enqueueing */
    MPWSD_ERR_UNSUPPORTED = -4  /* parameters outside the supported range */
};

enum { MPWSD_I8 = 0, MPWSD_F32 = 1 };

/* Message for the last failed call on this thread ("" if none). */
const char* mpwsd_last_error(void);

/*
 * mpwsd_build_moves - the code-weight sphere S_1(0) without the zero word
 * (Sec. II-C, Eq. (2)-(3); precomputed once, Sec. III-B).
 *
 * For RM(r, m) with 1 <= r < m <= 8 these are the P minimum-weight
 * codewords, of weight w = 2^(m-r): the incidence vectors of the
 * (m-r)-dimensional flats of EG(m, 2), coordinate j being the point whose
 * bits are the bits of j.  They are written in canonical order: ascending
 * by the sorted support (j_1 < ... < j_w) compared lexicographically; a
 * move index anywhere in this API is a row of this table.
 *
 * moves: HOST buffer of cap_bytes bytes receiving P rows of N/8 bytes, or
 *        NULL to query the sizes only.
 * P, N, w: out (any may be NULL).
 * Errors: MPWSD_ERR_UNSUPPORTED for r, m out of range; MPWSD_ERR_SIZE when
 * moves != NULL and cap_bytes < P * N / 8 (sizes are still reported).
 * Host-only, thread-safe.
 */
int mpwsd_build_moves(int r, int m, uint8_t* moves, size_t cap_bytes,
                      int64_t* P, int* N, int* w);

/*
 * mpwsd_build_sphere - the code-weight sphere S_radius(0) without the zero
 * word (Sec. II-C, Eq. (1)-(2)): every nonzero codeword of RM(r, m) whose
 * weight is one of the `radius` smallest nonzero weights of the code (the
 * shells d_1 .. d_radius).  radius = 1 is mpwsd_build_moves.  For radius >= 2
 * the code must have dimension K <= 30 (the shells are found by visiting all
 * 2^K codewords on the host's threads; RM(2,7), K = 29, takes a few seconds).
 *
 * Rows are sorted by weight, then canonically as in mpwsd_build_moves, so the
 * first rows are the table of radius 1.  The stage-2 search treats every row
 * the same way whatever its weight (Eq. (5) holds for any move).
 *
 * moves: HOST buffer of cap_bytes bytes receiving P rows of N/8 bytes, or
 *        NULL to query the sizes only.
 * P, N, w_max (the largest weight in the table): out (any may be NULL).
 * Errors: MPWSD_ERR_UNSUPPORTED for r, m out of range or K > 30 with
 * radius >= 2; MPWSD_ERR_ARG when the code has fewer than `radius` nonzero
 * weights; MPWSD_ERR_SIZE as for mpwsd_build_moves.  Host-only, thread-safe.
 */
int mpwsd_build_sphere(int r, int m, int radius, uint8_t* moves, size_t cap_bytes,
                       int64_t* P, int* N, int* w_max);

/*
 * mpwsd_quantize_llr - int8 LLR quantizer (device):
 *   q[i] = clamp(round_half_even(fl32(y[i] * scale)), -127, 127)
 * with scale typically 8 / sigma^2 (four times the LLR 2y/sigma^2).
 * Non-finite y[i] gives q[i] = 0 and bumps *bad (if bad != NULL; device
 * int32, not cleared by this call).
 * y: device float[n]; q: device int8[n].
 */
int mpwsd_quantize_llr(const float* y, int64_t n, float scale, int8_t* q,
                       int32_t* bad, hipStream_t stream);

/*
 * mpwsd_stage1_scl - stage 1, Sec. III-A: min-sum successive-cancellation
 * list decoding with list size L on RM(r, m), then the CRC test of the most
 * reliable candidate.
 *
 * Decoder: f(a,b) = sgn(a) sgn(b) min(|a|,|b|) with sgn(0) = +1,
 * g(a,b,v) = b + (1-2v) a, hard decision HD(l) = 1 iff l < 0, path metric
 * PM += |l| when the bit taken differs from HD(l), frozen bits are 0.  At
 * an information bit the 2n children are ranked by (PM, parent slot, bit)
 * and the first min(L, 2n) survive in that order.  Integer LLRs are decoded
 * in exact int32 arithmetic, float LLRs in IEEE binary32 without
 * contraction.
 *
 * llr: device [F][N], int8 (MPWSD_I8, read in [-127, 127]) or float
 *      (MPWSD_F32).
 * anchors: device out [F][L][N/8]: the list in ascending (PM, slot) order,
 *          the initial list of Sec. III-B.
 * crc_ok: device out [F]: 1 iff the first list entry's information bits
 *         pass the CRC (the frame is decided by stage 1); 0 otherwise, and
 *         always 0 when crc_len == 0 (no CRC: every frame goes on).
 * pm: device out [F][L] path metrics (int32 or float bits), may be NULL.
 * Supported: 5 <= m <= 8, 1 <= r < m, L in {1,2,4,8,16,32} with L <= 2^K,
 * 0 <= crc_len <= min(16, K).
 */
int mpwsd_stage1_scl(int r, int m, int crc_len, uint32_t crc_poly, int L,
                     const void* llr, int dtype, int64_t F,
                     uint8_t* anchors, uint8_t* crc_ok, int32_t* pm,
                     hipStream_t stream);

/*
 * mpwsd_stage1_scl_quantized - the int8 stage 1 from received values:
 * mpwsd_quantize_llr(y, F N, scale, q, bad) followed by
 * mpwsd_stage1_scl(r, m, crc_len, crc_poly, L, q, MPWSD_I8, F, ...), with
 * the same outputs bit for bit, in one launch when y is 16-byte and q 4-byte
 * aligned (each wave quantizes the values it decodes and writes them to q
 * for stage 2), else as those two launches.
 *
 * y: device float [F][N]; scale: finite; q: device out int8 [F][N];
 * bad: device int32 counter of non-finite y (those give q = 0), or NULL.
 * Other arguments, outputs, supported range and errors as mpwsd_stage1_scl
 * (Sec. III-A), plus MPWSD_ERR_ARG for a non-finite scale or a null y / q.
 */
int mpwsd_stage1_scl_quantized(int r, int m, int crc_len, uint32_t crc_poly, int L,
                               const float* y, float scale, int64_t F, int8_t* q, int32_t* bad,
                               uint8_t* anchors, uint8_t* crc_ok, int32_t* pm,
                               hipStream_t stream);

/*
 * mpwsd_stage1_osd - stage 1 by ordered-statistics decoding of order k
 * (Sec. III-A; the OSD initialisation of Sec. IV-A, whose complexity is
 * sum_{i<=k} C(K, i) candidates, Table I).  No CRC is involved: stage 2 then
 * runs on every frame (always-on mode, Sec. III-C: pass crc_ok = NULL to
 * mpwsd_decode_batch).
 *
 * Per frame:
 *   1. positions ranked by reliability |llr_j|, largest first, ties to the
 *      smaller position;
 *   2. the most reliable basis: the first K positions in that order whose
 *      generator columns are independent;
 *   3. the candidates: for every set e of at most `order` basis indices, the
 *      codeword that equals the hard decisions (HD(l) = 1 iff l < 0) on the
 *      basis except at the indices in e; candidate numbers run by |e|, then
 *      by the sorted index tuple of e in lexicographic order;
 *   4. the anchors: the L candidates of smallest metric, ties to the smaller
 *      candidate number, in ascending order.  Metric: int8 input M(c) =
 *      sum_{c_j = 1} q_j (exact); float input ||y - x(c)||^2 in IEEE
 *      binary32, summed in ascending position order without contraction.
 *
 * llr: device [F][N], int8 (MPWSD_I8, read in [-127, 127]) or float
 *      (MPWSD_F32), finite.
 * anchors: device out [F][L][N/8] (bit j of a row is byte j/8, bit j%8).
 * metric: device out [F][L] int32 (float input: the binary32 bit pattern),
 *         or NULL.
 * Supported: 5 <= m <= 8, 1 <= r < m, K <= 64, 0 <= order <= 4, 1 <= L <= 32,
 * L <= sum_{i<=order} C(K, i), F <= INT_MAX.  Errors: MPWSD_ERR_UNSUPPORTED /
 * MPWSD_ERR_ARG before anything is enqueued, MPWSD_ERR_DEVICE on a launch
 * failure.
 */
int mpwsd_stage1_osd(int r, int m, int order, int L, const void* llr, int dtype, int64_t F,
                     uint8_t* anchors, int32_t* metric, hipStream_t stream);

/*
 * mpwsd_group_moves - the paired-half layout of a move table, for a faster
 * int8 search over the same moves (same results, bit for bit).
 *
 * The search scores every move against every path's z (Eq. (5)).  A move of
 * RM(r, m) that is a flat of EG(m, 2) (Sec. II-C: the minimum-weight words)
 * lies in one half {x : u.x = c} of the positions for every normal u
 * orthogonal to its direction space, and its translate by a unit vector e_i
 * with u_i = 1 lies in the other half with the same pattern.  This call
 * picks one normal per direction space and stores each pair of translates as
 * ONE row of N/2 bits, so the search multiplies rows of length N/2 against
 * both halves of every z: half the matrix-core work of the N-long rows.
 * Only normals below N/4 serve (the search gathers the halves without moving
 * data between lanes); the moves of a direction space with none (e.g. 4096
 * of the 10668 moves of RM(2, 7)) are kept apart in the layout, with their
 * indices, and searched with plain rows into the same results.
 *
 * m: 7 or 8.  moves: HOST [P][N/8], the table given to mpwsd_decode_batch
 * (canonical order of mpwsd_build_moves).  out: HOST buffer of cap_bytes
 * bytes, or NULL for a query; it receives a self-contained byte layout that
 * the caller copies verbatim to the device and passes as the grouped,
 * grouped_chunks and grouped_extras fields of a segment or server code.
 * *chunks, *extras and *bytes receive the number of 128-row chunks, of moves
 * kept apart and the layout's size.  Moves keep their indices: the move logs
 * and results do not change.
 *
 * Returns MPWSD_ERR_UNSUPPORTED when a move has no translate partner in the
 * table (e.g. radius >= 2 spheres): use the plain table then.  MPWSD_ERR_SIZE
 * when out is too small (sizes are still reported).  Host-only, thread-safe;
 * O(P N) time.
 */
int mpwsd_group_moves(int m, const uint8_t* moves, int64_t P, uint8_t* out, size_t cap_bytes,
                      int64_t* chunks, int64_t* extras, size_t* bytes);

/*
 * One group of frames of one code for stage 2.
 */
typedef struct mpwsd_segment {
    int r, m;                  /* code RM(r, m) */
    const uint8_t* moves;      /* device [P][N/8], the table of mpwsd_build_moves
                                  or mpwsd_build_sphere */
    int64_t P;                 /* number of moves: the size of one of those
                                  tables for RM(r, m) (checked; for a radius
                                  >= 2 table the first check of a code walks
                                  its 2^K codewords on the host once per
                                  process, as mpwsd_build_sphere does, which
                                  fills the same memo: build the table before
                                  recording a graph) */
    const void* llr;           /* device [F][N]: int8 q (16-byte aligned; read
                                  in [-127, 127]) or float y (4-byte aligned) */
    int dtype;                 /* MPWSD_I8 or MPWSD_F32 */
    int64_t F;                 /* frames */
    const uint8_t* anchors;    /* device [F][L][N/8], list of stage 1
                                  (4-byte aligned) */
    const uint8_t* crc_ok;     /* device [F]; 1 = decided by stage 1.  NULL:
                                  every frame goes to stage 2 (always-on) */
    uint8_t* out_cw;           /* device out [F][N/8]: decision for every frame
                                  (4-byte aligned) */
    int32_t* out_k;            /* device out [F]: chosen path (0 when stage 1
                                  decided); may be NULL */
    int32_t* out_metric;       /* device out [F]: metric of the decision (int8:
                                  M(c) = sum_{c_j=1} q_j; float: the bits of
                                  ||y - x(c)||^2 in binary32); may be NULL */
    int32_t* out_moves;        /* device out [F][L][T]: accepted move index per
                                  path and iteration, -1 = none; may be NULL */
    const uint8_t* grouped;    /* device copy of mpwsd_group_moves' layout of
                                  this same table (256-byte aligned), or NULL;
                                  used by the int8 search only */
    int64_t grouped_chunks;    /* its chunk count (0 when grouped is NULL) */
    int64_t grouped_extras;    /* its count of moves kept apart (0 when
                                  grouped is NULL) */
} mpwsd_segment;

/*
 * mpwsd_workspace_bytes - device workspace needed by mpwsd_decode_batch for
 * these segments, L and T (0 on invalid arguments; see mpwsd_last_error).
 */
size_t mpwsd_workspace_bytes(const mpwsd_segment* segs, int nseg, int L, int T);

/*
 * mpwsd_decode_batch - stage 2, Sec. III-B, Eq. (4)-(5), Alg. 1.
 *
 * Frames with crc_ok = 1 take their first anchor as the decision.  The
 * others are compacted on the device into one list, and each of their L
 * anchors starts a path.  In each of T iterations every active path with
 * centre c scores all P moves w_p by
 *     S_p = sum_{j in supp(w_p)} z_j,   z_j = llr_j (1 - 2 c_j)
 * (the squared distance changes by 4 S_p; S_p = -G(w_p)/2 of Eq. (5)),
 * takes the smallest p attaining min_p S_p, and moves to c xor w_p iff
 * S_p < 0; otherwise the path stops (a stopped path could never move
 * again).  The decision is the path with the smallest metric, ties to the
 * smallest path index.  In int8 mode all sums are exact integers; in float
 * mode S_p is summed in binary32 in ascending j and the final metric is
 * ||y - x(c)||^2 summed in binary32 in ascending j.
 *
 * Paths of one frame that reach the same centre are merged (unless
 * mpwsd_options.no_merge): what a path does next depends on its centre
 * alone, so after each iteration a path that moved onto the centre of a
 * path that did not move stops, and one that moved onto the centre of a
 * moved path of smaller index follows that path; neither is searched again.
 * At the end a follower is given its leader's later moves, centre and
 * metric, so every output equals that of searching all paths.
 *
 * Several int8 segments (up to 4, e.g. codes of different lengths) are
 * decoded together: each iteration searches the failing paths of all of them
 * in ONE launch of the search kernel.
 *
 * segs[nseg]: host array.  All segments must use the same dtype.
 * ws: device workspace of ws_bytes >= mpwsd_workspace_bytes(...) bytes.
 * stats: device out int32[2 + T] or NULL: [0] = frames sent to stage 2
 *        (summed over segments), [1 + t] = paths searched in iteration t
 *        (after merging),
 *        [1 + T] = internal consistency failures (0 expected).
 * Supported: 5 <= m <= 8, 1 <= r < m, 1 <= L <= 32, 1 <= T <= 64.
 */
int mpwsd_decode_batch(const mpwsd_segment* segs, int nseg, int L, int T,
                       void* ws, size_t ws_bytes, int32_t* stats,
                       hipStream_t stream);

/*
 * mpwsd_decode_batch_noalloc - mpwsd_decode_batch without a workspace
 * argument, for callers that cannot allocate device memory (code recorded
 * into a HIP graph, tight serving loops, hosts that forbid allocation).
 *
 * Same segments, L, T, stats, results and errors as mpwsd_decode_batch; the
 * workspace is instead a fixed array of MPWSD_NOALLOC_SCRATCH_BYTES bytes
 * inside the library, one per GPU, that each GPU holds from the library's
 * first use on it until the process ends.  The call allocates nothing:
 * no hipMalloc or hipFree and no allocating library routine; the first call
 * on a device looks up that device's array address once.
 *
 * Limit: MPWSD_ERR_SIZE (nothing enqueued) when mpwsd_workspace_bytes of
 * the same arguments exceeds MPWSD_NOALLOC_SCRATCH_BYTES (64 MiB: about
 * 49000 RM(3,7) frames at L = 8, or 13000 RM(3,8) frames at L = 16).
 * Every call on one GPU uses that GPU's single array, and nothing in it
 * carries over between calls: calls whose work may overlap on one GPU (on
 * different streams, or from several host threads) race and must be
 * serialised by the caller, e.g. by issuing them on one stream.
 */
#define MPWSD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mpwsd_decode_batch_noalloc(const mpwsd_segment* segs, int nseg, int L, int T,
                               int32_t* stats, hipStream_t stream);

/*
 * Tuning of the stage-2 move search.  The search kernel comes in a few tile
 * shapes ("variants": column blocks of 16 per wave x waves per workgroup);
 * all give bit-identical results, only their speed differs with the code
 * and the number of active paths.
 */
typedef struct mpwsd_variant_info {
    int col_blocks;      /* 16-column MFMA blocks held per wave */
    int waves;           /* waves per workgroup (they share each LDS move chunk) */
    int columns;         /* paths per workgroup tile = 16 * col_blocks * waves */
    int blocks_per_cu;   /* default workgroups per CU of the persistent grid */
} mpwsd_variant_info;

/* Number of search variants (>= 1); info[i] filled for i < min(n, cap). */
int mpwsd_search_variants(mpwsd_variant_info* info, int cap);

typedef struct mpwsd_options {
    int search_variant;  /* 0 .. n-1, or -1 for the library default */
    int blocks_per_cu;   /* persistent grid = CUs x this; 0 = the variant's default */
    hipEvent_t* events;  /* NULL, or nseg * 2 * T events created by the caller:
                            events[2 (s T + t)] is recorded right before and
                            events[2 (s T + t) + 1] right after the search
                            kernel of iteration t of segment s, on the same
                            stream, for timing with hipEventElapsedTime; when
                            several int8 segments share one search launch,
                            only events[2 t] and events[2 t + 1] are recorded */
    const int* iter_variant;        /* NULL, or T host entries: the tile variant of
                                       iteration t's search (-1: library default);
                                       overrides search_variant */
    const int* iter_blocks_per_cu;  /* NULL, or T host entries overriding
                                       blocks_per_cu per iteration */
    int no_merge;                   /* 1: search every active path in every
                                       iteration, also paths of one frame
                                       that have reached the same centre
                                       (same outputs, more searched paths) */
} mpwsd_options;

/*
 * mpwsd_decode_batch_ex - mpwsd_decode_batch with options (NULL = defaults).
 * Nothing is synchronised in either form.
 */
int mpwsd_decode_batch_ex(const mpwsd_segment* segs, int nseg, int L, int T,
                          void* ws, size_t ws_bytes, int32_t* stats,
                          const mpwsd_options* options, hipStream_t stream);

/*
 * Recorded pipelines (HIP graphs).  Every call of this library is safe to
 * record: kernel launches only, with all counts kept in device memory, no
 * host synchronisation and no memset nodes.
 *
 * mpwsd_graph_begin creates a private stream in capture mode and returns
 * it; the caller enqueues any sequence of mpwsd calls on it (nothing runs).
 * mpwsd_graph_end stops the recording, instantiates the graph and destroys
 * the stream.  mpwsd_graph_launch replays the recorded calls on a stream with
 * the same buffers and sizes.  The graph object owns host-side driver
 * resources only; buffers stay owned by the caller and must outlive it.
 */
typedef struct mpwsd_graph mpwsd_graph;
int mpwsd_graph_begin(hipStream_t* record_stream);
int mpwsd_graph_end(hipStream_t record_stream, mpwsd_graph** graph);
int mpwsd_graph_launch(const mpwsd_graph* graph, hipStream_t stream);
int mpwsd_graph_destroy(mpwsd_graph* graph);

/*
 * Serving: continuous batching of arriving frames (int8 LLRs).
 *
 * A server holds, per code, a pool of frame slots in a device arena the
 * caller provides (the memory gate: at most `capacity` frames of that code
 * are in flight).  Each tick
 *   1. admits waiting frames into free slots, uploads their received values,
 *      quantizes them with their own scale and runs stage 1 on them; frames
 *      whose best list entry passes the CRC complete in this tick;
 *   2. appends the L paths of the other new frames to the code's pool of
 *      active paths, which holds the paths of frames admitted in earlier
 *      ticks as well;
 *   3. runs ONE stage-2 iteration (search + apply) over the whole pool: new
 *      and old paths share the same launches;
 *   4. merges paths of a frame that reach the same centre, as
 *      mpwsd_decode_batch does, and completes every frame with no path left
 *      to search (each stopped: no improving move, T accepted moves, or at
 *      the centre of a path that stopped; or follows a path of smaller
 *      index), with the same choice rule as mpwsd_decode_batch, and frees
 *      its slot once the host has read it.
 * A frame's result therefore does not depend on which other frames share
 * its ticks: it equals mpwsd_decode_batch's result for that frame alone.
 * Ticks run asynchronously on the server's stream; up to two are in flight.
 */
typedef struct mpwsd_server mpwsd_server;

typedef struct mpwsd_server_code {
    int r, m;                /* RM(r, m), 5 <= m <= 8 */
    const uint8_t* moves;    /* device [P][N/8] move table (mpwsd_build_moves or
                                mpwsd_build_sphere) */
    int64_t P;
    int L, T;                /* list size (power of two <= 32), iterations */
    int crc_len;             /* CRC length (0: no CRC, every frame goes on) */
    uint32_t crc_poly;
    int capacity;            /* frames of this code in flight at most */
    const uint8_t* grouped;  /* device copy of mpwsd_group_moves' layout of the
                                table, or NULL (as in mpwsd_segment) */
    int64_t grouped_chunks;
    int64_t grouped_extras;
} mpwsd_server_code;

typedef struct mpwsd_result {
    uint64_t tag;            /* the caller's tag of the frame */
    int32_t code;            /* index of the code in the server */
    int32_t stage;           /* 1: decided by stage 1, 2: by stage 2 */
    int32_t k;               /* chosen path (0 for stage 1) */
    int32_t metric;          /* M(c) = sum_{c_j=1} q_j of the decision */
    uint8_t cw[32];          /* decision in the first N/8 bytes, the rest 0 */
    double t_submit;         /* host seconds (steady clock) at submission */
    double t_done;           /* host seconds at which the host saw the result */
} mpwsd_result;

/* Device arena bytes needed by mpwsd_server_create for these codes. */
size_t mpwsd_server_arena_bytes(const mpwsd_server_code* codes, int ncodes);

/* Creates a server; arena (device, 256-byte aligned) stays owned by the
 * caller and must outlive the server.  The server allocates pinned host
 * staging buffers, one stream and events (host-side driver resources). */
int mpwsd_server_create(const mpwsd_server_code* codes, int ncodes, void* arena, size_t arena_bytes,
                        mpwsd_server** server);

/* Queues n frames of code `code`: y host [n][N] float, scale[n] quantizer
 * scales (8 / sigma^2), tags[n].  The data is copied; nothing is enqueued.
 * Submission may run on other threads than the one that calls
 * mpwsd_server_tick and mpwsd_server_poll (each call locks the code's
 * queue); tick, poll and destroy stay on one thread, and every submitting
 * thread must have returned before mpwsd_server_destroy. */
int mpwsd_server_submit(mpwsd_server* server, int code, int n, const float* y, const float* scale,
                        const uint64_t* tags);

/* Harvests finished ticks, admits waiting frames and enqueues one tick when
 * there is work.  *in_flight (may be NULL) receives the number of frames
 * submitted but not yet returned by mpwsd_server_poll. */
int mpwsd_server_tick(mpwsd_server* server, int64_t* in_flight);

/* Moves up to cap completed results to out; returns how many (>= 0). */
int mpwsd_server_poll(mpwsd_server* server, mpwsd_result* out, int cap);

/* Synchronises the server's stream and releases everything it owns. */
int mpwsd_server_destroy(mpwsd_server* server);

/*
 * mpwsd_serve_trace - a real-time load generator around a server: frame i of
 * the trace (code[i], y row row[i] of that code's pool, scale[i]) is
 * submitted when arrival[i] seconds have passed since the start (by a
 * producer thread of its own), the calling thread ticks the server
 * continuously, and the result of frame i is written to out[i] (tag = i),
 * its t_submit being the scheduled arrival (so latencies include any delay
 * in submitting).  pools[c] is a host [rows][N] float array for code c;
 * arrivals are seconds in [0, 1e9) (MPWSD_ERR_ARG otherwise, nothing run).
 * Returns 0 when every frame completed.
 */
int mpwsd_serve_trace(mpwsd_server* server, int64_t n, const int32_t* code, const int64_t* row,
                      const float* scale, const double* arrival, const float* const* pools,
                      mpwsd_result* out);

#ifdef __cplusplus
}
#endif

#endif /* MPWSD_H */
