// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>

#include <hip/hip_runtime_api.h>

#include "mpwsd.h"

namespace mpwsd {

// Records a message for mpwsd_last_error() on this thread and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Reed-Muller dimension K = sum_{d <= r} C(m, d).
int rm_dimension(int r, int m);

// Number of minimum-weight codewords of RM(r, m) (flats of dimension m - r).
int64_t rm_min_weight_count(int r, int m);

// Largest move table the kernels index (move indices are 32-bit in the
// search keys, with room for a 128-row tail chunk).
constexpr int64_t kMaxMoves = (int64_t(1) << 31) - 256;

// True when P is the size of a move table the library builds for RM(r, m):
// the minimum-weight words, or (K <= 30) the nonzero words of some S_rho(0).
bool valid_move_count(int r, int m, int64_t P);

// Compute units of the current device (cached per device).
int device_cu_count();

// Enqueue the int8 move search (stage 2) over the active columns act[0 .. *count)
// (count read on the device): per column the minimum (S << 32 | p) is folded
// into keys[column] with atomicMin.  zneg holds -z per column, padded to
// max(N, 64) bytes.  grouped (device, or NULL) is the paired-half layout of
// the same table with grouped_chunks chunks and grouped_extras moves kept
// apart.  variant / blocks_per_cu as in mpwsd_options.
void launch_search_i8(int N, const int8_t* zneg, const uint8_t* moves, int64_t P, const uint8_t* grouped,
                      int64_t grouped_chunks, int64_t grouped_extras, const int32_t* act, const int32_t* count,
                      long long* keys, int variant, int blocks_per_cu, hipStream_t s);

}  // namespace mpwsd
