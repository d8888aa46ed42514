// Internal helpers shared by the library's translation units.
#pragma once

#include <cstdarg>
#include <cstdint>

#include "mpwsd.h"

namespace mpwsd {

// Records a message for mpwsd_last_error() on this thread and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Reed-Muller dimension K = sum_{d <= r} C(m, d).
int rm_dimension(int r, int m);

// Number of minimum-weight codewords of RM(r, m) (flats of dimension m - r).
int64_t rm_min_weight_count(int r, int m);

}  // namespace mpwsd
