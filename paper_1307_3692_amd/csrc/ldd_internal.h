// Host-side helpers shared by the library's translation units.
#pragma once

void ldd_set_error(const char* fmt, ...);

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ldd.h"

// n Exp(beta) shifts of the library's recipe for `seed` into device memory, on stream st
// (ldd_shifts.hip).
ldd_status ldd_shifts_on_device(int32_t n, double beta, uint64_t seed, int64_t* out, hipStream_t st);
