// Shifts delta_u ~ Exp(beta) in fixed point (Algorithm 1 step 1, Sec. 2; Sec. 3's density
// beta exp(-beta x)), drawn by the library itself: on the host (ldd_make_shifts) and on the
// device (ldd_make_shifts_device), bit-identical, since the recipe uses integer arithmetic and
// two correctly rounded double operations only.
//
// Recipe (draw i for seed s):
//   x      = SplitMix64 output for state  stream(s) + (i + 1) * 0x9E3779B97F4A7C15  (Steele,
//            Lea, Flood, OOPSLA 2014), stream(s) = mix(mix(s + 0x9E3779B97F4A7C15) ^ 0xD1B54A32D192ED03)
//            (the shift stream of the library's seeded inputs);
//   U      = (x >> 11) 2^-53 in [0, 1);  M = 2^53 - (x >> 11) in [1, 2^53];
//   -ln(1 - U) = ln 2 (53 - log2 M), log2 M = e + log2 m with e = floor(log2 M), m in [1, 2);
//   47 bits of log2 m by repeated squaring (m^2 >= 2: bit 1 and m = m^2 / 2; else bit 0 and
//   m = m^2), with m a 64-bit fraction and each square truncated to 64 bits;
//   T      = 2^47 (53 - e) - bits  (an integer < 2^53, exact in double);
//   shift_fix = floor( (T * (ln 2 * 2^-27)) / beta ).
// The sampled delta is the inversion of the CDF 1 - exp(-beta x) at U (the logarithm to
// within 2^-47), truncated to 2^-20 units.  Each draw depends only on (seed, i): O(n) work,
// O(1) depth (the proof of Theorem 1.1, Sec. 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/ldd.h"
#include "ldd_internal.h"

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;
constexpr uint64_t TAG_SHIFT = 1;
constexpr uint64_t TAG_PERM = 6;
constexpr double LN2_2M27 = 0x1.62e42fefa39efp-28;  // ln 2 * 2^-27
constexpr int FIX_BITS = 20;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t stream_of(uint64_t seed, uint64_t tag) {
  return mix64(mix64(seed + GOLDEN) ^ (tag * 0xD1B54A32D192ED03ull));
}

__host__ __device__ inline uint64_t shift_stream(uint64_t seed) { return stream_of(seed, TAG_SHIFT); }

__host__ __device__ inline int top_bit(uint64_t v) {  // v > 0
  int e = 0;
  for (int step = 32; step > 0; step >>= 1)
    if (v >> (e + step)) e += step;
  return e;
}

// 2^47 (53 - log2 M) for M = 2^53 - (x >> 11), 47 fraction bits truncated
__host__ __device__ inline uint64_t neglog2_q47(uint64_t x) {
  const uint64_t M = (1ull << 53) - (x >> 11);
  const int e = top_bit(M);
  uint64_t m = M << (63 - e);  // m / 2^63 in [1, 2)
  uint64_t bits = 0;
  for (int k = 0; k < 47; ++k) {
    const unsigned __int128 sq = (unsigned __int128)m * m;  // sq / 2^126 in [1, 4)
    bits <<= 1;
    if ((uint64_t)(sq >> 127)) {
      bits |= 1;
      m = (uint64_t)(sq >> 64);
    } else {
      m = (uint64_t)(sq >> 63);
    }
  }
  return ((uint64_t)(53 - e) << 47) - bits;
}

__host__ __device__ inline int64_t shift_of(uint64_t stream, uint64_t i, double beta) {
  const double t = (double)neglog2_q47(mix64(stream + (i + 1) * GOLDEN));
  return (int64_t)floor((t * LN2_2M27) / beta);
}

__global__ __launch_bounds__(256) void k_make_shifts(long long n, double beta, uint64_t stream, long long* out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = shift_of(stream, (uint64_t)i, beta);
}

bool beta_ok(double beta) { return beta > 0.0 && std::isfinite(beta); }

}  // namespace

ldd_status ldd_shifts_on_device(int32_t n, double beta, uint64_t seed, int64_t* out, hipStream_t st) {
  if (n <= 0) return LDD_OK;
  const int grid = (int)std::min<long long>(4096, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_make_shifts, dim3(grid), dim3(256), 0, st, (long long)n, beta, shift_stream(seed),
                     (long long*)out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ldd_set_error("shift kernel launch failed: %s", hipGetErrorString(e));
    return LDD_ERR_HIP;
  }
  return LDD_OK;
}

extern "C" ldd_status ldd_make_shifts(int32_t n, double beta, uint64_t seed, int64_t* out_host) {
  if (n < 0 || (n > 0 && !out_host) || !beta_ok(beta)) {
    ldd_set_error("ldd_make_shifts: need n >= 0, an output buffer and a finite beta > 0");
    return LDD_ERR_INVALID_ARG;
  }
  const uint64_t stream = shift_stream(seed);
  for (int32_t i = 0; i < n; ++i) out_host[i] = shift_of(stream, (uint64_t)i, beta);
  return LDD_OK;
}

// The shift variants of the closing remarks of Sec. 5 (see ldd.h).  The random ranking orders
// the vertices by a 64-bit draw of stream (seed, 6), ties by id.
extern "C" ldd_status ldd_make_shifts_variant(int32_t n, double beta, uint64_t seed, int32_t kind, int64_t* out_host) {
  if (kind == LDD_SHIFTS_EXP) return ldd_make_shifts(n, beta, seed, out_host);
  if (n < 0 || (n > 0 && !out_host) || !beta_ok(beta) || (kind != LDD_SHIFTS_INT_PERM && kind != LDD_SHIFTS_PERM_ORDER)) {
    ldd_set_error("ldd_make_shifts_variant: need n >= 0, an output buffer, a finite beta > 0 and a known kind");
    return LDD_ERR_INVALID_ARG;
  }
  if (n == 0) return LDD_OK;
  std::vector<std::pair<uint64_t, int32_t>> order((size_t)n);
  const uint64_t ps = stream_of(seed, TAG_PERM);
  for (int32_t v = 0; v < n; ++v) order[v] = {mix64(ps + ((uint64_t)v + 1) * GOLDEN), v};
  std::sort(order.begin(), order.end());
  if (kind == LDD_SHIFTS_INT_PERM) {
    const uint64_t st = shift_stream(seed);
    for (int32_t i = 0; i < n; ++i) {
      const int32_t v = order[i].second;
      const int64_t whole = shift_of(st, (uint64_t)v, beta) >> FIX_BITS;
      const int64_t frac = (int64_t)(((unsigned __int128)(uint64_t)(n - 1 - i) << FIX_BITS) / (uint64_t)n);
      out_host[v] = (whole << FIX_BITS) | frac;
    }
  } else {
    // rank i takes (H_n - H_i) / beta: suffix sums of 1/j from the top, in this order
    std::vector<double> sfx((size_t)n + 1);
    sfx[n] = 0.0;
    for (int32_t i = n - 1; i >= 0; --i) sfx[i] = sfx[i + 1] + 1.0 / (double)(i + 1);
    for (int32_t i = 0; i < n; ++i) out_host[order[i].second] = (int64_t)floor((sfx[i] / beta) * 1048576.0);
  }
  return LDD_OK;
}

extern "C" ldd_status ldd_make_shifts_device(int32_t n, double beta, uint64_t seed, int64_t* out_device,
                                             void* hip_stream) {
  if (n < 0 || (n > 0 && !out_device) || !beta_ok(beta)) {
    ldd_set_error("ldd_make_shifts_device: need n >= 0, an output buffer and a finite beta > 0");
    return LDD_ERR_INVALID_ARG;
  }
  return ldd_shifts_on_device(n, beta, seed, out_device, (hipStream_t)hip_stream);
}
