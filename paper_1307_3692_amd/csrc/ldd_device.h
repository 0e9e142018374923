// Device-side building blocks of the decomposition kernels (gfx950, wave64).
//
// Labels.  Every vertex v carries one 64-bit label
//     P(v) = (key(v) << B) | c(v),   key(v) = Delta - shift_fix[c] + 2^20 * dist(c, v),
// with B = max(1, ceil(log2 n)) id bits.  Comparing labels as unsigned integers compares
// (key, centre) lexicographically, which is exactly the order of Algorithm 2 (Sec. 4):
// smaller shifted distance first, ties to the smaller centre id.  A neighbour u offers
// P(u) + (2^20 << B): one more unit of distance, same centre.  A vertex's own entry into
// the search (the delayed super-source arc of Sec. 5) offers ((Delta - shift_fix[v]) << B) | v.
// INF = 2^64 - 1 marks "not reached yet".
//
// Rounds.  Offers relayed along an edge add one unit, so a vertex first reached in round r
// has key in [r 2^20, (r+1) 2^20) and its label is final at the end of round r (Sec. 5:
// lengths with equal integer part are processed together, fractional parts break ties).
// Hence "settled before round r" is simply P(v) < base(r) = r << (B + 20).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldd {

typedef unsigned long long u64;
typedef long long i64;

constexpr int FIX = 20;
constexpr u64 INF = ~0ull;
constexpr int WAVE = 64;
constexpr int QCAP = 8192;  // integer parts of shifts bucketed in LDS by the preparation
// per preparation block, at most this many vertices of its highest q-buckets are listed for the
// first wake window (the buckets every block lists in full are placed before the rounds)
constexpr int CAND = 256;

// error bits raised by kernels (ctrl->err)
enum : unsigned {
  ERR_BAD_SHIFT = 1u,     // negative or huge shift
  ERR_BAD_ROWPTR = 2u,    // row_ptr not monotone / out of [0, nnz]
  ERR_BAD_COL = 4u,       // column id out of [0, n)
  ERR_BARRIER = 8u,       // grid barrier timed out
  ERR_WATCHDOG = 16u,     // more rounds than the shifts allow
  ERR_QUEUE = 32u         // queue overflow (more appends than vertices)
};

// Outcome of the preparation, decided on the device so that the host enqueues the whole
// decomposition without waiting for it.
enum : unsigned {
  SETUP_OK = 0,        // rounds run
  SETUP_EMPTY = 1,     // no vertex has an arc: every vertex is its own centre
  SETUP_INVALID = 2,   // bad row_ptr, shift or column id (ctrl->err says which)
  SETUP_OVERFLOW = 3,  // labels would not fit 64 bits, or too many rounds
  SETUP_WIDE = 4       // shifts span QCAP units or more: the host redoes the call on the wide path
};

// Control block in device memory, one per decomposition in flight.  Counters that many
// blocks update get a 128-byte line each: atomics to one line serialise (~12 ns apiece).
struct Ctrl {
  alignas(128) u64 delta;   // max shift_fix (atomicMax target)
  alignas(128) u64 n_active;  // vertices with at least one arc
  alignas(128) u64 hub;     // (degree << 32 | id) of the highest-degree vertex
  alignas(128) unsigned err;  // ERR_* bits
  unsigned wide;              // some shift has an integer part >= QCAP
  alignas(128) unsigned place_lo;  // lowest q-bucket every preparation block listed in full
  unsigned setup;                  // SETUP_*: what k_setup found (the rounds run only on SETUP_OK)
  alignas(128) u64 bar;     // grid barrier arrival counter (persistent engine)
  alignas(128) u64 cut_arcs;  // 2 per arc to H plus 1 per two-sided cut arc outside H
  alignas(128) u64 pieces;  // vertices that are their own centre
  alignas(128) u64 unreached;  // labels still INF after the rounds (must be 0)
  alignas(128) u64 list_cnt;  // (count << 32 | arcs) of the rows outside the hub's piece
};

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned rank_below(u64 mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ u64 shfl_u64(u64 v, int src) {
  unsigned lo = __shfl((unsigned)v, src, WAVE);
  unsigned hi = __shfl((unsigned)(v >> 32), src, WAVE);
  return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 wave_min_u64(u64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned lo = __shfl_xor((unsigned)v, o, WAVE);
    unsigned hi = __shfl_xor((unsigned)(v >> 32), o, WAVE);
    u64 w = ((u64)hi << 32) | lo;
    v = w < v ? w : v;
  }
  return v;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned lo = __shfl_xor((unsigned)v, o, WAVE);
    unsigned hi = __shfl_xor((unsigned)(v >> 32), o, WAVE);
    v += ((u64)hi << 32) | lo;
  }
  return v;
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned lo = __shfl_xor((unsigned)v, o, WAVE);
    unsigned hi = __shfl_xor((unsigned)(v >> 32), o, WAVE);
    u64 w = ((u64)hi << 32) | lo;
    v = w > v ? w : v;
  }
  return v;
}

// inclusive prefix sum over the wave (all 64 lanes must be active)
__device__ __forceinline__ unsigned wave_incl_scan(unsigned x) {
  const unsigned lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    unsigned y = __shfl_up(x, d, WAVE);
    if (lane >= (unsigned)d) x += y;
  }
  return x;
}

__device__ __forceinline__ u64 atomic_min_u64(u64* p, u64 v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 atomic_add_u64(u64* p, u64 v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_max_u64(u64* p, u64 v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or_u32(unsigned* p, unsigned v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned load_u32_acquire(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
// Last index i in [0, cnt) with a[i] <= x, for a non-decreasing array with a[0] <= x.  One
// wave splits the range 64 ways per pass (ceil(log64 cnt) + 1 dependent loads instead of
// log2 cnt); called by all lanes of the wave, every lane gets the answer.
__device__ __forceinline__ unsigned wave_search_le(const unsigned* a, unsigned cnt, unsigned x) {
  const unsigned lane = lane_id();
  unsigned lo = 0, hi = cnt;
  while (hi - lo > (unsigned)WAVE) {
    const u64 span = hi - lo;
    const unsigned idx = lo + (unsigned)(span * lane / WAVE);
    const u64 m = __ballot(a[idx] <= x);  // a prefix of the lanes; lane 0 holds a[lo] <= x
    const unsigned L = 63u - (unsigned)__builtin_clzll(m);
    const unsigned nlo = lo + (unsigned)(span * L / WAVE);
    if (L < (unsigned)WAVE - 1) hi = lo + (unsigned)(span * (L + 1) / WAVE);
    lo = nlo;
  }
  const unsigned idx = lo + lane;
  const u64 m = __ballot(idx < hi && a[idx] <= x);
  return lo + (63u - (unsigned)__builtin_clzll(m));
}

__device__ __forceinline__ u64 load_u64_relaxed(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Frontier queue: vertex ids plus the exclusive prefix of their degrees in append order,
// so that a round can split the frontier's arcs evenly over the grid.
struct Queue {
  int* vert;
  unsigned* aoff;
};

// Wave-aggregated append: lanes with `want` reserve consecutive slots and arc ranges with a
// single 64-bit atomic on `counter` = (count << 32) | arcs.  Must be called by a converged
// wave (all lanes active).
__device__ __forceinline__ void wave_append(bool want, int v, unsigned deg, Queue q, u64* counter, unsigned cap,
                                            unsigned* err) {
  const u64 mask = __ballot(want);
  if (mask == 0) return;
  const unsigned lane = lane_id();
  const unsigned incl = wave_incl_scan(want ? deg : 0u);
  const unsigned total = __shfl(incl, WAVE - 1, WAVE);
  const unsigned cnt = (unsigned)__popcll(mask);
  const int leader = __ffsll((long long)mask) - 1;
  u64 base = 0;
  if ((int)lane == leader) base = atomic_add_u64(counter, ((u64)cnt << 32) | total);
  base = shfl_u64(base, leader);
  if (want) {
    const unsigned idx = (unsigned)(base >> 32) + rank_below(mask);
    if (idx < cap) {
      q.vert[idx] = v;
      q.aoff[idx] = (unsigned)base + incl - deg;
    } else {
      atomic_or_u32(err, ERR_QUEUE);
    }
  }
}

// Grid-wide barrier for a co-resident (cooperatively launched) grid.  Arrival counter is
// monotone; generation `gen` is kept per block.  Every wave first waits for its own stores and
// atomics to complete (a workgroup barrier does not wait for other waves' stores to leave the
// CU); thread 0's release on arrival then writes them back at agent scope, and the acquire fence
// after leaving makes every write of the previous phase (plain stores and atomics) visible to
// every block at agent scope.  A bounded spin turns a hang into
// ERR_BARRIER; the caller then leaves its loop.
__device__ __forceinline__ void grid_sync(u64* bar, unsigned nblocks, u64& gen, unsigned* err) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores (and atomics) have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    gen += 1;
    const u64 target = gen * nblocks;
    __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 26)) {
        atomic_or_u32(err, ERR_BARRIER);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

}  // namespace ldd
