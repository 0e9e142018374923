// Block decomposition in the sense of Linial and Saks (Sec. 2): the edges are split into levels
// by running the (beta, O(log n / beta)) decomposition again and again on the edges not placed
// yet, beta = 1/2 by default.  Level L holds the edges whose endpoints fall into one piece of the
// L-th decomposition; the cut edges go on to level L + 1.  Each decomposition cuts an edge with
// probability below beta (Cor. 4.5), so the remaining edges shrink geometrically and O(log m)
// levels place them all; inside a level, every connected set of that level's edges lies in one
// piece, whose vertices are within O(log n / beta) of its centre (Lemma 4.2).
//
// Each level: shifts drawn on the device (the library's sampler, seed + level), one
// decomposition of the remaining graph (the single-graph engines), then one pass over the
// remaining arcs that assigns the level to arcs inside a piece and compacts the others into the
// next level's CSR (row counts, an exclusive scan, a scatter that keeps each arc's original id).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <vector>

#include "../../include/ldd.h"
#include "ldd_internal.h"

namespace {

#define BD_TRY(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      ldd_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      status = LDD_ERR_HIP;                                                                     \
      goto done;                                                                                \
    }                                                                                           \
  } while (0)

// Arcs of row u whose ends share a centre take the level; the others are counted for the next
// level's row u.  orig == nullptr: the arc ids are the positions themselves (the first level).
__global__ __launch_bounds__(256) void k_level_mark(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                    const int* __restrict__ orig, const int* __restrict__ centre,
                                                    int level, int* __restrict__ arc_level, int* __restrict__ keep_cnt,
                                                    unsigned long long* placed) {
  unsigned long long mine = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int cu = centre[u];
    int keep = 0;
    for (int a = rp[u]; a < rp[u + 1]; ++a) {
      const int v = col[a];
      if (centre[v] == cu) {
        arc_level[orig ? orig[a] : a] = level;
        ++mine;
      } else {
        ++keep;
      }
    }
    keep_cnt[u] = keep;
  }
  if (mine) atomicAdd(placed, mine);
}

// The kept arcs of row u, in order, to the next level's CSR (new_rp from the exclusive scan).
__global__ __launch_bounds__(256) void k_level_compact(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                       const int* __restrict__ orig, const int* __restrict__ centre,
                                                       const int* __restrict__ new_rp, int* __restrict__ new_col,
                                                       int* __restrict__ new_orig) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int cu = centre[u];
    int o = new_rp[u];
    for (int a = rp[u]; a < rp[u + 1]; ++a) {
      const int v = col[a];
      if (centre[v] != cu) {
        new_col[o] = v;
        new_orig[o] = orig ? orig[a] : a;
        ++o;
      }
    }
  }
}

__global__ void k_fill_i32(int* p, long long count, int value) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

int grid_of(long long items, int threads, int cap) {
  long long g = (items + threads - 1) / threads;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

extern "C" ldd_status ldd_block_decompose(const ldd_csr* g, double beta, uint64_t seed, int32_t max_levels,
                                          int32_t* arc_level, int32_t* levels, int64_t* level_edges,
                                          const ldd_options* opt, void* hip_stream) {
  if (!g || g->n < 0 || g->nnz < 0 || g->nnz >= (1ll << 31) || max_levels < 1 || !levels ||
      (g->n > 0 && !g->row_ptr) || (g->nnz > 0 && (!g->col_idx || !arc_level))) {
    ldd_set_error("ldd_block_decompose: bad graph, output or max_levels");
    return LDD_ERR_INVALID_ARG;
  }
  if (beta == 0.0) beta = 0.5;
  if (!(beta > 0.0 && beta < 1.0)) {
    ldd_set_error("ldd_block_decompose: beta must lie in (0, 1)");
    return LDD_ERR_INVALID_ARG;
  }
  const int n = g->n;
  const long long nnz = g->nnz;
  hipStream_t st = (hipStream_t)hip_stream;
  ldd_status status = LDD_OK;
  int* buf[6] = {};  // two generations of the remaining graph: row offsets, columns, original arc ids
  long long* shifts = nullptr;
  int* centre = nullptr;
  int* cnt = nullptr;
  unsigned long long* placed = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  *levels = 0;
  if (n == 0 || nnz == 0) return LDD_OK;  // no edge to place: zero levels
  {
    BD_TRY(hipMalloc(&buf[0], (size_t)(n + 1) * 4));
    BD_TRY(hipMalloc(&buf[1], (size_t)nnz * 4));
    BD_TRY(hipMalloc(&buf[2], (size_t)nnz * 4));
    BD_TRY(hipMalloc(&buf[3], (size_t)(n + 1) * 4));
    BD_TRY(hipMalloc(&buf[4], (size_t)nnz * 4));
    BD_TRY(hipMalloc(&buf[5], (size_t)nnz * 4));
    BD_TRY(hipMalloc(&shifts, (size_t)n * 8));
    BD_TRY(hipMalloc(&centre, (size_t)n * 4));
    BD_TRY(hipMalloc(&cnt, (size_t)(n + 1) * 4));
    BD_TRY(hipMalloc(&placed, 8));
    BD_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt, buf[0], n + 1, st));
    BD_TRY(hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(nnz, 256, 4096)), dim3(256), 0, st, arc_level, nnz, -1);
    // the level's graph: the input first, then the compacted generations in turn
    const int* rp = g->row_ptr;
    const int* col = g->col_idx;
    const int* orig = nullptr;
    long long remaining = nnz;
    int gen = 0;
    ldd_options o{};
    if (opt) o = *opt;
    for (int level = 0; level < max_levels && remaining > 0; ++level) {
      ldd_status s = ldd_make_shifts_device(n, beta, seed + (uint64_t)level, (int64_t*)shifts, st);
      if (s == LDD_OK) {
        ldd_csr lg{n, remaining, rp, col};
        s = ldd_decompose(&lg, (const int64_t*)shifts, beta, centre, nullptr, &o, nullptr, st);
      }
      if (s != LDD_OK) {
        status = s;
        goto done;
      }
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, (int*)placed, 2ll, 0);
      hipLaunchKernelGGL(k_level_mark, dim3(grid_of(n, 256, 8192)), dim3(256), 0, st, n, rp, col, orig,
                         (const int*)centre, level, arc_level, cnt, placed);
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, cnt + n, 1ll, 0);
      int* nrp = buf[gen ? 0 : 3];
      int* ncol = buf[gen ? 1 : 4];
      int* norig = buf[gen ? 2 : 5];
      BD_TRY(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, cnt, nrp, n + 1, st));
      hipLaunchKernelGGL(k_level_compact, dim3(grid_of(n, 256, 8192)), dim3(256), 0, st, n, rp, col, orig,
                         (const int*)centre, (const int*)nrp, ncol, norig);
      BD_TRY(hipGetLastError());
      unsigned long long placed_h = 0;
      BD_TRY(hipMemcpyAsync(&placed_h, placed, 8, hipMemcpyDeviceToHost, st));
      BD_TRY(hipStreamSynchronize(st));
      if (level_edges) level_edges[level] = (int64_t)(placed_h / 2);
      remaining -= (long long)placed_h;
      *levels = level + 1;
      rp = nrp;
      col = ncol;
      orig = norig;
      gen ^= 1;
    }
    if (remaining > 0) {
      ldd_set_error("%lld arcs not placed after %d levels (their level stays -1)", remaining, max_levels);
      status = LDD_ERR_RETRIES;
    }
  }
done:
  for (int* p : buf) (void)hipFree(p);
  (void)hipFree(shifts);
  (void)hipFree(centre);
  (void)hipFree(cnt);
  (void)hipFree(placed);
  (void)hipFree(tmp);
  return status;
}
