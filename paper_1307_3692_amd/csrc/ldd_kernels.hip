// HIP kernels of the exponential-shift low-diameter decomposition for gfx950.
//
// Pipeline for one graph (Sec. 5 of the paper: shortest paths from a super source whose
// arcs of length Delta - delta_u are added lazily, processed one integer distance at a time):
//   k_init          labels := INF, Delta := max shift (Algorithm 1 step 2), CSR bounds checks
//   k_wake_count    isolated vertices settle at once; others counted per wake round
//                   w(u) = (Delta - shift_fix[u]) >> 20 (the round the delayed arc s->u fires)
//   k_wake_scan     bucket offsets and "next non-empty bucket" links
//   k_wake_scatter  counting sort of vertices by wake round
//   k_rounds        all rounds in one persistent kernel with grid barriers (or the same
//                   phases launched one kernel each): wake bucket r, expand F_{r-1} top-down
//                   (push) or bottom-up (pull), append first-reached vertices to F_r
//   k_finalize      centre = low B bits of the label (Algorithm 1 step 4)
//   k_cut           edges whose endpoints have different centres (Def. 1.1)
#include "ldd_device.h"
#include "ldd_kernels.h"

namespace ldd {

// ------------------------------------------------------------------------------------------
// prep
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(int n, long long nnz, const int* __restrict__ row_ptr,
                                              const long long* __restrict__ shift, u64* __restrict__ P,
                                              Ctrl* ctrl) {
  u64 mx = 0, active = 0;
  unsigned bad = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const long long s = shift[v];
    if (s < 0 || s > (1ll << 52)) bad |= ERR_BAD_SHIFT;
    else mx = (u64)s > mx ? (u64)s : mx;
    const int a = row_ptr[v], b = row_ptr[v + 1];
    if (a < 0 || b < a || (long long)b > nnz) bad |= ERR_BAD_ROWPTR;
    if (v == 0 && a != 0) bad |= ERR_BAD_ROWPTR;
    if (v == n - 1 && (long long)b != nnz) bad |= ERR_BAD_ROWPTR;
    active += (b > a);
    P[v] = INF;
  }
  mx = wave_max_u64(mx);
  active = wave_sum_u64(active);
  if (lane_id() == 0) {
    if (mx) atomic_max_u64(&ctrl->delta, mx);
    if (active) atomic_add_u64(&ctrl->n_active, active);
  }
  if (bad) atomic_or_u32(&ctrl->err, bad);
}

// Optional O(nnz) check that every column id is in range (the round kernels also guard
// each access, so this only moves the error report before any traversal).
__global__ __launch_bounds__(256) void k_check_cols(int n, long long nnz, const int* __restrict__ col, Ctrl* ctrl) {
  unsigned bad = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nnz; a += stride) {
    const int w = col[a];
    if (w < 0 || w >= n) bad = ERR_BAD_COL;
  }
  if (bad) atomic_or_u32(&ctrl->err, bad);
}

// Count vertices per wake round; settle isolated vertices (their only offer is their own).
// Buckets are counted in LDS when they fit (lds_bins > 0), else directly in global memory.
__global__ __launch_bounds__(256) void k_wake_count(int n, int B, const int* __restrict__ row_ptr,
                                                    const long long* __restrict__ shift, const Ctrl* __restrict__ ctrl,
                                                    u64* __restrict__ P, unsigned* __restrict__ hist, int R,
                                                    int use_lds) {
  extern __shared__ unsigned lds_hist[];
  const u64 delta = ctrl->delta;
  if (use_lds) {
    for (int i = threadIdx.x; i < R; i += blockDim.x) lds_hist[i] = 0;
    __syncthreads();
  }
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const u64 off = delta - (u64)shift[v];
    if (row_ptr[v + 1] == row_ptr[v]) {
      P[v] = (off << B) | (u64)v;
    } else {
      const int w = (int)(off >> FIX);
      if (use_lds) atomicAdd(&lds_hist[w], 1u);
      else atomicAdd(&hist[w], 1u);
    }
  }
  if (use_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < R; i += blockDim.x)
      if (lds_hist[i]) atomicAdd(&hist[i], lds_hist[i]);
  }
}

// Exclusive scan of the R bucket counts (one block) and next-non-empty links:
// next_ne[r] = smallest r' >= r with a non-empty bucket, R if none.  Also copies the offsets
// into the scatter cursors.
__global__ __launch_bounds__(1024) void k_wake_scan(int R, const unsigned* __restrict__ hist, int* __restrict__ wake_off,
                                                    int* __restrict__ cursor, int* __restrict__ next_ne) {
  __shared__ unsigned part[1024];
  __shared__ int nxt[1024];
  const int t = threadIdx.x;
  const int per = (R + 1023) / 1024;
  const int lo = t * per, hi = min(R, lo + per);
  unsigned s = 0;
  int first = R;
  for (int i = lo; i < hi; ++i) {
    s += hist[i];
    if (hist[i] && first == R) first = i;
  }
  part[t] = s;
  nxt[t] = first;
  __syncthreads();
  // serial-by-thread-0 scan of 1024 partials is cheap relative to the launch
  if (t == 0) {
    unsigned acc = 0;
    for (int i = 0; i < 1024; ++i) {
      unsigned x = part[i];
      part[i] = acc;
      acc += x;
    }
    int nx = R;
    for (int i = 1023; i >= 0; --i) {
      if (nxt[i] != R) nx = nxt[i];
      nxt[i] = nx;
    }
  }
  __syncthreads();
  unsigned acc = part[t];
  int nx_after = (t + 1 < 1024) ? nxt[t + 1] : R;
  for (int i = lo; i < hi; ++i) {
    wake_off[i] = (int)acc;
    cursor[i] = (int)acc;
    acc += hist[i];
  }
  // next_ne over this thread's range, walking backwards
  for (int i = hi - 1; i >= lo; --i) {
    if (hist[i]) nx_after = i;
    next_ne[i] = nx_after;
  }
  if (t == 1023) {
    wake_off[R] = (int)acc;
    next_ne[R] = R;
  }
}

__global__ __launch_bounds__(256) void k_wake_scatter(int n, const int* __restrict__ row_ptr,
                                                      const long long* __restrict__ shift, const Ctrl* __restrict__ ctrl,
                                                      int* __restrict__ cursor, int* __restrict__ wake_ord) {
  const u64 delta = ctrl->delta;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    if (row_ptr[v + 1] == row_ptr[v]) continue;
    const int w = (int)((delta - (u64)shift[v]) >> FIX);
    const int pos = atomicAdd(&cursor[w], 1);
    wake_ord[pos] = (int)v;
  }
}

__global__ void k_fill_u64(u64* p, long long count, u64 value) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}


// ------------------------------------------------------------------------------------------
// output
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finalize(int n, int B, const u64* __restrict__ P, int* __restrict__ centre,
                                                  Ctrl* ctrl) {
  const u64 mask = ((u64)1 << B) - 1;
  u64 pieces = 0, unreached = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const u64 p = P[v];
    const int cv = (int)(p & mask);
    centre[v] = cv;
    pieces += (cv == (int)v);
    unreached += (p == INF);
  }
  pieces = wave_sum_u64(pieces);
  unreached = wave_sum_u64(unreached);
  if (lane_id() == 0 && pieces) atomic_add_u64(&ctrl->pieces, pieces);
  if (lane_id() == 0 && unreached) atomic_add_u64(&ctrl->unreached, unreached);
}

// Cut arcs: the nnz arcs are split evenly over the grid; each block walks its range in tiles
// of 256 arcs with a window of row offsets in LDS (zero-degree rows may be skipped over, so
// a window can end before the tile does; the loop then just advances the window).
__global__ __launch_bounds__(256) void k_cut(int n, long long nnz, const int* __restrict__ row_ptr,
                                             const int* __restrict__ col, const int* __restrict__ centre, Ctrl* ctrl) {
  constexpr int T = 256;
  __shared__ int w_rp[T + 1];
  __shared__ int s_v;
  const long long G = gridDim.x;
  const long long a_begin = nnz * blockIdx.x / G;
  const long long a_end = nnz * (blockIdx.x + 1) / G;
  u64 cut = 0;
  if (a_begin < a_end) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = n;  // last v with row_ptr[v] <= a_begin
      while (hi - lo > 1) {
        const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
        if (row_ptr[mid] <= a_begin) lo = mid;
        else hi = mid;
      }
      s_v = lo;
    }
    __syncthreads();
    int v0 = s_v;
    long long a_cur = a_begin;
    while (a_cur < a_end) {
      for (int k = threadIdx.x; k <= T; k += T) w_rp[k] = (v0 + k <= n) ? row_ptr[v0 + k] : (int)nnz;
      __syncthreads();
      const long long win_end = w_rp[T];  // arcs of rows v0 .. v0+T-1 end here
      long long t_end = a_cur + T;
      if (t_end > a_end) t_end = a_end;
      if (t_end > win_end) t_end = win_end;
      const long long a = a_cur + threadIdx.x;
      if (a < t_end) {
        int lo = 0, hi = T;  // last k with w_rp[k] <= a
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_rp[mid] <= a) lo = mid;
          else hi = mid;
        }
        const int v = v0 + lo;
        const int w = col[a];
        if ((unsigned)w < (unsigned)n) cut += (centre[w] != centre[v]);
      }
      __syncthreads();
      if (t_end >= win_end && t_end < a_end) {
        v0 += T;  // window exhausted before the tile: move the window
        // skip rows that end before t_end
        if (threadIdx.x == 0) {
          int lo = v0, hi = n;
          while (hi - lo > 1) {
            const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
            if (row_ptr[mid] <= t_end) lo = mid;
            else hi = mid;
          }
          s_v = lo;
        }
        __syncthreads();
        v0 = s_v;
        __syncthreads();
      } else if (t_end < a_end) {
        if (threadIdx.x == 0) {
          int lo = 0, hi = T;
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (w_rp[mid] <= t_end) lo = mid;
            else hi = mid;
          }
          s_v = v0 + lo;
        }
        __syncthreads();
        v0 = s_v;
        __syncthreads();
      }
      a_cur = t_end;
    }
  }
  cut = wave_sum_u64(cut);
  if (lane_id() == 0 && cut) atomic_add_u64(&ctrl->cut_arcs, cut);
}

}  // namespace ldd
