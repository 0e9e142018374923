// Serving: decomposition requests admitted continuously into one device-resident arena.
//
// Every admitted request owns a slot: a vertex range and an arc range of the arena holding its
// CSR rewritten to arena ids.  The round engine runs one global round per step over the whole
// arena, i.e. over the disjoint union of all admitted requests.  A request whose round 0 is the
// global round r0 gets the source-arc lengths Delta_g - shift + r0 * 2^20: every key of the
// request grows by the same constant, so its argmin and its tie order -- its result -- are those
// of the request alone (Sec. 5: the super-source search only compares keys within a component),
// and its round rho runs at global round r0 + rho.  It is complete once global round r0 + R - 1,
// its last wake round, has run.
//
// Requests join and leave between step chunks: admission (copy into the arena, wake-round sort),
// slot-table changes and result extraction are enqueued on the engine stream between graph
// replays, so they take effect at a round boundary without draining the device.  Keys grow with
// the global round; when they approach the label's key range, all live keys are lowered by the
// same number of rounds (a rebase), again between chunks.
//
// One engine thread owns the engine stream; submit, poll, wait and cancel touch host queues (and
// submit validates the request on a stream of its own).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ldd.h"
#include "ldd_internal.h"
#include "ldd_kernels.h"

namespace ldd {

constexpr u64 S_ONE = (u64)1 << FIX;
constexpr int CHECK_BLOCKS = 512;

// ------------------------------------------------------------------------------------------
// slot kernels
// ------------------------------------------------------------------------------------------
// Validation of a request before it is queued: shifts in [0, 2^52], row offsets from 0 to nnz
// and non-decreasing, column ids in [0, n).  Block b leaves its maximum shift and error bits in
// part[2b], part[2b+1].
__global__ __launch_bounds__(256) void k_req_check(int n, long long nnz, const int* __restrict__ rp,
                                                   const int* __restrict__ col, const long long* __restrict__ shift,
                                                   u64* __restrict__ part) {
  __shared__ u64 red[2][4];
  u64 mx = 0, bad = 0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long items = (long long)n > nnz ? (long long)n : nnz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += stride) {
    if (i < n) {
      const int a = rp[i], b = rp[i + 1];
      if (b < a || (i == 0 && a != 0) || (i == n - 1 && (long long)b != nnz)) bad |= ERR_BAD_ROWPTR;
      const long long s = shift[i];
      if (s < 0 || s > (1ll << 52)) bad |= ERR_BAD_SHIFT;
      else mx = (u64)s > mx ? (u64)s : mx;
    }
    if (i < nnz && (unsigned)col[i] >= (unsigned)n) bad |= ERR_BAD_COL;
  }
  mx = wave_max_u64(mx);
  // the OR over the wave, one error kind at a time (each a max over 0 / that bit)
  const u64 bits = wave_max_u64(bad & ERR_BAD_SHIFT) | wave_max_u64(bad & ERR_BAD_ROWPTR) |
                   wave_max_u64(bad & ERR_BAD_COL);
  if (lane_id() == 0) {
    red[0][threadIdx.x / WAVE] = mx;
    red[1][threadIdx.x / WAVE] = bits;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 m = 0, e = 0;
    for (int w = 0; w < 4; ++w) {
      m = red[0][w] > m ? red[0][w] : m;
      e |= red[1][w];
    }
    part[2 * blockIdx.x] = m;
    part[2 * blockIdx.x + 1] = e;
  }
}

// A request's CSR (local ids) into the arena: global row offsets and column ids, shifts stored
// as C - (Delta_g - shift + r0 2^20), so that the engine's C - shift is the request's source-arc
// length; labels INF for vertices with arcs and their own offer for isolated ones.  Vertex n of
// the slot is a separator closing the last row: settled (label 0) and never woken.
__global__ __launch_bounds__(256) void k_slot_load(long long vbeg, int n, long long abeg, long long nnz,
                                                   const int* __restrict__ s_rp, const int* __restrict__ s_col,
                                                   const long long* __restrict__ s_shift, u64 delta_s, long long r0,
                                                   u64 C, int B, int* __restrict__ rp_g, int* __restrict__ col_g,
                                                   long long* __restrict__ shift_g, u64* __restrict__ P) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long items = (long long)n + 1 > nnz ? (long long)n + 1 : nnz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += stride) {
    if (i < n) {
      const int a = s_rp[i], b = s_rp[i + 1];
      const u64 off = delta_s - (u64)s_shift[i] + (u64)r0 * S_ONE;
      rp_g[vbeg + i] = (int)(abeg + a);
      shift_g[vbeg + i] = (long long)(C - off);
      P[vbeg + i] = b > a ? INF : ((off << B) | (u64)(vbeg + i));
    } else if (i == n) {
      rp_g[vbeg + n] = (int)(abeg + nnz);
      shift_g[vbeg + n] = (long long)C;
      P[vbeg + n] = 0;
    }
    if (i < nnz) col_g[abeg + i] = (int)(vbeg + s_col[i]);
  }
}

// Per-block LDS histogram of the local wake rounds rho = (Delta_g - shift) >> 20 of the slot's
// vertices with arcs; block b owns [b n / G, (b+1) n / G).  mat[rho * G + b] as in k_init.
__global__ __launch_bounds__(1024) void k_slot_hist(int n, int R, const int* __restrict__ s_rp,
                                                    const long long* __restrict__ s_shift, u64 delta_s,
                                                    unsigned* __restrict__ mat, int* __restrict__ qmax) {
  __shared__ unsigned h[QCAP];
  for (int i = threadIdx.x; i < R; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const long long lo = (long long)n * blockIdx.x / gridDim.x, hi = (long long)n * (blockIdx.x + 1) / gridDim.x;
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x)
    if (s_rp[i + 1] > s_rp[i]) atomicAdd(&h[(delta_s - (u64)s_shift[i]) >> FIX], 1u);
  __syncthreads();
  const unsigned G = gridDim.x;
  for (int r = threadIdx.x; r < R; r += blockDim.x) mat[(size_t)r * G + blockIdx.x] = h[r];
  if (threadIdx.x == 0) qmax[blockIdx.x] = R - 1;
}

// Each vertex with arcs to its round's segment: roff[rho] + mat[rho * G + b] + rank in block b.
__global__ __launch_bounds__(1024) void k_slot_place(int n, int R, long long vbeg, const int* __restrict__ s_rp,
                                                     const long long* __restrict__ s_shift, u64 delta_s,
                                                     const unsigned* __restrict__ mat, const int* __restrict__ roff,
                                                     int* __restrict__ wake_ord) {
  __shared__ unsigned cur[QCAP];
  const unsigned G = gridDim.x;
  for (int r = threadIdx.x; r < R; r += blockDim.x) cur[r] = (unsigned)roff[r] + mat[(size_t)r * G + blockIdx.x];
  __syncthreads();
  const long long lo = (long long)n * blockIdx.x / gridDim.x, hi = (long long)n * (blockIdx.x + 1) / gridDim.x;
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x)
    if (s_rp[i + 1] > s_rp[i])
      wake_ord[vbeg + atomicAdd(&cur[(delta_s - (u64)s_shift[i]) >> FIX], 1u)] = (int)(vbeg + i);
}

// Centre (request-local id) of every vertex of a finished slot, into the caller's buffer.
__global__ __launch_bounds__(256) void k_slot_final(long long vbeg, int n, int B, const u64* __restrict__ P,
                                                    int* __restrict__ centre) {
  const u64 mask = ((u64)1 << B) - 1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    centre[i] = (int)((P[vbeg + i] & mask) - (u64)vbeg);
}

// Arcs of a finished slot whose ends have different centres (twice the cut edges).  The slot's
// nnz arcs are split evenly over the grid; a block walks its range in tiles of 256 arcs with a
// window of row offsets in LDS (rows of degree 0 can end a window before the tile; the walk
// then moves the window).  Row offsets are arena arc indices.
__global__ __launch_bounds__(256) void k_slot_cut(long long vbeg, int n, long long abeg, long long nnz,
                                                  const int* __restrict__ rp_g, const int* __restrict__ col_g,
                                                  const int* __restrict__ centre, u64* __restrict__ out) {
  constexpr int T = 256;
  __shared__ long long w_rp[T + 1];
  __shared__ int s_v;
  __shared__ u64 red[4];
  const int* rp = rp_g + vbeg;  // n + 1 entries (the separator closes the last row)
  const long long G = gridDim.x;
  const long long a_begin = nnz * blockIdx.x / G, a_end = nnz * (blockIdx.x + 1) / G;
  u64 cut = 0;
  if (a_begin < a_end) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = n;  // the last row v with start <= a_begin
      while (hi - lo > 1) {
        const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
        if (rp[mid] - abeg <= a_begin) lo = mid;
        else hi = mid;
      }
      s_v = lo;
    }
    __syncthreads();
    int v0 = s_v;
    long long a_cur = a_begin;
    while (a_cur < a_end) {
      for (int k = threadIdx.x; k <= T; k += T) w_rp[k] = (v0 + k <= n) ? (long long)rp[v0 + k] - abeg : nnz;
      __syncthreads();
      const long long win_end = w_rp[T];
      long long t_end = a_cur + T;
      if (t_end > a_end) t_end = a_end;
      if (t_end > win_end) t_end = win_end;
      const long long a = a_cur + threadIdx.x;
      if (a < t_end) {
        int lo = 0, hi = T;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_rp[mid] <= a) lo = mid;
          else hi = mid;
        }
        const int w = col_g[abeg + a] - (int)vbeg;
        cut += centre[w] != centre[v0 + lo];
      }
      __syncthreads();
      if (t_end >= win_end && t_end < a_end) {
        v0 += T;
        if (threadIdx.x == 0) {
          int lo = v0, hi = n;
          while (hi - lo > 1) {
            const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
            if (rp[mid] - abeg <= t_end) lo = mid;
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
  if (lane_id() == 0) red[threadIdx.x / WAVE] = cut;
  __syncthreads();
  if (threadIdx.x == 0) {
    const u64 t = red[0] + red[1] + red[2] + red[3];
    if (t) atomic_add_u64(out, t);
  }
}

__global__ void k_set_slot(SlotInfo* table, int s, SlotInfo e) {
  if (threadIdx.x == 0 && blockIdx.x == 0) table[s] = e;
}

// The engine's latest state (after step k_last) gains a new request's arcs.
__global__ void k_state_add(RoundState* st, long long k_last, long long arcs) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st[k_last & 1].unsettled_arcs += arcs;
}

// Rebase: every live key drops by X rounds.  Keys below X rounds belong to vertices outside the
// active slots (free ranges, separators, finished requests): they become 0, i.e. settled.
// The slots' r0 and the host's round numbering move by the same X.
__global__ __launch_bounds__(256) void k_rebase(long long V, int B, u64 C, long long X, u64* __restrict__ P,
                                                long long* __restrict__ shift_g, u64* __restrict__ lr_part, int n_lr,
                                                RoundState* st, long long k_last) {
  const u64 xf = (u64)X * S_ONE;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < V; i += stride) {
    const u64 p = P[i];
    if (p != INF) P[i] = (p >> B) >= xf ? p - (xf << B) : 0;
    const u64 off = C - (u64)shift_g[i];
    shift_g[i] = (long long)(off >= xf ? C - (off - xf) : C);
    if (i < n_lr) {
      const u64 l = lr_part[i];
      if (l != INF) lr_part[i] = (l >> B) >= xf ? l - (xf << B) : 0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[k_last & 1].round -= X;
}

}  // namespace ldd

using namespace ldd;

// ------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int log2_ceil(long long n) {
  int b = 0;
  while ((1ll << b) < n) ++b;
  return b < 1 ? 1 : b;
}

// first-fit allocator of ranges of [0, cap)
struct RangeAlloc {
  std::map<long long, long long> free_;  // start -> length
  void init(long long cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  long long take(long long len) {
    if (len == 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const long long at = it->first, rest = it->second - len;
        free_.erase(it);
        if (rest) free_[at + len] = rest;
        return at;
      }
    }
    return -1;
  }
  void give(long long at, long long len) {
    if (len == 0) return;
    auto it = free_.emplace(at, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum ReqState { RQ_QUEUED, RQ_ACTIVE, RQ_FINISHING, RQ_DONE };

struct Request {
  uint64_t ticket = 0;
  ldd_request q{};  // the caller's buffers (device)
  u64 delta = 0;    // max shift
  int R = 1;        // rounds: (delta >> 20) + 1
  int state = RQ_QUEUED;
  ldd_status status = LDD_ERR_PENDING;
  int slot = -1;
  long long vbeg = 0, abeg = 0, wbase = 0;
  long long r0 = 0;         // global round of its round 0 (numbering at admission)
  long long done_step = 0;  // complete once this step has run
  int64_t cut = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  hipEvent_t ev = nullptr;  // result written and cut copied out
};

}  // namespace

struct ldd_server {
  ldd_server_config cfg{};
  int dev = 0;
  long long vcap = 0, acap = 0;
  int B = 1;
  u64 C = 0;                  // engine Delta: a vertex's source-arc length is C - shift_g
  long long round_limit = 0;  // keys stay below round_limit * 2^20
  int max_rounds = 0;         // largest R a request may have
  hipStream_t stream = nullptr, check_stream = nullptr;
  hipEvent_t chunk_ev[2] = {};
  hipGraphExec_t graph = nullptr;
  int blocks = 0;
  // arena and engine buffers (device)
  void *P = nullptr, *qv0 = nullptr, *qv1 = nullptr, *qa0 = nullptr, *qa1 = nullptr, *wake_ord = nullptr;
  void *rp_g = nullptr, *col_g = nullptr, *shift_g = nullptr;
  void *mat = nullptr, *qmax = nullptr, *tot = nullptr, *scratch_ne = nullptr, *wake_tab = nullptr;
  void *slots = nullptr, *st = nullptr, *qcnt = nullptr, *lr_part = nullptr, *lb = nullptr, *ex_part = nullptr;
  void *ctrl = nullptr, *cuts = nullptr, *check = nullptr;
  u64* h_out = nullptr;    // pinned: per slot {cut arcs, engine error bits}
  u64* h_check = nullptr;  // pinned: k_req_check's block results
  int wake_tab_cap = 0;
  RangeAlloc valloc, aalloc, walloc;
  SlotInfo slot_tab[MAX_SLOTS] = {};
  Request* slot_req[MAX_SLOTS] = {};
  long long steps = 0;       // steps enqueued so far
  long long round_base = 0;  // global round of step 1 in the current numbering
  std::mutex check_mu;       // k_req_check's buffers
  std::mutex mu;             // everything below, and the allocators and slot_req
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  ldd_status fatal = LDD_OK;
  char fatal_msg[256] = {};
  std::thread engine;
  double t0 = 0;
  long long admitted = 0, completed = 0, max_active = 0, rebases = 0;
};

namespace {

#define SRV_TRY(expr)                                                                            \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      snprintf(srv->fatal_msg, sizeof(srv->fatal_msg), "%s: %s", #expr, hipGetErrorString(e_)); \
      return LDD_ERR_HIP;                                                                        \
    }                                                                                            \
  } while (0)

long long round_at(const ldd_server* srv, long long k) { return srv->round_base + (k - 1); }

ldd_status srv_alloc(ldd_server* srv, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    snprintf(srv->fatal_msg, sizeof(srv->fatal_msg), "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return LDD_ERR_OOM;
  }
  return LDD_OK;
}

// Device bytes per arena vertex (label, two queues with arc prefixes, wake order, row offset,
// shift) and per arena arc (column id).
constexpr long long BYTES_PER_VERTEX = 8 + 8 + 8 + 4 + 4 + 8;
constexpr long long BYTES_PER_ARC = 4;
constexpr int SORT_BLOCKS = 256;  // at most this many blocks in a slot's wake-round sort

ldd_status srv_setup(ldd_server* srv) {
  SRV_TRY(hipSetDevice(srv->dev));
  SRV_TRY(hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking));
  SRV_TRY(hipStreamCreateWithFlags(&srv->check_stream, hipStreamNonBlocking));
  for (auto& e : srv->chunk_ev) SRV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const long long V = srv->vcap, A = srv->acap;
  ldd_status s;
  if ((s = srv_alloc(srv, &srv->P, V * 8)) || (s = srv_alloc(srv, &srv->qv0, V * 4)) ||
      (s = srv_alloc(srv, &srv->qv1, V * 4)) || (s = srv_alloc(srv, &srv->qa0, V * 4)) ||
      (s = srv_alloc(srv, &srv->qa1, V * 4)) || (s = srv_alloc(srv, &srv->wake_ord, V * 4)) ||
      (s = srv_alloc(srv, &srv->rp_g, (V + 1) * 4)) || (s = srv_alloc(srv, &srv->col_g, A * 4)) ||
      (s = srv_alloc(srv, &srv->shift_g, V * 8)) || (s = srv_alloc(srv, &srv->mat, (size_t)QCAP * SORT_BLOCKS * 4)) ||
      (s = srv_alloc(srv, &srv->qmax, SORT_BLOCKS * 4)) || (s = srv_alloc(srv, &srv->tot, QCAP * 4)) ||
      (s = srv_alloc(srv, &srv->scratch_ne, (QCAP + 2) * 4)) ||
      (s = srv_alloc(srv, &srv->wake_tab, (size_t)srv->wake_tab_cap * 4)) ||
      (s = srv_alloc(srv, &srv->slots, sizeof(SlotInfo) * MAX_SLOTS)) ||
      (s = srv_alloc(srv, &srv->st, 2 * sizeof(RoundState))) || (s = srv_alloc(srv, &srv->qcnt, 3 * 16 * 8)) ||
      (s = srv_alloc(srv, &srv->lr_part, 2 * (size_t)RT * 8)) ||
      (s = srv_alloc(srv, &srv->lb, sizeof(LaunchBlock))) || (s = srv_alloc(srv, &srv->ex_part, (size_t)RT * 8)) ||
      (s = srv_alloc(srv, &srv->ctrl, sizeof(Ctrl))) || (s = srv_alloc(srv, &srv->cuts, MAX_SLOTS * 8)) ||
      (s = srv_alloc(srv, &srv->check, 2 * CHECK_BLOCKS * 8)))
    return s;
  SRV_TRY(hipHostMalloc((void**)&srv->h_out, MAX_SLOTS * 2 * 8, hipHostMallocDefault));
  SRV_TRY(hipHostMalloc((void**)&srv->h_check, 2 * CHECK_BLOCKS * 8, hipHostMallocDefault));
  memset(srv->h_out, 0, MAX_SLOTS * 2 * 8);
  const hipStream_t q = srv->stream;
  // every vertex is settled (label 0) until a request claims it
  SRV_TRY(hipMemsetAsync(srv->P, 0, V * 8, q));
  SRV_TRY(hipMemsetAsync(srv->shift_g, 0, V * 8, q));
  SRV_TRY(hipMemsetAsync(srv->slots, 0, sizeof(SlotInfo) * MAX_SLOTS, q));
  SRV_TRY(hipMemsetAsync(srv->qcnt, 0, 3 * 16 * 8, q));
  SRV_TRY(hipMemsetAsync(srv->ex_part, 0, (size_t)RT * 8, q));
  SRV_TRY(hipMemsetAsync(srv->ctrl, 0, sizeof(Ctrl), q));
  SRV_TRY(hipMemsetAsync(srv->lr_part, 0xff, 2 * (size_t)RT * 8, q));
  RoundState pair[2] = {};
  for (auto& x : pair) {
    x.mode = MODE_ROUNDS;
    x.round = -1;  // step 1 runs round 0
    x.dir = DIR_TD;
    x.tail_round = -1;
  }
  pair[1].seq = -1;
  SRV_TRY(hipMemcpyAsync(srv->st, pair, sizeof(pair), hipMemcpyHostToDevice, q));
  srv->valloc.init(V);
  srv->aalloc.init(A);
  srv->walloc.init(srv->wake_tab_cap);

  int ncu = 0;
  SRV_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, srv->dev));
  srv->blocks = srv->cfg.blocks > 0 ? std::min(srv->cfg.blocks, RT) : std::min(2 * ncu, RT);

  LaunchBlock lb{};
  RoundCtx& c = lb.c;
  c.n = (int)V;
  c.B = srv->B;
  c.R = INT32_MAX;
  c.nnz = A;
  c.delta = srv->C;
  c.n_active = 0;
  c.row_ptr = (const int*)srv->rp_g;
  c.col = (const int*)srv->col_g;
  c.shift = (const long long*)srv->shift_g;
  c.P = (u64*)srv->P;
  c.qv[0] = (int*)srv->qv0;
  c.qv[1] = (int*)srv->qv1;
  c.qa[0] = (unsigned*)srv->qa0;
  c.qa[1] = (unsigned*)srv->qa1;
  c.wake_ord = (const int*)srv->wake_ord;
  c.wake_off = nullptr;
  c.next_ne = nullptr;
  c.wake_q = 0;
  c.qcnt = (u64*)srv->qcnt;
  c.lr_part = (u64*)srv->lr_part;
  c.stamp = nullptr;  // the tail is never entered
  c.st = (RoundState*)srv->st;
  c.ctrl = (Ctrl*)srv->ctrl;
  c.dir_policy = srv->cfg.direction;
  c.td_to_bu = 14;
  c.bu_to_td = 24;
  c.tail_den = 0;
  c.tail_min_left = 0;
  c.host_st = nullptr;
  c.ex_part = (u64*)srv->ex_part;
  c.slots = (const SlotInfo*)srv->slots;
  c.nslots = srv->cfg.max_slots;
  c.wake_tab = (const int*)srv->wake_tab;
  lb.kbase = 1;
  SRV_TRY(hipMemcpyAsync(srv->lb, &lb, sizeof(LaunchBlock), hipMemcpyHostToDevice, q));
  SRV_TRY(hipStreamSynchronize(q));
  // the step graph: chunk_steps round steps, then the step base moves on
  hipStream_t cap = nullptr;
  SRV_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  SRV_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < srv->cfg.chunk_steps; ++j)
    hipLaunchKernelGGL(k_round_step_lb, dim3(srv->blocks), dim3(RT), 0, cap, (const LaunchBlock*)srv->lb, j);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, cap, (LaunchBlock*)srv->lb, srv->cfg.chunk_steps);
  SRV_TRY(hipStreamEndCapture(cap, &g));
  SRV_TRY(hipGraphInstantiate(&srv->graph, g, nullptr, nullptr, 0));
  SRV_TRY(hipGraphDestroy(g));
  SRV_TRY(hipStreamDestroy(cap));
  return LDD_OK;
}

// Enqueue the admission of r (ranges already taken), its round 0 being global round r0.
ldd_status srv_admit(ldd_server* srv, Request* r, int slot, long long r0) {
  const hipStream_t s = srv->stream;
  const int n = r->q.n, R = r->R;
  const long long nnz = r->q.nnz;
  r->slot = slot;
  r->r0 = r0;
  const long long items = std::max<long long>((long long)n + 1, nnz);
  hipLaunchKernelGGL(k_slot_load, dim3((unsigned)std::min<long long>(8192, (items + 255) / 256)), dim3(256), 0, s,
                     r->vbeg, n, r->abeg, nnz, r->q.row_ptr, r->q.col_idx, (const long long*)r->q.shift_fix, r->delta, r0, srv->C,
                     srv->B, (int*)srv->rp_g, (int*)srv->col_g, (long long*)srv->shift_g, (u64*)srv->P);
  // wake-round counting sort into the slot's part of wake_ord; round offsets into wake_tab
  const int gs = (int)std::max<long long>(1, std::min<long long>(SORT_BLOCKS, n / 8192));
  int* roff = (int*)srv->wake_tab + r->wbase;
  hipLaunchKernelGGL(k_slot_hist, dim3(gs), dim3(1024), 0, s, n, R, r->q.row_ptr, (const long long*)r->q.shift_fix, r->delta,
                     (unsigned*)srv->mat, (int*)srv->qmax);
  hipLaunchKernelGGL(k_qbucket_scan, dim3((unsigned)(((long long)R * WAVE + 255) / 256)), dim3(256), 0, s, R, gs,
                     (unsigned*)srv->mat, (const int*)srv->qmax, (unsigned*)srv->tot);
  hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, s, R - 1, (const unsigned*)srv->tot, roff,
                     (int*)srv->scratch_ne);
  hipLaunchKernelGGL(k_slot_place, dim3(gs), dim3(1024), 0, s, n, R, r->vbeg, r->q.row_ptr, (const long long*)r->q.shift_fix, r->delta,
                     (const unsigned*)srv->mat, (const int*)roff, (int*)srv->wake_ord);
  SlotInfo e{};
  e.vbeg = r->vbeg;
  e.r0 = r0;
  e.R = R;
  e.wbase = (int)r->wbase;
  e.active = 1;
  srv->slot_tab[slot] = e;
  hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(64), 0, s, (SlotInfo*)srv->slots, slot, e);
  hipLaunchKernelGGL(k_state_add, dim3(1), dim3(64), 0, s, (RoundState*)srv->st, srv->steps, nnz);
  SRV_TRY(hipGetLastError());
  r->done_step = (r0 + R - 1) - srv->round_base + 1;  // the step that runs global round r0 + R - 1
  return LDD_OK;
}

// Enqueue the result of a request whose last round has run: centres into the caller's buffer,
// the cut, the slot leaves the table.  Its ranges are freed once the event has completed.
ldd_status srv_finish(ldd_server* srv, Request* r) {
  const hipStream_t s = srv->stream;
  const int n = r->q.n;
  const long long nnz = r->q.nnz;
  hipLaunchKernelGGL(k_slot_final, dim3((unsigned)std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256))),
                     dim3(256), 0, s, r->vbeg, n, srv->B, (const u64*)srv->P, r->q.centre);
  SRV_TRY(hipMemsetAsync((u64*)srv->cuts + r->slot, 0, 8, s));
  if (nnz)
    hipLaunchKernelGGL(k_slot_cut, dim3((unsigned)std::max<long long>(1, std::min<long long>(2048, nnz / 4096))),
                       dim3(256), 0, s, r->vbeg, n, r->abeg, nnz, (const int*)srv->rp_g, (const int*)srv->col_g,
                       (const int*)r->q.centre, (u64*)srv->cuts + r->slot);
  SlotInfo off{};
  srv->slot_tab[r->slot] = off;
  hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(64), 0, s, (SlotInfo*)srv->slots, r->slot, off);
  SRV_TRY(hipMemcpyAsync(srv->h_out + 2 * r->slot, (u64*)srv->cuts + r->slot, 8, hipMemcpyDeviceToHost, s));
  SRV_TRY(hipMemcpyAsync(srv->h_out + 2 * r->slot + 1, &((Ctrl*)srv->ctrl)->err, 4, hipMemcpyDeviceToHost, s));
  SRV_TRY(hipEventCreateWithFlags(&r->ev, hipEventDisableTiming));
  SRV_TRY(hipEventRecord(r->ev, s));
  SRV_TRY(hipGetLastError());
  r->state = RQ_FINISHING;
  return LDD_OK;
}

// Lower the global round numbering by X rounds (X <= every active slot's r0).
ldd_status srv_rebase(ldd_server* srv, long long X) {
  hipLaunchKernelGGL(k_rebase, dim3((unsigned)std::min<long long>(8192, (srv->vcap + 255) / 256)), dim3(256), 0,
                     srv->stream, srv->vcap, srv->B, srv->C, X, (u64*)srv->P, (long long*)srv->shift_g,
                     (u64*)srv->lr_part, 2 * RT, (RoundState*)srv->st, srv->steps);
  for (int i = 0; i < MAX_SLOTS; ++i) {
    if (!srv->slot_tab[i].active) continue;
    srv->slot_tab[i].r0 -= X;
    hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(64), 0, srv->stream, (SlotInfo*)srv->slots, i, srv->slot_tab[i]);
  }
  SRV_TRY(hipGetLastError());
  srv->round_base -= X;
  ++srv->rebases;
  return LDD_OK;
}

// Hand a request whose event has completed back to its caller.
ldd_status srv_complete(ldd_server* srv, Request* r) {
  const u64 arcs = srv->h_out[2 * r->slot], err = srv->h_out[2 * r->slot + 1] & 0xffffffffull;
  SRV_TRY(hipEventDestroy(r->ev));
  r->ev = nullptr;
  if (err) {
    snprintf(srv->fatal_msg, sizeof(srv->fatal_msg), "round engine error flags 0x%llx", (unsigned long long)err);
    return LDD_ERR_INTERNAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->valloc.give(r->vbeg, (long long)r->q.n + 1);
  srv->aalloc.give(r->abeg, r->q.nnz);
  srv->walloc.give(r->wbase, (long long)r->R + 1);
  srv->slot_req[r->slot] = nullptr;
  r->cut = (int64_t)(arcs / 2);
  r->status = LDD_OK;
  r->state = RQ_DONE;
  r->t_done = now_s();
  ++srv->completed;
  return LDD_OK;
}

ldd_status engine_loop(ldd_server* srv) {
  SRV_TRY(hipSetDevice(srv->dev));
  const int nslots = srv->cfg.max_slots;
  std::vector<Request*> finishing;
  int inflight = 0, oldest = 0;
  for (;;) {
    // 1. results whose copies have completed
    bool handed = false;
    for (size_t i = 0; i < finishing.size();) {
      const hipError_t e = hipEventQuery(finishing[i]->ev);
      if (e == hipErrorNotReady) {
        ++i;
        continue;
      }
      SRV_TRY(e);
      const ldd_status st = srv_complete(srv, finishing[i]);
      if (st != LDD_OK) return st;
      handed = true;
      finishing[i] = finishing.back();
      finishing.pop_back();
    }
    if (handed) srv->cv_done.notify_all();
    // 2. admission, first come first served, while the head of the queue fits
    int active = 0;
    long long min_r0 = -1;
    for (int i = 0; i < nslots; ++i)
      if (srv->slot_req[i] && srv->slot_req[i]->state == RQ_ACTIVE) {
        ++active;
        min_r0 = min_r0 < 0 ? srv->slot_tab[i].r0 : std::min(min_r0, srv->slot_tab[i].r0);
      }
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      if (active == 0 && inflight == 0 && finishing.empty()) {
        if (srv->stop && srv->queue.empty()) return LDD_OK;
        if (srv->queue.empty()) {
          srv->cv_work.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
          continue;
        }
      }
      const long long r_next = round_at(srv, srv->steps + 1);
      if (!srv->queue.empty() && r_next + srv->max_rounds > srv->round_limit) {
        const long long X = min_r0 < 0 ? r_next : std::min(min_r0, r_next);
        if (X > 0) {
          lk.unlock();
          const ldd_status st = srv_rebase(srv, X);
          if (st != LDD_OK) return st;
          lk.lock();
        }
      }
      while (!srv->queue.empty()) {
        Request* r = srv->queue.front();
        int slot = -1;
        for (int i = 0; i < nslots && slot < 0; ++i)
          if (!srv->slot_req[i]) slot = i;
        const long long r0 = round_at(srv, srv->steps + 1);
        if (slot < 0 || r0 + r->R > srv->round_limit) break;
        const long long vb = srv->valloc.take((long long)r->q.n + 1);
        const long long ab = vb < 0 ? -1 : srv->aalloc.take(r->q.nnz);
        const long long wb = ab < 0 ? -1 : srv->walloc.take((long long)r->R + 1);
        if (wb < 0) {
          if (ab >= 0) srv->aalloc.give(ab, r->q.nnz);
          if (vb >= 0) srv->valloc.give(vb, (long long)r->q.n + 1);
          break;
        }
        srv->queue.pop_front();
        r->vbeg = vb;
        r->abeg = ab;
        r->wbase = wb;
        r->state = RQ_ACTIVE;
        r->t_admit = now_s();
        srv->slot_req[slot] = r;
        ++srv->admitted;
        ++active;
        srv->max_active = std::max<long long>(srv->max_active, active);
        lk.unlock();
        const ldd_status st = srv_admit(srv, r, slot, r0);
        lk.lock();
        if (st != LDD_OK) return st;
      }
    }
    // 3. one more step chunk while any request is active (two chunks in flight)
    if (active > 0) {
      SRV_TRY(hipGraphLaunch(srv->graph, srv->stream));
      srv->steps += srv->cfg.chunk_steps;
      SRV_TRY(hipEventRecord(srv->chunk_ev[(oldest + inflight) & 1], srv->stream));
      ++inflight;
    }
    // 4. requests whose last round is enqueued: their results follow in stream order
    for (int i = 0; i < nslots; ++i) {
      Request* r = srv->slot_req[i];
      if (r && r->state == RQ_ACTIVE && r->done_step <= srv->steps) {
        const ldd_status st = srv_finish(srv, r);
        if (st != LDD_OK) return st;
        finishing.push_back(r);
        --active;
      }
    }
    // 5. wait: for the older chunk once two are in flight, else for whatever is outstanding
    if (inflight == 2 || (inflight > 0 && active == 0)) {
      SRV_TRY(hipEventSynchronize(srv->chunk_ev[oldest]));
      oldest ^= 1;
      --inflight;
    } else if (inflight == 0 && active == 0 && !finishing.empty()) {
      SRV_TRY(hipEventSynchronize(finishing.front()->ev));
    }
  }
}

void fail_all(ldd_server* srv, ldd_status st) {
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->fatal = st;
  srv->queue.clear();
  for (auto& kv : srv->all)
    if (kv.second->state != RQ_DONE) {
      kv.second->status = st;
      kv.second->state = RQ_DONE;
      kv.second->t_done = now_s();
    }
  srv->cv_done.notify_all();
}

void fill_result(const ldd_server* srv, const Request* r, ldd_result* out) {
  out->status = r->status;
  out->cut_edges = r->cut;
  out->rounds = r->R;
  out->first_round = r->r0;
  out->t_submit = r->t_submit - srv->t0;
  out->t_admit = r->t_admit > 0 ? r->t_admit - srv->t0 : 0;
  out->t_done = r->t_done - srv->t0;
  out->latency_ms = (r->t_done - r->t_submit) * 1e3;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------
extern "C" ldd_status ldd_server_create(const ldd_server_config* cfg, ldd_server** out) {
  if (!cfg || !out) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  *out = nullptr;
  ldd_server* srv = new ldd_server();
  srv->cfg = *cfg;
  srv->t0 = now_s();
  if (srv->cfg.max_slots <= 0 || srv->cfg.max_slots > MAX_SLOTS) srv->cfg.max_slots = MAX_SLOTS;
  if (srv->cfg.chunk_steps <= 0) srv->cfg.chunk_steps = 8;
  if (srv->cfg.chunk_steps > 64 || srv->cfg.direction < 0 || srv->cfg.direction > 2 || srv->cfg.blocks < 0 ||
      srv->cfg.max_rounds < 0) {
    delete srv;
    ldd_set_error("bad server configuration");
    return LDD_ERR_INVALID_ARG;
  }
  if (hipGetDevice(&srv->dev) != hipSuccess) {
    delete srv;
    ldd_set_error("no HIP device");
    return LDD_ERR_HIP;
  }
  long long V = srv->cfg.max_vertices, A = srv->cfg.max_arcs;
  if (V <= 0 || A <= 0) {  // split the budget for graphs of about 16 arcs per vertex
    V = srv->cfg.hbm_budget_bytes / (BYTES_PER_VERTEX + 16 * BYTES_PER_ARC);
    A = 16 * V;
  }
  const long long used = V * BYTES_PER_VERTEX + A * BYTES_PER_ARC;
  if (V < 2 || V > (1ll << 30) || A < 1 || A >= (1ll << 31) ||
      (srv->cfg.hbm_budget_bytes > 0 && used > srv->cfg.hbm_budget_bytes)) {
    delete srv;
    ldd_set_error("budget gives an unusable arena (%lld vertices, %lld arcs, %lld bytes)", V, A, used);
    return LDD_ERR_BUDGET;
  }
  srv->vcap = V;
  srv->acap = A;
  srv->B = log2_ceil(V);
  srv->round_limit = std::min<long long>(1ll << 30, 1ll << (64 - srv->B - FIX - 1));
  if (srv->cfg.max_rounds > 0) srv->round_limit = std::min<long long>(srv->round_limit, srv->cfg.max_rounds);
  srv->C = (u64)srv->round_limit << FIX;  // keys stay below C, and (C + 2^20) << B < 2^64
  srv->max_rounds = (int)std::min<long long>(QCAP, srv->round_limit / 2 - 1);
  if (srv->max_rounds < 1) {
    delete srv;
    ldd_set_error("max_rounds must be at least 4");
    return LDD_ERR_INVALID_ARG;
  }
  srv->wake_tab_cap = srv->cfg.max_slots * (srv->max_rounds + 1);
  const ldd_status s = srv_setup(srv);
  if (s != LDD_OK) {
    ldd_set_error("%s", srv->fatal_msg);
    ldd_server_destroy(srv);
    return s;
  }
  srv->engine = std::thread([srv] {
    const ldd_status st = engine_loop(srv);
    if (st != LDD_OK) fail_all(srv, st);
  });
  *out = srv;
  return LDD_OK;
}

extern "C" ldd_status ldd_server_submit(ldd_server* srv, const ldd_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || req->n < 0 || req->nnz < 0 || req->nnz >= (1ll << 31) ||
      (req->n > 0 && (!req->row_ptr || !req->shift_fix || !req->centre)) || (req->nnz > 0 && !req->col_idx) ||
      (req->nnz > 0 && req->n == 0)) {
    ldd_set_error("bad request");
    return LDD_ERR_INVALID_ARG;
  }
  if ((long long)req->n + 1 > srv->vcap || req->nnz > srv->acap) {
    ldd_set_error("request of %d vertices and %lld arcs exceeds the arena (%lld, %lld)", req->n,
                  (long long)req->nnz, srv->vcap, srv->acap);
    return LDD_ERR_BUDGET;
  }
  Request* r = new Request();
  r->q = *req;
  r->t_submit = now_s();
  if (req->n > 0) {
    // validate on the check stream, after the work the caller's stream has queued so far
    std::lock_guard<std::mutex> ck(srv->check_mu);
    int prev = 0;
    hipEvent_t ready = nullptr;
    bool ok = hipGetDevice(&prev) == hipSuccess && hipSetDevice(srv->dev) == hipSuccess &&
              hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess &&
              hipEventRecord(ready, (hipStream_t)req->hip_stream) == hipSuccess &&
              hipStreamWaitEvent(srv->check_stream, ready, 0) == hipSuccess;
    const long long items = std::max<long long>(req->n, req->nnz);
    const int gb = (int)std::max<long long>(1, std::min<long long>(CHECK_BLOCKS, (items + 1023) / 1024));
    if (ok) {
      hipLaunchKernelGGL(k_req_check, dim3(gb), dim3(256), 0, srv->check_stream, req->n, (long long)req->nnz,
                         req->row_ptr, req->col_idx, (const long long*)req->shift_fix, (u64*)srv->check);
      ok = hipGetLastError() == hipSuccess &&
           hipMemcpyAsync(srv->h_check, srv->check, 2 * gb * 8, hipMemcpyDeviceToHost, srv->check_stream) ==
               hipSuccess &&
           hipStreamSynchronize(srv->check_stream) == hipSuccess;
    }
    if (ready) (void)hipEventDestroy(ready);
    (void)hipSetDevice(prev);
    if (!ok) {
      delete r;
      ldd_set_error("request check failed: %s", hipGetErrorString(hipGetLastError()));
      return LDD_ERR_HIP;
    }
    u64 mx = 0, bad = 0;
    for (int b = 0; b < gb; ++b) {
      mx = std::max(mx, srv->h_check[2 * b]);
      bad |= srv->h_check[2 * b + 1];
    }
    if (bad) {
      delete r;
      ldd_set_error("invalid request:%s%s%s", (bad & ERR_BAD_SHIFT) ? " shift out of [0, 2^52]" : "",
                    (bad & ERR_BAD_ROWPTR) ? " row offsets" : "", (bad & ERR_BAD_COL) ? " column id out of range" : "");
      return LDD_ERR_INVALID_ARG;
    }
    r->delta = mx;
    const long long R = (long long)(mx >> FIX) + 1;
    if (R > srv->max_rounds) {
      delete r;
      ldd_set_error("request needs %lld rounds; this server takes at most %d", R, srv->max_rounds);
      return LDD_ERR_OVERFLOW;
    }
    r->R = (int)R;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->fatal != LDD_OK || srv->stop) {
      delete r;
      ldd_set_error("server is not running: %s", srv->fatal_msg);
      return srv->fatal != LDD_OK ? srv->fatal : LDD_ERR_INVALID_ARG;
    }
    r->ticket = srv->next_ticket++;
    srv->all[r->ticket] = r;
    if (req->n == 0) {  // nothing to decompose
      r->status = LDD_OK;
      r->state = RQ_DONE;
      r->t_admit = r->t_done = now_s();
    } else {
      srv->queue.push_back(r);
    }
  }
  srv->cv_work.notify_all();
  *ticket = r->ticket;
  return LDD_OK;
}

extern "C" ldd_status ldd_server_poll(ldd_server* srv, uint64_t ticket, ldd_result* out) {
  if (!srv || !out) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) {
    ldd_set_error("unknown ticket %llu", (unsigned long long)ticket);
    return LDD_ERR_INVALID_ARG;
  }
  Request* r = it->second;
  if (r->state != RQ_DONE) return LDD_ERR_PENDING;
  fill_result(srv, r, out);
  srv->all.erase(it);
  delete r;
  if (out->status != LDD_OK && srv->fatal != LDD_OK) ldd_set_error("server failed: %s", srv->fatal_msg);
  return out->status;
}

extern "C" ldd_status ldd_server_wait(ldd_server* srv, uint64_t ticket, ldd_result* out) {
  if (!srv || !out) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) {
    ldd_set_error("unknown ticket %llu", (unsigned long long)ticket);
    return LDD_ERR_INVALID_ARG;
  }
  Request* r = it->second;
  srv->cv_done.wait(lk, [&] { return r->state == RQ_DONE; });
  fill_result(srv, r, out);
  srv->all.erase(it);
  delete r;
  if (out->status != LDD_OK && srv->fatal != LDD_OK) ldd_set_error("server failed: %s", srv->fatal_msg);
  return out->status;
}

extern "C" ldd_status ldd_server_cancel(ldd_server* srv, uint64_t ticket) {
  if (!srv) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) {
    ldd_set_error("unknown ticket %llu", (unsigned long long)ticket);
    return LDD_ERR_INVALID_ARG;
  }
  Request* r = it->second;
  if (r->state != RQ_QUEUED) return LDD_ERR_PENDING;  // admitted or done: it runs to the end
  srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), r));
  r->status = LDD_ERR_CANCELLED;
  r->state = RQ_DONE;
  r->t_done = now_s();
  srv->cv_done.notify_all();
  return LDD_OK;
}

extern "C" ldd_status ldd_server_query(ldd_server* srv, ldd_server_info* out) {
  if (!srv || !out) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  out->arena_vertices = srv->vcap;
  out->arena_arcs = srv->acap;
  out->max_rounds = srv->max_rounds;
  out->max_slots = srv->cfg.max_slots;
  out->admitted = srv->admitted;
  out->completed = srv->completed;
  out->queued = (int64_t)srv->queue.size();
  out->max_active = srv->max_active;
  out->steps = srv->steps;
  out->rebases = srv->rebases;
  return srv->fatal;
}

extern "C" ldd_status ldd_server_destroy(ldd_server* srv) {
  if (!srv) {
    ldd_set_error("NULL argument");
    return LDD_ERR_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->engine.joinable()) srv->engine.join();
  const ldd_status fatal = srv->fatal;
  if (srv->stream) (void)hipStreamSynchronize(srv->stream);
  if (srv->check_stream) (void)hipStreamSynchronize(srv->check_stream);
  for (void* p : {srv->P, srv->qv0, srv->qv1, srv->qa0, srv->qa1, srv->wake_ord, srv->rp_g, srv->col_g, srv->shift_g,
                  srv->mat, srv->qmax, srv->tot, srv->scratch_ne, srv->wake_tab, srv->slots, srv->st, srv->qcnt,
                  srv->lr_part, srv->lb, srv->ex_part, srv->ctrl, srv->cuts, srv->check})
    if (p) (void)hipFree(p);
  if (srv->h_out) (void)hipHostFree(srv->h_out);
  if (srv->h_check) (void)hipHostFree(srv->h_check);
  if (srv->graph) (void)hipGraphExecDestroy(srv->graph);
  for (auto& e : srv->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  if (srv->check_stream) (void)hipStreamDestroy(srv->check_stream);
  for (auto& kv : srv->all) {
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    delete kv.second;
  }
  delete srv;
  return fatal;
}
