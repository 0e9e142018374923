// Host side of libldd: argument checks, device workspace, kernel sequencing, error mapping.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/ldd.h"
#include "ldd_block.h"
#include "ldd_internal.h"
#include "ldd_kernels.h"

using namespace ldd;

// ------------------------------------------------------------------------------------------
// errors
// ------------------------------------------------------------------------------------------
static thread_local char g_err[512];

void ldd_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" const char* ldd_last_error(void) { return g_err; }

extern "C" const char* ldd_status_string(ldd_status s) {
  switch (s) {
    case LDD_OK: return "ok";
    case LDD_ERR_INVALID_ARG: return "invalid argument";
    case LDD_ERR_OOM: return "out of device memory";
    case LDD_ERR_OVERFLOW: return "label width overflow";
    case LDD_ERR_HIP: return "HIP runtime error";
    case LDD_ERR_BUDGET: return "request exceeds memory budget";
    case LDD_ERR_CANCELLED: return "cancelled";
    case LDD_ERR_INTERNAL: return "internal error";
    case LDD_ERR_PENDING: return "pending";
    case LDD_ERR_RETRIES: return "no draw met the bounds";
  }
  return "unknown status";
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ldd_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return LDD_ERR_HIP;                                                               \
    }                                                                                   \
  } while (0)

// ------------------------------------------------------------------------------------------
// workspace: one per device, grown on demand, guarded by a mutex for the whole call
// ------------------------------------------------------------------------------------------
namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

ldd_status grow(Buf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return LDD_OK;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  size_t want = bytes < 256 ? 256 : bytes;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ldd_set_error("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    return LDD_ERR_OOM;
  }
  b.bytes = want;
  return LDD_OK;
}

struct HostMirror {  // pinned, mapped host memory
  Ctrl ctrl;
  u64 ex_part[RT];
  Report report;   // written by the device as a decomposition ends
  BlockOut bout;   // the workgroup engine's result for one graph
};

constexpr int CHUNK = 8;     // steps per graph replay
constexpr int INFLIGHT = 2;  // replays enqueued ahead of the one running
// Replays enqueued after the last step that has work return at once, but the output pass
// queues behind them: so the second replay is a short one, and once the tail has started (a
// few sweeps are left) the next replays are short again, growing back to CHUNK.
constexpr int CHUNK_SIZES[] = {2, 4, CHUNK};

struct StepGraph {
  int blocks = 0, steps = 0;
  hipGraphExec_t exec = nullptr;
};

struct Workspace {
  std::mutex mu;
  Buf P, qv0, qv1, qa0, qa1, wake_ord, stamp, hub_bits;  // per vertex
  unsigned stamp_base = 0;     // every tail stamp in `stamp` is <= stamp_base ...
  void* stamp_clean = nullptr;  // ... while this equals stamp.p
  Buf hist, cursor, wake_off, next_ne, mat, qmax;        // per round / q-bucket (mat: per bucket and prep block)
  Buf cand, cand_cnt;                                    // per prep block: first-window candidates
  Buf ctrl, st, qcnt, lr_part, lb, ex_part, vr;
  // workgroup engine: queues and wake order (3 ints per vertex), jobs, order, results, job counter
  Buf bk_wq, bk_jobs, bk_order, bk_out, bk_cnt, bk_team, bk_sync;
  // batch: union CSR with global ids, adjusted shifts, graph of each vertex, per-graph data
  Buf b_rp, b_col, b_shift, b_gid, b_off, b_dg, b_cut;
  HostMirror* host = nullptr;
  hipEvent_t ev[6] = {};
  hipEvent_t chunk_ev[INFLIGHT] = {};
  hipEvent_t out_ev = nullptr;
  hipStream_t capture = nullptr;
  hipStream_t out = nullptr;  // the output pass, concurrent with the replays still queued
  std::vector<StepGraph> graphs;
  int num_cu = 0;
  int max_coresident = 0;  // co-resident blocks of the persistent round kernel
  int block_coresident = 0;  // co-resident workgroups of the workgroup engine (a team's bound)
  int lds_bytes = 0;       // dynamic LDS the workgroup engine may take (0: the device refused the size)
};

std::mutex g_ws_mu;
std::vector<Workspace*> g_ws;

Workspace* workspace_for(int dev) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1, nullptr);
  if (!g_ws[dev]) g_ws[dev] = new Workspace();
  return g_ws[dev];
}

ldd_status ws_setup(Workspace& w) {
  if (!w.host) {
    HIP_TRY(hipHostMalloc((void**)&w.host, sizeof(HostMirror), hipHostMallocMapped | hipHostMallocCoherent));
    for (auto& e : w.ev) HIP_TRY(hipEventCreate(&e));
    for (auto& e : w.chunk_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIP_TRY(hipStreamCreateWithFlags(&w.capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&w.out, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&w.out_ev, hipEventDisableTiming));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&w.num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_rounds_persistent),
                                                         RT, 0));
    // one block per CU at most: measured co-residency of large cooperative grids falls short
    // of what the occupancy query reports, and barrier cost grows with the block count
    w.max_coresident = w.num_cu * (per_cu < 1 ? 0 : 1);
    int per_cu_block = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_block, reinterpret_cast<const void*>(k_block_decompose),
                                                         1024, 0));
    w.block_coresident = w.num_cu * std::max(per_cu_block, 1);
    // the workgroup engine's dynamic LDS for small graphs (beside its static LDS)
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_block_decompose), hipFuncAttributeMaxDynamicSharedMemorySize,
                            BLOCK_LDS_BYTES) == hipSuccess)
      w.lds_bytes = BLOCK_LDS_BYTES;
    else
      (void)hipGetLastError();
  }
  ldd_status s;
  if ((s = grow(w.ctrl, sizeof(Ctrl))) || (s = grow(w.st, 2 * sizeof(RoundState))) ||
      (s = grow(w.qcnt, 3 * 16 * sizeof(u64))) || (s = grow(w.lr_part, 2 * (size_t)RT * sizeof(u64))) ||
      (s = grow(w.lb, sizeof(LaunchBlock))) || (s = grow(w.ex_part, (size_t)RT * sizeof(u64))))
    return s;
  return LDD_OK;
}

// A graph of `steps` step launches (reading their arguments from the workspace's LaunchBlock)
// followed by one k_advance; instantiated once per grid size and length, replayed for every call.
ldd_status step_graph(Workspace& w, int blocks, int steps, hipGraphExec_t* out) {
  for (auto& g : w.graphs)
    if (g.blocks == blocks && g.steps == steps) {
      *out = g.exec;
      return LDD_OK;
    }
  const LaunchBlock* lbp = (const LaunchBlock*)w.lb.p;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(w.capture, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < steps; ++j) hipLaunchKernelGGL(k_round_step_lb, dim3(blocks), dim3(RT), 0, w.capture, lbp, j);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, w.capture, (LaunchBlock*)w.lb.p, steps);
  HIP_TRY(hipStreamEndCapture(w.capture, &graph));
  hipGraphExec_t exec = nullptr;
  HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  HIP_TRY(hipGraphDestroy(graph));
  w.graphs.push_back({blocks, steps, exec});
  *out = exec;
  return LDD_OK;
}

int ceil_log2(long long n) {
  int b = 0;
  while ((1ll << b) < n) ++b;
  return b;
}

int grid_for(long long items, int threads, int cap) {
  long long g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

extern "C" size_t ldd_workspace_bytes(int32_t n, int64_t nnz) {
  (void)nnz;
  const size_t nv = n > 0 ? (size_t)n : 1;
  // labels 8 + two queues (4 + 4 each) + wake order 4 + tail stamp 4 = 32 bytes per vertex, the
  // piece bitmap, the preparation's per-block bucket counts and window lists, rounds arrays
  // sized by the shift range (bounded here by 2^16 rounds) and the control block; and the
  // workgroup engines' wake list and queues (16 bytes per vertex) with a team's record and the
  // result record, which one call may hold beside the rest (a team that refuses a graph)
  const size_t gp = std::min<size_t>(1024, std::max<size_t>(1, nv / 16384));
  return nv * 48 + (nv + 63) / 64 * 8 + gp * ((size_t)QCAP * 4 + (size_t)CAND * 8 + 8) +
         (size_t)(65536 + 2) * (4 * 4) + sizeof(Ctrl) + 2 * sizeof(RoundState) + 3 * 16 * 8 + 2 * (size_t)RT * 8 +
         sizeof(TeamSync) + sizeof(BlockOut);
}

extern "C" void ldd_release_workspace(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  Workspace* w = workspace_for(dev);
  std::lock_guard<std::mutex> lk(w->mu);
  (void)hipDeviceSynchronize();  // round steps a call left queued (they return at once) may still read it
  for (auto& g : w->graphs) (void)hipGraphExecDestroy(g.exec);  // they hold workspace pointers
  w->graphs.clear();
  for (Buf* b : {&w->P, &w->qv0, &w->qv1, &w->qa0, &w->qa1, &w->wake_ord, &w->stamp, &w->hub_bits, &w->hist,
                 &w->cursor, &w->wake_off, &w->next_ne, &w->mat, &w->qmax, &w->cand, &w->cand_cnt, &w->ctrl, &w->st, &w->qcnt, &w->lr_part,
                 &w->lb, &w->ex_part, &w->vr, &w->bk_wq, &w->bk_jobs, &w->bk_order, &w->bk_out, &w->bk_cnt, &w->bk_team, &w->bk_sync, &w->b_rp, &w->b_col, &w->b_shift, &w->b_gid, &w->b_off, &w->b_dg,
                 &w->b_cut}) {
    if (b->p) (void)hipFree(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
}

// ------------------------------------------------------------------------------------------
// single graph
// ------------------------------------------------------------------------------------------
static ldd_status finish_error(unsigned err) {
  if (err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) {
    ldd_set_error("invalid input:%s%s%s", (err & ERR_BAD_SHIFT) ? " shift out of [0, 2^52]" : "",
                  (err & ERR_BAD_ROWPTR) ? " row_ptr not a valid offset array" : "",
                  (err & ERR_BAD_COL) ? " column id out of range" : "");
    return LDD_ERR_INVALID_ARG;
  }
  if (err) {
    ldd_set_error("internal error flags 0x%x%s%s%s", err, (err & ERR_BARRIER) ? " barrier-timeout" : "",
                  (err & ERR_WATCHDOG) ? " round-watchdog" : "", (err & ERR_QUEUE) ? " queue-overflow" : "");
    return LDD_ERR_INTERNAL;
  }
  return LDD_OK;
}

// Per-graph bookkeeping when the graph being decomposed is the disjoint union of a batch.
struct BatchView {
  const int* gid;          // device [n]: graph of every vertex
  u64* cut_g;              // device [G]: 2 x cut edges per graph (see k_cut)
};

static ldd_status decompose_impl(Workspace& w, const ldd_csr* g, const int64_t* shift_fix, int32_t* centre,
                                 int64_t* cut_edges, const ldd_options& o, ldd_stats* stats, hipStream_t st,
                                 const BatchView* bv);

extern "C" ldd_status ldd_decompose(const ldd_csr* g, const int64_t* shift_fix, double beta, int32_t* centre,
                                    int64_t* cut_edges, const ldd_options* opt, ldd_stats* stats, void* hip_stream) {
  g_err[0] = 0;
  if (!g) {
    ldd_set_error("graph is NULL");
    return LDD_ERR_INVALID_ARG;
  }
  const int n = g->n;
  const long long nnz = g->nnz;
  if (n < 0 || nnz < 0 || nnz >= (1ll << 31)) {
    ldd_set_error("bad sizes n=%d nnz=%lld (need n >= 0, 0 <= nnz < 2^31)", n, nnz);
    return LDD_ERR_INVALID_ARG;
  }
  if (!(beta > 0.0)) {
    ldd_set_error("beta must be positive");
    return LDD_ERR_INVALID_ARG;
  }
  if (n > 0 && (!g->row_ptr || !shift_fix || !centre || (nnz > 0 && !g->col_idx))) {
    ldd_set_error("NULL device pointer");
    return LDD_ERR_INVALID_ARG;
  }
  ldd_options o{};
  if (opt) o = *opt;
  if (o.direction < 0 || o.direction > 2 || o.engine < 0 || o.engine > 4 || o.blocks < 0) {
    ldd_set_error("bad options");
    return LDD_ERR_INVALID_ARG;
  }
  if (stats) memset(stats, 0, sizeof(*stats));
  if (n == 0) {
    if (cut_edges) *cut_edges = 0;
    return LDD_OK;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace& w = *workspace_for(dev);
  std::lock_guard<std::mutex> lk(w.mu);
  return decompose_impl(w, g, shift_fix, centre, cut_edges, o, stats, st, nullptr);
}

static const ldd_status REDO_WIDE = static_cast<ldd_status>(100);  // internal: run again on the wide layout

// The largest distance from a vertex to its centre, from the final labels still in the workspace.
static ldd_status max_radius(Workspace& w, int n, const int64_t* shift_fix, u64 delta, hipStream_t st, int64_t* out) {
  ldd_status s = grow(w.vr, 256);
  if (s != LDD_OK) return s;
  const int B = ceil_log2(n) < 1 ? 1 : ceil_log2(n);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (u64*)w.vr.p, 1ll, 0ull);
  hipLaunchKernelGGL(k_max_radius, dim3(grid_for(n, 256 * 8, 2048)), dim3(256), 0, st, n, B, (const u64*)w.P.p,
                     (const long long*)shift_fix, delta, (u64*)w.vr.p);
  HIP_TRY(hipGetLastError());
  u64 radius = 0;
  HIP_TRY(hipMemcpyAsync(&radius, w.vr.p, sizeof(u64), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = (int64_t)radius;
  return LDD_OK;
}

// One decomposition.  wide = false: the sorted (q-bucket) layout, enqueued in full without the
// host waiting (k_setup decides on the device whether the rounds run); if the shifts turn out to
// span QCAP units or more, the run reports REDO_WIDE and is redone with wide = true, whose
// preparation reads Delta on the host to size its per-round arrays.
static ldd_status decompose_run(Workspace& w, const ldd_csr* g, const int64_t* shift_fix, int32_t* centre,
                                int64_t* cut_edges, const ldd_options& o, ldd_stats* stats, hipStream_t st,
                                const BatchView* bv, bool wide) {
  const int n = g->n;
  const long long nnz = g->nnz;
  ldd_status s = ws_setup(w);
  if (s != LDD_OK) return s;
  const size_t nv = (size_t)n;
  if ((s = grow(w.P, nv * 8)) || (s = grow(w.qv0, nv * 4)) || (s = grow(w.qv1, nv * 4)) || (s = grow(w.qa0, nv * 4)) ||
      (s = grow(w.qa1, nv * 4)) || (s = grow(w.wake_ord, nv * 4)) || (s = grow(w.stamp, nv * 4)) ||
      (s = grow(w.hub_bits, (nv + 63) / 64 * 8)))
    return s;
  Ctrl* ctrl = (Ctrl*)w.ctrl.p;
  u64* P = (u64*)w.P.p;
  const int B = ceil_log2(n) < 1 ? 1 : ceil_log2(n);

  // the previous call on this workspace may have left idle steps queued on its stream, which
  // read the argument block and the state this call is about to rewrite: start after them
  HIP_TRY(hipStreamWaitEvent(st, w.ev[2], 0));
  HIP_TRY(hipEventRecord(w.ev[0], st));
  const int g_n = grid_for(n, 256 * 4, 2048);
  // preparation pass A: labels, Delta, checks and the q-bucket histogram (per block)
  const int gp = (int)std::min<long long>(1024, std::max<long long>(1, n / 16384));
  if ((s = grow(w.mat, (size_t)QCAP * gp * 4)) || (s = grow(w.qmax, (size_t)gp * 4)) ||
      (s = grow(w.cand, (size_t)CAND * gp * 8)) || (s = grow(w.cand_cnt, (size_t)gp * 4)))
    return s;
  HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(Ctrl), st));
  hipLaunchKernelGGL(k_init, dim3(gp), dim3(1024), 0, st, n, nnz, g->row_ptr, (const long long*)shift_fix, P, ctrl,
                     (unsigned*)w.mat.p, (int*)w.qmax.p, (u64*)w.cand.p, (unsigned*)w.cand_cnt.p);
  if (o.validate && nnz > 0)
    hipLaunchKernelGGL(k_check_cols, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, st, n, nnz, g->col_idx, ctrl);
  HIP_TRY(hipGetLastError());

  long long R_bound;  // rounds bound for the host's step limit
  if (!wide) {
    // pass B: vertices sorted by the integer part of their shift, no global atomics; only the
    // first window of buckets is placed now (the round steps place the rest when needed)
    const size_t nq = (size_t)QCAP + 2;
    if ((s = grow(w.hist, nq * 4)) || (s = grow(w.wake_off, nq * 4)) || (s = grow(w.next_ne, nq * 4))) return s;
    R_bound = QCAP;
    hipLaunchKernelGGL(k_qbucket_scan, dim3(std::min(QCAP, 1024)), dim3(256), 0, st, gp, (unsigned*)w.mat.p,
                       (const int*)w.qmax.p, (unsigned*)w.hist.p, (const Ctrl*)ctrl);
    hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, st, (const Ctrl*)ctrl, (const unsigned*)w.hist.p,
                       (int*)w.wake_off.p, (int*)w.next_ne.p);
    hipLaunchKernelGGL(k_place_window, dim3(gp), dim3(256), 0, st, (const Ctrl*)ctrl, (const unsigned*)w.mat.p,
                       (const int*)w.qmax.p, (const int*)w.wake_off.p, (const u64*)w.cand.p,
                       (const unsigned*)w.cand_cnt.p, (int*)w.wake_ord.p);
  } else {
    // shifts spanning QCAP units or more: exact wake rounds via global atomics, arrays sized
    // by the rounds bound the host reads first
    HIP_TRY(hipMemcpyAsync(&w.host->ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    {
      ldd_status e = finish_error(w.host->ctrl.err);
      if (e != LDD_OK) return e;
    }
    const u64 delta = w.host->ctrl.delta;
    if ((delta + (1ull << FIX)) >= (1ull << (64 - B))) {
      ldd_set_error("labels need (Delta + 2^20) << %d < 2^64 (Delta = %llu)", B, (unsigned long long)delta);
      return LDD_ERR_OVERFLOW;
    }
    const long long R = (long long)(delta >> FIX) + 1;
    if (R > (1ll << 28)) {
      ldd_set_error("shift range needs %lld rounds", R);
      return LDD_ERR_OVERFLOW;
    }
    R_bound = R;
    const size_t nr = (size_t)R + 2;
    if ((s = grow(w.hist, nr * 4)) || (s = grow(w.cursor, nr * 4)) || (s = grow(w.wake_off, nr * 4)) ||
        (s = grow(w.next_ne, nr * 4)))
      return s;
    HIP_TRY(hipMemsetAsync(w.hist.p, 0, nr * 4, st));
    hipLaunchKernelGGL(k_wake_count, dim3(g_n), dim3(256), 0, st, n, B, g->row_ptr, (const long long*)shift_fix,
                       (const Ctrl*)ctrl, P, (unsigned*)w.hist.p, (int)R, 0);
    hipLaunchKernelGGL(k_wake_scan, dim3(1), dim3(1024), 0, st, (int)R, (const unsigned*)w.hist.p,
                       (int*)w.wake_off.p, (int*)w.cursor.p, (int*)w.next_ne.p);
    hipLaunchKernelGGL(k_wake_scatter, dim3(g_n), dim3(256), 0, st, n, g->row_ptr, (const long long*)shift_fix,
                       (const Ctrl*)ctrl, (int*)w.cursor.p, (int*)w.wake_ord.p);
  }
  HIP_TRY(hipGetLastError());

  const int tail_den = o.tail_vertices < 0 ? 0 : (o.tail_vertices > 0 ? o.tail_vertices : 32);
  // tail stamps: cleared only when the buffer is new, was left in an unknown state, or the
  // base has come within 2^30 of wrapping; otherwise this call's tags lie above every old one
  if (tail_den && (w.stamp_clean != w.stamp.p || w.stamp_base >= (1u << 30))) {
    HIP_TRY(hipMemsetAsync(w.stamp.p, 0, w.stamp.bytes, st));
    w.stamp_base = 0;
  }
  const unsigned stamp_base = w.stamp_base;
  w.stamp_clean = nullptr;  // unknown until this call's steps are counted

  // round arguments; Delta, the rounds bound and the vertices with arcs are filled in by k_setup
  RoundCtx c{};
  c.n = n;
  c.B = B;
  c.nnz = nnz;
  c.row_ptr = g->row_ptr;
  c.col = g->col_idx;
  c.shift = (const long long*)shift_fix;
  c.P = P;
  c.qv[0] = (int*)w.qv0.p;
  c.qv[1] = (int*)w.qv1.p;
  c.qa[0] = (unsigned*)w.qa0.p;
  c.qa[1] = (unsigned*)w.qa1.p;
  c.wake_ord = (int*)w.wake_ord.p;
  c.wake_off = (const int*)w.wake_off.p;
  c.next_ne = (const int*)w.next_ne.p;
  c.wake_q = wide ? 0 : 1;
  c.prep_blocks = gp;
  c.mat = (const unsigned*)w.mat.p;
  c.qmax = (const int*)w.qmax.p;
  c.qcnt = (u64*)w.qcnt.p;
  c.lr_part = (u64*)w.lr_part.p;
  c.stamp = (unsigned*)w.stamp.p;
  c.stamp_base = stamp_base;
  c.st = (RoundState*)w.st.p;
  c.ctrl = ctrl;
  c.dir_policy = o.direction;
  c.td_to_bu = o.td_to_bu > 0 ? o.td_to_bu : 14;
  c.bu_to_td = o.bu_to_td > 0 ? o.bu_to_td : 24;
  c.tail_den = tail_den;
  c.tail_min_left = 16;
  c.ex_part = (u64*)w.ex_part.p;
  void* report_dev = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&report_dev, &w.host->report, 0));
  c.report = (Report*)report_dev;
  volatile Report* rep = &w.host->report;
  rep->ready = 0;
  rep->out_ready = 0;
  rep->tail_hint = 0;

  const int engine = o.engine == LDD_ENGINE_PERSISTENT ? LDD_ENGINE_PERSISTENT : LDD_ENGINE_LAUNCH;
  int blocks = o.blocks > 0 ? o.blocks : 2 * w.num_cu;
  if (blocks > RT) blocks = RT;  // the per-block minima of a step are reduced by one block
  if (engine == LDD_ENGINE_PERSISTENT && blocks > w.max_coresident) blocks = w.max_coresident;
  // rounds, placement steps, tail sweeps (each settles or lowers at least one label) and slack
  const long long kmax = R_bound + R_bound / ABUF + 1 + (long long)n + 2;
  long long steps = 0;
  hipGraphExec_t exec[3] = {};
  if (engine != LDD_ENGINE_PERSISTENT)
    for (int i = 0; i < 3; ++i)
      if ((s = step_graph(w, blocks, CHUNK_SIZES[i], &exec[i]))) return s;
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, c, (LaunchBlock*)w.lb.p, wide ? 0 : 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(w.ev[1], st));
  // The host spins on the report (written by the step that finds the rounds done) and on the
  // oldest replay's completion, which makes room for another.  Replays still queued after the
  // report return at once; the output pass runs on its own stream beside them.
  if (engine == LDD_ENGINE_PERSISTENT) {
    const LaunchBlock* lbp = (const LaunchBlock*)w.lb.p;
    void* args[] = {&lbp};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_rounds_persistent), dim3(blocks), dim3(RT), args,
                                       0, st));
    HIP_TRY(hipEventRecord(w.chunk_ev[0], st));
    while (!rep->ready) {
      const hipError_t q = hipEventQuery(w.chunk_ev[0]);
      if (q == hipErrorNotReady) {
        __builtin_ia32_pause();
        continue;
      }
      HIP_TRY(q);
      break;  // ended: the report is there, or missing (checked below)
    }
    steps = 1;
  } else {
    long long submitted = 0;
    int head = 0;
    // replay lengths: CHUNK, then short; after the tail hint short again, then growing
    int size_i = 2, hint_seen = 0;
    auto launch = [&](int slot, int i) -> hipError_t {
      hipError_t e = hipGraphLaunch(exec[i], st);
      if (e == hipSuccess) e = hipEventRecord(w.chunk_ev[slot], st);
      submitted += CHUNK_SIZES[i];
      return e;
    };
    HIP_TRY(launch(0, 2));
    HIP_TRY(launch(1, 0));
    while (!rep->ready) {
      const hipError_t q = hipEventQuery(w.chunk_ev[head]);
      if (q == hipErrorNotReady) {
        __builtin_ia32_pause();
        continue;
      }
      HIP_TRY(q);
      if (rep->ready) break;
      if (submitted > kmax) {
        HIP_TRY(hipStreamSynchronize(st));
        ldd_set_error("round steps exceeded their bound (%lld)", kmax);
        return LDD_ERR_INTERNAL;
      }
      if (!hint_seen && rep->tail_hint) {
        hint_seen = 1;
        size_i = 0;
      }
      HIP_TRY(launch(head, size_i));
      if (size_i < 2) ++size_i;
      head = (head + 1) % INFLIGHT;
    }
    steps = submitted;
    // step k tags at most stamp_base + k + 1 (k <= submitted): the next call starts above that
    w.stamp_base = stamp_base + (unsigned)submitted + 2;
    w.stamp_clean = w.stamp.p;
  }
  HIP_TRY(hipEventRecord(w.ev[2], st));  // after every step enqueued, idle ones included
  if (!rep->ready) {
    HIP_TRY(hipStreamSynchronize(st));
    ldd_set_error("the rounds ended without a report");
    return LDD_ERR_INTERNAL;
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  switch (rep->setup) {
    case SETUP_OK:
    case SETUP_EMPTY:
      break;
    case SETUP_WIDE:
      HIP_TRY(hipStreamSynchronize(st));
      return REDO_WIDE;
    case SETUP_OVERFLOW:
      ldd_set_error("labels need (Delta + 2^20) << %d < 2^64 and at most 2^28 rounds (Delta = %llu)", B,
                    (unsigned long long)rep->delta);
      return LDD_ERR_OVERFLOW;
    default: {
      ldd_status e = finish_error(rep->err);
      return e != LDD_OK ? e : LDD_ERR_INTERNAL;
    }
  }
  {
    ldd_status e = finish_error(rep->err);
    if (e != LDD_OK) return e;
  }
  // output pass: every label is final once the report is there
  const hipStream_t so = w.out;
  HIP_TRY(hipEventRecord(w.ev[3], so));
  const int g_f = grid_for((n + 63) / 64, 128, 2048);  // whole bitmap words per block
  hipLaunchKernelGGL(k_finalize, dim3(g_f), dim3(512), 0, so, n, B, g->row_ptr, (const u64*)P, centre,
                     (u64*)w.hub_bits.p, (int*)w.qv0.p, (unsigned*)w.qa0.p, ctrl);
  HIP_TRY(hipEventRecord(w.ev[4], so));
  if (nnz > 0)
    hipLaunchKernelGGL(k_cut, dim3(grid_for(nnz, 256 * 8, 2048)), dim3(256), 0, so, n, g->row_ptr, g->col_idx,
                       (const int*)centre, (const u64*)w.hub_bits.p, (const int*)w.qv0.p, (const unsigned*)w.qa0.p,
                       ctrl, bv ? bv->gid : nullptr, bv ? bv->cut_g : nullptr);
  HIP_TRY(hipEventRecord(w.ev[5], so));
  hipLaunchKernelGGL(k_out_report, dim3(1), dim3(64), 0, so, (const Ctrl*)ctrl, c.report);
  HIP_TRY(hipGetLastError());
  if (stats) HIP_TRY(hipMemcpyAsync(w.host->ex_part, w.ex_part.p, (size_t)blocks * sizeof(u64), hipMemcpyDeviceToHost, so));
  HIP_TRY(hipEventRecord(w.out_ev, so));
  HIP_TRY(hipStreamWaitEvent(st, w.out_ev, 0));  // later work on the caller's stream sees the output
  if (stats) {
    HIP_TRY(hipEventSynchronize(w.out_ev));
    HIP_TRY(hipEventSynchronize(w.ev[2]));
  } else {
    while (!rep->out_ready) {
      const hipError_t q = hipEventQuery(w.out_ev);
      if (q == hipErrorNotReady) {
        __builtin_ia32_pause();
        continue;
      }
      HIP_TRY(q);
      break;
    }
  }
  if (!rep->out_ready) {
    ldd_set_error("the output pass ended without a report");
    return LDD_ERR_INTERNAL;
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  {
    ldd_status e = finish_error(rep->out_err);
    if (e != LDD_OK) return e;
  }
  const u64 delta = rep->delta, n_active = rep->n_active;
  const long long R = (long long)(delta >> FIX) + 1;
  const RoundState fs = *(const RoundState*)&rep->st;
  if (rep->unreached != 0 || (n_active > 0 && fs.mode != MODE_DONE)) {
    ldd_set_error("rounds ended with %llu labels unset (mode %lld)", (unsigned long long)rep->unreached, fs.mode);
    return LDD_ERR_INTERNAL;
  }
  if (cut_edges) *cut_edges = (int64_t)(rep->cut_arcs / 2);
  if (stats) {
    stats->rounds = n_active ? (int32_t)fs.rounds : 0;
    stats->rounds_bound = (int32_t)R;
    stats->td_rounds = n_active ? (int32_t)fs.td_rounds : 0;
    stats->bu_rounds = n_active ? (int32_t)fs.bu_rounds : 0;
    stats->tail_iters = n_active ? (int32_t)fs.tail_iters : 0;
    stats->tail_round = n_active ? (int32_t)fs.tail_round : -1;
    stats->blocks = blocks;
    stats->steps = (int32_t)steps;
    stats->delta = (int64_t)delta;
    stats->pieces = (int64_t)rep->pieces;
    stats->max_frontier = n_active ? (int64_t)fs.max_frontier : 0;
    u64 ex = 0;
    for (int b = 0; b < blocks; ++b) ex += w.host->ex_part[b];
    stats->arcs_examined = (int64_t)ex;
    stats->n_active = (int64_t)n_active;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, w.ev[0], w.ev[1]);
    stats->ms_prep = ms;
    (void)hipEventElapsedTime(&ms, w.ev[1], w.ev[2]);
    stats->ms_rounds = ms;
    (void)hipEventElapsedTime(&ms, w.ev[3], w.ev[4]);
    stats->ms_finalize = ms;
    (void)hipEventElapsedTime(&ms, w.ev[4], w.ev[5]);
    stats->ms_cut = ms;
    if (!bv) {
      ldd_status sr = max_radius(w, n, shift_fix, delta, st, &stats->max_radius);
      if (sr != LDD_OK) return sr;
    }
  }
  return LDD_OK;
}

// ------------------------------------------------------------------------------------------
// the workgroup engine for one graph: one workgroup runs all rounds (small graphs)
// ------------------------------------------------------------------------------------------
// The automatic engine choice.  Graphs of more than AUTO_TEAM_DEGREE arcs per vertex on average
// (RMAT and other skewed graphs, random graphs of small diameter) go to the multi-block engines,
// whose bottom-up pulls and grid-wide arc splits they need.  Sparser graphs (meshes, geometric and
// road-like graphs: many rounds with small frontiers) go to one workgroup when they have at most
// BLOCK_AUTO_ARCS arcs (one workgroup reads them faster than round steps over the whole GPU
// synchronise), else to a team, which refuses a graph with a vertex of more than AUTO_TEAM_DEG_CAP
// arcs (one member would expand it alone), and that graph goes to the multi-block engines too.
// Measured (ms, launch engine -> team): rgg (6 arcs per vertex) 50K/200K/1M/4M vertices
// 3.8/5.3/6.5/10.3 -> 1.6/2.3/2.6/4.5, grid2d-1000/3000 6.6/12.5 -> 2.7/5.3, grid3d-128 4.4 -> 1.8,
// ER with 4 arcs per vertex, 2M vertices 0.69 -> 0.63; but ER with 8-10 arcs per vertex (small
// diameter, huge frontiers, where the top-down team reads every arc) 4M/8M vertices 1.0/1.3 ->
// 1.4/3.6 (50K/200K: 0.28/0.32 -> 0.16/0.20), and RMAT 10-20 0.18-0.30 -> 0.3-36.
constexpr long long BLOCK_AUTO_ARCS = 1ll << 15;
constexpr long long AUTO_TEAM_DEGREE = 7;
constexpr int AUTO_TEAM_DEG_CAP = 4096;

static const ldd_status REDO_MULTI = static_cast<ldd_status>(101);  // internal: shifts too wide for a workgroup

static ldd_status block_status(unsigned err, u64 delta, int n) {
  if (err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) return finish_error(err);
  if (err & BLK_OVERFLOW) {
    ldd_set_error("labels need (Delta + 2^20) << %d < 2^64 (Delta = %llu)", ceil_log2(n) < 1 ? 1 : ceil_log2(n),
                  (unsigned long long)delta);
    return LDD_ERR_OVERFLOW;
  }
  if (err & (BLK_WIDE | BLK_SKEW)) return REDO_MULTI;
  if (err) {
    ldd_set_error("workgroup engine error flags 0x%x", err);
    return LDD_ERR_INTERNAL;
  }
  return LDD_OK;
}

static int tail_den_of(const ldd_options& o) {
  return o.tail_vertices < 0 ? 0 : (o.tail_vertices > 0 ? o.tail_vertices : 32);
}

// One graph on the workgroup engine: one workgroup (WORKGROUP), or a team of K workgroups
// (TEAM: blocks of them, default one per CU, at most the workgroups that can be resident at once, at
// least 64 vertices per member) meeting at a device-memory barrier once per round.
static ldd_status decompose_block(Workspace& w, const ldd_csr* g, const int64_t* shift_fix, int32_t* centre,
                                  int64_t* cut_edges, const ldd_options& opt, ldd_stats* stats, hipStream_t st,
                                  bool team, int deg_cap) {
  const int n = g->n;
  const size_t nv = (size_t)n;
  ldd_status s = ws_setup(w);  // first: it reads the device's CU count and residency
  if (s != LDD_OK) return s;
  int K = 1;
  if (team) {
    K = opt.blocks > 0 ? opt.blocks : w.num_cu;
    K = std::min(K, std::min(w.block_coresident, TEAM_GROUP * TEAM_GROUPS));
    K = std::min(K, n / 64);
    K = std::max(K, 1);
  }
  if ((s = grow(w.P, nv * 8)) || (s = grow(w.bk_wq, nv * 16)) || (s = grow(w.bk_out, sizeof(BlockOut))) ||
      (s = grow(w.bk_sync, sizeof(TeamSync))))
    return s;
  // the job, by value: one kernel launch in all (a team's record is cleared by a fill before it)
  BlockJob j{};
  j.n = n;
  j.nnz = g->nnz;
  j.row_ptr = g->row_ptr;
  j.col = g->col_idx;
  j.shift = (const long long*)shift_fix;
  j.centre = centre;
  j.P = (u64*)w.P.p;
  j.wk = (u64*)w.bk_wq.p;
  j.wake = (int*)w.bk_wq.p;
  j.q0 = (int*)w.bk_wq.p + 2 * (long long)n;
  j.q1 = (int*)w.bk_wq.p + 3 * (long long)n;
  j.tail_den = tail_den_of(opt);
  j.team = K;
  j.sync = K > 1 ? (TeamSync*)w.bk_sync.p : nullptr;
  j.deg_cap = deg_cap;
  // the dynamic LDS the graph's mode needs (the label-correcting iteration, or the rounds in LDS)
  long long lds = 0;
  if (K == 1 && fix_lds_bytes(n, g->nnz) <= w.lds_bytes) lds = fix_lds_bytes(n, g->nnz);
  else if (K == 1 && rounds_lds_bytes(n) <= w.lds_bytes) lds = rounds_lds_bytes(n);
  const int lds_bytes = (int)((lds + 15) & ~15ll);
  HIP_TRY(hipStreamWaitEvent(st, w.ev[2], 0));  // after any step a previous call left queued
  if (stats) HIP_TRY(hipEventRecord(w.ev[0], st));
  if (K > 1)
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, (u64*)w.bk_sync.p, (long long)(sizeof(TeamSync) / 8),
                       0ull);
  if (stats) HIP_TRY(hipEventRecord(w.ev[1], st));
  // the result record goes straight to mapped host memory; the host waits for its ready flag (or
  // for the stream, if the kernel ended without setting it)
  void* bout_dev = nullptr;
  HIP_TRY(hipHostGetDevicePointer(&bout_dev, &w.host->bout, 0));
  volatile BlockOut* vb = &w.host->bout;
  vb->ready = 0;
  hipLaunchKernelGGL(k_block_decompose, dim3(K), dim3(1024), (size_t)lds_bytes, st, (const BlockJob*)nullptr,
                     (const TeamJob*)nullptr, K, (unsigned*)nullptr, (BlockOut*)bout_dev, j, lds_bytes);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(w.ev[2], st));
  for (unsigned spin = 0; !vb->ready; ++spin) {
    if ((spin & 255) == 255) {
      const hipError_t q = hipEventQuery(w.ev[2]);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) HIP_TRY(q);
    }
  }
  if (!vb->ready) {
    ldd_set_error("the workgroup engine ended without a result");
    return LDD_ERR_HIP;
  }
  if (stats) HIP_TRY(hipEventSynchronize(w.ev[2]));
  BlockOut o;
  std::memcpy(&o, (const void*)vb, sizeof(BlockOut));
  w.host->report.delta = o.delta;  // read by the verification pass
  s = block_status(o.err, o.delta, n);
  if (s != LDD_OK) return s;
  if (cut_edges) *cut_edges = (int64_t)(o.cut_arcs / 2);
  if (stats) {
    stats->rounds = (int32_t)o.rounds;
    stats->rounds_bound = (int32_t)((o.delta >> FIX) + 1);
    stats->td_rounds = (int32_t)o.rounds;
    stats->bu_rounds = 0;
    stats->tail_iters = (int32_t)o.sweeps;
    stats->tail_round = o.sweeps ? (int32_t)o.rounds : -1;
    stats->blocks = K;
    stats->steps = 1;
    stats->delta = (int64_t)o.delta;
    stats->pieces = (int64_t)o.pieces;
    stats->max_frontier = 0;
    stats->arcs_examined = (int64_t)o.examined;
    stats->n_active = (int64_t)o.n_active;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, w.ev[0], w.ev[1]);
    stats->ms_prep = ms;
    (void)hipEventElapsedTime(&ms, w.ev[1], w.ev[2]);
    stats->ms_rounds = ms;
    stats->ms_finalize = 0;
    stats->ms_cut = 0;
    s = max_radius(w, n, shift_fix, o.delta, st, &stats->max_radius);
    if (s != LDD_OK) return s;
  }
  return LDD_OK;
}

static ldd_status decompose_impl(Workspace& w, const ldd_csr* g, const int64_t* shift_fix, int32_t* centre,
                                 int64_t* cut_edges, const ldd_options& o, ldd_stats* stats, hipStream_t st,
                                 const BatchView* bv) {
  // a forced bottom-up policy needs the multi-block engines (the workgroup engines run top-down)
  const bool sparse = g->nnz <= AUTO_TEAM_DEGREE * (long long)g->n && o.direction != LDD_DIR_BOTTOM_UP;
  const bool auto_wg = o.engine == LDD_ENGINE_AUTO && sparse && g->nnz <= BLOCK_AUTO_ARCS;
  const bool auto_team = o.engine == LDD_ENGINE_AUTO && sparse && g->nnz > BLOCK_AUTO_ARCS;
  if (!bv && (o.engine == LDD_ENGINE_WORKGROUP || o.engine == LDD_ENGINE_TEAM || auto_wg || auto_team)) {
    const bool team = o.engine == LDD_ENGINE_TEAM || auto_team;
    ldd_status s = decompose_block(w, g, shift_fix, centre, cut_edges, o, stats, st, team,
                                   auto_team ? AUTO_TEAM_DEG_CAP : 0);
    if (s != REDO_MULTI) return s;
  }
  ldd_status s = decompose_run(w, g, shift_fix, centre, cut_edges, o, stats, st, bv, false);
  if (s == REDO_WIDE) s = decompose_run(w, g, shift_fix, centre, cut_edges, o, stats, st, bv, true);
  return s;
}

// ------------------------------------------------------------------------------------------
// Las Vegas: draw, decompose, verify, draw again (proof of Theorem 1.1, Sec. 5)
// ------------------------------------------------------------------------------------------
extern "C" ldd_status ldd_decompose_verified(const ldd_csr* g, double beta, uint64_t seed, int64_t* shift_fix,
                                             int32_t* centre, const ldd_verify_options* vopt, const ldd_options* opt,
                                             ldd_verify_report* report, void* hip_stream) {
  g_err[0] = 0;
  if (!g || g->n < 0 || g->nnz < 0 || g->nnz >= (1ll << 31)) {
    ldd_set_error("bad graph");
    return LDD_ERR_INVALID_ARG;
  }
  const int n = g->n;
  if (!(beta > 0.0) || !std::isfinite(beta)) {
    ldd_set_error("beta must be finite and positive");
    return LDD_ERR_INVALID_ARG;
  }
  if (n > 0 && (!g->row_ptr || !shift_fix || !centre || (g->nnz > 0 && !g->col_idx))) {
    ldd_set_error("NULL device pointer");
    return LDD_ERR_INVALID_ARG;
  }
  ldd_verify_options v{};
  if (vopt) v = *vopt;
  if (v.cut_factor < 0 || v.radius_factor < 0 || v.max_attempts < 0 || !std::isfinite(v.cut_factor) ||
      !std::isfinite(v.radius_factor)) {
    ldd_set_error("bad verification options");
    return LDD_ERR_INVALID_ARG;
  }
  const double cut_factor = v.cut_factor > 0 ? v.cut_factor : 2.0;
  const double radius_factor = v.radius_factor > 0 ? v.radius_factor : 3.0;
  const int max_attempts = v.max_attempts > 0 ? v.max_attempts : 16;
  ldd_options o{};
  if (opt) o = *opt;
  if (o.direction < 0 || o.direction > 2 || o.engine < 0 || o.engine > 4 || o.blocks < 0) {
    ldd_set_error("bad options");
    return LDD_ERR_INVALID_ARG;
  }
  ldd_verify_report r{};
  r.cut_bound = cut_factor * beta * ((double)g->nnz / 2.0);
  r.radius_bound = n > 1 ? radius_factor * std::log((double)n) / beta : 0.0;
  if (n == 0) {
    r.attempts = 1;
    r.accepted = 1;
    r.seed = seed;
    if (report) *report = r;
    return LDD_OK;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace& w = *workspace_for(dev);
  std::lock_guard<std::mutex> lk(w.mu);
  ldd_status s = LDD_OK;
  for (int a = 0; a < max_attempts; ++a) {
    const uint64_t sd = seed + (uint64_t)a;
    if ((s = ldd_shifts_on_device(n, beta, sd, shift_fix, st))) return s;
    int64_t cut = 0;
    if ((s = decompose_impl(w, g, shift_fix, centre, &cut, o, nullptr, st, nullptr))) return s;
    // the labels of this draw are still in the workspace: the largest distance to a centre
    int64_t radius = 0;
    if ((s = max_radius(w, n, shift_fix, w.host->report.delta, st, &radius))) return s;
    r.attempts = a + 1;
    r.seed = sd;
    r.cut_edges = cut;
    r.max_radius = radius;
    r.accepted = (double)cut <= r.cut_bound && (double)radius <= r.radius_bound;
    if (r.accepted) break;
  }
  if (report) *report = r;
  if (!r.accepted) {
    ldd_set_error("no draw of %d met cut <= %.6g and radius <= %.6g (last: cut %lld, radius %lld)", max_attempts,
                  r.cut_bound, r.radius_bound, (long long)r.cut_edges, (long long)r.max_radius);
    return LDD_ERR_RETRIES;
  }
  return LDD_OK;
}

// ------------------------------------------------------------------------------------------
// many graphs, one after another (the one-graph-per-launch path)
// ------------------------------------------------------------------------------------------
ldd_status ldd_batch_sequential(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off,
                                const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                                int32_t* centre, int64_t* cut_edges, const ldd_options* opt, void* hip_stream) {
  for (int32_t gi = 0; gi < num_graphs; ++gi) {
    ldd_csr g{(int32_t)(vtx_off[gi + 1] - vtx_off[gi]), arc_off[gi + 1] - arc_off[gi], row_ptr + vtx_off[gi] + gi,
              col_idx + arc_off[gi]};
    int64_t cut = 0;
    ldd_status s = ldd_decompose(&g, shift_fix + vtx_off[gi], 1.0, centre + vtx_off[gi], &cut, opt, nullptr,
                                 hip_stream);
    if (s != LDD_OK) return s;
    if (cut_edges) cut_edges[gi] = cut;
  }
  return LDD_OK;
}

// ------------------------------------------------------------------------------------------
// many graphs at once on the workgroup engine: one workgroup per graph, largest first
// ------------------------------------------------------------------------------------------
ldd_status ldd_batch_workgroup(int32_t G, const int64_t* vtx_off, const int64_t* arc_off, const int32_t* row_ptr,
                               const int32_t* col_idx, const int64_t* shift_fix, int32_t* centre, int64_t* cut_edges,
                               const ldd_options* opt, void* hip_stream) {
  const long long N = vtx_off[G];
  if (N > INT32_MAX) {
    ldd_set_error("batch too large (%lld vertices)", N);
    return LDD_ERR_INVALID_ARG;
  }
  if (N == 0 || G == 0) {
    if (cut_edges)
      for (int g = 0; g < G; ++g) cut_edges[g] = 0;
    return LDD_OK;
  }
  ldd_options o{};
  if (opt) o = *opt;
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace& w = *workspace_for(dev);
  std::vector<int> redo;  // graphs whose shifts span too many rounds for a workgroup
  {
    std::lock_guard<std::mutex> lk(w.mu);
    ldd_status s = ws_setup(w);
    if (s != LDD_OK) return s;
    // one workgroup per CU by default: on the 512-graph benchmark batch one per CU ran 17% faster
    // than two (6.35 vs 7.69 ms), the memory system being the shared resource
    int grid = o.blocks > 0 ? o.blocks : w.num_cu;
    // Teams: a graph with more arcs than a workgroup's share of the batch (all arcs over the grid,
    // at least 2^14; or team_arcs when given) runs on K = ceil(arcs / share) workgroups (at most
    // TEAM_MAX, at most a quarter of the grid, at least 64 vertices per member), so that no graph
    // holds one workgroup long after the others are done.
    const long long M = arc_off[G];
    std::vector<int> team((size_t)G, 1);
    const long long share = o.team_arcs > 0 ? o.team_arcs : std::max(M / grid, 1ll << 14);
    const int kcap = o.team_arcs < 0 ? 1 : std::min(TEAM_MAX, grid / 4);
    for (int g = 0; g < G; ++g) {
      const long long e = arc_off[g + 1] - arc_off[g], nv = vtx_off[g + 1] - vtx_off[g];
      long long k = (e + share - 1) / share;
      k = std::min<long long>(k, kcap);
      k = std::min<long long>(k, nv / 64);
      team[g] = k > 1 ? (int)k : 1;
    }
    // jobs, the heaviest per workgroup (arcs / team size, then vertices) first; a team's members
    // are consecutive
    std::vector<int> order((size_t)G);
    for (int g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const long long ea = (arc_off[a + 1] - arc_off[a]) / team[a], eb = (arc_off[b + 1] - arc_off[b]) / team[b];
      if (ea != eb) return ea > eb;
      return vtx_off[a + 1] - vtx_off[a] > vtx_off[b + 1] - vtx_off[b];
    });
    std::vector<TeamJob> jobs;
    jobs.reserve((size_t)G);
    std::vector<int> tinfo((size_t)G * 2, 0);
    int nteams = 0;
    for (int g : order) {
      tinfo[2 * (size_t)g] = team[g];
      if (team[g] > 1) tinfo[2 * (size_t)g + 1] = nteams++;
      for (int m = 0; m < team[g]; ++m) jobs.push_back(TeamJob{g, m});
    }
    const int njobs = (int)jobs.size();
    if ((s = grow(w.P, (size_t)N * 8)) || (s = grow(w.bk_wq, (size_t)N * 16)) ||
        (s = grow(w.bk_jobs, (size_t)G * sizeof(BlockJob))) || (s = grow(w.bk_order, (size_t)njobs * sizeof(TeamJob))) ||
        (s = grow(w.bk_out, (size_t)G * sizeof(BlockOut))) || (s = grow(w.bk_cnt, 8)) ||
        (s = grow(w.b_off, (size_t)(G + 1) * 16)) || (s = grow(w.bk_team, (size_t)G * 8)) ||
        (s = grow(w.bk_sync, (size_t)(nteams > 0 ? nteams : 1) * sizeof(TeamSync))))
      return s;
    long long* d_vo = (long long*)w.b_off.p;
    long long* d_ao = d_vo + (G + 1);
    int* d_team = (int*)w.bk_team.p;
    HIP_TRY(hipStreamWaitEvent(st, w.ev[2], 0));  // after any step a previous call left queued
    HIP_TRY(hipMemcpyAsync(d_vo, vtx_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_ao, arc_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w.bk_order.p, jobs.data(), (size_t)njobs * sizeof(TeamJob), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_team, tinfo.data(), (size_t)G * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_block_jobs, dim3(grid_for(G, 256, 1024)), dim3(256), 0, st, G, N, (const long long*)d_vo,
                       (const long long*)d_ao, row_ptr, col_idx, (const long long*)shift_fix, centre, (u64*)w.P.p,
                       (int*)w.bk_wq.p, tail_den_of(o), (const int*)d_team, (TeamSync*)w.bk_sync.p,
                       (BlockJob*)w.bk_jobs.p);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (u64*)w.bk_cnt.p, 1ll, 0ull);
    if (nteams > 0)
      hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((long long)nteams * sizeof(TeamSync) / 8, 256, 1024)), dim3(256), 0,
                         st, (u64*)w.bk_sync.p, (long long)nteams * (long long)(sizeof(TeamSync) / 8), 0ull);
    if (grid > njobs) grid = njobs;
    // small graphs keep their state in LDS when the grid is one workgroup per CU (the LDS then costs
    // no residency: one workgroup of 1024 threads per CU either way)
    const int lds_bytes = grid <= w.num_cu ? w.lds_bytes : 0;
    hipLaunchKernelGGL(k_block_decompose, dim3(grid), dim3(1024), (size_t)lds_bytes, st, (const BlockJob*)w.bk_jobs.p,
                       (const TeamJob*)w.bk_order.p, njobs, (unsigned*)w.bk_cnt.p, (BlockOut*)w.bk_out.p, BlockJob{},
                       lds_bytes);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(w.ev[2], st));
    std::vector<BlockOut> outs((size_t)G);
    HIP_TRY(hipMemcpyAsync(outs.data(), w.bk_out.p, (size_t)G * sizeof(BlockOut), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int g = 0; g < G; ++g) {
      s = block_status(outs[g].err, outs[g].delta, (int)(vtx_off[g + 1] - vtx_off[g]));
      if (s == REDO_MULTI) {
        redo.push_back(g);
        continue;
      }
      if (s != LDD_OK) {
        char msg[512];
        snprintf(msg, sizeof(msg), "graph %d: %s", g, ldd_last_error());
        ldd_set_error("%s", msg);
        return s;
      }
      if (cut_edges) cut_edges[g] = (int64_t)(outs[g].cut_arcs / 2);
    }
  }
  // a graph whose shifts span too many rounds for a workgroup's wake sort: the multi-block engine
  for (int g : redo) {
    ldd_csr gg{(int32_t)(vtx_off[g + 1] - vtx_off[g]), arc_off[g + 1] - arc_off[g], row_ptr + vtx_off[g] + g,
               col_idx + arc_off[g]};
    ldd_options og = o;
    og.engine = LDD_ENGINE_LAUNCH;
    int64_t cut = 0;
    const ldd_status s = ldd_decompose(&gg, shift_fix + vtx_off[g], 1.0, centre + vtx_off[g], &cut, &og, nullptr,
                                       hip_stream);
    if (s != LDD_OK) return s;
    if (cut_edges) cut_edges[g] = cut;
  }
  return LDD_OK;
}

// ------------------------------------------------------------------------------------------
// many graphs at once: the disjoint union, one launch per round for all of them
// ------------------------------------------------------------------------------------------
// The batch is decomposed as one graph, the disjoint union, with global vertex ids.  Graph g's
// shifts are raised by Delta_max - Delta_g, so that the union's per-vertex offset
// Delta_max - shift' equals Delta_g - shift: every key is the one the graph has alone, and
// global ids keep each graph's tie order.  So each graph's centres and cut equal those of
// ldd_decompose on that graph, bit for bit, and all graphs advance one round per launch.
ldd_status ldd_batch_union(int32_t G, const int64_t* vtx_off, const int64_t* arc_off, const int32_t* row_ptr,
                           const int32_t* col_idx, const int64_t* shift_fix, int32_t* centre, int64_t* cut_edges,
                           const ldd_options* opt, void* hip_stream) {
  const long long N = vtx_off[G], M = arc_off[G];
  if (N > INT32_MAX || M >= (1ll << 31)) {
    ldd_set_error("batch too large for int32 ids (%lld vertices, %lld arcs)", N, M);
    return LDD_ERR_INVALID_ARG;
  }
  if (N == 0) {
    if (cut_edges)
      for (int g = 0; g < G; ++g) cut_edges[g] = 0;
    return LDD_OK;
  }
  ldd_options o{};
  if (opt) o = *opt;
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  Workspace& w = *workspace_for(dev);
  std::lock_guard<std::mutex> lk(w.mu);
  ldd_status s = ws_setup(w);
  if (s != LDD_OK) return s;
  if ((s = grow(w.b_rp, (size_t)(N + 1) * 4)) || (s = grow(w.b_col, (size_t)(M > 0 ? M : 1) * 4)) ||
      (s = grow(w.b_shift, (size_t)N * 8)) || (s = grow(w.b_gid, (size_t)N * 4)) ||
      (s = grow(w.b_off, (size_t)(G + 1) * 16)) || (s = grow(w.b_dg, (size_t)(G + 1) * 128)) ||
      (s = grow(w.b_cut, (size_t)G * 8)))
    return s;
  long long* d_vo = (long long*)w.b_off.p;
  long long* d_ao = d_vo + (G + 1);
  u64* d_dg = (u64*)w.b_dg.p;  // max shift of graph g at [16 g] (one line each), overall max at [16 G]
  // offsets to the device through pinned staging
  HIP_TRY(hipMemcpyAsync(d_vo, vtx_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_ao, arc_off, (size_t)(G + 1) * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(w.b_dg.p, 0, (size_t)(G + 1) * 128, st));
  HIP_TRY(hipMemsetAsync(w.b_cut.p, 0, (size_t)G * 8, st));
  HIP_TRY(hipMemsetAsync(w.ctrl.p, 0, sizeof(Ctrl), st));
  Ctrl* ctrl = (Ctrl*)w.ctrl.p;
  hipLaunchKernelGGL(k_batch_rows, dim3(grid_for(N, 256 * 4, 4096)), dim3(256), 0, st, G, (long long)N, d_vo, d_ao,
                     row_ptr, (const long long*)shift_fix, (int*)w.b_rp.p, (int*)w.b_gid.p, d_dg, ctrl);
  if (M > 0)
    hipLaunchKernelGGL(k_batch_cols, dim3(grid_for(M, 256 * 4, 4096)), dim3(256), 0, st, G, (long long)M, d_vo, d_ao,
                       col_idx, (int*)w.b_col.p, ctrl);
  hipLaunchKernelGGL(k_batch_dmax, dim3(1), dim3(1024), 0, st, G, d_dg);
  hipLaunchKernelGGL(k_batch_shift, dim3(grid_for(N, 256 * 4, 4096)), dim3(256), 0, st, G, (long long)N,
                     (const int*)w.b_gid.p, (const long long*)shift_fix, (const u64*)d_dg, (long long*)w.b_shift.p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&w.host->ctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (w.host->ctrl.err) {
    (void)finish_error(w.host->ctrl.err);
    ldd_set_error("batch: %s", ldd_last_error());
    return LDD_ERR_INVALID_ARG;
  }
  ldd_csr ug{(int32_t)N, M, (const int32_t*)w.b_rp.p, (const int32_t*)w.b_col.p};
  BatchView bv{(const int*)w.b_gid.p, (u64*)w.b_cut.p};
  s = decompose_impl(w, &ug, (const int64_t*)w.b_shift.p, centre, nullptr, o, nullptr, st, &bv);
  if (s != LDD_OK) return s;
  hipLaunchKernelGGL(k_batch_localize, dim3(grid_for(N, 256 * 4, 4096)), dim3(256), 0, st, (long long)N,
                     (const int*)w.b_gid.p, (const long long*)d_vo, centre);
  HIP_TRY(hipGetLastError());
  std::vector<u64> hc((size_t)G);
  HIP_TRY(hipMemcpyAsync(hc.data(), w.b_cut.p, (size_t)G * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (cut_edges)
    for (int g = 0; g < G; ++g) cut_edges[g] = (int64_t)(hc[g] / 2);
  return LDD_OK;
}
