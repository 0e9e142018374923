// ldd_decompose_static: the single-graph decomposition with every device buffer it needs beyond
// the caller's inputs and outputs taken from one file-scope device array, so that the call
// allocates nothing (no hipMalloc / hipFree, no pinned host memory, no events, streams or
// graphs).  Each device the library runs on holds its own copy of the array until the process
// ends; its device address is looked up once per device with hipGetSymbolAddress and only that
// address is handed to kernels.  Every call on a device shares its array, which keeps the last
// call's contents: whatever must start at zero is cleared by a fill kernel at the start of the
// call, and calls that overlap on one device race (the caller serialises them).
//
// Same kernels and the same exact result as ldd_decompose (Algorithm 2, Sec. 4, by the round
// search of Sec. 5): preparation, round steps launched directly on the caller's stream in
// chunks (the host reads the device-side report after each chunk with a stream-ordered copy and
// a stream synchronisation), centre extraction and the cut.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/ldd.h"
#include "ldd_internal.h"
#include "ldd_kernels.h"

using namespace ldd;

namespace {

constexpr long long SMAX = LDD_STATIC_MAX_VERTICES;

// preparation blocks for n vertices (as in the workspace path), at most for SMAX vertices
constexpr long long prep_blocks(long long n) {
  return n / 16384 < 1 ? 1 : (n / 16384 > 1024 ? 1024 : n / 16384);
}
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the array, for SMAX vertices; every part starts on a 256-byte boundary.
struct Layout {
  size_t P, qv0, qv1, qa0, qa1, wake_ord, stamp, hub_bits, mat, qmax, cand, cand_cnt, hist, wake_off, next_ne, ctrl,
      st, qcnt, lr_part, lb, ex_part, report, total;
};
constexpr Layout make_layout() {
  Layout L{};
  size_t o = 0;
  const size_t nv = (size_t)SMAX, gp = (size_t)prep_blocks(SMAX), nq = (size_t)QCAP + 2;
  L.P = o; o = align256(o + nv * 8);
  L.qv0 = o; o = align256(o + nv * 4);
  L.qv1 = o; o = align256(o + nv * 4);
  L.qa0 = o; o = align256(o + nv * 4);
  L.qa1 = o; o = align256(o + nv * 4);
  L.wake_ord = o; o = align256(o + nv * 4);
  L.stamp = o; o = align256(o + nv * 4);
  L.hub_bits = o; o = align256(o + (nv + 63) / 64 * 8);
  L.mat = o; o = align256(o + (size_t)QCAP * gp * 4);
  L.qmax = o; o = align256(o + gp * 4);
  L.cand = o; o = align256(o + (size_t)CAND * gp * 8);
  L.cand_cnt = o; o = align256(o + gp * 4);
  L.hist = o; o = align256(o + nq * 4);
  L.wake_off = o; o = align256(o + nq * 4);
  L.next_ne = o; o = align256(o + nq * 4);
  L.ctrl = o; o = align256(o + sizeof(Ctrl));
  L.st = o; o = align256(o + 2 * sizeof(RoundState));
  L.qcnt = o; o = align256(o + 3 * 16 * 8);
  L.lr_part = o; o = align256(o + 2 * (size_t)RT * 8);
  L.lb = o; o = align256(o + sizeof(LaunchBlock));
  L.ex_part = o; o = align256(o + (size_t)RT * 8);
  L.report = o; o = align256(o + sizeof(Report));
  L.total = o;
  return L;
}
constexpr Layout LAY = make_layout();
static_assert(LAY.total == LDD_STATIC_SCRATCH_BYTES, "the header's scratch size matches the layout");

// The library's scratch memory for this entry point: one copy per device, alive until the
// process ends.  In host code `scratch` is a host-side stand-in, never a device address: only
// the address from hipGetSymbolAddress (kept per device below) is passed to kernels.
static __device__ __align__(256) unsigned char scratch[LAY.total];

constexpr int MAX_DEVICES = 64;
constexpr int STEPS_PER_CHUNK = 8;

struct DeviceState {
  unsigned char* base = nullptr;  // device address of this device's `scratch`
  int num_cu = 0;
  unsigned stamp_base = 0;        // every tail stamp in the array is <= stamp_base
  bool stamps_clean = false;      // the stamp part has been cleared once
};
std::mutex g_mu;
DeviceState g_dev[MAX_DEVICES];

#define ST_TRY(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      ldd_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return LDD_ERR_HIP;                                                                 \
    }                                                                                     \
  } while (0)

// Set-up for the current device, once: the array's device address and the CU count.
ldd_status device_state(int dev, DeviceState** out) {
  DeviceState& d = g_dev[dev];
  if (!d.base) {
    void* ptr = nullptr;
    ST_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      ldd_set_error("hipGetSymbolAddress returned no address for the static scratch");
      return LDD_ERR_HIP;
    }
    ST_TRY(hipDeviceGetAttribute(&d.num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    d.base = (unsigned char*)ptr;
  }
  *out = &d;
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

ldd_status input_error(unsigned err) {
  ldd_set_error("invalid input:%s%s%s", (err & ERR_BAD_SHIFT) ? " shift out of [0, 2^52]" : "",
                (err & ERR_BAD_ROWPTR) ? " row_ptr not a valid offset array" : "",
                (err & ERR_BAD_COL) ? " column id out of range" : "");
  return LDD_ERR_INVALID_ARG;
}

ldd_status internal_error(unsigned err) {
  ldd_set_error("internal error flags 0x%x", err);
  return LDD_ERR_INTERNAL;
}

ldd_status run_static(DeviceState& d, const ldd_csr* g, const int64_t* shift_fix, int32_t* centre, int64_t* cut_edges,
                      const ldd_options& o, hipStream_t st) {
  const int n = g->n;
  const long long nnz = g->nnz;
  unsigned char* b = d.base;
  u64* P = (u64*)(b + LAY.P);
  Ctrl* ctrl = (Ctrl*)(b + LAY.ctrl);
  Report* rep_dev = (Report*)(b + LAY.report);
  LaunchBlock* lb = (LaunchBlock*)(b + LAY.lb);
  const int B = ceil_log2(n) < 1 ? 1 : ceil_log2(n);
  const int gp = (int)prep_blocks(n);

  // what must start at zero: the control block and the report (and the stamps, once)
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, (u64*)ctrl, (long long)(sizeof(Ctrl) / 8), 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, (u64*)rep_dev, (long long)(sizeof(Report) / 8), 0ull);
  const int tail_den = o.tail_vertices < 0 ? 0 : (o.tail_vertices > 0 ? o.tail_vertices : 32);
  if (tail_den && (!d.stamps_clean || d.stamp_base >= (1u << 30))) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(SMAX / 2, 256, 1024)), dim3(256), 0, st, (u64*)(b + LAY.stamp),
                       (long long)(SMAX / 2), 0ull);
    d.stamp_base = 0;
    d.stamps_clean = true;
  }
  // preparation: labels, Delta, checks, the wake-round buckets and their first window
  hipLaunchKernelGGL(k_init, dim3(gp), dim3(1024), 0, st, n, nnz, g->row_ptr, (const long long*)shift_fix, P, ctrl,
                     (unsigned*)(b + LAY.mat), (int*)(b + LAY.qmax), (u64*)(b + LAY.cand),
                     (unsigned*)(b + LAY.cand_cnt));
  if (o.validate && nnz > 0)
    hipLaunchKernelGGL(k_check_cols, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, st, n, nnz, g->col_idx, ctrl);
  hipLaunchKernelGGL(k_qbucket_scan, dim3(std::min(QCAP, 1024)), dim3(256), 0, st, gp, (unsigned*)(b + LAY.mat),
                     (const int*)(b + LAY.qmax), (unsigned*)(b + LAY.hist), (const Ctrl*)ctrl);
  hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, st, (const Ctrl*)ctrl, (const unsigned*)(b + LAY.hist),
                     (int*)(b + LAY.wake_off), (int*)(b + LAY.next_ne));
  hipLaunchKernelGGL(k_place_window, dim3(gp), dim3(256), 0, st, (const Ctrl*)ctrl, (const unsigned*)(b + LAY.mat),
                     (const int*)(b + LAY.qmax), (const int*)(b + LAY.wake_off), (const u64*)(b + LAY.cand),
                     (const unsigned*)(b + LAY.cand_cnt), (int*)(b + LAY.wake_ord));
  ST_TRY(hipGetLastError());

  RoundCtx c{};
  c.n = n;
  c.B = B;
  c.nnz = nnz;
  c.row_ptr = g->row_ptr;
  c.col = g->col_idx;
  c.shift = (const long long*)shift_fix;
  c.P = P;
  c.qv[0] = (int*)(b + LAY.qv0);
  c.qv[1] = (int*)(b + LAY.qv1);
  c.qa[0] = (unsigned*)(b + LAY.qa0);
  c.qa[1] = (unsigned*)(b + LAY.qa1);
  c.wake_ord = (int*)(b + LAY.wake_ord);
  c.wake_off = (const int*)(b + LAY.wake_off);
  c.next_ne = (const int*)(b + LAY.next_ne);
  c.wake_q = 1;
  c.prep_blocks = gp;
  c.mat = (const unsigned*)(b + LAY.mat);
  c.qmax = (const int*)(b + LAY.qmax);
  c.qcnt = (u64*)(b + LAY.qcnt);
  c.lr_part = (u64*)(b + LAY.lr_part);
  c.stamp = (unsigned*)(b + LAY.stamp);
  c.stamp_base = d.stamp_base;
  c.st = (RoundState*)(b + LAY.st);
  c.ctrl = ctrl;
  c.dir_policy = o.direction;
  c.td_to_bu = o.td_to_bu > 0 ? o.td_to_bu : 14;
  c.bu_to_td = o.bu_to_td > 0 ? o.bu_to_td : 24;
  c.tail_den = tail_den;
  c.tail_min_left = 16;
  c.ex_part = (u64*)(b + LAY.ex_part);
  c.report = rep_dev;
  hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, st, c, lb, 1);
  ST_TRY(hipGetLastError());

  int blocks = o.blocks > 0 ? o.blocks : 2 * d.num_cu;
  if (blocks > RT) blocks = RT;
  // rounds (at most QCAP on this layout), placement steps, tail sweeps (each lowers a label) and slack
  const long long kmax = (long long)QCAP + QCAP / ABUF + 1 + (long long)n + 2;
  Report rep{};
  long long steps = 0;
  for (;;) {
    for (int j = 0; j < STEPS_PER_CHUNK; ++j) hipLaunchKernelGGL(k_round_step_lb, dim3(blocks), dim3(RT), 0, st, lb, j);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, lb, STEPS_PER_CHUNK);
    steps += STEPS_PER_CHUNK;
    ST_TRY(hipGetLastError());
    ST_TRY(hipMemcpyAsync(&rep, rep_dev, sizeof(Report), hipMemcpyDeviceToHost, st));
    ST_TRY(hipStreamSynchronize(st));
    if (rep.ready) break;
    if (steps > kmax) {
      ldd_set_error("round steps exceeded their bound (%lld)", kmax);
      return LDD_ERR_INTERNAL;
    }
  }
  d.stamp_base += (unsigned)steps + 2;  // step k tags at most stamp_base + k + 1
  switch (rep.setup) {
    case SETUP_OK:
    case SETUP_EMPTY:
      break;
    case SETUP_WIDE:
      ldd_set_error("shifts span %d or more units of distance; the static workspace holds only %d wake rounds "
                    "(use ldd_decompose)", QCAP, QCAP);
      return LDD_ERR_BUDGET;
    case SETUP_OVERFLOW:
      ldd_set_error("labels need (Delta + 2^20) << %d < 2^64 (Delta = %llu)", B, (unsigned long long)rep.delta);
      return LDD_ERR_OVERFLOW;
    default:
      return (rep.err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) ? input_error(rep.err) : internal_error(rep.err);
  }
  if (rep.err) return (rep.err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) ? input_error(rep.err) : internal_error(rep.err);
  // output pass: centre per vertex, the hub-piece bitmap and the list of other rows, the cut
  const int g_f = grid_for((n + 63) / 64, 128, 2048);
  hipLaunchKernelGGL(k_finalize, dim3(g_f), dim3(512), 0, st, n, B, g->row_ptr, (const u64*)P, centre,
                     (u64*)(b + LAY.hub_bits), (int*)(b + LAY.qv0), (unsigned*)(b + LAY.qa0), ctrl);
  if (nnz > 0)
    hipLaunchKernelGGL(k_cut, dim3(grid_for(nnz, 256 * 8, 2048)), dim3(256), 0, st, n, g->row_ptr, g->col_idx,
                       (const int*)centre, (const u64*)(b + LAY.hub_bits), (const int*)(b + LAY.qv0),
                       (const unsigned*)(b + LAY.qa0), ctrl, (const int*)nullptr, (u64*)nullptr);
  hipLaunchKernelGGL(k_out_report, dim3(1), dim3(64), 0, st, (const Ctrl*)ctrl, rep_dev);
  ST_TRY(hipGetLastError());
  ST_TRY(hipMemcpyAsync(&rep, rep_dev, sizeof(Report), hipMemcpyDeviceToHost, st));
  ST_TRY(hipStreamSynchronize(st));
  if (!rep.out_ready) {
    ldd_set_error("the output pass ended without a report");
    return LDD_ERR_INTERNAL;
  }
  if (rep.out_err) return (rep.out_err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) ? input_error(rep.out_err)
                                                                                         : internal_error(rep.out_err);
  if (rep.unreached != 0 || (rep.n_active > 0 && rep.st.mode != MODE_DONE)) {
    ldd_set_error("rounds ended with %llu labels unset", (unsigned long long)rep.unreached);
    return LDD_ERR_INTERNAL;
  }
  if (cut_edges) *cut_edges = (int64_t)(rep.cut_arcs / 2);
  return LDD_OK;
}

}  // namespace

extern "C" ldd_status ldd_decompose_static(const ldd_csr* g, const int64_t* shift_fix, double beta, int32_t* centre,
                                           int64_t* cut_edges, const ldd_options* opt, void* hip_stream) {
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
  if (n > LDD_STATIC_MAX_VERTICES) {
    ldd_set_error("n=%d exceeds the static workspace's %d vertices (use ldd_decompose)", n, LDD_STATIC_MAX_VERTICES);
    return LDD_ERR_BUDGET;
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
  if (o.direction < 0 || o.direction > 2 || o.blocks < 0 || o.engine == LDD_ENGINE_PERSISTENT) {
    ldd_set_error("bad options (the static entry point runs the launch engine only)");
    return LDD_ERR_INVALID_ARG;
  }
  if (n == 0) {
    if (cut_edges) *cut_edges = 0;
    return LDD_OK;
  }
  int dev = 0;
  ST_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    ldd_set_error("device %d beyond the %d the static entry point supports", dev, MAX_DEVICES);
    return LDD_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState* d = nullptr;
  ldd_status s = device_state(dev, &d);
  if (s != LDD_OK) return s;
  return run_static(*d, g, shift_fix, centre, cut_edges, o, (hipStream_t)hip_stream);
}
