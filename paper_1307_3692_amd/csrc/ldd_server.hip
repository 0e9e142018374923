// Serving: decomposition requests admitted continuously into one device-resident arena.
//
// Every admitted request owns a slot: a range of arena vertices (labels, queues, wake order),
// while its CSR and shifts stay in the caller's device buffers.  The round engine runs one
// global round per step over the whole arena, i.e. over the disjoint union of all admitted
// requests.  A request whose round 0 is the global round r0 gets the source-arc lengths
// Delta_g - shift + r0 * 2^20: every key of the request grows by the same constant, so its
// argmin and its tie order -- its result -- are those of the request alone (Sec. 5: the
// super-source search only compares keys within a component), and its round rho runs at global
// round r0 + rho.  Each request has its own mode (rounds, then a label-correcting tail once few
// of its vertices remain) and is done as soon as its labels are final.
//
// Requests join and leave between step chunks.  Admission (validation, labels, wake-round
// sort) and finishing (centres, cut, report) each run as a few kernels for a whole batch of
// requests, their descriptors passed as kernel arguments, enqueued on the engine stream between
// graph replays; results reach the host through mapped memory.  So the host cost per engine
// iteration does not grow with the number of requests that join or leave.  Keys grow with the
// global round; when they approach the label's key range, all live keys are lowered by the same
// number of rounds (a rebase), again between chunks.
//
// One engine thread owns the engine stream; submit, poll, wait and cancel touch host queues
// (submit also records an event on the caller's stream, which admission waits for).
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
constexpr int MAX_BATCH = 16;         // requests per admission / finishing launch
// most arcs of the requests on the device at once (32-bit arc offsets of a step's top-down split)
constexpr unsigned long long MAX_ACTIVE_ARCS = 0xffffffffull;
constexpr int ADM_T = 1024;           // threads of the admission kernels
constexpr int FIN_T = 256;            // threads of the finishing kernel (its arc tile)
constexpr unsigned ERR_ROUNDS = 64u;  // the request needs more rounds than the server takes
constexpr unsigned ROW_ERRS = ERR_BAD_SHIFT | ERR_BAD_ROWPTR;

// One request of an admission batch.  Block j of the item (j < nblk) owns vertices
// [n j / nblk, n (j+1) / nblk) and arcs [nnz j / nblk, nnz (j+1) / nblk).
struct AdmItem {
  const int* rp;
  const int* col;
  const long long* shift;
  long long vbeg, nnz, r0;
  int n, slot, blk0, nblk;
};
struct AdmBatch {
  AdmItem it[MAX_BATCH];
  int count;
};

struct FinItem {
  int* centre;
  const int* rp;
  const int* col;
  long long vbeg, nnz;
  int n, slot, blk0, nblk;
};
struct FinBatch {
  FinItem it[MAX_BATCH];
  int count;
};

// Per-slot report in mapped host memory.  Admission writes adm_err then R (release), finishing
// writes cut and fin_err then done (release); the host clears R and done before reuse.
struct SlotReport {
  long long R;     // rounds of the request once admitted (0: not runnable), -1 until then
  long long cut;   // cut edges
  long long done;  // 1 once cut and fin_err are written
  unsigned adm_err, fin_err;
};

template <typename Batch>
__device__ __forceinline__ int item_of(const Batch& b, int blk) {
  int i = b.count - 1;
  while (i > 0 && blk < b.it[i].blk0) --i;
  return i;
}

__device__ __forceinline__ long long chunk(long long total, int j, int nb) { return total * j / nb; }

// the request's rounds and whether its rows and shifts passed the check (column errors do not
// stop a request: such columns were redirected inside the slot and only its status changes)
__device__ __forceinline__ int request_rounds(u64 delta, unsigned err, int max_rounds) {
  const u64 R = (delta >> FIX) + 1;
  return ((err & ROW_ERRS) == 0 && R <= (u64)max_rounds) ? (int)R : 0;
}

// the block's maximum (or error bits), in thread 0 only
__device__ __forceinline__ u64 block_max_or(u64 v, u64* red, bool is_or) {
  if (is_or) {
    v = wave_max_u64(v & ERR_BAD_SHIFT) | wave_max_u64(v & ERR_BAD_ROWPTR);
  } else {
    v = wave_max_u64(v);
  }
  if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  u64 r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) r = is_or ? (r | red[w]) : (red[w] > r ? red[w] : r);
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------------------------------
// admission: scan (checks, labels, bucket histogram) -> commit (bucket offsets, slot entry)
// -> place
// ------------------------------------------------------------------------------------------
// One pass over a request's rows and shifts: rows non-decreasing from 0 to nnz, shifts in
// [0, 2^52], the request's max shift and hub ((degree << 32 | id) of a vertex of largest degree,
// for the cut); labels INF (an isolated vertex keeps INF, which the finishing maps to the vertex
// itself); and the vertices with arcs counted by the integer part q of their shift.  The wake
// round of a vertex is D - q or D - q - 1 (D = Delta >> 20), depending on whether its shift's
// fractional part exceeds Delta's, so the q-buckets need no Delta and give every round's
// wakers in two adjacent segments.  Vertex n of the slot is settled (label 0).
__global__ __launch_bounds__(ADM_T) void k_adm_scan(AdmBatch b, int max_rounds, u64* __restrict__ adm_max,
                                                    unsigned* __restrict__ adm_err, u64* __restrict__ adm_hub,
                                                    u64* __restrict__ P, unsigned* __restrict__ cnt) {
  __shared__ unsigned h[QCAP];
  __shared__ u64 red[ADM_T / WAVE];
  const AdmItem& t = b.it[item_of(b, blockIdx.x)];
  const int j = blockIdx.x - t.blk0;
  const int Q = max_rounds < QCAP ? max_rounds : QCAP;  // buckets a runnable request can have
  for (int q = threadIdx.x; q < Q; q += ADM_T) h[q] = 0;
  __syncthreads();
  const long long lo = chunk(t.n, j, t.nblk), hi = chunk(t.n, j + 1, t.nblk);
  u64 mx = 0, bad = 0, hub = 0;
  for (long long v = lo + threadIdx.x; v < hi; v += ADM_T) {
    const int a = t.rp[v], e = t.rp[v + 1];
    const long long s = t.shift[v];
    P[t.vbeg + v] = INF;
    if (e < a || (v == 0 && a != 0) || (v == t.n - 1 && (long long)e != t.nnz)) bad |= ERR_BAD_ROWPTR;
    else if (e > a && (((u64)(unsigned)(e - a) << 32) | (u64)v) > hub) hub = ((u64)(unsigned)(e - a) << 32) | (u64)v;
    if (s < 0 || s > (1ll << 52)) {
      bad |= ERR_BAD_SHIFT;
    } else {
      mx = (u64)s > mx ? (u64)s : mx;
      const u64 q = (u64)s >> FIX;
      if (e > a && q < (u64)Q) atomicAdd(&h[q], 1u);  // a larger q: too many rounds to run anyway
    }
  }
  if (j == t.nblk - 1 && threadIdx.x == 0) P[t.vbeg + t.n] = 0;
  mx = block_max_or(mx, red, false);
  hub = block_max_or(hub, red, false);
  bad = block_max_or(bad, red, true);
  if (threadIdx.x == 0) {
    if (mx) atomic_max_u64(&adm_max[t.slot], mx);
    if (hub) atomic_max_u64(&adm_hub[t.slot], hub);
    if (bad) atomic_or_u32(&adm_err[t.slot], (unsigned)bad);
  }
  unsigned* row = cnt + (size_t)t.slot * max_rounds;
  for (int q = threadIdx.x; q < Q; q += ADM_T)
    if (h[q]) atomicAdd(&row[q], h[q]);
}

// One block per request: bucket offsets (wake_tab row of the slot, indexed by q, R + 1 entries)
// and the place cursors from the counts (the whole row of counts is cleared for the next
// occupant; a cursor holds the bucket's next front position in its low half and the entries
// placed from its end in its high half), the slot's table entry, the engine state's unsettled arcs, and the report
// (adm_err, then R).  The request's rounds before its first possible waker, fr = D - q_max - 1
// (q_max its highest non-empty bucket), wake nobody: its origin moves fr rounds back (r0 - fr),
// so that its first wakers wake in the first step after admission.  Its keys stay >= the round
// of admission (every vertex with arcs has Delta - shift >= fr units), so nothing it writes is
// settled before that step.
__global__ __launch_bounds__(ADM_T) void k_adm_commit(AdmBatch b, int max_rounds, const u64* __restrict__ adm_max,
                                                      unsigned* __restrict__ adm_err, unsigned* __restrict__ cnt,
                                                      u64* __restrict__ cur, int* __restrict__ wake_tab,
                                                      SlotInfo* __restrict__ slots, RoundState* st, long long k_last,
                                                      SlotState* __restrict__ sst, u64* __restrict__ s_cnt,
                                                      u64* __restrict__ s_lr, SlotReport* rep) {
  __shared__ unsigned w_sum[ADM_T / WAVE];
  __shared__ int q_top;
  const AdmItem& t = b.it[blockIdx.x];
  const u64 delta = adm_max[t.slot];
  const unsigned err = adm_err[t.slot];
  const int R = request_rounds(delta, err, max_rounds);
  unsigned* crow = cnt + (size_t)t.slot * max_rounds;
  u64* urow = cur + (size_t)t.slot * (max_rounds + 1);
  int* wrow = wake_tab + (size_t)t.slot * (max_rounds + 1);
  // thread i takes buckets [i per, (i + 1) per) of the whole row (cleared), the first R counted
  const int per = (max_rounds + ADM_T - 1) / ADM_T;
  const int lo = threadIdx.x * per, hi = min(max_rounds, lo + per);
  unsigned s = 0;
  int top = -1;
  for (int q = lo; q < hi; ++q) {
    if (q < R) {
      s += crow[q];
      if (crow[q]) top = q;
    }
  }
  if (threadIdx.x == 0) q_top = -1;
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  const unsigned incl = wave_incl_scan(s);
  if (lane == WAVE - 1) w_sum[wid] = incl;
  __syncthreads();
  if (top >= 0) atomicMax(&q_top, top);
  unsigned acc = incl - s, total = 0;
  for (int w = 0; w < ADM_T / WAVE; ++w) {
    if (w < (int)wid) acc += w_sum[w];
    total += w_sum[w];
  }
  for (int q = lo; q < hi; ++q) {
    if (q < R) {
      const unsigned x = crow[q];
      wrow[q] = (int)acc;
      urow[q] = acc;
      acc += x;
    }
    crow[q] = 0;
  }
  if (threadIdx.x == 0 && R) wrow[R] = (int)total;
  __syncthreads();
  const int D = R - 1;
  const int first_ne = q_top >= 0 && D - q_top - 1 > 0 ? D - q_top - 1 : 0;
  if (threadIdx.x == 0) {
    SlotInfo e;
    e.rp = t.rp;
    e.col = t.col;
    e.shift = t.shift;
    e.delta = delta;
    e.nnz = t.nnz;
    e.vbeg = t.vbeg;
    e.r0 = t.r0 - first_ne;
    e.R = R;
    e.wbase = t.slot * (max_rounds + 1);
    e.active = R > 0;
    e.n = t.n;
    slots[t.slot] = e;
    if (R) atomic_add_u64((u64*)&st[k_last & 1].unsettled_arcs, (u64)t.nnz);
    // the slot's traversal state as step k_last + 1 reads it: all arcs unsettled, no frontier
    SlotState q;
    q.ua = t.nnz;
    q.dir = DIR_TD;
    q.mode = SM_ROUNDS;
    q.settled = 0;
    sst[(k_last & 1) * MAX_SLOTS + t.slot] = q;
    s_cnt[(k_last % 3) * MAX_SLOTS + t.slot] = 0;
    s_lr[(k_last % 3) * MAX_SLOTS + t.slot] = INF;
    // too many rounds: the request is inert, and its finishing reports why
    const unsigned rerr = err | (((delta >> FIX) + 1 > (u64)max_rounds && !(err & ROW_ERRS)) ? ERR_ROUNDS : 0u);
    if (rerr != err) adm_err[t.slot] = rerr;
    __hip_atomic_store(&rep[t.slot].adm_err, rerr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&rep[t.slot].R, (long long)R, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Each vertex with arcs to its q-bucket's segment of the slot's part of wake_ord: to the front
// of the segment if its shift's fractional part is at most Delta's (it wakes in round D - q),
// to the back otherwise (round D - q - 1).  Buckets ascend, so the wakers of round rho are one
// range, from the split of bucket D - rho - 1 to the split of bucket D - rho, and the split of
// bucket q is the low half of its cursor once every block has placed its vertices.
__global__ __launch_bounds__(ADM_T) void k_adm_place(AdmBatch b, int max_rounds, const u64* __restrict__ adm_max,
                                                     const unsigned* __restrict__ adm_err, u64* __restrict__ cur,
                                                     const int* __restrict__ wake_tab, int* __restrict__ wake_ord) {
  __shared__ unsigned hf[QCAP], hb[QCAP];
  const AdmItem& t = b.it[item_of(b, blockIdx.x)];
  const int j = blockIdx.x - t.blk0;
  const u64 delta = adm_max[t.slot];
  const int R = request_rounds(delta, adm_err[t.slot], max_rounds);
  if (R == 0) return;  // whole block leaves together
  const u64 dfrac = delta & (S_ONE - 1);
  for (int q = threadIdx.x; q < R; q += ADM_T) hf[q] = hb[q] = 0;
  __syncthreads();
  const long long lo = chunk(t.n, j, t.nblk), hi = chunk(t.n, j + 1, t.nblk);
  for (long long v = lo + threadIdx.x; v < hi; v += ADM_T)
    if (t.rp[v + 1] > t.rp[v]) {
      const u64 s = (u64)t.shift[v];
      atomicAdd((s & (S_ONE - 1)) > dfrac ? &hb[s >> FIX] : &hf[s >> FIX], 1u);
    }
  __syncthreads();
  u64* urow = cur + (size_t)t.slot * (max_rounds + 1);
  const int* wrow = wake_tab + (size_t)t.slot * (max_rounds + 1);
  for (int q = threadIdx.x; q < R; q += ADM_T)
    if (hf[q] | hb[q]) {
      const u64 old = atomicAdd((unsigned long long*)&urow[q], ((u64)hb[q] << 32) | hf[q]);
      hf[q] = (unsigned)old;
      hb[q] = (unsigned)wrow[q + 1] - (unsigned)(old >> 32) - hb[q];
    }
  __syncthreads();
  for (long long v = lo + threadIdx.x; v < hi; v += ADM_T)
    if (t.rp[v + 1] > t.rp[v]) {
      const u64 s = (u64)t.shift[v];
      const unsigned pos = atomicAdd((s & (S_ONE - 1)) > dfrac ? &hb[s >> FIX] : &hf[s >> FIX], 1u);
      wake_ord[t.vbeg + pos] = (int)(t.vbeg + v);
    }
}

// ------------------------------------------------------------------------------------------
// finishing: centres, hub piece and rows outside it -> cut over those rows -> report
// ------------------------------------------------------------------------------------------
// The cut counts the arcs whose ends have different centres, twice per cut edge.  With H the
// piece of the request's hub, an edge between H and the rest is cut, an edge inside H is not:
// so only the rows outside H are read.  An arc from outside H into H counts 2 (its reverse is
// not read), an arc between two vertices outside H counts 1 if their centres differ (its
// reverse counts the other 1).  RMAT-like requests have almost all arcs inside H.

// Vertex chunks aligned to 64 vertices (the slot starts on a multiple of 64), so every bitmap
// word belongs to one block of one request.
__device__ __forceinline__ long long chunk64(long long n, int j, int nb) {
  return j == nb ? n : (((n * j / nb) >> 6) << 6);
}

// Centres (request-local ids) into the caller's buffer, the bit of H of every vertex, and the
// rows outside H with arcs, listed (local id, arc prefix) in the slot's range of one queue pair
// (a request found done has nothing queued and is never expanded again).
__global__ __launch_bounds__(FIN_T) void k_fin_vertices(FinBatch b, int B, const u64* __restrict__ P,
                                                        const SlotInfo* __restrict__ slots,
                                                        const u64* __restrict__ adm_hub, u64* __restrict__ hbits,
                                                        int* __restrict__ list_v, unsigned* __restrict__ list_a,
                                                        u64* __restrict__ lcnt) {
  constexpr int NWF = FIN_T / WAVE;
  __shared__ unsigned w_cnt[NWF], w_arcs[NWF];
  __shared__ u64 base;
  const FinItem& t = b.it[item_of(b, blockIdx.x)];
  const int j = blockIdx.x - t.blk0;
  const u64 mask = ((u64)1 << B) - 1;
  const bool ran = slots[t.slot].active != 0;
  const long long lo = chunk64(t.n, j, t.nblk), hi = chunk64(t.n, j + 1, t.nblk);
  const long long hv = t.vbeg + (long long)(adm_hub[t.slot] & 0xffffffffull);
  const u64 hubc = P[hv] == INF ? (u64)hv : (P[hv] & mask);
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  for (long long v0 = lo; v0 < hi; v0 += FIN_T) {  // uniform trip count over the block
    const long long v = v0 + threadIdx.x;
    bool out = false;
    unsigned deg = 0;
    bool inH = false;
    // loads first, at an index clamped into the chunk, so that they need no branch
    const long long vc = v < hi ? v : hi - 1;
    const u64 p = P[t.vbeg + vc];
    const u64 c = p == INF ? (u64)(t.vbeg + vc) : (p & mask);  // INF: isolated, its own centre
    const int r0 = t.rp[vc], r1 = t.rp[vc + 1];
    if (v < hi) {
      t.centre[v] = ran ? (int)(c - (u64)t.vbeg) : -1;
      deg = (unsigned)(r1 - r0);
      inH = c == hubc;
      out = ran && !inH && deg > 0;
    }
    const u64 hb = __ballot(inH);
    if (lane == 0 && v0 + wid * WAVE < hi) hbits[(t.vbeg + v0 + wid * WAVE) >> 6] = hb;
    const u64 om = __ballot(out);
    const unsigned incl = wave_incl_scan(out ? deg : 0u);
    if (lane == WAVE - 1) {
      w_cnt[wid] = (unsigned)__popcll(om);
      w_arcs[wid] = incl;
    }
    __syncthreads();
    unsigned bc = 0, ba = 0, tc = 0, ta = 0;
    for (int w = 0; w < NWF; ++w) {
      if (w < (int)wid) {
        bc += w_cnt[w];
        ba += w_arcs[w];
      }
      tc += w_cnt[w];
      ta += w_arcs[w];
    }
    if (tc) {  // uniform
      if (threadIdx.x == 0) base = atomic_add_u64(&lcnt[t.slot], ((u64)tc << 32) | ta);
      __syncthreads();
      if (out) {
        const unsigned idx = (unsigned)(base >> 32) + bc + rank_below(om);
        const unsigned pre = (unsigned)base + ba + incl - deg;
        list_v[t.vbeg + idx] = (int)v;
        list_a[t.vbeg + idx] = pre;
      }
    }
    __syncthreads();
  }
}

// The listed rows' arcs, split evenly over the item's blocks, walked in tiles of FIN_T arcs with
// a window of list entries in LDS.
__global__ __launch_bounds__(FIN_T) void k_fin_cut(FinBatch b, int B, const u64* __restrict__ P,
                                                   const u64* __restrict__ hbits, const int* __restrict__ list_v,
                                                   const unsigned* __restrict__ list_a, const u64* __restrict__ lcnt,
                                                   u64* __restrict__ cut_acc) {
  constexpr int T = FIN_T;
  __shared__ unsigned w_pre[T + 1];
  __shared__ int w_first[T + 1];
  __shared__ u64 w_c[T + 1];
  __shared__ unsigned s_ent;
  __shared__ u64 red[T / WAVE];
  const FinItem& t = b.it[item_of(b, blockIdx.x)];
  const int j = blockIdx.x - t.blk0;
  const u64 mask = ((u64)1 << B) - 1;
  const u64 lc = lcnt[t.slot];
  const unsigned ne = (unsigned)(lc >> 32), na = (unsigned)lc;
  const unsigned a_begin = (unsigned)(((u64)na * j) / t.nblk), a_end = (unsigned)(((u64)na * (j + 1)) / t.nblk);
  const int* LV = list_v + t.vbeg;
  const unsigned* LA = list_a + t.vbeg;
  const u64* Ps = P + t.vbeg;
  u64 cut = 0;
  if (a_begin < a_end) {  // uniform
    if (threadIdx.x < WAVE) {  // the last entry whose arcs start at or before a_begin
      const unsigned e = wave_search_le(LA, ne, a_begin);
      if (threadIdx.x == 0) s_ent = e;
    }
    __syncthreads();
    unsigned ent = s_ent;
    for (unsigned tile = a_begin; tile < a_end; tile += T) {
      for (int kk = threadIdx.x; kk <= T; kk += T) {
        const unsigned e = ent + kk;
        if (e < ne) {
          const int v = LV[e];
          w_pre[kk] = LA[e];
          w_first[kk] = t.rp[v];
          w_c[kk] = Ps[v] & mask;
        } else {
          w_pre[kk] = na;
          w_first[kk] = 0;
          w_c[kk] = 0;
        }
      }
      __syncthreads();
      const unsigned a = tile + threadIdx.x;
      if (a < a_end) {
        int lo = 0, hi = T;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_pre[mid] <= a) lo = mid;
          else hi = mid;
        }
        const int wl = t.col[(long long)w_first[lo] + (a - w_pre[lo])];
        if ((unsigned)wl < (unsigned)t.n) {  // (a request with a bad column id fails anyway)
          const long long w = t.vbeg + wl;  // arena id
          if ((hbits[w >> 6] >> (w & 63)) & 1) cut += 2;
          else cut += (P[w] & mask) != w_c[lo];
        }
      }
      const unsigned next = tile + T;
      __syncthreads();
      if (threadIdx.x == 0) {
        int lo = 0, hi = T + 1;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_pre[mid] <= next) lo = mid;
          else hi = mid;
        }
        s_ent = ent + lo;
      }
      __syncthreads();
      ent = s_ent;
    }
  }
  cut = wave_sum_u64(cut);
  if (lane_id() == 0) red[threadIdx.x / WAVE] = cut;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 s = 0;
    for (int w = 0; w < T / WAVE; ++w) s += red[w];
    if (s) atomic_add_u64(&cut_acc[t.slot], s);
  }
}

// One thread per finished request: the report (cut, error bits, then done), and the slot's
// per-request state cleared for the next occupant.
__global__ void k_fin_out(FinBatch b, u64* __restrict__ cut_acc, unsigned* __restrict__ adm_err,
                          u64* __restrict__ adm_max, u64* __restrict__ adm_hub, u64* __restrict__ lcnt,
                          const Ctrl* __restrict__ ctrl, SlotInfo* __restrict__ slots, SlotReport* rep) {
  const int i = threadIdx.x;
  if (blockIdx.x != 0 || i >= b.count) return;
  const int s = b.it[i].slot;
  const unsigned e = adm_err[s] | __hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&rep[s].cut, (long long)(cut_acc[s] / 2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&rep[s].fin_err, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  cut_acc[s] = 0;
  adm_err[s] = 0;
  adm_max[s] = 0;
  adm_hub[s] = 0;
  lcnt[s] = 0;
  slots[s].active = 0;
  __hip_atomic_store(&rep[s].done, 1ll, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Rebase: every live key drops by X rounds.  Keys below X rounds belong to vertices outside the
// active slots (free ranges, separators, finished requests): they become 0, i.e. settled.
// The slots' r0 and the host's round numbering move by the same X.
__global__ __launch_bounds__(256) void k_rebase(long long V, int B, long long X, u64* __restrict__ P,
                                                u64* __restrict__ lr_part, int n_lr,
                                                u64* __restrict__ s_lr, SlotInfo* __restrict__ slots, int nslots,
                                                RoundState* st, long long k_last) {
  const u64 xf = (u64)X * S_ONE;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long items = V > n_lr ? V : n_lr;
  items = items > 3 * MAX_SLOTS ? items : 3 * MAX_SLOTS;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < items; i += stride) {
    if (i < V) {
      const u64 p = P[i];
      if (p != INF) P[i] = (p >> B) >= xf ? p - (xf << B) : 0;
    }
    if (i < n_lr) {
      const u64 l = lr_part[i];
      if (l != INF) lr_part[i] = (l >> B) >= xf ? l - (xf << B) : 0;
    }
    if (i < 3 * MAX_SLOTS) {
      const u64 l = s_lr[i];
      if (l != INF) s_lr[i] = (l >> B) >= xf ? l - (xf << B) : 0;
    }
    if (i < nslots) slots[i].r0 -= X;
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
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  int state = RQ_QUEUED;
  ldd_status status = LDD_ERR_PENDING;
  int slot = -1;
  long long vbeg = 0;
  long long r0 = 0;          // global round of its round 0 (numbering at admission)
  long long first_step = 0;  // the step that runs its round 0
  int R = -1;                // rounds, once the admission has reported them
  int64_t cut = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct ldd_server {
  ldd_server_config cfg{};
  int dev = 0;
  long long vcap = 0;
  int B = 1;
  long long round_limit = 0;  // keys stay below round_limit * 2^20
  int max_rounds = 0;         // largest R a request may have
  hipStream_t stream = nullptr;
  // finishing runs on its own stream, beside the steps that follow: it reads only the finished
  // requests' vertex ranges and slots, which no step and no admission touches until the reports
  // arrive; fin_dep orders it after the steps enqueued before it
  hipStream_t fin_stream = nullptr;
  hipEvent_t fin_dep = nullptr, fin_done = nullptr;
  hipEvent_t chunk_ev[2] = {};
  hipGraphExec_t graph = nullptr;
  int blocks = 0;
  // arena and engine buffers (device)
  void *P = nullptr, *qv0 = nullptr, *qv1 = nullptr, *qa0 = nullptr, *qa1 = nullptr, *wake_ord = nullptr;
  void *wake_tab = nullptr, *cnt = nullptr, *cur = nullptr;
  void *slots = nullptr, *st = nullptr, *qcnt = nullptr, *lr_part = nullptr, *lb = nullptr, *ex_part = nullptr;
  void *ctrl = nullptr, *adm_max = nullptr, *adm_err = nullptr, *cut_acc = nullptr;
  void *sst = nullptr, *s_cnt = nullptr, *s_lr = nullptr, *stamp = nullptr;
  void *adm_hub = nullptr, *hbits = nullptr, *lcnt = nullptr;
  SlotEnd* s_end = nullptr;      // mapped host memory: the step each slot was found done
  SlotEnd* s_end_dev = nullptr;  // its device address
  SlotReport* rep = nullptr;      // mapped host memory
  SlotReport* rep_dev = nullptr;  // its device address
  RangeAlloc valloc;
  Request* slot_req[MAX_SLOTS] = {};
  long long steps = 0;       // steps enqueued so far
  long long round_base = 0;  // global round of step 1 in the current numbering
  std::mutex ev_mu;          // the event pool
  std::vector<hipEvent_t> ev_pool;
  std::mutex mu;  // everything below, and the allocators and slot_req
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
  // arcs of the requests on the device: a step splits the top-down slots' frontier arcs over the
  // grid with 32-bit prefix sums, so admission keeps this sum below 2^32
  long long active_arcs = 0;
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

// A request's vertex range: its n vertices and the separator, rounded up to 64 vertices so that
// every range starts on a bitmap word.
long long vrange(int n) { return (((long long)n + 1 + 63) >> 6) << 6; }

hipEvent_t get_event(ldd_server* srv) {
  {
    std::lock_guard<std::mutex> lk(srv->ev_mu);
    if (!srv->ev_pool.empty()) {
      hipEvent_t e = srv->ev_pool.back();
      srv->ev_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void put_event(ldd_server* srv, hipEvent_t e) {
  std::lock_guard<std::mutex> lk(srv->ev_mu);
  srv->ev_pool.push_back(e);
}

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

// Device bytes per arena vertex: label, two queues with arc prefixes, wake order, tail stamp
// and a bit of the finishing bitmap (rounded up).  The requests' CSR and shifts stay in the
// callers' buffers.
constexpr long long BYTES_PER_VERTEX = 8 + 8 + 8 + 4 + 4 + 1;

ldd_status srv_setup(ldd_server* srv) {
  SRV_TRY(hipSetDevice(srv->dev));
  SRV_TRY(hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking));
  SRV_TRY(hipStreamCreateWithFlags(&srv->fin_stream, hipStreamNonBlocking));
  SRV_TRY(hipEventCreateWithFlags(&srv->fin_dep, hipEventDisableTiming));
  SRV_TRY(hipEventCreateWithFlags(&srv->fin_done, hipEventDisableTiming));
  for (auto& e : srv->chunk_ev) SRV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  const long long V = srv->vcap;
  const size_t per_slot = (size_t)MAX_SLOTS * (srv->max_rounds + 1);
  ldd_status s;
  if ((s = srv_alloc(srv, &srv->P, V * 8)) || (s = srv_alloc(srv, &srv->qv0, V * 4)) ||
      (s = srv_alloc(srv, &srv->qv1, V * 4)) || (s = srv_alloc(srv, &srv->qa0, V * 4)) ||
      (s = srv_alloc(srv, &srv->qa1, V * 4)) || (s = srv_alloc(srv, &srv->wake_ord, V * 4)) ||
      (s = srv_alloc(srv, &srv->wake_tab, per_slot * 4)) ||
      (s = srv_alloc(srv, &srv->cnt, per_slot * 4)) || (s = srv_alloc(srv, &srv->cur, per_slot * 8)) ||
      (s = srv_alloc(srv, &srv->slots, sizeof(SlotInfo) * MAX_SLOTS)) ||
      (s = srv_alloc(srv, &srv->st, 2 * sizeof(RoundState))) || (s = srv_alloc(srv, &srv->qcnt, 3 * 16 * 8)) ||
      (s = srv_alloc(srv, &srv->lr_part, 2 * (size_t)RT * 8)) ||
      (s = srv_alloc(srv, &srv->lb, sizeof(LaunchBlock))) || (s = srv_alloc(srv, &srv->ex_part, (size_t)RT * 8)) ||
      (s = srv_alloc(srv, &srv->ctrl, sizeof(Ctrl))) || (s = srv_alloc(srv, &srv->adm_max, MAX_SLOTS * 8)) ||
      (s = srv_alloc(srv, &srv->adm_err, MAX_SLOTS * 4)) || (s = srv_alloc(srv, &srv->cut_acc, MAX_SLOTS * 8)) ||
      (s = srv_alloc(srv, &srv->sst, 2 * MAX_SLOTS * sizeof(SlotState))) ||
      (s = srv_alloc(srv, &srv->s_cnt, 3 * MAX_SLOTS * 8)) || (s = srv_alloc(srv, &srv->s_lr, 3 * MAX_SLOTS * 8)) ||
      (s = srv_alloc(srv, &srv->stamp, V * 4)) || (s = srv_alloc(srv, &srv->adm_hub, MAX_SLOTS * 8)) ||
      (s = srv_alloc(srv, &srv->hbits, (V / 64 + 2) * 8)) || (s = srv_alloc(srv, &srv->lcnt, MAX_SLOTS * 8)))
    return s;
  SRV_TRY(hipHostMalloc((void**)&srv->rep, sizeof(SlotReport) * MAX_SLOTS,
                        hipHostMallocMapped | hipHostMallocCoherent));
  memset(srv->rep, 0, sizeof(SlotReport) * MAX_SLOTS);
  SRV_TRY(hipHostGetDevicePointer((void**)&srv->rep_dev, srv->rep, 0));
  SRV_TRY(hipHostMalloc((void**)&srv->s_end, sizeof(SlotEnd) * MAX_SLOTS, hipHostMallocMapped | hipHostMallocCoherent));
  memset(srv->s_end, 0, sizeof(SlotEnd) * MAX_SLOTS);
  SRV_TRY(hipHostGetDevicePointer((void**)&srv->s_end_dev, srv->s_end, 0));
  const hipStream_t q = srv->stream;
  // every vertex is settled (label 0) until a request claims it
  SRV_TRY(hipMemsetAsync(srv->P, 0, V * 8, q));
  SRV_TRY(hipMemsetAsync(srv->cnt, 0, per_slot * 4, q));
  SRV_TRY(hipMemsetAsync(srv->slots, 0, sizeof(SlotInfo) * MAX_SLOTS, q));
  SRV_TRY(hipMemsetAsync(srv->qcnt, 0, 3 * 16 * 8, q));
  SRV_TRY(hipMemsetAsync(srv->ex_part, 0, (size_t)RT * 8, q));
  SRV_TRY(hipMemsetAsync(srv->ctrl, 0, sizeof(Ctrl), q));
  SRV_TRY(hipMemsetAsync(srv->adm_max, 0, MAX_SLOTS * 8, q));
  SRV_TRY(hipMemsetAsync(srv->adm_err, 0, MAX_SLOTS * 4, q));
  SRV_TRY(hipMemsetAsync(srv->cut_acc, 0, MAX_SLOTS * 8, q));
  SRV_TRY(hipMemsetAsync(srv->lr_part, 0xff, 2 * (size_t)RT * 8, q));
  SRV_TRY(hipMemsetAsync(srv->stamp, 0, V * 4, q));  // stamps are step numbers (>= 1)
  SRV_TRY(hipMemsetAsync(srv->adm_hub, 0, MAX_SLOTS * 8, q));
  SRV_TRY(hipMemsetAsync(srv->lcnt, 0, MAX_SLOTS * 8, q));
  SRV_TRY(hipMemsetAsync(srv->sst, 0, 2 * MAX_SLOTS * sizeof(SlotState), q));
  SRV_TRY(hipMemsetAsync(srv->s_cnt, 0, 3 * MAX_SLOTS * 8, q));
  SRV_TRY(hipMemsetAsync(srv->s_lr, 0xff, 3 * MAX_SLOTS * 8, q));
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

  int ncu = 0;
  SRV_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, srv->dev));
  srv->blocks = srv->cfg.blocks > 0 ? std::min(srv->cfg.blocks, RT) : std::min(2 * ncu, RT);

  LaunchBlock lb{};
  RoundCtx& c = lb.c;
  c.n = (int)V;
  c.B = srv->B;
  c.R = INT32_MAX;
  c.nnz = 0;  // the requests' CSR and shifts are read through their slots
  c.delta = 0;
  c.n_active = 0;
  c.row_ptr = nullptr;
  c.col = nullptr;
  c.shift = nullptr;
  c.P = (u64*)srv->P;
  c.qv[0] = (int*)srv->qv0;
  c.qv[1] = (int*)srv->qv1;
  c.qa[0] = (unsigned*)srv->qa0;
  c.qa[1] = (unsigned*)srv->qa1;
  c.wake_ord = (int*)srv->wake_ord;
  c.wake_off = nullptr;
  c.next_ne = nullptr;
  c.wake_q = 0;
  c.qcnt = (u64*)srv->qcnt;
  c.lr_part = (u64*)srv->lr_part;
  c.stamp = (unsigned*)srv->stamp;
  c.st = (RoundState*)srv->st;
  c.ctrl = (Ctrl*)srv->ctrl;
  c.dir_policy = srv->cfg.direction;
  c.td_to_bu = 14;
  c.bu_to_td = 24;
  c.tail_den = srv->cfg.tail_vertices == 0 ? 32 : (srv->cfg.tail_vertices < 0 ? 0 : srv->cfg.tail_vertices);
  c.tail_min_left = 16;
  c.report = nullptr;
  c.ex_part = (u64*)srv->ex_part;
  c.slots = (const SlotInfo*)srv->slots;
  c.nslots = srv->cfg.max_slots;
  c.wake_tab = (const int*)srv->wake_tab;
  c.wake_cur = (const u64*)srv->cur;
  c.sst = (SlotState*)srv->sst;
  c.s_cnt = (u64*)srv->s_cnt;
  c.s_lr = (u64*)srv->s_lr;
  c.s_end = srv->s_end_dev;
  c.slot_err = (unsigned*)srv->adm_err;
  lb.kbase = 1;
  SRV_TRY(hipMemcpyAsync(srv->lb, &lb, sizeof(LaunchBlock), hipMemcpyHostToDevice, q));
  SRV_TRY(hipStreamSynchronize(q));
  // the step graph: chunk_steps round steps, then the step base moves on
  hipStream_t cap = nullptr;
  SRV_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  SRV_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < srv->cfg.chunk_steps; ++j)
    hipLaunchKernelGGL(k_round_step_srv, dim3(srv->blocks), dim3(RT), 0, cap, (const LaunchBlock*)srv->lb, j);
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, cap, (LaunchBlock*)srv->lb, srv->cfg.chunk_steps);
  SRV_TRY(hipStreamEndCapture(cap, &g));
  SRV_TRY(hipGraphInstantiate(&srv->graph, g, nullptr, nullptr, 0));
  SRV_TRY(hipGraphDestroy(g));
  SRV_TRY(hipStreamDestroy(cap));
  return LDD_OK;
}

volatile SlotReport& report(ldd_server* srv, int slot) { return ((volatile SlotReport*)srv->rep)[slot]; }

// The slot's report is cleared before its admission is enqueued (the device writes it later).
void rep_reset(ldd_server* srv, int slot) {
  ((volatile SlotEnd*)srv->s_end)[slot].step = 0;
  volatile SlotReport& rp = report(srv, slot);
  rp.done = 0;
  rp.R = -1;
  rp.adm_err = 0;
  rp.fin_err = 0;
  rp.cut = 0;
}

int blocks_for(long long n, long long nnz, long long per_block) {
  return (int)std::max<long long>(1, std::min<long long>(1024, (n + nnz / 8 + per_block - 1) / per_block));
}

// Enqueue the admission of a batch of requests (ranges and slots already taken).
ldd_status srv_admit(ldd_server* srv, const std::vector<Request*>& rs) {
  const hipStream_t s = srv->stream;
  for (size_t b0 = 0; b0 < rs.size(); b0 += MAX_BATCH) {
    AdmBatch ab{};
    int nblk = 0;
    for (size_t i = b0; i < rs.size() && ab.count < MAX_BATCH; ++i) {
      Request* r = rs[i];
      if (r->ready) {
        SRV_TRY(hipStreamWaitEvent(s, r->ready, 0));
        put_event(srv, r->ready);  // the wait took the recorded state; the event may be reused
        r->ready = nullptr;
      }
      AdmItem& t = ab.it[ab.count++];
      t.rp = r->q.row_ptr;
      t.col = r->q.col_idx;
      t.shift = (const long long*)r->q.shift_fix;
      t.vbeg = r->vbeg;
      t.nnz = r->q.nnz;
      t.r0 = r->r0;
      t.n = r->q.n;
      t.slot = r->slot;
      t.blk0 = nblk;
      t.nblk = blocks_for(r->q.n, r->q.nnz, 16384);
      nblk += t.nblk;
      rep_reset(srv, r->slot);
    }
    hipLaunchKernelGGL(k_adm_scan, dim3(nblk), dim3(ADM_T), 0, s, ab, srv->max_rounds, (u64*)srv->adm_max,
                       (unsigned*)srv->adm_err, (u64*)srv->adm_hub, (u64*)srv->P, (unsigned*)srv->cnt);
    hipLaunchKernelGGL(k_adm_commit, dim3(ab.count), dim3(ADM_T), 0, s, ab, srv->max_rounds,
                       (const u64*)srv->adm_max, (unsigned*)srv->adm_err, (unsigned*)srv->cnt,
                       (u64*)srv->cur, (int*)srv->wake_tab, (SlotInfo*)srv->slots, (RoundState*)srv->st,
                       srv->steps, (SlotState*)srv->sst, (u64*)srv->s_cnt, (u64*)srv->s_lr, srv->rep_dev);
    hipLaunchKernelGGL(k_adm_place, dim3(nblk), dim3(ADM_T), 0, s, ab, srv->max_rounds, (const u64*)srv->adm_max,
                       (const unsigned*)srv->adm_err, (u64*)srv->cur, (const int*)srv->wake_tab,
                       (int*)srv->wake_ord);
    SRV_TRY(hipGetLastError());
  }
  return LDD_OK;
}

// Enqueue the finishing of a batch of requests whose last round and the step after it are
// enqueued: centres into the callers' buffers, cuts, reports.
ldd_status srv_finish(ldd_server* srv, const std::vector<Request*>& rs) {
  const hipStream_t s = srv->fin_stream;
  SRV_TRY(hipEventRecord(srv->fin_dep, srv->stream));
  SRV_TRY(hipStreamWaitEvent(s, srv->fin_dep, 0));
  for (size_t b0 = 0; b0 < rs.size(); b0 += MAX_BATCH) {
    FinBatch fv{}, fc{};
    int nv = 0, nc = 0;
    for (size_t i = b0; i < rs.size() && fv.count < MAX_BATCH; ++i) {
      Request* r = rs[i];
      FinItem t{};
      t.centre = r->q.centre;
      t.rp = r->q.row_ptr;
      t.col = r->q.col_idx;
      t.vbeg = r->vbeg;
      t.nnz = r->q.nnz;
      t.n = r->q.n;
      t.slot = r->slot;
      t.blk0 = nv;
      t.nblk = (int)std::max<long long>(1, std::min<long long>(4096, ((long long)r->q.n + 2047) / 2048));
      nv += t.nblk;
      fv.it[fv.count++] = t;
      t.blk0 = nc;
      t.nblk = (int)std::max<long long>(1, std::min<long long>(4096, r->q.nnz / 8192));
      nc += t.nblk;
      fc.it[fc.count++] = t;
      r->state = RQ_FINISHING;
    }
    hipLaunchKernelGGL(k_fin_vertices, dim3(nv), dim3(FIN_T), 0, s, fv, srv->B, (const u64*)srv->P,
                       (const SlotInfo*)srv->slots, (const u64*)srv->adm_hub, (u64*)srv->hbits, (int*)srv->qv0,
                       (unsigned*)srv->qa0, (u64*)srv->lcnt);
    hipLaunchKernelGGL(k_fin_cut, dim3(nc), dim3(FIN_T), 0, s, fc, srv->B, (const u64*)srv->P, (const u64*)srv->hbits,
                       (const int*)srv->qv0, (const unsigned*)srv->qa0, (const u64*)srv->lcnt,
                       (u64*)srv->cut_acc);
    hipLaunchKernelGGL(k_fin_out, dim3(1), dim3(64), 0, s, fv, (u64*)srv->cut_acc, (unsigned*)srv->adm_err,
                       (u64*)srv->adm_max, (u64*)srv->adm_hub, (u64*)srv->lcnt, (const Ctrl*)srv->ctrl,
                       (SlotInfo*)srv->slots, srv->rep_dev);
    SRV_TRY(hipGetLastError());
  }
  SRV_TRY(hipEventRecord(srv->fin_done, s));
  return LDD_OK;
}

// Lower the global round numbering by X rounds (X <= every active slot's r0).
ldd_status srv_rebase(ldd_server* srv, long long X) {
  SRV_TRY(hipStreamWaitEvent(srv->stream, srv->fin_done, 0));  // finishing reads labels the rebase rewrites
  hipLaunchKernelGGL(k_rebase, dim3((unsigned)std::min<long long>(8192, (std::max<long long>(srv->vcap, 2 * RT) + 255) / 256)), dim3(256), 0,
                     srv->stream, srv->vcap, srv->B, X, (u64*)srv->P, (u64*)srv->lr_part, 2 * RT, (u64*)srv->s_lr, (SlotInfo*)srv->slots, MAX_SLOTS,
                     (RoundState*)srv->st, srv->steps);
  SRV_TRY(hipGetLastError());
  srv->round_base -= X;
  ++srv->rebases;
  return LDD_OK;
}

ldd_status status_of(unsigned err) {
  if (err & (ERR_BARRIER | ERR_WATCHDOG | ERR_QUEUE)) return LDD_ERR_INTERNAL;
  if (err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) return LDD_ERR_INVALID_ARG;
  if (err & ERR_ROUNDS) return LDD_ERR_OVERFLOW;
  return LDD_OK;
}

ldd_status engine_loop(ldd_server* srv) {
  SRV_TRY(hipSetDevice(srv->dev));
  const int nslots = srv->cfg.max_slots;
  std::vector<Request*> finishing, batch;
  int inflight = 0, oldest = 0;
  for (;;) {
    // 1. finished requests whose reports have arrived go back to their callers
    bool handed = false;
    for (size_t i = 0; i < finishing.size();) {
      Request* r = finishing[i];
      volatile SlotReport& rp = report(srv, r->slot);
      if (__atomic_load_n(&rp.done, __ATOMIC_ACQUIRE) == 0) {
        ++i;
        continue;
      }
      const unsigned err = rp.fin_err;
      if (status_of(err) == LDD_ERR_INTERNAL) {
        snprintf(srv->fatal_msg, sizeof(srv->fatal_msg), "round engine error flags 0x%x", err);
        return LDD_ERR_INTERNAL;
      }
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->valloc.give(r->vbeg, vrange(r->q.n));
        srv->active_arcs -= r->q.nnz;
        srv->slot_req[r->slot] = nullptr;
        r->status = status_of(err);
        r->cut = r->status == LDD_OK ? (int64_t)rp.cut : 0;
        r->state = RQ_DONE;
        r->t_done = now_s();
        ++srv->completed;
      }
      handed = true;
      finishing[i] = finishing.back();
      finishing.pop_back();
    }
    if (handed) srv->cv_done.notify_all();
    // 2. rounds of admitted requests, as their admission reports them
    int active = 0;
    long long min_r0 = -1;
    for (int i = 0; i < nslots; ++i) {
      Request* r = srv->slot_req[i];
      if (!r || r->state != RQ_ACTIVE) continue;
      if (r->R < 0) {
        volatile SlotReport& rp = report(srv, i);
        const long long R = __atomic_load_n(&rp.R, __ATOMIC_ACQUIRE);
        if (R >= 0) r->R = (int)R;
      }
      ++active;
      min_r0 = min_r0 < 0 ? r->r0 : std::min(min_r0, r->r0);
    }
    // 3. admission, first come first served, while the head of the queue fits
    batch.clear();
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
          const ldd_status st = srv_rebase(srv, X);
          if (st != LDD_OK) return st;
          for (int i = 0; i < nslots; ++i)
            if (srv->slot_req[i] && srv->slot_req[i]->state == RQ_ACTIVE) srv->slot_req[i]->r0 -= X;
        }
      }
      const long long r0 = round_at(srv, srv->steps + 1);
      while (!srv->queue.empty() && r0 + srv->max_rounds <= srv->round_limit) {
        Request* r = srv->queue.front();
        int slot = -1;
        for (int i = 0; i < nslots && slot < 0; ++i)
          if (!srv->slot_req[i]) slot = i;
        if (slot < 0) break;
        if (srv->active_arcs + r->q.nnz > (long long)MAX_ACTIVE_ARCS) break;
        const long long vb = srv->valloc.take(vrange(r->q.n));
        if (vb < 0) break;
        srv->queue.pop_front();
        srv->active_arcs += r->q.nnz;
        r->vbeg = vb;
        r->slot = slot;
        r->r0 = r0;
        r->first_step = srv->steps + 1;
        r->R = -1;
        r->state = RQ_ACTIVE;
        r->t_admit = now_s();
        srv->slot_req[slot] = r;
        ++srv->admitted;
        ++active;
        srv->max_active = std::max<long long>(srv->max_active, active);
        batch.push_back(r);
      }
    }
    if (!batch.empty()) {
      const ldd_status st = srv_admit(srv, batch);
      if (st != LDD_OK) return st;
    }
    // 4. one more step chunk while any request is active (two chunks in flight)
    if (active > 0) {
      SRV_TRY(hipGraphLaunch(srv->graph, srv->stream));
      srv->steps += srv->cfg.chunk_steps;
      SRV_TRY(hipEventRecord(srv->chunk_ev[(oldest + inflight) & 1], srv->stream));
      ++inflight;
    }
    // 5. requests whose last round and the step after it are enqueued (that step consumes the
    // last frontier, so no later step refers to their vertex ids once they are released)
    batch.clear();
    for (int i = 0; i < nslots; ++i) {
      Request* r = srv->slot_req[i];
      if (!r || r->state != RQ_ACTIVE || r->R < 0) continue;
      // inert (failed its check), or found done by a step: that step consumed the request's
      // last frontier, so no later step refers to its vertex ids once they are released
      const long long end = __atomic_load_n(&((volatile SlotEnd*)srv->s_end)[i].step, __ATOMIC_ACQUIRE);
      if (r->R == 0 || end > 0) {
        batch.push_back(r);
        finishing.push_back(r);
        --active;
      } else if (srv->steps > r->first_step + r->R + 4 * std::max(srv->cfg.chunk_steps, 8) + 8) {
        snprintf(srv->fatal_msg, sizeof(srv->fatal_msg), "request in slot %d not done %lld steps after its last round",
                 i, srv->steps - (r->first_step + r->R));
        return LDD_ERR_INTERNAL;
      }
    }
    if (!batch.empty()) {
      const ldd_status st = srv_finish(srv, batch);
      if (st != LDD_OK) return st;
    }
    // 6. wait: for the older chunk once two are in flight, else for whatever is outstanding
    if (inflight == 2 || (inflight > 0 && active == 0)) {
      SRV_TRY(hipEventSynchronize(srv->chunk_ev[oldest]));
      oldest ^= 1;
      --inflight;
    } else if (inflight == 0 && active == 0 && !finishing.empty()) {
      SRV_TRY(hipStreamSynchronize(srv->fin_stream));
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
  out->rounds = r->R > 0 ? r->R : 0;
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
  if (srv->cfg.chunk_steps <= 0) srv->cfg.chunk_steps = 4;
  if (srv->cfg.chunk_steps > 64 || srv->cfg.direction < 0 || srv->cfg.direction > 2 || srv->cfg.blocks < 0 ||
      srv->cfg.max_rounds < 0 || srv->cfg.tail_vertices < -1) {
    delete srv;
    ldd_set_error("bad server configuration");
    return LDD_ERR_INVALID_ARG;
  }
  if (hipGetDevice(&srv->dev) != hipSuccess) {
    delete srv;
    ldd_set_error("no HIP device");
    return LDD_ERR_HIP;
  }
  long long V = srv->cfg.max_vertices;
  if (V <= 0) V = std::min<long long>(1ll << 30, srv->cfg.hbm_budget_bytes / BYTES_PER_VERTEX);
  const long long used = V * BYTES_PER_VERTEX;
  if (V < 64 || V > (1ll << 30) || (srv->cfg.hbm_budget_bytes > 0 && used > srv->cfg.hbm_budget_bytes)) {
    delete srv;
    ldd_set_error("budget gives an unusable arena (%lld vertices, %lld bytes)", V, used);
    return LDD_ERR_BUDGET;
  }
  srv->vcap = V;
  srv->B = log2_ceil(V);
  srv->round_limit = std::min<long long>(1ll << 30, 1ll << (64 - srv->B - FIX - 1));
  if (srv->cfg.max_rounds > 0) srv->round_limit = std::min<long long>(srv->round_limit, srv->cfg.max_rounds);
  // keys stay below round_limit * 2^20, so (key + 2^20) << B < 2^64
  srv->max_rounds = (int)std::min<long long>(QCAP, srv->round_limit / 2 - 1);
  if (srv->max_rounds < 1) {
    delete srv;
    ldd_set_error("max_rounds must be at least 4");
    return LDD_ERR_INVALID_ARG;
  }
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
  if (vrange(req->n) > srv->vcap) {
    ldd_set_error("request of %d vertices exceeds the arena (%lld vertices)", req->n, srv->vcap);
    return LDD_ERR_BUDGET;
  }
  Request* r = new Request();
  r->q = *req;
  r->t_submit = now_s();
  if (req->n > 0) {  // admission waits for the work the caller's stream has queued so far
    r->ready = get_event(srv);
    if (!r->ready || hipEventRecord(r->ready, (hipStream_t)req->hip_stream) != hipSuccess) {
      if (r->ready) put_event(srv, r->ready);
      delete r;
      ldd_set_error("recording the request's ready event failed: %s", hipGetErrorString(hipGetLastError()));
      return LDD_ERR_HIP;
    }
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->fatal != LDD_OK || srv->stop) {
      if (r->ready) put_event(srv, r->ready);
      delete r;
      ldd_set_error("server is not running: %s", srv->fatal_msg);
      return srv->fatal != LDD_OK ? srv->fatal : LDD_ERR_INVALID_ARG;
    }
    r->ticket = srv->next_ticket++;
    srv->all[r->ticket] = r;
    if (req->n == 0) {  // nothing to decompose
      r->status = LDD_OK;
      r->state = RQ_DONE;
      r->R = 0;
      r->t_admit = r->t_done = now_s();
    } else {
      srv->queue.push_back(r);
    }
  }
  srv->cv_work.notify_all();
  *ticket = r->ticket;
  return LDD_OK;
}

static ldd_status collect(ldd_server* srv, std::map<uint64_t, Request*>::iterator it, ldd_result* out) {
  Request* r = it->second;
  fill_result(srv, r, out);
  srv->all.erase(it);
  if (r->ready) put_event(srv, r->ready);
  delete r;
  if (out->status == LDD_ERR_INVALID_ARG) ldd_set_error("invalid request (row offsets, shifts or column ids)");
  else if (out->status == LDD_ERR_OVERFLOW) ldd_set_error("request needs more than %d rounds", srv->max_rounds);
  else if (out->status == LDD_ERR_CANCELLED) ldd_set_error("request cancelled");
  else if (out->status != LDD_OK && srv->fatal != LDD_OK) ldd_set_error("server failed: %s", srv->fatal_msg);
  return out->status;
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
  if (it->second->state != RQ_DONE) return LDD_ERR_PENDING;
  return collect(srv, it, out);
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
  return collect(srv, it, out);
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
  out->arena_arcs = 0;  // arcs stay in the callers' buffers
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
  if (srv->fin_stream) (void)hipStreamSynchronize(srv->fin_stream);
  for (void* p : {srv->P, srv->qv0, srv->qv1, srv->qa0, srv->qa1, srv->wake_ord,
                  srv->wake_tab, srv->cnt, srv->cur, srv->slots, srv->st, srv->qcnt, srv->lr_part, srv->lb,
                  srv->ex_part, srv->ctrl, srv->adm_max, srv->adm_err, srv->cut_acc, srv->sst,
                  srv->s_cnt, srv->s_lr, srv->stamp, srv->adm_hub, srv->hbits, srv->lcnt})
    if (p) (void)hipFree(p);
  if (srv->rep) (void)hipHostFree(srv->rep);
  if (srv->s_end) (void)hipHostFree(srv->s_end);
  if (srv->graph) (void)hipGraphExecDestroy(srv->graph);
  for (auto& e : srv->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : srv->ev_pool) (void)hipEventDestroy(e);
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  if (srv->fin_stream) (void)hipStreamDestroy(srv->fin_stream);
  if (srv->fin_dep) (void)hipEventDestroy(srv->fin_dep);
  if (srv->fin_done) (void)hipEventDestroy(srv->fin_done);
  for (auto& kv : srv->all) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  delete srv;
  return fatal;
}
