// Round kernels of the exponential-shift low-diameter decomposition (gfx950).
//
// The search of Sec. 5 runs one integer distance ("round") per step.  Step k reads the state
// left by step k-1 (device memory, double-buffered by parity), so the host can enqueue steps
// without waiting for them; a step whose state says "done" returns at once.  Every block
// derives the same next state from the same counters, so no grid-wide agreement is needed
// inside a step.  The same step function also runs inside one persistent kernel with grid
// barriers between steps.
//
// Step kinds
//   round r, top-down   wake bucket r; every arc of F_{r-1} offers P(u) + unit to its far end
//   round r, bottom-up  wake bucket r; every vertex not settled before r pulls the best offer
//                       of its neighbours in F_{r-1}, stopping at the lower bound L_r
//   tail sweep          once few vertices remain, all remaining delayed source arcs are added
//                       at once and offers are relaxed until nothing changes (the labels are
//                       the unique fixpoint of P(v) = min(own arc, min_w P(w) + unit), so
//                       relaxing in any order reaches the same, exact result)
//
// Frontier appends are staged per block in LDS and reserved in the global queue with one
// 64-bit atomic (count << 32 | arcs) per flush, so the queue stays contiguous with a running
// arc prefix that the next top-down step splits evenly over the grid.
#include "ldd_device.h"
#include "ldd_kernels.h"

namespace ldd {

constexpr int NW = RT / WAVE;

struct AppendBuf {
  int vert[ABUF];
  unsigned off[ABUF];  // exclusive arc prefix inside the buffer
  unsigned wave_cnt[NW];
  unsigned wave_arcs[NW];
  unsigned n;
  unsigned arcs;
  u64 base;
  int wpar;  // queue buffer the step writes
};

// the tail seed scans SEED_SCAN vertices per thread per window and lists the unsettled ones (as
// 16-bit offsets in the window)
constexpr int SEED_SCAN = 8;
constexpr int SLIST = SEED_SCAN * RT;
static_assert(SLIST <= 65536, "window offsets fit 16 bits");

struct StepShared {
  RoundState S;
  u64 lr;
  unsigned start;
  unsigned nlist;   // tail seed: vertices listed in the current window
  u64 red[NW];
  // top-down window: RT+1 queue entries (arc prefix, first arc in col_idx, offer)
  unsigned w_pre[RT + 1];
  int w_first[RT + 1];
  u64 w_offer[RT + 1];
};

__device__ __forceinline__ u64* qcounter(const RoundCtx& c, int k) { return c.qcnt + (size_t)(k % 3) * 16; }

// Copy the LDS buffer to the global queue of step k behind one reservation.
__device__ __forceinline__ void block_flush(AppendBuf& ab, const RoundCtx& c, int k) {
  __syncthreads();
  const unsigned cnt = ab.n, arcs = ab.arcs;
  if (cnt == 0) return;
  if (threadIdx.x == 0) ab.base = atomic_add_u64(qcounter(c, k), ((u64)cnt << 32) | arcs);
  __syncthreads();
  const u64 base = ab.base;
  const unsigned b_cnt = (unsigned)(base >> 32), b_arcs = (unsigned)base;
  int* qv = c.qv[ab.wpar];
  unsigned* qa = c.qa[ab.wpar];
  for (unsigned i = threadIdx.x; i < cnt; i += RT) {
    const unsigned idx = b_cnt + i;
    if (idx < (unsigned)c.n) {
      qv[idx] = ab.vert[i];
      qa[idx] = b_arcs + ab.off[i];
    } else {
      atomic_or_u32(&c.ctrl->err, ERR_QUEUE);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ab.n = 0;
    ab.arcs = 0;
  }
  __syncthreads();
}

// Block-wide append of one tile: ballot and wave scans give each appending thread its slot
// and arc offset; wave totals are combined through LDS.  Called by every thread of the block.
__device__ __forceinline__ void block_append(AppendBuf& ab, bool want, int v, unsigned deg, const RoundCtx& c, int k) {
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  const u64 mask = __ballot(want);
  const unsigned incl = wave_incl_scan(want ? deg : 0u);
  if (lane == WAVE - 1) {
    ab.wave_cnt[wid] = (unsigned)__popcll(mask);
    ab.wave_arcs[wid] = incl;
  }
  __syncthreads();
  unsigned wc = 0, wa = 0, tc = 0, ta = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const unsigned a = ab.wave_cnt[w], b = ab.wave_arcs[w];
    if (w < (int)wid) {
      wc += a;
      wa += b;
    }
    tc += a;
    ta += b;
  }
  if (tc == 0) {
    __syncthreads();
    return;
  }
  if (ab.n + tc > (unsigned)ABUF) block_flush(ab, c, k);
  const unsigned fill = ab.n, fill_arcs = ab.arcs;
  if (want) {
    const unsigned idx = fill + wc + rank_below(mask);
    ab.vert[idx] = v;
    ab.off[idx] = fill_arcs + wa + incl - deg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ab.n = fill + tc;
    ab.arcs = fill_arcs + ta;
  }
  __syncthreads();
}

__device__ __forceinline__ u64 block_min_u64(u64 v, StepShared& sh) {
  v = wave_min_u64(v);
  const unsigned wid = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) sh.red[wid] = v;
  __syncthreads();
  u64 m = INF;
#pragma unroll
  for (int w = 0; w < NW; ++w) m = sh.red[w] < m ? sh.red[w] : m;
  __syncthreads();
  return m;
}

__device__ __forceinline__ unsigned degree(const RoundCtx& c, int v) {
  return (unsigned)(c.row_ptr[v + 1] - c.row_ptr[v]);
}

__device__ __forceinline__ u64 own_offer(const RoundCtx& c, int v) {
  return ((c.delta - (u64)c.shift[v]) << c.B) | (u64)v;
}

// ---- round r: wake bucket r (the delayed source arcs of length in [r, r+1) units) ----------
// With the q-layout, round r's wakers are the vertices of bucket q = D - r whose shift's
// fractional part is <= that of Delta, and those of bucket D - r - 1 whose fractional part
// is larger; the two buckets are adjacent in wake_ord.
__device__ __forceinline__ void phase_wake(const RoundCtx& c, int r, int k, AppendBuf& ab, u64& wmin) {
  constexpr u64 FMASK = ((u64)1 << FIX) - 1;
  int lo, mid, hi;
  const int D = (int)(c.delta >> FIX);
  const u64 dfrac = c.delta & FMASK;
  if (c.wake_q) {
    const int qa = D - r;  // >= 0 for every round r < R
    lo = c.wake_off[qa > 0 ? qa - 1 : 0];
    mid = c.wake_off[qa];
    hi = c.wake_off[qa + 1];
  } else {
    lo = mid = c.wake_off[r];
    hi = c.wake_off[r + 1];
  }
  const int cnt = hi - lo;
  for (long long base = (long long)blockIdx.x * RT; base < cnt; base += (long long)gridDim.x * RT) {
    const long long i = base + threadIdx.x;
    bool want = false;
    int v = 0;
    unsigned deg = 0;
    if (i < cnt) {
      v = c.wake_ord[lo + i];
      const u64 sv = (u64)c.shift[v];
      // in bucket D - r: wakes now iff frac <= dfrac; in bucket D - r - 1: iff frac > dfrac
      const bool wakes = !c.wake_q || ((lo + i >= mid) ? (sv & FMASK) <= dfrac : (sv & FMASK) > dfrac);
      const u64 self = ((c.delta - sv) << c.B) | (u64)v;
      if (wakes && c.P[v] > self) {
        const u64 old = atomic_min_u64(&c.P[v], self);
        if (old > self) {
          wmin = self < wmin ? self : wmin;
          if (old == INF) {
            want = true;
            deg = degree(c, v);
          }
        }
      }
    }
    block_append(ab, want, v, deg, c, k);
  }
}

// ---- top-down: the af arcs of queue (qv, qa, nf entries) split evenly over the grid ---------
// Each block walks its arc range in tiles of RT arcs.  The RT+1 queue entries that can touch
// a tile are staged in LDS (arc prefix, first arc in col_idx, offer); each thread finds its
// arc's entry by binary search.  Entries have degree >= 1, so a tile whose first arc lies in
// entry e only touches entries e .. e+RT-1.
// TAIL = false: round step; an arc appends its far end if it is reached for the first time.
// TAIL = true: tail sweep `sweep`; an arc appends its far end whenever it lowered the label
// and the far end is not queued for the next sweep yet.
template <bool TAIL>
__device__ __forceinline__ void phase_top_down(const RoundCtx& c, int k, const int* qv, const unsigned* qa, unsigned nf, unsigned af,
                               AppendBuf& ab, StepShared& sh, u64& wmin, unsigned sweep) {
  unsigned* w_pre = sh.w_pre;
  int* w_first = sh.w_first;
  u64* w_offer = sh.w_offer;
  const u64 unit = (u64)1 << (FIX + c.B);
  const unsigned G = gridDim.x;
  const unsigned a_begin = (unsigned)(((u64)af * blockIdx.x) / G);
  const unsigned a_end = (unsigned)(((u64)af * (blockIdx.x + 1)) / G);
  if (a_begin >= a_end) return;
  if (threadIdx.x < WAVE) {  // last entry with qa <= a_begin
    const unsigned e = wave_search_le(qa, nf, a_begin);
    if (threadIdx.x == 0) sh.start = e;
  }
  __syncthreads();
  unsigned ent = sh.start;
  for (unsigned tile = a_begin; tile < a_end; tile += RT) {
    for (int kk = threadIdx.x; kk <= RT; kk += RT) {
      const unsigned e = ent + kk;
      if (e < nf) {
        const int u = qv[e];
        w_pre[kk] = qa[e];
        const bool ok = (unsigned)u < (unsigned)c.n;
        w_first[kk] = ok ? c.row_ptr[u] : 0;
        const u64 pu = ok ? load_u64_relaxed(&c.P[u]) : INF;
        w_offer[kk] = pu == INF ? INF : pu + unit;
      } else {
        w_pre[kk] = af;
        w_first[kk] = 0;
        w_offer[kk] = INF;
      }
    }
    __syncthreads();
    const unsigned a = tile + threadIdx.x;
    bool want = false;
    int w = 0;
    unsigned deg = 0;
    if (a < a_end) {
      int lo = 0, hi = RT;  // last kk in [0, RT) with w_pre[kk] <= a
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= a) lo = mid;
        else hi = mid;
      }
      const u64 offer = w_offer[lo];
      const unsigned j = a - w_pre[lo];
      const long long arc = (long long)w_first[lo] + j;
      // j < degree and arc < nnz hold for a symmetric CSR; checked so that malformed input
      // cannot cause an out-of-range read
      const bool in_range = j < w_pre[lo + 1] - w_pre[lo] && arc < c.nnz && offer != INF;
      w = in_range ? c.col[arc] : -1;
      if ((unsigned)w < (unsigned)c.n) {
        if (c.P[w] > offer) {
          const u64 old = atomic_min_u64(&c.P[w], offer);
          if (old > offer) {
            if (TAIL) {
              const unsigned tag = c.stamp_base + sweep + 1;
              if (__hip_atomic_fetch_max(&c.stamp[w], tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tag) {
                want = true;
                deg = degree(c, w);
              }
            } else {
              wmin = offer < wmin ? offer : wmin;
              if (old == INF) {
                want = true;
                deg = degree(c, w);
              }
            }
          }
        }
      } else if (in_range) {
        atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
      }
    }
    block_append(ab, want, w, deg, c, k);
    // the entry holding the next tile's first arc is one of ent .. ent+RT (all staged)
    const unsigned next = tile + RT;
    __syncthreads();
    if (threadIdx.x == 0) {
      int lo = 0, hi = RT + 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= next) lo = mid;
        else hi = mid;
      }
      sh.start = ent + lo;
    }
    __syncthreads();
    ent = sh.start;
  }
}

// ---- pull: bottom-up rounds and the tail seed -------------------------------------------
// Bottom-up round r: every vertex not settled before r pulls the best offer of its neighbours
// in F_{r-1} (a neighbour u is in F_{r-1} iff its label lies in [base(r-1), base(r))), stopping
// as soon as the offer reaches L_r, the smallest offer F_{r-1} makes.
// Tail seed (SEED): every vertex not settled before round r takes the best of its own arc and
// the offers of its neighbours in F_{r-1} (the only settled vertices whose offers have not been
// propagated yet); the sweeps then relax to the fixpoint.
// A thread scans its vertex's row for up to PULL_CAP arcs.  Rows still undecided after that
// are finished by their whole wave, one at a time, 64 arcs per pass with a wave minimum and the
// same stop at L_r: a high-degree vertex no longer holds its wave for a serial scan of its row.
constexpr int PULL_CAP = 16;

// A pulled vertex v whose best offer is below its label: the label drops (atomic minimum);
// bottom-up queues v if it was not reached before, the seed if it is not queued yet.
template <bool SEED>
__device__ __forceinline__ void pull_update(const RoundCtx& c, int v, u64 best, int degree, u64& wmin, bool& want,
                                            unsigned& deg) {
  if (SEED) {
    atomic_min_u64(&c.P[v], best);
    const unsigned tag = c.stamp_base + 1;  // the seed is sweep 0
    want = __hip_atomic_fetch_max(&c.stamp[v], tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < tag;
    deg = (unsigned)degree;
  } else {
    const u64 old = atomic_min_u64(&c.P[v], best);
    if (old > best) {
      wmin = best < wmin ? best : wmin;
      if (old == INF) {
        want = true;
        deg = (unsigned)degree;
      }
    }
  }
}

// The rows the lanes in `rows` left undecided, each finished by the whole wave in turn: 64 arcs
// per pass, a wave minimum, the stop at L_r.  A listed lane's next arc, row end and best offer
// so far are in the step's LDS windows at its thread index (free during a pull); its best offer
// comes back there.  Out of line: it is the rare path, and inlined it costs the common path
// registers.  Returns the arcs read (in lane 0).
__device__ __attribute__((noinline)) unsigned pull_rows_wave(const RoundCtx& c, u64 rows, unsigned* w_a, int* w_a1,
                                                             u64* w_best, u64 Lr, int r) {
  unsigned examined = 0;
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const unsigned lane = lane_id(), wave0 = threadIdx.x - lane;
  for (; rows; rows &= rows - 1) {
    const int src = __ffsll((long long)rows) - 1;
    int ra = (int)w_a[wave0 + src];
    const int ra1 = w_a1[wave0 + src];
    u64 rb = w_best[wave0 + src];
    while (ra < ra1 && rb > Lr) {  // uniform over the wave
      const int ai = ra + (int)lane;
      u64 mine = INF;
      bool bad = false;
      if (ai < ra1) {
        const int u = c.col[ai];
        bad = (unsigned)u >= (unsigned)c.n;
        if (!bad) {
          const u64 pu = load_u64_relaxed(&c.P[u]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF) mine = pu + unit;
        }
      }
      if (lane == 0) examined += (unsigned)min(ra1 - ra, WAVE);
      if (__ballot(bad)) {
        if (lane == 0) atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
        break;
      }
      const u64 wm = wave_min_u64(mine);
      rb = wm < rb ? wm : rb;
      ra += WAVE;
    }
    if ((int)lane == src) w_best[wave0 + src] = rb;
  }
  return examined;
}

template <bool SEED>
__device__ __forceinline__ void phase_pull(const RoundCtx& c, int r, int k, u64 Lr, AppendBuf& ab, StepShared& sh,
                                           u64& wmin, u64& examined_total) {
  unsigned examined = 0;
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const long long stride = (long long)gridDim.x * RT;
  // each tile's labels are loaded during the tile before, so that the load is in flight across
  // the append's barriers (a label read early can only be higher than the current one: labels
  // only drop, so the worst case is a pull that finds nothing to lower)
  u64 pv_next = (long long)blockIdx.x * RT + threadIdx.x < c.n ? c.P[blockIdx.x * RT + threadIdx.x] : 0;
  for (long long base = (long long)blockIdx.x * RT; base < c.n; base += stride) {
    const long long vi = base + threadIdx.x;
    const int v = (int)vi;
    bool want = false, defer = false;
    unsigned deg = 0;
    const u64 pv = pv_next;
    if (vi < c.n) {
      if (pv >= base_r && (SEED || pv > Lr)) {
        const int a0 = c.row_ptr[v], a1 = c.row_ptr[v + 1];
        if (!SEED || a1 > a0) {
          u64 best = SEED ? own_offer(c, v) : pv;
          int a = a0;
          bool bad = false;
          const int a_cap = a1 - a0 > PULL_CAP ? a0 + PULL_CAP : a1;
          for (; a < a_cap && best > Lr; ++a) {
            ++examined;
            const int u = c.col[a];
            if ((unsigned)u >= (unsigned)c.n) {
              atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
              bad = true;
              break;
            }
            const u64 pu = load_u64_relaxed(&c.P[u]);
            if ((pu >> (FIX + B)) == prev_round && pu != INF && pu + unit < best) best = pu + unit;
          }
          if (!bad && a < a1 && best > Lr) {  // long row, undecided: the wave finishes it below
            defer = true;
            sh.w_pre[threadIdx.x] = (unsigned)a;
            sh.w_first[threadIdx.x] = a1;
            sh.w_offer[threadIdx.x] = best;
          } else if (best < pv) {
            pull_update<SEED>(c, v, best, a1 - a0, wmin, want, deg);
          }
        }
      }
    }
    const u64 m = __ballot(defer);
    if (m) {
      examined += pull_rows_wave(c, m, sh.w_pre, sh.w_first, sh.w_offer, Lr, r);
      if (defer) {
        const u64 best = sh.w_offer[threadIdx.x];
        if (best < c.P[v]) pull_update<SEED>(c, v, best, c.row_ptr[v + 1] - c.row_ptr[v], wmin, want, deg);
      }
    }
    pv_next = vi + stride < c.n ? c.P[vi + stride] : 0;
    block_append(ab, want, v, deg, c, k);
  }
  examined_total += examined;
}

// ---- tail seed, listed -------------------------------------------------------------------
// Every vertex with arcs not settled before round r takes the best of its own label (whatever its
// wake round) and the offers of its neighbours in F_{r-1}.  The seed step writes nothing else, so
// a vertex's label is INF until its own thread writes it.  Each block takes a contiguous vertex
// range and walks it in windows of SLIST vertices: a coalesced scan of labels and row offsets
// lists the window's unsettled vertices with arcs in LDS, then the listed vertices pull, RT at a
// time (rows undecided after PULL_CAP arcs finished by their wave, as in the bottom-up pull).
// Settled and isolated vertices cost one coalesced label read (and, unsettled, the row offsets).
__device__ __forceinline__ void phase_seed(const RoundCtx& c, int r, int k, u64 Lr, AppendBuf& ab, StepShared& sh,
                                           unsigned short* list, u64& wmin, u64& examined_total) {
  unsigned examined = 0;
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const long long v0 = (long long)c.n * blockIdx.x / gridDim.x, v1 = (long long)c.n * (blockIdx.x + 1) / gridDim.x;
  for (long long w0 = v0; w0 < v1; w0 += SLIST) {
    __syncthreads();  // every thread has read the previous window's list count
    if (threadIdx.x == 0) sh.nlist = 0;
    __syncthreads();
    u64 pv[SEED_SCAN];
#pragma unroll
    for (int j = 0; j < SEED_SCAN; ++j) {
      const long long v = w0 + (long long)j * RT + threadIdx.x;
      pv[j] = v < v1 ? c.P[v] : 0;
    }
#pragma unroll
    for (int j = 0; j < SEED_SCAN; ++j) {
      const long long v = w0 + (long long)j * RT + threadIdx.x;
      if (v < v1 && pv[j] >= base_r && c.row_ptr[v + 1] > c.row_ptr[v])
        list[atomicAdd(&sh.nlist, 1u)] = (unsigned short)(v - w0);
    }
    __syncthreads();
    const unsigned cnt = sh.nlist;
    for (unsigned c0 = 0; c0 < cnt; c0 += RT) {
      const unsigned i = c0 + threadIdx.x;
      bool want = false, defer = false;
      int v = 0;
      unsigned deg = 0;
      if (i < cnt) {
        v = (int)(w0 + list[i]);
        const int a0 = c.row_ptr[v], a1 = c.row_ptr[v + 1];
        u64 best = own_offer(c, v);
        int a = a0;
        bool bad = false;
        const int a_cap = a1 - a0 > PULL_CAP ? a0 + PULL_CAP : a1;
        for (; a < a_cap && best > Lr; ++a) {
          ++examined;
          const int u = c.col[a];
          if ((unsigned)u >= (unsigned)c.n) {
            atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
            bad = true;
            break;
          }
          const u64 pu = load_u64_relaxed(&c.P[u]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF && pu + unit < best) best = pu + unit;
        }
        if (!bad && a < a1 && best > Lr) {  // long row, undecided: the wave finishes it below
          defer = true;
          sh.w_pre[threadIdx.x] = (unsigned)a;
          sh.w_first[threadIdx.x] = a1;
          sh.w_offer[threadIdx.x] = best;
        } else {
          pull_update<true>(c, v, best, a1 - a0, wmin, want, deg);
        }
      }
      const u64 m = __ballot(defer);
      if (m) {
        examined += pull_rows_wave(c, m, sh.w_pre, sh.w_first, sh.w_offer, Lr, r);
        if (defer) pull_update<true>(c, v, sh.w_offer[threadIdx.x], c.row_ptr[v + 1] - c.row_ptr[v], wmin, want, deg);
      }
      block_append(ab, want, v, deg, c, k);
    }
  }
  examined_total += examined;
}

// Direction of the next round.  Top-down touches every arc of the frontier (random accesses);
// bottom-up reads every label once (sequential) plus at most the arcs of unsettled vertices,
// usually far fewer thanks to the early exit.  Bottom-up is taken once the frontier's arcs
// outweigh that work, and kept until the frontier is small again and top-down is cheaper.
__device__ __forceinline__ int choose_dir(const RoundCtx& c, int dir, u64 nf, u64 af, u64 unsettled_arcs) {
  if (c.dir_policy == DIR_TD) return DIR_TD;
  if (c.dir_policy == DIR_BU) return DIR_BU;
  const bool bu_better = af * (u64)c.td_to_bu > unsettled_arcs + (u64)c.n / 4;
  if (dir == DIR_TD) return bu_better ? DIR_BU : DIR_TD;
  return (bu_better || nf * (u64)c.bu_to_td >= (u64)c.n) ? DIR_BU : DIR_TD;
}

// State of step k from the state of step k-1 and what step k-1 appended.
// The state is read with coherent loads: in the persistent kernel it was written by another
// block during the previous step.
__device__ RoundState load_state(const RoundState* p) {
  RoundState s;
#define LDD_LOAD(f) s.f = __hip_atomic_load(&p->f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  LDD_STATE_FIELDS(LDD_LOAD)
#undef LDD_LOAD
  return s;
}

template <int SCOPE>
__device__ void store_state(RoundState* p, const RoundState& s) {
#define LDD_STORE(f) __hip_atomic_store(&p->f, s.f, __ATOMIC_RELAXED, SCOPE);
  LDD_STATE_FIELDS(LDD_STORE)
#undef LDD_STORE
}

// Round r wakes buckets D - r and D - r - 1 (bucket 0 alone when r = D).
__device__ __forceinline__ bool needs_place(const RoundCtx& c, int r, long long placed_lo) {
  const long long D = (long long)(c.delta >> FIX);
  const long long need = D - r - 1 > 0 ? D - r - 1 : 0;
  return c.wake_q && need < placed_lo;
}

// ---- placement: wake buckets [max(0, placed_lo - ABUF), placed_lo) ------------------------
// Same slots as the preparation would have given them: per preparation block pb, a cursor per
// bucket starts at the bucket's offset plus the counts of earlier blocks (mat); the block's
// vertices of those buckets are scattered through the cursors (kept in the append buffer's LDS).
__device__ __forceinline__ void phase_place(const RoundCtx& c, long long placed_lo, AppendBuf& ab) {
  const int hi_q = (int)placed_lo, lo_q = hi_q > ABUF ? hi_q - ABUF : 0;
  const int G = c.prep_blocks;
  int* cur = ab.vert;
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  for (int pb = blockIdx.x; pb < G; pb += gridDim.x) {
    __syncthreads();
    const int qm = min(c.qmax[pb], hi_q - 1);
    for (int q = lo_q + (int)threadIdx.x; q <= qm; q += RT)
      cur[q - lo_q] = c.wake_off[q] + (int)c.mat[(size_t)q * G + pb];
    __syncthreads();
    const long long lo = (long long)c.n * pb / G, hi = (long long)c.n * (pb + 1) / G;
    for (long long base = lo + 256ll * wid; base < hi; base += 256ll * NW) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long v = base + 64 * j + lane;
        if (v < hi) {
          const long long q = (long long)((u64)c.shift[v] >> FIX);
          if (q >= lo_q && q <= qm && c.row_ptr[v + 1] > c.row_ptr[v])
            c.wake_ord[atomicAdd(&cur[q - lo_q], 1)] = (int)v;
        }
      }
    }
  }
}

__device__ __forceinline__ RoundState next_state(const RoundCtx& c, int k) {
  const RoundState P = load_state(&c.st[(k - 1) & 1]);
  const u64 out = load_u64_relaxed(qcounter(c, k - 1));
  RoundState S = P;
  S.seq = k;
  if (P.mode == MODE_DONE) return S;
  if (P.mode == MODE_PLACE) {
    // step k-1 placed buckets [lo, placed_lo) and queued nothing: round P.round runs now, on
    // the queue step k-2 wrote (hence the parity flip), unless it needs still lower buckets
    S.placed_lo = P.placed_lo > ABUF ? P.placed_lo - ABUF : 0;
    S.flip = P.flip ^ 1;
    S.mode = needs_place(c, (int)S.round, S.placed_lo) ? MODE_PLACE : MODE_ROUNDS;
    return S;
  }
  const unsigned nf = min((unsigned)(out >> 32), (unsigned)c.n), af = (unsigned)out;
  if (P.mode == MODE_ROUNDS) {
    int next_r;
    if (k > 1) {
      S.settled += nf;
      S.unsettled_arcs -= af;
      S.rounds += 1;
      if (P.prev >> 32) {
        S.td_rounds += P.dir == DIR_TD;
        S.bu_rounds += P.dir == DIR_BU;
      }
      S.max_frontier = (long long)nf > S.max_frontier ? (long long)nf : S.max_frontier;
      next_r = nf ? (int)P.round + 1 : c.next_ne[P.round + 1];
    } else {
      next_r = c.next_ne[0];
    }
    S.prev = (long long)out;
    const u64 left = c.n_active - (u64)S.settled;
    if ((u64)S.settled >= c.n_active) {
      S.mode = MODE_DONE;
    } else if (next_r >= c.R) {
      S.mode = MODE_DONE;
      if (blockIdx.x == 0) atomic_or_u32(&c.ctrl->err, ERR_WATCHDOG);
    } else if (c.tail_den > 0 && left * (u64)c.tail_den <= c.n_active && c.R - next_r > c.tail_min_left) {
      S.mode = MODE_TAIL;
      S.round = 0;
      S.tail_round = next_r;
    } else {
      S.round = next_r;
      S.dir = nf ? choose_dir(c, (int)P.dir, nf, af, (u64)S.unsettled_arcs) : P.dir;
      if (needs_place(c, next_r, S.placed_lo)) S.mode = MODE_PLACE;
    }
  } else {  // MODE_TAIL: step k-1 ran sweep P.round and queued `out`
    S.tail_iters += 1;
    S.round = P.round + 1;
    S.prev = (long long)out;
    if (nf == 0) S.mode = MODE_DONE;
  }
  return S;
}

// per-block statistics slot: no atomics (each block owns its slot for the whole call)
__device__ __forceinline__ void add_examined(const RoundCtx& c, u64 examined, StepShared& sh) {
  examined = wave_sum_u64(examined);
  __syncthreads();
  if (lane_id() == 0) sh.red[threadIdx.x / WAVE] = examined;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 t = 0;
    for (int w = 0; w < NW; ++w) t += sh.red[w];
    if (t) c.ex_part[blockIdx.x] += t;
  }
}

// One step; returns the mode it ran in (MODE_DONE: nothing was left to do).
__device__ __forceinline__ int round_step(const RoundCtx& c, int k, AppendBuf& ab, StepShared& sh,
                                          unsigned short* slist) {
  if (threadIdx.x == 0) {
    // Once a step has written "done" into either slot no step writes a slot again, so later
    // steps only need the two mode words to leave.
    const bool done = __hip_atomic_load(&c.st[0].mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == MODE_DONE ||
                      __hip_atomic_load(&c.st[1].mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == MODE_DONE;
    if (done) {
      sh.S.mode = MODE_DONE;
      sh.S.seq = -1;
    } else {
      sh.S = next_state(c, k);
    }
    ab.n = 0;
    ab.arcs = 0;
  }
  __syncthreads();
  // the fields the step uses, as wave-uniform scalars (the rest of the state stays in LDS)
  const int mode = __builtin_amdgcn_readfirstlane((int)sh.S.mode);
  if (__builtin_amdgcn_readfirstlane((int)(sh.S.seq < 0))) return MODE_DONE;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_state<__HIP_MEMORY_SCOPE_AGENT>(&c.st[k & 1], sh.S);
    __hip_atomic_store(qcounter(c, k + 1), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the host stops enqueueing steps once it reads the report; written once per
    // decomposition, since a store to host memory delays the completion of the kernel that
    // makes it.  Likewise the hint that the tail has started (few steps are left), once.
    if (c.report && mode == MODE_TAIL && sh.S.round == 0)
      __hip_atomic_store(&c.report->tail_hint, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (c.report && mode == MODE_DONE) {
      Report* r = c.report;
      r->st = sh.S;
      r->delta = c.delta;
      r->n_active = c.n_active;
      r->err = __hip_atomic_load(&c.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      r->setup = SETUP_OK;
      __threadfence_system();  // the fields before the flag
      __hip_atomic_store(&r->ready, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  if (mode == MODE_DONE) return MODE_DONE;
  if (mode == MODE_PLACE) {
    phase_place(c, sh.S.placed_lo, ab);
    return MODE_PLACE;
  }
  const int round = __builtin_amdgcn_readfirstlane((int)sh.S.round);
  const int dir = __builtin_amdgcn_readfirstlane((int)sh.S.dir);
  const int rpar = (int)((k - 1 + __builtin_amdgcn_readfirstlane((int)sh.S.flip)) & 1), wpar = rpar ^ 1;
  const u64 prev = (u64)sh.S.prev;
  if (threadIdx.x == 0) ab.wpar = wpar;
  const unsigned nf = __builtin_amdgcn_readfirstlane(min((unsigned)(prev >> 32), (unsigned)c.n));
  const unsigned af = __builtin_amdgcn_readfirstlane((unsigned)prev);
  const int* qv = c.qv[rpar];
  const unsigned* qa = c.qa[rpar];
  u64 wmin = INF, examined = 0;
  const bool need_lr = nf && ((mode == MODE_ROUNDS && dir == DIR_BU) || (mode == MODE_TAIL && round == 0));
  if (need_lr) {
    // L_r: the smallest offer of F_{r-1}, from the per-block minima the previous step left
    u64 m = INF;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += RT) {
      const u64 x = load_u64_relaxed(&c.lr_part[(size_t)rpar * gridDim.x + b]);
      m = x < m ? x : m;
    }
    m = block_min_u64(m, sh);
    if (threadIdx.x == 0) sh.lr = m == INF ? INF : m + ((u64)1 << (FIX + c.B));
    __syncthreads();
  }
  if (mode == MODE_ROUNDS) {
    const int r = round;
    phase_wake(c, r, k, ab, wmin);
    if (nf) {
      if (dir == DIR_BU) {
        phase_pull<false>(c, r, k, sh.lr, ab, sh, wmin, examined);
      } else {
        phase_top_down<false>(c, k, qv, qa, nf, af, ab, sh, wmin, 0);
        if (blockIdx.x == 0 && threadIdx.x == 0) examined += af;
      }
    }
  } else {
    const unsigned sweep = (unsigned)round;
    if (sweep == 0) {
      phase_seed(c, __builtin_amdgcn_readfirstlane((int)sh.S.tail_round), k, nf ? sh.lr : INF, ab, sh, slist, wmin,
                 examined);
    } else if (nf) {
      phase_top_down<true>(c, k, qv, qa, nf, af, ab, sh, wmin, sweep);
      if (blockIdx.x == 0 && threadIdx.x == 0) examined += af;
    }
  }
  block_flush(ab, c, k);
  const u64 bm = block_min_u64(wmin, sh);
  if (threadIdx.x == 0) c.lr_part[(size_t)wpar * gridDim.x + blockIdx.x] = bm;
  add_examined(c, examined, sh);
  return mode;
}

// (RT, 8): eight waves per SIMD, i.e. two 1024-thread blocks per CU, which caps VGPRs at 64
__global__ __launch_bounds__(RT, 8) void k_round_step_lb(const LaunchBlock* __restrict__ lb, int j) {
  __shared__ AppendBuf ab;
  __shared__ StepShared sh;
  __shared__ unsigned short slist[SLIST];
  round_step(lb->c, (int)(lb->kbase + j), ab, sh, slist);
}

__global__ void k_advance(LaunchBlock* lb, int C) {
  if (threadIdx.x == 0 && blockIdx.x == 0) lb->kbase += C;
}

// All steps in one kernel with grid barriers between them (the grid must be co-resident).
__global__ __launch_bounds__(RT) void k_rounds_persistent(const LaunchBlock* __restrict__ lb) {
  __shared__ AppendBuf ab;
  __shared__ StepShared sh;
  __shared__ unsigned short slist[SLIST];
  const RoundCtx& c = lb->c;
  u64 gen = 0;
  const long long kmax = (long long)c.R + c.n + 2;
  for (int k = 1; k <= kmax; ++k) {
    if (round_step(c, k, ab, sh, slist) == MODE_DONE) break;
    grid_sync(&c.ctrl->bar, gridDim.x, gen, &c.ctrl->err);
    if (__hip_atomic_load(&c.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (ERR_BARRIER | ERR_QUEUE)) break;
  }
}

// =============================================================================================
// Server mode
// =============================================================================================
// The server's arena is the disjoint union of the admitted requests ("slots").  One step is the
// next global round for every slot; each slot is in its own mode (rounds, seed, tail sweeps,
// done) and, in rounds mode, takes its own direction, as next_state and choose_dir decide for
// one graph.  Each slot's frontier is queued in the slot's own vertex range of the queue arrays
// (a vertex is queued at most once per step) behind a per-slot reservation counter
// (count << 32 | arcs), so top-down splits exactly the top-down slots' arcs evenly over the
// grid, and those counters are each slot's frontier statistics for the next step.

constexpr int SABUF = 1792;  // entries of a block's LDS append buffer in server mode
static_assert(SABUF >= RT, "a whole tile's appends fit the buffer");
static_assert(MAX_SLOTS <= 256, "buffered appends keep their slot in one byte");
enum { TD_SKIP = 0, TD_ROUND = 1, TD_SWEEP = 2 };

struct SrvAppend {
  int vert[SABUF];
  u64 loc[SABUF];  // (rank << 32 | arc offset) among the buffered appends of the same slot
  unsigned char slot[SABUF];
  u64 tot[MAX_SLOTS];   // (count << 32 | arcs) buffered per slot
  u64 base[MAX_SLOTS];  // the flush's reservation in each slot's queue
  unsigned wave_cnt[NW];
  unsigned n;
};

struct SrvShared {
  const int* rp[MAX_SLOTS];  // each slot's request: CSR and shifts (local ids)
  const int* col[MAX_SLOTS];
  const long long* shift[MAX_SLOTS];
  u64 off0[MAX_SLOTS];       // delta + r0 * 2^20: a vertex's own arc is off0 - shift
  long long nnz[MAX_SLOTS];
  int td[MAX_SLOTS];    // TD_* of each slot in this step
  int wake[MAX_SLOTS];  // the slot takes part in this round's wake
  int seed[MAX_SLOTS];  // the slot's pull in this step is its tail seed
  int n[MAX_SLOTS];
  long long vbeg[MAX_SLOTS];
  u64 L[MAX_SLOTS];      // each slot's L_r: the smallest offer its F_{r-1} makes
  u64 front[MAX_SLOTS];  // (count << 32 | arcs) of each slot's queue from the previous step
  u64 lr[MAX_SLOTS];     // this block's smallest label written per slot
  long long seg_beg[MAX_SLOTS];  // this round's wake segment of every slot
  int seg_off[MAX_SLOTS + 1];
  long long pull_beg[MAX_SLOTS];  // vertex ranges that pull (bottom-up or seed)
  int pull_off[MAX_SLOTS + 1];
  unsigned td_off[MAX_SLOTS + 1];  // prefix of the top-down slots' frontier arcs
  unsigned start;
  int pslot[RT];  // pull: slot of a thread's row left to its wave
};

// Reserve the buffered appends in their slots' queues of step k and copy them there.
__device__ __forceinline__ void srv_flush(SrvAppend& ab, const RoundCtx& c, int k, const SrvShared& ss) {
  __syncthreads();
  const unsigned cnt = ab.n;
  if (cnt == 0) return;
  if (threadIdx.x < MAX_SLOTS) {
    const u64 t = ab.tot[threadIdx.x];
    ab.base[threadIdx.x] = t ? atomic_add_u64(&c.s_cnt[(k % 3) * MAX_SLOTS + threadIdx.x], t) : 0;
  }
  __syncthreads();
  int* qv = c.qv[k & 1];
  unsigned* qa = c.qa[k & 1];
  for (unsigned i = threadIdx.x; i < cnt; i += RT) {
    const int s = ab.slot[i];
    const u64 b = ab.base[s], x = ab.loc[i];
    const unsigned idx = (unsigned)(b >> 32) + (unsigned)(x >> 32);
    if (idx < (unsigned)ss.n[s]) {
      qv[ss.vbeg[s] + idx] = ab.vert[i];
      qa[ss.vbeg[s] + idx] = (unsigned)b + (unsigned)x;
    } else {
      atomic_or_u32(&c.ctrl->err, ERR_QUEUE);
    }
  }
  __syncthreads();
  if (threadIdx.x < MAX_SLOTS) ab.tot[threadIdx.x] = 0;
  if (threadIdx.x == 0) ab.n = 0;
  __syncthreads();
}

// Block-wide append of one tile (every thread calls it): a buffer index per appending thread
// from ballots, and its rank and arc offset within its slot from a wave-level grouping by slot
// (one LDS atomic per slot present in the wave).
__device__ __forceinline__ void srv_append(SrvAppend& ab, bool want, int v, unsigned deg, int slot, const RoundCtx& c,
                                           int k, const SrvShared& ss) {
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  const u64 mask = __ballot(want);
  if (lane == 0) ab.wave_cnt[wid] = (unsigned)__popcll(mask);
  __syncthreads();
  unsigned wc = 0, tc = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const unsigned a = ab.wave_cnt[w];
    if (w < (int)wid) wc += a;
    tc += a;
  }
  if (tc == 0) {
    __syncthreads();
    return;
  }
  if (ab.n + tc > (unsigned)SABUF) srv_flush(ab, c, k, ss);
  const unsigned fill = ab.n;
  u64 myloc = 0;
  u64 pending = mask;
  while (pending) {  // wave-uniform
    const int leader = (int)__builtin_ctzll(pending);
    const int sl = __shfl(slot, leader, WAVE);
    const bool mine = want && slot == sl;
    const u64 m = __ballot(mine);
    const unsigned d = mine ? deg : 0u;
    const unsigned incl = wave_incl_scan(d);
    const unsigned dtot = __shfl(incl, WAVE - 1, WAVE);
    u64 g = 0;
    if ((int)lane == leader) g = atomicAdd(&ab.tot[sl], ((u64)__popcll(m) << 32) | (u64)dtot);
    g = shfl_u64(g, leader);
    if (mine) myloc = ((u64)((unsigned)(g >> 32) + rank_below(m)) << 32) | (u64)((unsigned)g + incl - d);
    pending &= ~m;
  }
  if (want) {
    const unsigned idx = fill + wc + rank_below(mask);
    ab.vert[idx] = v;
    ab.slot[idx] = (unsigned char)slot;
    ab.loc[idx] = myloc;
  }
  __syncthreads();
  if (threadIdx.x == 0) ab.n = fill + tc;
  __syncthreads();
}

// The smallest label each slot had written in this tile (wave-level grouping by slot).
__device__ __forceinline__ void srv_note_lr(SrvShared& ss, bool wrote, int slot, u64 label) {
  u64 pending = __ballot(wrote);
  while (pending) {  // wave-uniform
    const int leader = (int)__builtin_ctzll(pending);
    const int sl = __shfl(slot, leader, WAVE);
    const bool mine = wrote && slot == sl;
    const u64 m = __ballot(mine);
    const u64 lab = wave_min_u64(mine ? label : INF);
    if ((int)lane_id() == leader) atomicMin(&ss.lr[sl], lab);
    pending &= ~m;
  }
}

__device__ __forceinline__ unsigned srv_degree(const SrvShared& ss, int s, int v) {
  const int lv = v - (int)ss.vbeg[s];
  return (unsigned)(ss.rp[s][lv + 1] - ss.rp[s][lv]);
}

// The request's own arc of arena vertex v: its source-arc length raised by r0 units.
__device__ __forceinline__ u64 srv_own_offer(const RoundCtx& c, const SrvShared& ss, int s, int v) {
  return ((ss.off0[s] - (u64)ss.shift[s][v - ss.vbeg[s]]) << c.B) | (u64)v;
}

// The per-slot prefix sums are taken one wave per WAVE slots; each later wave adds the total of
// the waves before it (one barrier per wave after the first; nothing when one wave holds them all).
template <typename A, typename B>
__device__ __forceinline__ void slot_carry(A* a, B* b) {
  for (int w = 1; w < MAX_SLOTS / WAVE; ++w) {
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= w * WAVE && t < (w + 1) * WAVE) {
      a[t + 1] += a[w * WAVE];
      if (b) b[t + 1] += b[w * WAVE];
    }
  }
}

// Start of step k, round r (one lane per slot): each slot's mode for this step and, in
// rounds mode, its direction from its own frontier; its L_r; the wake, pull and top-down work
// lists.  Block 0 records the slots' state after step k, clears the counters step k+1 fills,
// and reports a slot found done (through mapped host memory).
__device__ __forceinline__ void srv_slot_setup(const RoundCtx& c, int k, int r, SrvShared& ss) {
  static_assert(MAX_SLOTS % WAVE == 0, "slots fill whole waves");
  if (threadIdx.x >= MAX_SLOTS) return;
  const int s = threadIdx.x;
  int td = TD_SKIP, wake = 0, seed = 0, pull_len = 0, n = 0;
  long long pull_beg = 0, vbeg = 0;
  u64 L = INF, front = 0;
  if (s < c.nslots) {
    const SlotInfo sl = c.slots[s];
    ss.rp[s] = sl.rp;
    ss.col[s] = sl.col;
    ss.shift[s] = sl.shift;
    ss.off0[s] = sl.delta + (u64)sl.r0 * ((u64)1 << FIX);
    ss.nnz[s] = sl.nnz;
    const SlotState p = c.sst[((k - 1) & 1) * MAX_SLOTS + s];
    front = c.s_cnt[((k - 1) % 3) * MAX_SLOTS + s];
    const u64 lr = c.s_lr[((k - 1) % 3) * MAX_SLOTS + s];
    const u64 nf = front >> 32, af = front & 0xffffffffull;
    n = sl.n;
    vbeg = sl.vbeg;
    SlotState q = p;
    q.dir = DIR_TD;
    bool report = false;
    if (sl.active && p.mode == SM_ROUNDS) {
      q.settled += (long long)nf;
      q.ua -= (long long)af;
      const long long n_act = c.wake_tab[sl.wbase + sl.R];
      const long long left = n_act - q.settled;
      const long long rho = (long long)r - sl.r0;
      if (left <= 0) {  // every vertex reached: the round that reached the last one has ended
        q.mode = SM_DONE;
        report = true;
      } else if (c.tail_den > 0 && left * c.tail_den <= n_act && sl.R - rho > c.tail_min_left) {
        q.mode = SM_SEED;
        seed = 1;
        pull_len = sl.n;
        pull_beg = sl.vbeg;
      } else {
        wake = 1;
        int dir = DIR_TD;
        if (nf) {
          if (c.dir_policy == DIR_TD || c.dir_policy == DIR_BU) {
            dir = c.dir_policy;
          } else {
            const u64 nn = (u64)sl.n;
            const bool bu_better = af * (u64)c.td_to_bu > (u64)(q.ua > 0 ? q.ua : 0) + nn / 4;
            dir = (p.dir == DIR_BU) ? ((bu_better || nf * (u64)c.bu_to_td >= nn) ? DIR_BU : DIR_TD)
                                    : (bu_better ? DIR_BU : DIR_TD);
          }
        }
        q.dir = dir;
        if (dir == DIR_BU) {
          pull_len = sl.n;
          pull_beg = sl.vbeg;
        } else {
          td = TD_ROUND;
        }
      }
    } else if (sl.active && (p.mode == SM_SEED || p.mode == SM_TAIL)) {
      if (nf == 0) {  // the last sweep lowered nothing: the labels are the fixpoint
        q.mode = SM_DONE;
        report = true;
      } else {
        q.mode = SM_TAIL;
        td = TD_SWEEP;
      }
    }
    L = lr == INF ? INF : lr + ((u64)1 << (FIX + c.B));
    if (blockIdx.x == 0) {
      c.sst[(k & 1) * MAX_SLOTS + s] = q;
      c.s_cnt[((k + 1) % 3) * MAX_SLOTS + s] = 0;
      c.s_lr[((k + 1) % 3) * MAX_SLOTS + s] = INF;
      if (report) __hip_atomic_store(&c.s_end[s].step, (long long)k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
  const unsigned pull_incl = wave_incl_scan((unsigned)pull_len);
  const unsigned td_incl = wave_incl_scan(td != TD_SKIP ? (unsigned)(front & 0xffffffffull) : 0u);
  ss.td[s] = td;
  ss.wake[s] = wake;
  ss.seed[s] = seed;
  ss.n[s] = n;
  ss.vbeg[s] = vbeg;
  ss.L[s] = L;
  ss.front[s] = front;
  ss.lr[s] = INF;
  ss.pull_beg[s] = pull_beg;
  ss.pull_off[s + 1] = (int)pull_incl;
  ss.td_off[s + 1] = td_incl;
  if (s == 0) {
    ss.pull_off[0] = 0;
    ss.td_off[0] = 0;
  }
}

// Wake: for every slot in rounds mode with r0 <= r < r0 + R, the vertices of its local round
// rho = r - r0 take their own arc: the back of shift bucket D - rho - 1 and the front of bucket
// D - rho (D = R - 1), one range of its part of wake_ord.
__device__ __forceinline__ void srv_wake(const RoundCtx& c, int r, int k, SrvAppend& ab, SrvShared& ss) {
  if (threadIdx.x < MAX_SLOTS) {
    const int t = threadIdx.x;
    int len = 0;
    long long beg = 0;
    if (t < c.nslots && ss.wake[t]) {
      const SlotInfo sl = c.slots[t];
      const long long rho = (long long)r - sl.r0;
      if (rho >= 0 && rho < sl.R) {
        const long long q = sl.R - 1 - rho;
        const unsigned hi = (unsigned)c.wake_cur[sl.wbase + q];
        const unsigned lo = q > 0 ? (unsigned)c.wake_cur[sl.wbase + q - 1] : 0u;
        len = (int)(hi - lo);
        beg = sl.vbeg + lo;
      }
    }
    const unsigned incl = wave_incl_scan((unsigned)len);
    ss.seg_beg[t] = beg;
    ss.seg_off[t + 1] = (int)incl;
    if (t == 0) ss.seg_off[0] = 0;
  }
  slot_carry(ss.seg_off, (int*)nullptr);
  __syncthreads();
  const int cnt = ss.seg_off[MAX_SLOTS];
  for (long long base = (long long)blockIdx.x * RT; base < cnt; base += (long long)gridDim.x * RT) {
    const long long i = base + threadIdx.x;
    bool want = false, wrote = false;
    int v = 0, slot = 0;
    unsigned deg = 0;
    u64 self = INF;
    if (i < cnt) {
      int lo = 0, hi = MAX_SLOTS;  // the last slot with seg_off <= i
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ss.seg_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      slot = lo;
      v = c.wake_ord[ss.seg_beg[lo] + (i - ss.seg_off[lo])];
      self = srv_own_offer(c, ss, lo, v);
      if (c.P[v] > self) {
        const u64 old = atomic_min_u64(&c.P[v], self);
        if (old > self) {
          wrote = true;
          if (old == INF) {
            want = true;
            deg = srv_degree(ss, lo, v);
          }
        }
      }
    }
    srv_note_lr(ss, wrote, slot, self);
    srv_append(ab, want, v, deg, slot, c, k, ss);
  }
}

// Top-down over slot s's queue (its frontier from step k-1), slot-local arcs [lo, hi): the
// windowed search of phase_top_down.  Rounds: a far end reached for the first time is queued;
// tail sweep: a far end is queued whenever its label drops (once per step, by its stamp).
__device__ __forceinline__ void srv_td_segment(const RoundCtx& c, int k, SrvAppend& ab, StepShared& sh, SrvShared& ss,
                                               int s, unsigned lo_a, unsigned hi_a) {
  unsigned* w_pre = sh.w_pre;
  int* w_first = sh.w_first;
  u64* w_offer = sh.w_offer;
  const u64 unit = (u64)1 << (FIX + c.B);
  const int* qv = c.qv[(k - 1) & 1] + ss.vbeg[s];
  const unsigned* qa = c.qa[(k - 1) & 1] + ss.vbeg[s];
  const unsigned nf = (unsigned)(ss.front[s] >> 32), af = (unsigned)ss.front[s];
  const bool sweep = ss.td[s] == TD_SWEEP;
  const int* rp = ss.rp[s];
  const int* col = ss.col[s];
  const long long vbeg = ss.vbeg[s], nnz = ss.nnz[s];
  const int n = ss.n[s];
  __syncthreads();
  if (threadIdx.x < WAVE) {  // the last entry with qa <= lo_a
    const unsigned e = wave_search_le(qa, nf, lo_a);
    if (threadIdx.x == 0) ss.start = e;
  }
  __syncthreads();
  unsigned ent = ss.start;
  for (unsigned tile = lo_a; tile < hi_a; tile += RT) {
    for (int kk = threadIdx.x; kk <= RT; kk += RT) {
      const unsigned e = ent + kk;
      if (e < nf) {
        const int u = qv[e];
        w_pre[kk] = qa[e];
        const long long lu = (long long)u - vbeg;
        const bool ok = lu >= 0 && lu < n;
        w_first[kk] = ok ? rp[lu] : 0;
        const u64 pu = ok ? load_u64_relaxed(&c.P[u]) : INF;
        w_offer[kk] = pu == INF ? INF : pu + unit;
      } else {
        w_pre[kk] = af;
        w_first[kk] = 0;
        w_offer[kk] = INF;
      }
    }
    __syncthreads();
    const unsigned a = tile + threadIdx.x;
    bool want = false, wrote = false;
    int w = 0;
    unsigned deg = 0;
    u64 offer = INF;
    if (a < hi_a) {
      int lo = 0, hi = RT;  // the last kk in [0, RT) with w_pre[kk] <= a
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= a) lo = mid;
        else hi = mid;
      }
      offer = w_offer[lo];
      const unsigned j = a - w_pre[lo];
      const long long arc = (long long)w_first[lo] + j;
      const bool in_range = j < w_pre[lo + 1] - w_pre[lo] && arc < nnz && offer != INF;
      const int wl = in_range ? col[arc] : -1;
      w = (int)(vbeg + wl);
      if ((unsigned)wl < (unsigned)n) {
        if (c.P[w] > offer) {
          const u64 old = atomic_min_u64(&c.P[w], offer);
          if (old > offer) {
            wrote = true;
            if (sweep) {
              want = __hip_atomic_fetch_max(&c.stamp[w], (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                     (unsigned)k;
            } else {
              want = old == INF;
            }
            if (want) deg = (unsigned)(rp[wl + 1] - rp[wl]);
          }
        }
      } else if (in_range) {
        atomic_or_u32(&c.slot_err[s], ERR_BAD_COL);
      }
    }
    srv_note_lr(ss, wrote, s, offer);
    srv_append(ab, want, w, deg, s, c, k, ss);
    const unsigned next = tile + RT;
    __syncthreads();
    if (threadIdx.x == 0) {
      int lo = 0, hi = RT + 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= next) lo = mid;
        else hi = mid;
      }
      ss.start = ent + lo;
    }
    __syncthreads();
    ent = ss.start;
  }
}

// Top-down over the top-down slots' frontier arcs, split evenly over the grid.
__device__ __forceinline__ void srv_top_down(const RoundCtx& c, int k, SrvAppend& ab, StepShared& sh, SrvShared& ss) {
  const unsigned T = ss.td_off[MAX_SLOTS];
  const unsigned G = gridDim.x;
  const unsigned a_begin = (unsigned)(((u64)T * blockIdx.x) / G);
  const unsigned a_end = (unsigned)(((u64)T * (blockIdx.x + 1)) / G);
  if (a_begin >= a_end) return;  // uniform
  int s = 0, hi = MAX_SLOTS;  // the last slot with td_off <= a_begin
  while (hi - s > 1) {
    const int mid = (s + hi) >> 1;
    if (ss.td_off[mid] <= a_begin) s = mid;
    else hi = mid;
  }
  for (; s < MAX_SLOTS && ss.td_off[s] < a_end; ++s) {
    const unsigned s0 = ss.td_off[s], s1 = ss.td_off[s + 1];
    const unsigned lo = a_begin > s0 ? a_begin - s0 : 0u, hi_a = (a_end < s1 ? a_end : s1) - s0;
    if (s1 > s0 && lo < hi_a) srv_td_segment(c, k, ab, sh, ss, s, lo, hi_a);
  }
}

// Pull over the vertex ranges of the slots that go bottom-up (each with its own L_r) or take
// their tail seed this step (own arc, whatever its wake round, and offers from F_{r-1}).
// The rows the lanes in `rows` left undecided (as in the single-graph pull, the row state in
// the step's LDS windows at the thread index, the slot beside it), each finished by the whole
// wave in turn with its slot's CSR, id range and L_r.
__device__ __attribute__((noinline)) void srv_pull_rows_wave(const RoundCtx& c, u64 rows, unsigned* w_a, int* w_a1,
                                                             u64* w_best, const int* w_slot, const SrvShared& ss,
                                                             int r) {
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const unsigned lane = lane_id(), wave0 = threadIdx.x - lane;
  for (; rows; rows &= rows - 1) {
    const int src = __ffsll((long long)rows) - 1;
    const int s = w_slot[wave0 + src];
    const int* col = ss.col[s];
    const long long vbeg = ss.vbeg[s];
    const unsigned n = (unsigned)ss.n[s];
    const u64 Lr = ss.L[s];
    int ra = (int)w_a[wave0 + src];
    const int ra1 = w_a1[wave0 + src];
    u64 rb = w_best[wave0 + src];
    while (ra < ra1 && rb > Lr) {  // uniform over the wave
      const int ai = ra + (int)lane;
      u64 mine = INF;
      bool bad = false;
      if (ai < ra1) {
        const int ul = col[ai];
        bad = (unsigned)ul >= n;
        if (!bad) {
          const u64 pu = load_u64_relaxed(&c.P[vbeg + ul]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF) mine = pu + unit;
        }
      }
      if (__ballot(bad)) {
        if (lane == 0) atomic_or_u32(&c.slot_err[s], ERR_BAD_COL);
        break;
      }
      const u64 wm = wave_min_u64(mine);
      rb = wm < rb ? wm : rb;
      ra += WAVE;
    }
    if ((int)lane == src) w_best[wave0 + src] = rb;
  }
}

// A pulled vertex whose best offer is below its label: the label drops; a bottom-up vertex is
// queued if it was not reached before, a seeded one if it is not queued in this step yet.
__device__ __forceinline__ void srv_pull_update(const RoundCtx& c, int k, int v, bool seed, u64 best, unsigned degree,
                                                bool& wrote, bool& want, unsigned& deg) {
  if (seed) {
    atomic_min_u64(&c.P[v], best);
    wrote = true;
    want = __hip_atomic_fetch_max(&c.stamp[v], (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)k;
    deg = degree;
  } else {
    const u64 old = atomic_min_u64(&c.P[v], best);
    if (old > best) {
      wrote = true;
      if (old == INF) {
        want = true;
        deg = degree;
      }
    }
  }
}

__device__ __forceinline__ void srv_pull(const RoundCtx& c, int r, int k, SrvAppend& ab, StepShared& sh, SrvShared& ss) {
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const int cnt = ss.pull_off[MAX_SLOTS];
  for (long long base = (long long)blockIdx.x * RT; base < cnt; base += (long long)gridDim.x * RT) {
    const long long i = base + threadIdx.x;
    bool want = false, wrote = false, defer = false;
    int v = 0, slot = 0;
    unsigned deg = 0;
    u64 best = INF;
    if (i < cnt) {
      int lo = 0, hi = MAX_SLOTS;  // the last slot with pull_off <= i
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ss.pull_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      slot = lo;
      const long long lv = ss.pull_beg[lo] - ss.vbeg[lo] + (i - ss.pull_off[lo]);
      v = (int)(ss.vbeg[lo] + lv);
      const u64 Lr = ss.L[lo];
      const u64 pv = c.P[v];
      const int* rp = ss.rp[lo];
      const int* col = ss.col[lo];
      const long long vbeg = ss.vbeg[lo];
      const unsigned n = (unsigned)ss.n[lo];
      const bool seed = ss.seed[lo];
      if (pv >= base_r && (seed || pv > Lr)) {
        const int a0 = rp[lv], a1 = rp[lv + 1];
        if (!seed || a1 > a0) {
          best = seed ? srv_own_offer(c, ss, lo, v) : pv;
          int a = a0;
          bool bad = false;
          const int a_cap = a1 - a0 > PULL_CAP ? a0 + PULL_CAP : a1;
          // the first arc alone (most rows stop there), then four per group: their column ids,
          // then their labels, so that a group costs two dependent loads
          while (a < a_cap && best > Lr) {
            const int lim = min(a_cap, a + (a == a0 ? 1 : 4));
            int ul[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) ul[j] = a + j < lim ? col[a + j] : 0;
            bool bad_g = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) bad_g |= a + j < lim && (unsigned)ul[j] >= n;
            if (bad_g) {
              atomic_or_u32(&c.slot_err[lo], ERR_BAD_COL);
              bad = true;
              break;
            }
            u64 pu[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) pu[j] = a + j < lim ? load_u64_relaxed(&c.P[vbeg + ul[j]]) : INF;
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if ((pu[j] >> (FIX + B)) == prev_round && pu[j] != INF && pu[j] + unit < best) best = pu[j] + unit;
            a = lim;
          }
          if (!bad && a < a1 && best > Lr) {  // long row, undecided: the wave finishes it below
            defer = true;
            sh.w_pre[threadIdx.x] = (unsigned)a;
            sh.w_first[threadIdx.x] = a1;
            sh.w_offer[threadIdx.x] = best;
            ss.pslot[threadIdx.x] = lo;
          } else if (best < pv) {
            srv_pull_update(c, k, v, seed, best, (unsigned)(a1 - a0), wrote, want, deg);
          }
        }
      }
    }
    const u64 m = __ballot(defer);
    if (m) {
      srv_pull_rows_wave(c, m, sh.w_pre, sh.w_first, sh.w_offer, ss.pslot, ss, r);
      if (defer) {
        best = sh.w_offer[threadIdx.x];
        const long long lv = v - ss.vbeg[slot];
        if (best < c.P[v])
          srv_pull_update(c, k, v, ss.seed[slot], best, (unsigned)(ss.rp[slot][lv + 1] - ss.rp[slot][lv]), wrote, want,
                          deg);
      }
    }
    srv_note_lr(ss, wrote, slot, best);
    srv_append(ab, want, v, deg, slot, c, k, ss);
  }
}

// One server step: the next global round over every admitted request.
__device__ __forceinline__ void srv_step(const RoundCtx& c, int k, SrvAppend& ab, StepShared& sh, SrvShared& ss) {
  if (threadIdx.x == 0) {
    const RoundState P = load_state(&c.st[(k - 1) & 1]);
    RoundState S = P;
    S.seq = k;
    S.round = P.round + 1;
    S.rounds += 1;
    sh.S = S;
    ab.n = 0;
  }
  if (threadIdx.x < MAX_SLOTS) ab.tot[threadIdx.x] = 0;
  __syncthreads();
  const int r = (int)sh.S.round;
  srv_slot_setup(c, k, r, ss);
  slot_carry(ss.pull_off, ss.td_off);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) store_state<__HIP_MEMORY_SCOPE_AGENT>(&c.st[k & 1], sh.S);
  srv_wake(c, r, k, ab, ss);
  srv_top_down(c, k, ab, sh, ss);
  if (ss.pull_off[MAX_SLOTS]) srv_pull(c, r, k, ab, sh, ss);
  srv_flush(ab, c, k, ss);
  if (threadIdx.x < MAX_SLOTS && threadIdx.x < c.nslots && ss.lr[threadIdx.x] != INF)
    atomic_min_u64(&c.s_lr[(k % 3) * MAX_SLOTS + threadIdx.x], ss.lr[threadIdx.x]);
}

__global__ __launch_bounds__(RT, 8) void k_round_step_srv(const LaunchBlock* __restrict__ lb, int j) {
  __shared__ SrvAppend ab;
  __shared__ StepShared sh;
  __shared__ SrvShared ss;
  srv_step(lb->c, (int)(lb->kbase + j), ab, sh, ss);
}

}  // namespace ldd
