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
};

struct StepShared {
  RoundState S;
  u64 lr;
  unsigned start;
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
  int* qv = c.qv[k & 1];
  unsigned* qa = c.qa[k & 1];
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

// Server mode: per-slot LDS state of a step.
// what the top-down phase does with a slot's queue entries
enum { TD_SKIP = 0, TD_ROUND = 1, TD_SWEEP = 2 };
struct SrvShared {
  int std_[MAX_SLOTS];   // TD_* of each slot in this step
  int swake[MAX_SLOTS];  // the slot takes part in this round's wake
  int sseed[MAX_SLOTS];  // the slot's pull in this step is its tail seed
  u64 sL[MAX_SLOTS];     // each slot's L_r (its smallest possible offer this round)
  u64 s_cnt[MAX_SLOTS];  // this block's (count << 32 | arcs) appended per slot
  u64 s_lr[MAX_SLOTS];   // this block's smallest label written per slot
  // this round's wake segment of every slot (start in wake_ord, prefix of lengths)
  long long seg_beg[MAX_SLOTS];
  int seg_off[MAX_SLOTS + 1];
  // vertex ranges of the slots that go bottom-up (start, prefix of lengths)
  long long bseg_beg[MAX_SLOTS];
  int bseg_off[MAX_SLOTS + 1];
  unsigned char w_slot[RT + 1];  // slot of each staged top-down entry
  int skip_to;
  int any_td;  // some slot with a frontier goes top-down
};

// Per-slot notes of a tile (server mode): the count and arcs of the vertices appended and the
// smallest label written, summed per slot over the wave, then one LDS atomic per slot present.
// Called by every lane of the wave (the loop count is wave-uniform).
__device__ __forceinline__ void slot_note(SrvShared& ss, bool wrote, bool want, int slot, unsigned deg, u64 label) {
  const bool any = wrote || want;
  u64 pending = __ballot(any);
  while (pending) {
    const int leader = (int)__builtin_ctzll(pending);
    const int sl = __shfl(slot, leader, WAVE);
    const bool mine = any && slot == sl;
    const u64 m = __ballot(mine);
    const u64 cnt = wave_sum_u64(mine && want ? (((u64)1 << 32) | deg) : 0);
    const u64 lab = wave_min_u64(mine && wrote ? label : INF);
    if ((int)lane_id() == leader) {
      if (cnt) atomicAdd(&ss.s_cnt[sl], cnt);
      if (lab != INF) atomicMin(&ss.s_lr[sl], lab);
    }
    pending &= ~m;
  }
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
// Server mode: the wakers of global round r are, for every active slot with r0 <= r < r0 + R,
// the vertices of its local round r - r0 (a segment of its part of wake_ord).
__device__ __forceinline__ void phase_wake_slots(const RoundCtx& c, int r, int k, AppendBuf& ab, SrvShared& sh) {
  if (threadIdx.x < WAVE) {
    const int t = threadIdx.x;
    int len = 0;
    long long beg = 0;
    if (t < c.nslots) {
      const SlotInfo sl = c.slots[t];
      const long long rho = (long long)r - sl.r0;
      if (sh.swake[t] && rho >= 0 && rho < sl.R) {
        const int lo = c.wake_tab[sl.wbase + rho], hi = c.wake_tab[sl.wbase + rho + 1];
        len = hi - lo;
        beg = sl.vbeg + lo;
      }
    }
    const unsigned incl = wave_incl_scan((unsigned)len);
    if (t < MAX_SLOTS) {
      sh.seg_beg[t] = beg;
      sh.seg_off[t + 1] = (int)incl;
    }
    if (t == 0) sh.seg_off[0] = 0;
  }
  __syncthreads();
  const int ns = c.nslots < MAX_SLOTS ? c.nslots : MAX_SLOTS;
  const int cnt = sh.seg_off[ns];
  for (long long base = (long long)blockIdx.x * RT; base < cnt; base += (long long)gridDim.x * RT) {
    const long long i = base + threadIdx.x;
    bool want = false, wrote = false;
    int v = 0, slot = 0;
    unsigned deg = 0;
    u64 self = INF;
    if (i < cnt) {
      int lo = 0, hi = ns;  // last slot with seg_off <= i
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sh.seg_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      slot = lo;
      v = c.wake_ord[sh.seg_beg[lo] + (i - sh.seg_off[lo])];
      self = own_offer(c, v);
      if (c.P[v] > self) {
        const u64 old = atomic_min_u64(&c.P[v], self);
        if (old > self) {
          wrote = true;
          if (old == INF) {
            want = true;
            deg = degree(c, v);
          }
        }
      }
    }
    slot_note(sh, wrote, want, slot, deg, self);
    block_append(ab, want, v, deg, c, k);
  }
}

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
// SRV: server mode; the entries of slots that go bottom-up this round are skipped, a whole
// staged window at a time where they are contiguous.
template <bool TAIL, bool SRV>
__device__ __forceinline__ void phase_top_down(const RoundCtx& c, int k, const int* qv, const unsigned* qa, unsigned nf, unsigned af,
                               AppendBuf& ab, StepShared& sh, u64& wmin, unsigned sweep, SrvShared* ss) {
  unsigned* w_pre = sh.w_pre;
  int* w_first = sh.w_first;
  u64* w_offer = sh.w_offer;
  const u64 unit = (u64)1 << (FIX + c.B);
  const unsigned G = gridDim.x;
  const unsigned a_begin = (unsigned)(((u64)af * blockIdx.x) / G);
  const unsigned a_end = (unsigned)(((u64)af * (blockIdx.x + 1)) / G);
  if (a_begin >= a_end) return;
  if (threadIdx.x == 0) {
    unsigned lo = 0, hi = nf;  // last entry with qa <= a_begin
    while (hi - lo > 1) {
      const unsigned mid = (lo + hi) >> 1;
      if (qa[mid] <= a_begin) lo = mid;
      else hi = mid;
    }
    sh.start = lo;
  }
  __syncthreads();
  unsigned ent = sh.start;
  unsigned tile = a_begin;
  while (tile < a_end) {
    for (int kk = threadIdx.x; kk <= RT; kk += RT) {
      const unsigned e = ent + kk;
      if (e < nf) {
        const int u = qv[e];
        w_pre[kk] = qa[e];
        bool ok = (unsigned)u < (unsigned)c.n;
        if (SRV) {
          const int sl = ok ? c.vslot[u] : 0;
          ss->w_slot[kk] = (unsigned char)sl;
          ok = ok && ss->std_[sl] != TD_SKIP;
        }
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
    bool want = false, wrote = false;
    int w = 0, slot = 0;
    unsigned deg = 0;
    u64 offer = INF;
    if (a < a_end) {
      int lo = 0, hi = RT;  // last kk in [0, RT) with w_pre[kk] <= a
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= a) lo = mid;
        else hi = mid;
      }
      offer = w_offer[lo];
      if (SRV) slot = ss->w_slot[lo];
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
            if (SRV && ss->std_[slot] == TD_SWEEP) {  // the slot's tail: queue on any lowering
              wrote = true;
              if (__hip_atomic_fetch_max(&c.stamp[w], (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                  (unsigned)k) {
                want = true;
                deg = degree(c, w);
              }
            } else if (TAIL) {
              if (__hip_atomic_fetch_max(&c.stamp[w], sweep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                  sweep + 1) {
                want = true;
                deg = degree(c, w);
              }
            } else {
              wmin = offer < wmin ? offer : wmin;
              wrote = true;
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
    if (SRV) slot_note(*ss, wrote, want, slot, deg, offer);
    block_append(ab, want, w, deg, c, k);
    // the entry holding the next tile's first arc is one of ent .. ent+RT (all staged)
    unsigned next = tile + RT;
    __syncthreads();
    if (threadIdx.x == 0) {
      int lo = 0, hi = RT + 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (w_pre[mid] <= next) lo = mid;
        else hi = mid;
      }
      sh.start = lo;
      if (SRV) ss->skip_to = RT;
    }
    __syncthreads();
    if (SRV) {
      // skipped entries from there on: the next tile starts at the first entry that is not
      // skipped (or at entry RT, the last one staged)
      const int lo = (int)sh.start;
      for (int kk = threadIdx.x; kk < RT; kk += RT)
        if (kk >= lo && w_offer[kk] != INF) atomicMin(&ss->skip_to, kk);
      __syncthreads();
      const int to = ss->skip_to;
      if (to > lo && w_pre[to] > next) next = w_pre[to];
      __syncthreads();
      if (threadIdx.x == 0) {
        int l2 = lo, h2 = RT + 1;  // the entry holding the (possibly moved) tile start
        while (h2 - l2 > 1) {
          const int mid = (l2 + h2) >> 1;
          if (w_pre[mid] <= next) l2 = mid;
          else h2 = mid;
        }
        sh.start = l2;
      }
      __syncthreads();
    }
    ent += sh.start;
    tile = next;
  }
}

// ---- bottom-up: vertices not settled before round r pull from their neighbours in F_{r-1} ---
// A neighbour u is in F_{r-1} iff its label lies in [base(r-1), base(r)).  L_r (the smallest
// offer F_{r-1} makes) ends the scan as soon as it is attained.
__device__ __forceinline__ void phase_bottom_up(const RoundCtx& c, int r, int k, u64 Lr, AppendBuf& ab, u64& wmin, u64& examined) {
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  for (long long base = (long long)blockIdx.x * RT; base < c.n; base += (long long)gridDim.x * RT) {
    const long long vi = base + threadIdx.x;
    bool want = false;
    unsigned deg = 0;
    const int v = (int)vi;
    if (vi < c.n) {
      const u64 pv = c.P[v];
      if (pv >= base_r && pv > Lr) {
        const int a0 = c.row_ptr[v], a1 = c.row_ptr[v + 1];
        u64 best = pv;
        for (int a = a0; a < a1; ++a) {
          ++examined;
          const int u = c.col[a];
          if ((unsigned)u >= (unsigned)c.n) {
            atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
            break;
          }
          const u64 pu = load_u64_relaxed(&c.P[u]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF) {
            const u64 offer = pu + unit;
            if (offer < best) best = offer;
            if (best <= Lr) break;
          }
        }
        if (best < pv) {
          const u64 old = atomic_min_u64(&c.P[v], best);
          if (old > best) {
            wmin = best < wmin ? best : wmin;
            if (old == INF) {
              want = true;
              deg = (unsigned)(a1 - a0);
            }
          }
        }
      }
    }
    block_append(ab, want, v, deg, c, k);
  }
}

// Server mode: the same pull over the vertex ranges of the slots that go bottom-up this round,
// each with its own L_r.
__device__ __forceinline__ void phase_bottom_up_slots(const RoundCtx& c, int r, int k, AppendBuf& ab, SrvShared& ss) {
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  const int ns = c.nslots < MAX_SLOTS ? c.nslots : MAX_SLOTS;
  const int cnt = ss.bseg_off[ns];
  for (long long base = (long long)blockIdx.x * RT; base < cnt; base += (long long)gridDim.x * RT) {
    const long long i = base + threadIdx.x;
    bool want = false, wrote = false;
    int v = 0, slot = 0;
    unsigned deg = 0;
    u64 best = INF;
    if (i < cnt) {
      int lo = 0, hi = ns;  // last slot with bseg_off <= i
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ss.bseg_off[mid] <= i) lo = mid;
        else hi = mid;
      }
      slot = lo;
      v = (int)(ss.bseg_beg[lo] + (i - ss.bseg_off[lo]));
      const u64 Lr = ss.sL[lo];
      const bool seed = ss.sseed[lo] != 0;
      const u64 pv = c.P[v];
      const int a0 = c.row_ptr[v], a1 = c.row_ptr[v + 1];
      if (seed && pv >= base_r && a1 > a0) {
        // tail seed: the vertex's own arc (whatever its wake round) and its neighbours in
        // F_{r-1}; the sweeps relax the rest, queueing every vertex whose label drops
        best = own_offer(c, v);
        for (int a = a0; a < a1 && best > Lr; ++a) {
          const int u = c.col[a];
          if ((unsigned)u >= (unsigned)c.n) {
            atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
            break;
          }
          const u64 pu = load_u64_relaxed(&c.P[u]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF && pu + unit < best) best = pu + unit;
        }
        if (best < pv) {
          atomic_min_u64(&c.P[v], best);
          wrote = true;
          want = __hip_atomic_fetch_max(&c.stamp[v], (unsigned)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                 (unsigned)k;
          deg = (unsigned)(a1 - a0);
        }
      } else if (!seed && pv >= base_r && pv > Lr) {
        best = pv;
        for (int a = a0; a < a1; ++a) {
          const int u = c.col[a];
          if ((unsigned)u >= (unsigned)c.n) {
            atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
            break;
          }
          const u64 pu = load_u64_relaxed(&c.P[u]);
          if ((pu >> (FIX + B)) == prev_round && pu != INF) {
            const u64 offer = pu + unit;
            if (offer < best) best = offer;
            if (best <= Lr) break;
          }
        }
        if (best < pv) {
          const u64 old = atomic_min_u64(&c.P[v], best);
          if (old > best) {
            wrote = true;
            if (old == INF) {
              want = true;
              deg = (unsigned)(a1 - a0);
            }
          }
        }
      }
    }
    slot_note(ss, wrote, want, slot, deg, best);
    block_append(ab, want, v, deg, c, k);
  }
}

// ---- tail seed: every vertex not settled before round r takes the best of its own arc and
// the offers of its neighbours in F_{r-1} (the only settled vertices whose offers have not
// been propagated yet); the sweeps then relax to the fixpoint.  Pulling touches only the
// rows of unsettled vertices, which are few when the tail starts.
__device__ __forceinline__ void phase_tail_seed(const RoundCtx& c, int r, int k, u64 Lr, AppendBuf& ab,
                                                u64& examined) {
  const int B = c.B;
  const u64 unit = (u64)1 << (FIX + B);
  const u64 base_r = (u64)r << (FIX + B);
  const u64 prev_round = (u64)(r - 1);
  for (long long base = (long long)blockIdx.x * RT; base < c.n; base += (long long)gridDim.x * RT) {
    const long long vi = base + threadIdx.x;
    bool want = false;
    unsigned deg = 0;
    const int v = (int)vi;
    if (vi < c.n) {
      const u64 pv = c.P[v];
      if (pv >= base_r) {
        const int a0 = c.row_ptr[v], a1 = c.row_ptr[v + 1];
        deg = (unsigned)(a1 - a0);
        if (deg > 0) {
          u64 best = own_offer(c, v);
          for (int a = a0; a < a1 && best > Lr; ++a) {
            ++examined;
            const int u = c.col[a];
            if ((unsigned)u >= (unsigned)c.n) {
              atomic_or_u32(&c.ctrl->err, ERR_BAD_COL);
              break;
            }
            const u64 pu = load_u64_relaxed(&c.P[u]);
            if ((pu >> (FIX + B)) == prev_round && pu != INF && pu + unit < best) best = pu + unit;
          }
          if (best < pv) {
            atomic_min_u64(&c.P[v], best);
            want = __hip_atomic_fetch_max(&c.stamp[v], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 1u;
          }
        }
      }
    }
    block_append(ab, want, v, deg, c, k);
  }
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

template <bool SRV>
__device__ __forceinline__ RoundState next_state(const RoundCtx& c, int k) {
  const RoundState P = load_state(&c.st[(k - 1) & 1]);
  const u64 out = load_u64_relaxed(qcounter(c, k - 1));
  RoundState S = P;
  S.seq = k;
  if (P.mode == MODE_DONE) return S;
  const unsigned nf = min((unsigned)(out >> 32), (unsigned)c.n), af = (unsigned)out;
  if (SRV) {  // server: the next global round, always (directions are per slot)
    S.settled += nf;
    S.rounds += 1;
    S.max_frontier = (long long)nf > S.max_frontier ? (long long)nf : S.max_frontier;
    S.round = P.round + 1;
    S.prev = (long long)out;
    return S;
  }
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

// Server mode, start of step k (wave 0, one lane per slot), round r: each slot's mode and, in
// rounds mode, its direction from its own frontier (the notes of step k-1), as next_state and
// choose_dir decide for one graph; its L_r; the ranges that pull.  Block 0 records the slots'
// state after step k and reports a slot found done (through mapped host memory).
__device__ __forceinline__ void slot_setup(const RoundCtx& c, int k, int r, SrvShared& ss) {
  if (threadIdx.x >= WAVE) return;
  const int s = threadIdx.x;  // MAX_SLOTS == WAVE
  int td = TD_SKIP, wake = 0, seed = 0, pull_len = 0;
  long long pull_beg = 0;
  u64 L = INF, nf = 0;
  if (s < c.nslots) {
    const SlotInfo sl = c.slots[s];
    const SlotState p = c.sst[((k - 1) & 1) * MAX_SLOTS + s];
    const u64 cnt = c.s_cnt[((k - 1) % 3) * MAX_SLOTS + s];
    const u64 lr = c.s_lr[((k - 1) % 3) * MAX_SLOTS + s];
    nf = cnt >> 32;
    const u64 af = cnt & 0xffffffffull;
    SlotState q = p;
    q.dir = DIR_TD;
    bool report = false;
    if (sl.active && p.mode == SM_ROUNDS) {
      q.settled += (long long)nf;
      q.ua -= (long long)af;
      const long long n_act = c.wake_tab[sl.wbase + sl.R];
      const long long left = n_act - q.settled;
      const long long rho = (long long)r - sl.r0;
      if (left <= 0) {  // every vertex reached: the round that reached the last one ended
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
            const u64 n = (u64)sl.n;
            const bool bu_better = af * (u64)c.td_to_bu > (u64)(q.ua > 0 ? q.ua : 0) + n / 4;
            dir = (p.dir == DIR_BU) ? ((bu_better || nf * (u64)c.bu_to_td >= n) ? DIR_BU : DIR_TD)
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
  const u64 td_front = __ballot(td != TD_SKIP && nf > 0);
  const unsigned incl = wave_incl_scan((unsigned)pull_len);
  ss.std_[s] = td;
  ss.swake[s] = wake;
  ss.sseed[s] = seed;
  ss.sL[s] = L;
  ss.s_cnt[s] = 0;
  ss.s_lr[s] = INF;
  ss.bseg_beg[s] = pull_beg;
  ss.bseg_off[s + 1] = (int)incl;
  if (s == 0) {
    ss.bseg_off[0] = 0;
    ss.any_td = td_front != 0;
  }
}

// Server mode, end of step k: the block's per-slot notes into the step's counters.
__device__ __forceinline__ void slot_flush(const RoundCtx& c, int k, SrvShared& ss) {
  __syncthreads();
  const int s = threadIdx.x;
  if (s < MAX_SLOTS && s < c.nslots) {
    if (ss.s_cnt[s]) atomic_add_u64(&c.s_cnt[(k % 3) * MAX_SLOTS + s], ss.s_cnt[s]);
    if (ss.s_lr[s] != INF) atomic_min_u64(&c.s_lr[(k % 3) * MAX_SLOTS + s], ss.s_lr[s]);
  }
}

// One step; returns the mode it ran in (MODE_DONE: nothing was left to do).
// SRV: server mode (the next global round over all slots, each in its own direction).
template <bool SRV>
__device__ __forceinline__ int round_step(const RoundCtx& c, int k, AppendBuf& ab, StepShared& sh, SrvShared* ss) {
  if (threadIdx.x == 0) {
    // Once a step has written "done" into either slot no step writes a slot again, so later
    // steps only need the two mode words to leave.
    const bool done = !SRV && (__hip_atomic_load(&c.st[0].mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == MODE_DONE ||
                               __hip_atomic_load(&c.st[1].mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == MODE_DONE);
    if (done) {
      sh.S.mode = MODE_DONE;
      sh.S.seq = -1;
    } else {
      sh.S = next_state<SRV>(c, k);
    }
    ab.n = 0;
    ab.arcs = 0;
  }
  __syncthreads();
  if (SRV) {
    slot_setup(c, k, (int)sh.S.round, *ss);
    __syncthreads();
  }
  const RoundState S = sh.S;
  if (S.seq < 0) return MODE_DONE;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_state<__HIP_MEMORY_SCOPE_AGENT>(&c.st[k & 1], S);
    __hip_atomic_store(qcounter(c, k + 1), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the host stops enqueueing steps once it reads "done"; written once per decomposition,
    // since a store to host memory delays the completion of the kernel that makes it
    if (c.host_st && S.mode == MODE_DONE) store_state<__HIP_MEMORY_SCOPE_SYSTEM>(c.host_st, S);
  }
  if (S.mode == MODE_DONE) return MODE_DONE;
  const unsigned nf = min((unsigned)((u64)S.prev >> 32), (unsigned)c.n), af = (unsigned)S.prev;
  const int* qv = c.qv[(k - 1) & 1];
  const unsigned* qa = c.qa[(k - 1) & 1];
  u64 wmin = INF, examined = 0;
  if (SRV) {
    const int r = (int)S.round;
    phase_wake_slots(c, r, k, ab, *ss);
    if (nf && ss->any_td) phase_top_down<false, true>(c, k, qv, qa, nf, af, ab, sh, wmin, 0, ss);
    if (ss->bseg_off[MAX_SLOTS]) phase_bottom_up_slots(c, r, k, ab, *ss);
    block_flush(ab, c, k);
    slot_flush(c, k, *ss);
    return MODE_ROUNDS;
  }
  const bool need_lr = nf && ((S.mode == MODE_ROUNDS && S.dir == DIR_BU) || (S.mode == MODE_TAIL && S.round == 0));
  if (need_lr) {
    // L_r: the smallest offer of F_{r-1}, from the per-block minima the previous step left
    u64 m = INF;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += RT) {
      const u64 x = load_u64_relaxed(&c.lr_part[(size_t)((k - 1) & 1) * gridDim.x + b]);
      m = x < m ? x : m;
    }
    m = block_min_u64(m, sh);
    if (threadIdx.x == 0) sh.lr = m == INF ? INF : m + ((u64)1 << (FIX + c.B));
    __syncthreads();
  }
  if (S.mode == MODE_ROUNDS) {
    const int r = (int)S.round;
    phase_wake(c, r, k, ab, wmin);
    if (nf) {
      if (S.dir == DIR_BU) {
        phase_bottom_up(c, r, k, sh.lr, ab, wmin, examined);
      } else {
        phase_top_down<false, false>(c, k, qv, qa, nf, af, ab, sh, wmin, 0, nullptr);
        if (blockIdx.x == 0 && threadIdx.x == 0) examined += af;
      }
    }
  } else {
    const unsigned sweep = (unsigned)S.round;
    if (sweep == 0) {
      phase_tail_seed(c, (int)S.tail_round, k, nf ? sh.lr : INF, ab, examined);
    } else if (nf) {
      phase_top_down<true, false>(c, k, qv, qa, nf, af, ab, sh, wmin, sweep, nullptr);
      if (blockIdx.x == 0 && threadIdx.x == 0) examined += af;
    }
  }
  block_flush(ab, c, k);
  const u64 bm = block_min_u64(wmin, sh);
  if (threadIdx.x == 0) c.lr_part[(size_t)(k & 1) * gridDim.x + blockIdx.x] = bm;
  add_examined(c, examined, sh);
  return (int)S.mode;
}

// (RT, 8): eight waves per SIMD, i.e. two 1024-thread blocks per CU, which caps VGPRs at 64
__global__ __launch_bounds__(RT, 8) void k_round_step_lb(const LaunchBlock* __restrict__ lb, int j) {
  __shared__ AppendBuf ab;
  __shared__ StepShared sh;
  round_step<false>(lb->c, (int)(lb->kbase + j), ab, sh, nullptr);
}

// The server's step: the next global round over every admitted request.
__global__ __launch_bounds__(RT, 8) void k_round_step_srv(const LaunchBlock* __restrict__ lb, int j) {
  __shared__ AppendBuf ab;
  __shared__ StepShared sh;
  __shared__ SrvShared ss;
  round_step<true>(lb->c, (int)(lb->kbase + j), ab, sh, &ss);
}

__global__ void k_advance(LaunchBlock* lb, int C) {
  if (threadIdx.x == 0 && blockIdx.x == 0) lb->kbase += C;
}

// All steps in one kernel with grid barriers between them (the grid must be co-resident).
__global__ __launch_bounds__(RT) void k_rounds_persistent(RoundCtx c) {
  __shared__ AppendBuf ab;
  __shared__ StepShared sh;
  u64 gen = 0;
  const long long kmax = (long long)c.R + c.n + 2;
  for (int k = 1; k <= kmax; ++k) {
    if (round_step<false>(c, k, ab, sh, nullptr) == MODE_DONE) break;
    grid_sync(&c.ctrl->bar, gridDim.x, gen, &c.ctrl->err);
    if (__hip_atomic_load(&c.ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & (ERR_BARRIER | ERR_QUEUE)) break;
  }
}

}  // namespace ldd
