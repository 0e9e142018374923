// Workgroup-owned decomposition: one workgroup runs every round of one graph, with workgroup
// barriers between rounds and no grid-wide step.  This is the search of Sec. 5 (Algorithm 2 via
// the delayed-start breadth-first search), round by round, as the multi-block engine runs it:
//
//   preparation  Delta = max shift; labels INF; the vertices with arcs sorted by wake round
//                w(v) = (Delta - shift[v]) >> 20 (counting sort in LDS)
//   round r      wake: every vertex of bucket r offers its own label ((Delta - shift[v]) << B) | v;
//                top-down: every vertex u of F_{r-1} offers P(u) + (2^20 << B) along its arcs;
//                offers are applied with an atomic minimum on the 64-bit label (exact), and the
//                first offer a vertex receives appends it to F_r
//   empty F_r    the next round is the next non-empty wake bucket
//   output       centre = low B bits of the label (INF: an isolated vertex, its own centre) and
//                the cut (Def. 1.1)
//
// A round costs a few workgroup barriers and a handful of dependent cache accesses instead of a
// kernel launch and a grid-wide state exchange, so graphs with many rounds and small frontiers
// (small graphs, high-diameter graphs) run far faster here; a batch runs one graph per workgroup,
// the largest first, each workgroup taking the next graph when it finishes one.
//
// Top-down is arc-balanced inside the workgroup: a chunk of RT frontier entries is staged in LDS
// (first arc, degree prefix, offer) and every thread takes arcs of the chunk by index, finding its
// entry by binary search, so a high-degree vertex is shared by all threads.
//
// A graph too large for one workgroup (a batch's largest graphs, or one large high-diameter graph)
// runs on a team of K workgroups, all resident at once: member m owns a slice of the vertices
// (its preparation, wake buckets, tail seed and output) and the m-th K-th of every frontier; the
// next frontier is one shared queue, to which each member appends through a staging buffer in LDS
// and one reservation per round; the members meet once per round at a barrier in device memory,
// where the queue's length and the error bits are read.  The labels are then shared by several
// CUs, so their loads and atomics take device scope.
#include "ldd_block.h"

namespace ldd {

namespace {

constexpr int BT = 1024;         // threads per workgroup
constexpr int BNW = BT / WAVE;   // waves per workgroup
constexpr int WPT = BLOCK_WCAP / BT;  // wake buckets per thread in the scans
constexpr unsigned TB_CAP = 2048;     // a team member's staged appends per round (more go straight out)

struct BlockShared {
  int woff[BLOCK_WCAP + 1];  // wake bucket offsets (exclusive prefix), then the scatter cursors
  unsigned pre[BT + 1];      // top-down chunk: exclusive degree prefix
  int first[BT];             // first arc of each staged entry
  u64 offer[BT];             // offer of each staged entry
  u64 red64[BNW];
  unsigned red32[BNW];
  int job;
  int nxt;                   // next non-empty wake bucket (block minimum)
  unsigned cnt;              // appends to the next frontier in this round (team, tail)
  unsigned cnt3[3];          // the same, alone: round k counts in cnt3[k % 3], so one barrier per round
  unsigned err;
  u64 delta, n_active;       // preparation results
  u64 settled, examined;     // round results
  long long rounds, sweeps;
  // team of several workgroups on one graph
  TeamSync* ts;
  int tK, tm, tlo, thi;      // team size, this member, this member's vertex slice
  unsigned epoch;            // barriers passed
  unsigned bn;               // appends staged in tbuf this round
  unsigned tnf;              // the queue length the last team barrier published
  unsigned tcount;           // this member's appends to the shared queue in this step
  unsigned tbase;            // the staged appends' place in the shared queue
  u64 nz[BLOCK_WCAP / 64];   // non-empty wake buckets of the whole graph
  int tbuf[TB_CAP];          // staged appends of this member
};

__device__ __forceinline__ u64 block_max64(u64 v, BlockShared& sh) {
  v = wave_max_u64(v);
  __syncthreads();
  if (lane_id() == 0) sh.red64[threadIdx.x / WAVE] = v;
  __syncthreads();
  u64 m = 0;
#pragma unroll
  for (int w = 0; w < BNW; ++w) m = sh.red64[w] > m ? sh.red64[w] : m;
  return m;
}

__device__ __forceinline__ u64 block_sum64(u64 v, BlockShared& sh) {
  v = wave_sum_u64(v);
  __syncthreads();
  if (lane_id() == 0) sh.red64[threadIdx.x / WAVE] = v;
  __syncthreads();
  u64 s = 0;
#pragma unroll
  for (int w = 0; w < BNW; ++w) s += sh.red64[w];
  return s;
}

// exclusive prefix sum of x over the workgroup; *total receives the sum (all threads call)
__device__ __forceinline__ unsigned block_excl_scan(unsigned x, BlockShared& sh, unsigned* total) {
  const unsigned incl = wave_incl_scan(x);
  const unsigned wid = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == WAVE - 1) sh.red32[wid] = incl;
  __syncthreads();
  unsigned before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < BNW; ++w) {
    const unsigned t = sh.red32[w];
    before += w < (int)wid ? t : 0u;
    all += t;
  }
  *total = all;
  return before + incl - x;
}

// The first non-empty wake bucket at or after r (D + n + 1 when none is left: past the end);
// all threads call.  Found by a block-wide minimum over the bucket offsets.
__device__ __forceinline__ int next_nonempty(BlockShared& sh, int r, int D) {
  __syncthreads();
  if (threadIdx.x == 0) sh.nxt = 0x7fffffff;
  __syncthreads();
  for (int q = r + (int)threadIdx.x; q <= D; q += BT)
    if (sh.woff[q + 1] > sh.woff[q]) atomicMin(&sh.nxt, q);
  __syncthreads();
  const int q = sh.nxt;
  __syncthreads();
  return q <= D ? q : 0x3fffffff;
}

// A graph's labels are touched by its own workgroup only while it runs, so their loads and atomics
// need workgroup scope alone (all waves of a workgroup share one CU and its vector L1).  A team's
// labels are shared by its members' CUs, which may sit on different XCDs, each with its own L2.
// Within the rounds every access another member may read or write is itself coherent at device
// scope: the claims are device-scope atomics, the queue entries device-scope stores and loads, and
// the loads that decide something (an offer, a queue entry) device-scope loads; so the per-round
// barrier only has to wait for the member's own accesses to complete, with no L2 writeback or
// invalidation (which would also drop the cached CSR every round).  A label load that only filters
// atomics (is the label still larger than the offer?) stays at workgroup scope and may see an
// older value, which is never smaller (labels only decrease, and the preparation's barriers,
// which do write back and invalidate, order every cached copy after the labels' initialisation),
// so at worst it lets through an atomic that finds nothing to do.  The phases that use plain
// loads and stores on shared data (preparation, the tail's seed, the output) are bracketed by
// barriers or fences that do write back and invalidate.
constexpr int WG = __HIP_MEMORY_SCOPE_WORKGROUP;
constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;

template <int SC>
__device__ __forceinline__ u64 lab_load(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ u64 lab_min(u64* p, u64 v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ void lab_store(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, SC);
}
__device__ __forceinline__ u64 wg_load(const u64* p) { return lab_load<WG>(p); }

__device__ __forceinline__ void append(unsigned* cnt, int* next, int v) {
  const unsigned idx = atomicAdd(cnt, 1u);
  next[idx] = v;
}

// Appends to the next frontier.  Alone: counted in LDS, written at once.  step() is called by
// every thread after each pass of at most BT appends (nothing to do here).
struct LocalAppend {
  unsigned* cnt;
  int* next;
  __device__ __forceinline__ void operator()(int v) const { append(cnt, next, v); }
  __device__ __forceinline__ void step() const {}
};

// The staged appends of a team member go to the team's shared queue behind one reservation
// (all threads call; `c` entries staged, c <= TB_CAP).
__device__ __forceinline__ void team_flush(BlockShared& sh, int* next, u64* gcnt, unsigned c) {
  if (threadIdx.x == 0) {
    sh.tbase = (unsigned)__hip_atomic_fetch_add(gcnt, (u64)c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh.tcount += c;
  }
  __syncthreads();
  for (unsigned i = threadIdx.x; i < c; i += BT)
    __hip_atomic_store(&next[sh.tbase + i], sh.tbuf[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (threadIdx.x == 0) sh.bn = 0;
  __syncthreads();
}

// A team member: staged in LDS; after a pass that may leave fewer than BT free entries, the
// staged entries are placed in the shared queue (step(), uniform: one reservation per 1024 or
// more appends), and the rest at the end of the round.  An append past the staging capacity
// (which the passes never reach) would reserve its own slot.
struct TeamAppend {
  BlockShared* sh;
  int* next;
  u64* gcnt;
  __device__ __forceinline__ void operator()(int v) const {
    const unsigned i = atomicAdd(&sh->bn, 1u);
    if (i < TB_CAP) {
      sh->tbuf[i] = v;
    } else {
      __hip_atomic_store(&next[__hip_atomic_fetch_add(gcnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)], v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      atomicAdd(&sh->tcount, 1u);
    }
  }
  __device__ __forceinline__ void step() const {
    __syncthreads();
    const unsigned c = sh->bn;
    if (c > TB_CAP - BT) team_flush(*sh, next, gcnt, c < TB_CAP ? c : TB_CAP);
  }
};

// The slice loops (preparation, wake sort, output) are latency-bound with one vertex per thread at a
// time: a thread takes VU vertices at once (v, v + BT, ...), and in the output AU arcs of each,
// so that each of its loads has others in flight.
constexpr int VU = 4, AU = 2;

// Vertices v0 + k * BT (k < VU) below hi: has[k] when the vertex has arcs, key[k] = Delta - shift.
__device__ __forceinline__ void slice_load(const int* __restrict__ rp, const long long* __restrict__ shift, int v0,
                                           int hi, u64 delta, u64 (&key)[VU], bool (&has)[VU]) {
  int a0[VU], a1[VU];
  long long sv[VU];
#pragma unroll
  for (int k = 0; k < VU; ++k) {
    const int v = v0 + k * BT;
    a0[k] = a1[k] = 0;
    sv[k] = 0;
    if (v < hi) {
      a0[k] = rp[v];
      a1[k] = rp[v + 1];
      sv[k] = shift[v];
    }
  }
#pragma unroll
  for (int k = 0; k < VU; ++k) {
    has[k] = a1[k] > a0[k];
    key[k] = delta - (u64)sv[k];
  }
}

// Wake buckets of the vertices with arcs in [lo, hi): counting sort by w(v) = (Delta - shift) >> 20
// in LDS; the vertices' own labels ((Delta - shift[v]) << B) | v go to wk[lo ...] in bucket order
// (a wake then needs no shift load) and sh.woff[q] is bucket q's offset from lo (all threads call).
__device__ __forceinline__ void wake_sort(const BlockJob& j, BlockShared& sh, int lo, int hi, u64 delta) {
  const int* __restrict__ rp = j.row_ptr;
  const long long* __restrict__ shift = j.shift;
  const int tid = threadIdx.x;
  const int B = j.n > 1 ? 32 - __builtin_clz((unsigned)(j.n - 1)) : 1;
  for (int q = tid; q <= BLOCK_WCAP; q += BT) sh.woff[q] = 0;
  __syncthreads();
  for (int v0 = lo + tid; v0 < hi; v0 += VU * BT) {
    u64 key[VU];
    bool has[VU];
    slice_load(rp, shift, v0, hi, delta, key, has);
#pragma unroll
    for (int k = 0; k < VU; ++k)
      if (has[k]) atomicAdd(&sh.woff[(int)(key[k] >> FIX)], 1);
  }
  __syncthreads();
  {
    unsigned loc[WPT], sum = 0;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      loc[i] = (unsigned)sh.woff[tid * WPT + i];
      sum += loc[i];
    }
    unsigned total;
    unsigned run = block_excl_scan(sum, sh, &total);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const unsigned c = loc[i];
      sh.woff[tid * WPT + i] = (int)run;
      run += c;
    }
    if (tid == 0) sh.woff[BLOCK_WCAP] = (int)total;
  }
  __syncthreads();
  // scatter: woff[q] serves as bucket q's cursor (it ends at the start of bucket q + 1) and is
  // shifted back by one bucket afterwards
  for (int v0 = lo + tid; v0 < hi; v0 += VU * BT) {
    u64 key[VU];
    bool has[VU];
    slice_load(rp, shift, v0, hi, delta, key, has);
#pragma unroll
    for (int k = 0; k < VU; ++k)
      if (has[k]) j.wk[lo + atomicAdd(&sh.woff[(int)(key[k] >> FIX)], 1)] = (key[k] << B) | (u64)(v0 + k * BT);
  }
  __syncthreads();
  {
    int vals[WPT];
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const int q = tid * WPT + i;
      vals[i] = q == 0 ? 0 : sh.woff[q - 1];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < WPT; ++i) sh.woff[tid * WPT + i] = vals[i];
    __syncthreads();
  }
}

// Checks, Delta and the count of vertices with arcs over [lo, hi), which also get label INF
// (all threads call; results are the workgroup's: *dmax and *active reduced, errors in sh.err,
// which the caller cleared).
__device__ __forceinline__ void prepare_scan(const BlockJob& j, BlockShared& sh, int lo, int hi, bool ends,
                                             u64* dmax_out, u64* active_out, u64* degmax_out = nullptr) {
  const int n = j.n;
  const long long nnz = j.nnz;
  const int* __restrict__ rp = j.row_ptr;
  const long long* __restrict__ shift = j.shift;
  u64* P = j.P;
  const int tid = threadIdx.x;
  unsigned err = 0;
  u64 dmax = 0, active = 0, degmax = 0;
  if (ends && n > 0 && (rp[0] != 0 || (long long)rp[n] != nnz) && tid == 0) err |= ERR_BAD_ROWPTR;
  for (int v0 = lo + tid; v0 < hi; v0 += VU * BT) {
    long long sv[VU];
    int a0[VU], a1[VU];
#pragma unroll
    for (int k = 0; k < VU; ++k) {
      const int v = v0 + k * BT;
      sv[k] = 0;
      a0[k] = a1[k] = 0;
      if (v < hi) {
        sv[k] = shift[v];
        a0[k] = rp[v];
        a1[k] = rp[v + 1];
      }
    }
#pragma unroll
    for (int k = 0; k < VU; ++k) {
      const int v = v0 + k * BT;
      if (v < hi) {
        if (sv[k] < 0 || sv[k] > (1ll << 52)) err |= ERR_BAD_SHIFT;
        if (a1[k] < a0[k]) err |= ERR_BAD_ROWPTR;
        active += a1[k] > a0[k];
        dmax = (u64)sv[k] > dmax ? (u64)sv[k] : dmax;
        degmax = a1[k] > a0[k] && (u64)(a1[k] - a0[k]) > degmax ? (u64)(a1[k] - a0[k]) : degmax;
        P[v] = INF;
      }
    }
  }
  if (err) atomicOr(&sh.err, err);
  *dmax_out = block_max64(dmax, sh);
  *active_out = block_sum64(active, sh);
  if (degmax_out) *degmax_out = block_max64(degmax, sh);
  __syncthreads();
}

// The checks that need Delta: labels fit 64 bits, and the shifts span fewer than BLOCK_WCAP units.
__device__ __forceinline__ unsigned range_err(int n, u64 delta) {
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  if ((delta + ((u64)1 << FIX)) >= ((u64)1 << (64 - B))) return BLK_OVERFLOW;
  if ((delta >> FIX) >= (u64)BLOCK_WCAP) return BLK_WIDE;
  return 0;
}

// Preparation of one graph: checks, Delta, the vertices with arcs, labels INF, and the wake
// buckets.  Results in sh (delta, n_active, err, woff).
__device__ __attribute__((noinline)) void block_prepare(const BlockJob& j, BlockShared& sh) {
  if (threadIdx.x == 0) sh.err = 0;
  __syncthreads();
  u64 delta, n_active;
  prepare_scan(j, sh, 0, j.n, true, &delta, &n_active);
  if (threadIdx.x == 0) {
    unsigned e = sh.err;
    if (!e) e = range_err(j.n, delta);
    sh.err = e;
    sh.delta = delta;
    sh.n_active = n_active;
  }
  __syncthreads();
  if (sh.err) return;
  wake_sort(j, sh, 0, j.n, delta);
}

// Relax the arcs of a staged chunk (ne entries: first arc, degree prefix, offer in LDS; total
// arcs): every arc offers its entry's label plus one unit to its far end (atomic minimum).  A
// round appends a far end reached for the first time (old label INF); a tail sweep appends a far
// end whose label dropped, once per sweep (its stamp takes the sweep's tag).  U arcs per thread
// are issued together (entries by binary search in LDS, column ids, far labels, minima); one at a
// time measured fastest (more in flight cost registers and did not pay on batches or small graphs).
template <int SC, bool SWEEP, class App>
__device__ __forceinline__ void relax_chunk(const BlockJob& j, BlockShared& sh, unsigned ne, unsigned total, int tag,
                                            const App& app) {
  constexpr int U = 1;
  const int n = j.n;
  const long long nnz = j.nnz;
  const int* __restrict__ col = j.col;
  u64* P = j.P;
  const int top = ne > 1 ? 1 << (31 - __builtin_clz(ne - 1)) : 0;
  for (unsigned b0 = 0; b0 < total; b0 += U * BT) {  // the same passes in every thread (app.step)
    const unsigned base = b0 + threadIdx.x;
    int w[U];
    u64 off[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const unsigned a = base + (unsigned)k * BT;
      int lo = 0;  // last entry with pre <= a (steps from the largest power of two below ne)
      for (int step = top; step >= 1; step >>= 1)
        if (lo + step < (int)ne && sh.pre[lo + step] <= a) lo += step;
      const long long arc = (long long)sh.first[lo] + (a - sh.pre[lo]);
      w[k] = a < total ? (arc < nnz ? col[arc] : -1) : -2;
      off[k] = sh.offer[lo];
    }
    u64 pw[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const bool ok = (unsigned)w[k] < (unsigned)n;
      if (!ok && w[k] != -2) atomicOr(&sh.err, ERR_BAD_COL);
      pw[k] = ok ? wg_load(&P[w[k]]) : 0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (pw[k] > off[k]) {
        const u64 old = lab_min<SC>(&P[w[k]], off[k]);
        if (SWEEP) {
          if (old > off[k] && __hip_atomic_exchange(&j.wake[w[k]], tag, __ATOMIC_RELAXED, SC) != tag) app(w[k]);
        } else if (old == INF) {
          app(w[k]);
        }
      }
    }
    app.step();
  }
}

// Relax the arcs of frontier entries cur[e0 .. e1), staged in LDS a chunk of BT entries at a time
// (all threads call).
template <int SC, bool SWEEP, class App>
__device__ __forceinline__ u64 expand_frontier(const BlockJob& j, BlockShared& sh, const int* cur, unsigned e0,
                                               unsigned e1, u64 unit, int tag, const App& app) {
  const int* __restrict__ rp = j.row_ptr;
  u64 examined = 0;
  for (unsigned c0 = e0; c0 < e1; c0 += BT) {
    const unsigned e = c0 + threadIdx.x;
    unsigned deg = 0;
    if (e < e1) {
      // a team's queue entries and offers: device-scope loads (the round's barrier invalidates nothing)
      int u;
      if constexpr (SC == AG) u = __hip_atomic_load(const_cast<int*>(&cur[e]), __ATOMIC_RELAXED, AG);
      else u = cur[e];
      if (SC == WG || (unsigned)u < (unsigned)j.n) {  // a team's entries are checked (never out of range)
        const u64 pu = SC == AG ? lab_load<AG>(&j.P[u]) : wg_load(&j.P[u]);
        const int a0 = rp[u], a1 = rp[u + 1];
        deg = (unsigned)(a1 - a0);
        sh.first[threadIdx.x] = a0;
        sh.offer[threadIdx.x] = pu + unit;
      } else {
        atomicOr(&sh.err, ERR_QUEUE);
      }
    }
    unsigned total;
    const unsigned ex = block_excl_scan(deg, sh, &total);
    sh.pre[threadIdx.x] = ex;
    __syncthreads();
    examined += threadIdx.x == 0 ? total : 0;
    relax_chunk<SC, SWEEP>(j, sh, e1 - c0 < (unsigned)BT ? e1 - c0 : (unsigned)BT, total, tag, app);
    __syncthreads();
  }
  return examined;
}

// The rounds of one prepared graph (results in sh: settled, examined, rounds, sweeps, err).
// Once few vertices are left (unreached vertices * tail_den <= vertices with arcs) and more than
// TAIL_MIN_LEFT rounds remain, the tail finishes by label correction: every unreached vertex
// takes the best of its own label and its neighbours' in F_{r-1} (the only settled vertices
// whose offers are still pending), then sweeps relax the changed labels until none drops.  The
// labels are the unique fixpoint of P(v) = min(own label, min_w P(w) + unit), so the result is
// the same exact one.
constexpr int TAIL_MIN_LEFT = 16;

__device__ __attribute__((noinline)) void block_rounds(const BlockJob& j, BlockShared& sh) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  const long long* __restrict__ shift = j.shift;
  u64* P = j.P;
  const int tid = threadIdx.x;
  const u64 delta = sh.delta, n_active = sh.n_active;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const int D = (int)(delta >> FIX);
  const u64 unit = (u64)1 << (FIX + B);
  int* cur = j.q0;
  int* next = j.q1;
  unsigned nf = 0;
  u64 settled = 0, examined = 0;
  long long rounds = 0, sweeps = 0;
  const u64 mask = ((u64)1 << B) - 1;
  if (tid < 3) sh.cnt3[tid] = 0;
  int ci = 0;  // this round's append counter: cnt3[ci]; cnt3[(ci + 2) % 3] is cleared for two rounds on
  int r = next_nonempty(sh, 0, D);
  bool tail = false;
  while (settled < n_active && r <= D + n && rounds <= (long long)D + n + 2) {  // r past the end: stop
    unsigned* cnt = &sh.cnt3[ci];
    const int w0 = r <= D ? sh.woff[r] : 0, w1 = r <= D ? sh.woff[r + 1] : 0;
    // wake bucket r: each vertex offers its own label (a load first: a vertex reached earlier with
    // a smaller label needs no atomic)
    for (int i = w0 + tid; i < w1; i += BT) {
      const u64 self = j.wk[i];
      const int v = (int)(self & mask);
      if (wg_load(&P[v]) > self && lab_min<WG>(&P[v], self) == INF) append(cnt, next, v);
    }
    examined += expand_frontier<WG, false>(j, sh, cur, 0, nf, unit, 0, LocalAppend{cnt, next});
    __syncthreads();  // this round's appends are done; every thread has read the count of round k - 1
    nf = *cnt;
    if (tid == 0) sh.cnt3[ci == 0 ? 2 : ci - 1] = 0;  // round k - 1's counter, next used by round k + 2
    ci = ci == 2 ? 0 : ci + 1;
    if (sh.err) break;
    settled += nf;
    ++rounds;
    int* t = cur;
    cur = next;
    next = t;
    if (nf) ++r;
    else r = next_nonempty(sh, r + 1, D);
    const u64 left = n_active - settled;
    if (j.tail_den > 0 && left > 0 && left * (u64)j.tail_den <= n_active && D - r > TAIL_MIN_LEFT) {
      tail = true;
      break;
    }
  }
  if (tail && !sh.err) {
    // seed: F_{r-1} is cur (nf entries, final labels); every unreached vertex with arcs takes the
    // best of its own label and its neighbours' in F_{r-1}, and is queued for the first sweep
    unsigned* cnt = &sh.cnt3[ci];
    const u64 prev_round = (u64)(r - 1);
    for (int v = tid; v < n; v += BT) {
      const int a0 = rp[v], a1 = rp[v + 1];
      if (a1 == a0 || wg_load(&P[v]) != INF) continue;
      u64 best = ((delta - (u64)shift[v]) << B) | (u64)v;
      for (int a = a0; a < a1; ++a) {
        const int u = col[a];
        if ((unsigned)u >= (unsigned)n) {
          atomicOr(&sh.err, ERR_BAD_COL);
          break;
        }
        const u64 pu = wg_load(&P[u]);
        if (pu != INF && (pu >> (FIX + B)) == prev_round && pu + unit < best) best = pu + unit;
      }
      examined += (u64)(a1 - a0);
      lab_store<WG>(&P[v], best);
      j.wake[v] = -1;  // the stamp of the first sweep
      append(cnt, next, v);
    }
    __syncthreads();
    nf = *cnt;
    if (tid == 0) sh.cnt3[ci == 0 ? 2 : ci - 1] = 0;
    ci = ci == 2 ? 0 : ci + 1;
    int* t = cur;
    cur = next;
    next = t;
    // sweeps: sweep k relaxes the labels queued by the step before and queues those that drop
    for (int k = 1; nf && !sh.err && sweeps <= n; ++k) {
      unsigned* cnt = &sh.cnt3[ci];
      examined += expand_frontier<WG, true>(j, sh, cur, 0, nf, unit, -(k + 1), LocalAppend{cnt, next});
      __syncthreads();
      nf = *cnt;
      if (tid == 0) sh.cnt3[ci == 0 ? 2 : ci - 1] = 0;
      ci = ci == 2 ? 0 : ci + 1;
      ++sweeps;
      t = cur;
      cur = next;
      next = t;
    }
    settled = n_active;
  }
  __syncthreads();
  examined = block_sum64(examined, sh);
  if (tid == 0) {
    sh.settled = settled;
    sh.examined = examined;
    sh.rounds = rounds;
    sh.sweeps = sweeps;
  }
  __syncthreads();
}

// Centres (INF: an isolated vertex, its own centre) and the cut, from the final labels.
// Centres and cut arcs of the vertices [lo, hi), added to *cut2 and *pieces; an arc to a vertex out
// of range (arcs of the last frontier were not read by a round) sets ERR_BAD_COL.
__device__ __forceinline__ void output_slice(const BlockJob& j, BlockShared& sh, int lo, int hi, u64 mask, u64* cut2,
                                             u64* pieces) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  const u64* P = j.P;
  for (int v0 = lo + (int)threadIdx.x; v0 < hi; v0 += VU * BT) {
    int a[VU], a1[VU], c[VU];
    u64 p[VU];
#pragma unroll
    for (int k = 0; k < VU; ++k) {
      const int v = v0 + k * BT;
      a[k] = a1[k] = 0;
      p[k] = INF;
      if (v < hi) {
        a[k] = rp[v];
        a1[k] = rp[v + 1];
        p[k] = wg_load(&P[v]);
      }
    }
#pragma unroll
    for (int k = 0; k < VU; ++k) {
      const int v = v0 + k * BT;
      c[k] = p[k] == INF ? v : (int)(p[k] & mask);
      if (v < hi) {
        j.centre[v] = c[k];
        *pieces += c[k] == v;
      }
    }
    for (bool more = true; more;) {  // AU arcs of each vertex per pass
      int w[VU][AU];
      bool has[VU][AU];
#pragma unroll
      for (int k = 0; k < VU; ++k)
#pragma unroll
        for (int t = 0; t < AU; ++t) {
          has[k][t] = a[k] + t < a1[k];
          w[k][t] = has[k][t] ? col[a[k] + t] : 0;
        }
      u64 pw[VU][AU];
#pragma unroll
      for (int k = 0; k < VU; ++k)
#pragma unroll
        for (int t = 0; t < AU; ++t) pw[k][t] = has[k][t] && (unsigned)w[k][t] < (unsigned)n ? wg_load(&P[w[k][t]]) : 0;
      more = false;
#pragma unroll
      for (int k = 0; k < VU; ++k) {
#pragma unroll
        for (int t = 0; t < AU; ++t) {
          if (!has[k][t]) continue;
          if ((unsigned)w[k][t] >= (unsigned)n) {
            atomicOr(&sh.err, ERR_BAD_COL);
            a1[k] = a[k];
            break;
          }
          const int cw = pw[k][t] == INF ? w[k][t] : (int)(pw[k][t] & mask);
          *cut2 += cw != c[k];
        }
        a[k] += AU;
        more |= a[k] < a1[k];
      }
    }
  }
}

__device__ __attribute__((noinline)) void block_output(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  const int tid = threadIdx.x;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const u64 mask = ((u64)1 << B) - 1;
  const unsigned e0 = sh.err | (sh.settled < sh.n_active ? ERR_WATCHDOG : 0u);
  u64 cut2 = 0, pieces = 0;
  if (!e0) output_slice(j, sh, 0, n, mask, &cut2, &pieces);
  cut2 = block_sum64(cut2, sh);
  pieces = block_sum64(pieces, sh);
  if (tid == 0) {
    out->err = e0 | sh.err;
    out->cut_arcs = cut2;
    out->pieces = pieces;
    out->delta = sh.delta;
    out->n_active = sh.n_active;
    out->rounds = sh.rounds;
    out->sweeps = sh.sweeps;
    out->examined = sh.examined;
  }
}

extern __shared__ __attribute__((aligned(16))) unsigned char blk_dyn[];  // the launch's dynamic LDS

// One graph, the whole workgroup.
__device__ void block_graph(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  block_prepare(j, sh);
  if (sh.err) {
    if (threadIdx.x == 0) {
      out->err = sh.err;
      out->delta = sh.delta;
    }
    return;
  }
  block_rounds(j, sh);
  block_output(j, sh, out);
}

// One small graph, the whole workgroup, with its labels, wake order and queues in the dynamic LDS
// (P: 8 B, wake order: 8 B, queues: 2 x 4 B per vertex); the same code reaches them through
// generic pointers.  The labels are copied to the graph's label array at the end.
__device__ void block_graph_lds(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  BlockJob l = j;
  u64* base = reinterpret_cast<u64*>(blk_dyn);
  l.P = base;
  l.wk = base + n;
  l.wake = reinterpret_cast<int*>(l.wk);
  l.q0 = reinterpret_cast<int*>(base + 2 * (long long)n);
  l.q1 = l.q0 + n;
  block_graph(l, sh, out);
  __syncthreads();
  for (int v = threadIdx.x; v < n; v += BT) j.P[v] = l.P[v];
}

// One small graph whose labels and CSR fit the dynamic LDS, the whole workgroup: every vertex
// starts from its own label ((Delta - shift) << B) | v and the labels are relaxed,
// P(v) = min(P(v), min over arcs (v, u) of P(u) + unit), in place, until a pass lowers none.
// That is the unique fixpoint the rounds reach (the minimum over centres of the shifted
// distance, ties to the smaller centre; Sec. 5's search, by label correction from every source at
// once), so the result is the same; no wake buckets, frontier or queue, and every access but
// the first loads of the CSR and shifts stays in LDS.  A pass costs about n / 1024 vertices per
// thread; there are at most as many passes as the largest number of hops from a vertex to its
// centre, plus one block of passes (fewer, since labels lowered early in a pass are read later in
// the same pass).
// Labels are 8-byte LDS words written whole, so a concurrent read sees the old or the new label.
__device__ __attribute__((noinline)) void block_graph_fix(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  const long long nnz = j.nnz;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  const long long* __restrict__ shift = j.shift;
  const int tid = threadIdx.x;
  u64* P = reinterpret_cast<u64*>(blk_dyn);
  int* lrp = reinterpret_cast<int*>(P + n);
  int* lcol = lrp + n + 1;
  if (tid == 0) sh.err = 0;
  __syncthreads();
  unsigned err = 0;
  u64 dmax = 0, active = 0;
  if (tid == 0 && n > 0 && (rp[0] != 0 || (long long)rp[n] != nnz)) err |= ERR_BAD_ROWPTR;
  for (int v = tid; v <= n; v += BT) {
    const int a0 = rp[v];
    lrp[v] = a0;
    if (v == n) break;
    const int a1 = rp[v + 1];
    const long long s = shift[v];
    if (s < 0 || s > (1ll << 52)) err |= ERR_BAD_SHIFT;
    if (a1 < a0) err |= ERR_BAD_ROWPTR;
    active += a1 > a0;
    dmax = (u64)s > dmax ? (u64)s : dmax;
  }
  for (long long a = tid; a < nnz; a += BT) {
    const int c = col[a];
    if ((unsigned)c >= (unsigned)n) err |= ERR_BAD_COL;
    lcol[a] = c;
  }
  if (err) atomicOr(&sh.err, err);
  const u64 delta = block_max64(dmax, sh);
  const u64 n_active = block_sum64(active, sh);
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  __syncthreads();
  if (tid == 0) {
    unsigned e = sh.err;
    if (!e && (delta + ((u64)1 << FIX)) >= ((u64)1 << (64 - B))) e |= BLK_OVERFLOW;
    sh.err = e;
  }
  __syncthreads();
  if (sh.err) {
    if (tid == 0) {
      out->err = sh.err;
      out->delta = delta;
    }
    return;
  }
  for (int v = tid; v < n; v += BT) P[v] = ((delta - (u64)shift[v]) << B) | (u64)v;
  __syncthreads();
  const u64 unit = (u64)1 << (FIX + B);
  // Passes run FIX_BLOCK at a time with no barrier between them (in-place relaxation is exact in
  // any interleaving); a block of passes in which no thread lowered any label read only final
  // labels, so the labels are the fixpoint.
  constexpr int FIX_BLOCK = 4;
  long long passes = 0;
  bool converged = false;
  const int* __restrict__ rrp = lrp;   // the CSR in LDS is never written during the passes
  const int* __restrict__ rcol = lcol;
  for (;;) {
    int changed = 0;
    for (int k = 0; k < FIX_BLOCK; ++k) {
      for (int v = tid; v < n; v += BT) {
        const int a0 = rrp[v], a1 = rrp[v + 1];
        const u64 p = P[v];
        u64 best = p;
        for (int a = a0; a < a1; ++a) {
          const u64 q = P[rcol[a]] + unit;
          best = q < best ? q : best;
        }
        if (best < p) {
          P[v] = best;
          changed = 1;
        }
      }
    }
    passes += FIX_BLOCK;
    converged = !__syncthreads_or(changed);
    if (converged || passes > (long long)n + 1 + FIX_BLOCK) break;
  }
  // centres, pieces, cut; the labels to the graph's label array
  const u64 mask = ((u64)1 << B) - 1;
  u64 cut2 = 0, pieces = 0;
  for (int v = tid; v < n; v += BT) {
    const u64 p = P[v];
    const int c = (int)(p & mask);
    j.centre[v] = c;
    j.P[v] = p;
    pieces += c == v;
    const int a1 = lrp[v + 1];
    for (int a = lrp[v]; a < a1; ++a) cut2 += (int)(P[lcol[a]] & mask) != c;
  }
  cut2 = block_sum64(cut2, sh);
  pieces = block_sum64(pieces, sh);
  if (tid == 0) {
    out->err = converged ? 0u : (unsigned)ERR_WATCHDOG;
    out->cut_arcs = cut2;
    out->pieces = pieces;
    out->delta = delta;
    out->n_active = n_active;
    out->rounds = passes;
    out->sweeps = 0;
    out->examined = (u64)passes * (u64)nnz;
  }
}

// ---- a team of workgroups on one graph ----------------------------------------------------

// Member 0 clears the words of the next step's slot before it arrives at this step's barrier:
// every member read them (as the slot of the step before last) before arriving at the last
// barrier, and the next step uses them only after this step's barrier (all threads call).
__device__ __forceinline__ void team_clear_next(BlockShared& sh) {
  if (sh.tm != 0) return;
  const int nx = (int)((sh.epoch + 1) % 3);
  const int ng = (sh.tK + TEAM_GROUP - 1) / TEAM_GROUP;
  if ((int)threadIdx.x < ng) __hip_atomic_store(&sh.ts->gw[nx][threadIdx.x].v, 0ull, __ATOMIC_RELAXED, AG);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&sh.ts->tw[nx].v, 0ull, __ATOMIC_RELAXED, AG);
    __hip_atomic_store(&sh.ts->qcnt[nx], 0ull, __ATOMIC_RELAXED, AG);
  }
}

// The team's barrier k (all threads call; k = sh.epoch, slot k % 3).  Every wave first waits for
// its own stores and atomics to complete (a workgroup barrier does not wait for other waves'
// stores to leave the CU).  Then thread 0 arrives, adding (1 << 42) | (error ? 1 << 32 : 0) | (its
// appends this step) to its group's word; the group's last arrival adds the group's sums to the
// team's word, and the team's last arrival publishes the step's queue length (the sum of the
// appends; 0xffffffff if any member had an error) with the barrier's number in gen, which the
// others wait for.  In a team of at most TEAM_GROUP members the arrivals go to the team's word
// directly.  full: arrivals are acquire-release read-modify-writes, gen a release store and the
// wait ends with an acquire, so every plain write of the members before the barrier is visible to
// plain loads after it (each member writes back and invalidates its L2).  Otherwise everything is
// relaxed: the members' shared accesses are device-scope themselves and complete before the
// arrival (the waits above), and every load after the barrier is issued after the wait observed
// gen.  A bounded wait raises ERR_BARRIER instead of hanging.  Returns the queue length; after an
// error every member ORs the team's error bits into sh.err.
template <bool FULL>
__device__ unsigned team_barrier(BlockShared& sh) {
  constexpr int RMW = FULL ? __ATOMIC_ACQ_REL : __ATOMIC_RELAXED;
  constexpr int PUB = FULL ? __ATOMIC_RELEASE : __ATOMIC_RELAXED;
  team_clear_next(sh);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    TeamSync* ts = sh.ts;
    const unsigned K = (unsigned)sh.tK, g = (unsigned)sh.tm / TEAM_GROUP;
    const unsigned ng = (K + TEAM_GROUP - 1) / TEAM_GROUP;
    const unsigned in_g = K - g * TEAM_GROUP < (unsigned)TEAM_GROUP ? K - g * TEAM_GROUP : (unsigned)TEAM_GROUP;
    const unsigned e1 = sh.epoch + 1;
    const int slot = (int)(sh.epoch % 3);
    if (sh.err) __hip_atomic_fetch_or(&ts->err, sh.err, __ATOMIC_RELAXED, AG);
    constexpr u64 ONE = 1ull << 42, SUMS = ONE - 1;
    const u64 mine = ONE | (sh.err ? 1ull << 32 : 0ull) | (u64)sh.tcount;
    bool last = false;
    u64 sum = 0;
    if (ng == 1) {
      const u64 old = __hip_atomic_fetch_add(&ts->tw[slot].v, mine, RMW, AG);
      last = (old >> 42) + 1 == K;
      sum = (old & SUMS) + (mine & SUMS);
    } else {
      const u64 old = __hip_atomic_fetch_add(&ts->gw[slot][g].v, mine, RMW, AG);
      if ((old >> 42) + 1 == in_g) {
        const u64 grp = ONE | ((old & SUMS) + (mine & SUMS));
        const u64 top = __hip_atomic_fetch_add(&ts->tw[slot].v, grp, RMW, AG);
        last = (top >> 42) + 1 == ng;
        sum = (top & SUMS) + (grp & SUMS);
      }
    }
    u64 word;
    if (last) {
      const unsigned nf = (sum >> 32) ? 0xffffffffu : (unsigned)sum;
      word = ((u64)nf << 32) | e1;
      __hip_atomic_store(&ts->gen, word, PUB, AG);
    } else {
      unsigned spins = 0;
      while ((unsigned)(word = __hip_atomic_load(&ts->gen, __ATOMIC_RELAXED, AG)) < e1) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 22)) {  // seconds: far beyond any round, or a member's late start
          __hip_atomic_fetch_or(&ts->err, (unsigned)ERR_BARRIER, __ATOMIC_RELAXED, AG);
          word = (u64)0xffffffffu << 32;
          break;
        }
      }
    }
    if (FULL) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    unsigned nf = (unsigned)(word >> 32);
    if (nf == 0xffffffffu) {
      const unsigned e = __hip_atomic_load(&ts->err, __ATOMIC_RELAXED, AG);
      sh.err |= e ? e : (unsigned)ERR_BARRIER;
      nf = 0;
    }
    sh.tnf = nf;
    sh.tcount = 0;
    sh.epoch = e1;
  }
  __syncthreads();
  return sh.tnf;
}

// End of a member's step: its staged appends go to the shared queue `next`, then the barrier,
// which returns the queue's length, the same in every member (all threads call).
template <bool FULL>
__device__ unsigned team_round_end(BlockShared& sh, int* next, u64* gcnt) {
  __syncthreads();
  const unsigned c = sh.bn < TB_CAP ? sh.bn : TB_CAP;
  if (c) team_flush(sh, next, gcnt, c);
  return team_barrier<FULL>(sh);
}

// Before plain loads of labels that other members wrote since the last full barrier: an acquire
// that invalidates this CU's L1 and its XCD's L2 (all threads call).
__device__ __forceinline__ void team_acquire() {
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
}

// The first non-empty wake bucket of the whole graph at or after r, from the bitmap sh.nz (D + n +
// 1 past the end, as next_nonempty; all threads call).
__device__ __forceinline__ int team_next_nonempty(BlockShared& sh, int r, int D) {
  __syncthreads();
  if (threadIdx.x == 0) sh.nxt = 0x7fffffff;
  __syncthreads();
  const int w = (int)threadIdx.x;
  if (w < BLOCK_WCAP / 64 && r < BLOCK_WCAP) {
    const int b0 = w * 64;
    u64 bits = sh.nz[w];
    if (b0 + 63 < r) bits = 0;
    else if (b0 < r) bits &= ~0ull << (r - b0);
    if (bits) atomicMin(&sh.nxt, b0 + __builtin_ctzll(bits));
  }
  __syncthreads();
  const int q = sh.nxt;
  __syncthreads();
  return q <= D ? q : 0x3fffffff;
}

// Team preparation: every member scans its slice (checks, labels INF, Delta and the vertices with
// arcs, combined by atomics in the team's record) and sorts its slice's wake buckets; the members'
// non-empty buckets are ORed into the record and read back after a second barrier.
__device__ __attribute__((noinline)) void team_prepare(const BlockJob& j, BlockShared& sh) {
  const int tid = threadIdx.x;
  TeamSync* ts = sh.ts;
  if (tid == 0) {
    sh.err = 0;
    sh.bn = 0;
  }
  __syncthreads();
  u64 dmax, active, degmax;
  prepare_scan(j, sh, sh.tlo, sh.thi, sh.tm == 0, &dmax, &active, &degmax);
  if (tid == 0) {
    if (j.deg_cap > 0 && degmax > (u64)j.deg_cap) __hip_atomic_fetch_max(&ts->maxdeg, degmax, __ATOMIC_RELAXED, AG);
    if (dmax) __hip_atomic_fetch_max(&ts->delta, dmax, __ATOMIC_RELAXED, AG);
    if (active) __hip_atomic_fetch_add(&ts->active, active, __ATOMIC_RELAXED, AG);
    if (sh.err) __hip_atomic_fetch_or(&ts->err, sh.err, __ATOMIC_RELAXED, AG);
  }
  team_barrier<true>(sh);
  const u64 delta = __hip_atomic_load(&ts->delta, __ATOMIC_RELAXED, AG);
  const u64 n_active = __hip_atomic_load(&ts->active, __ATOMIC_RELAXED, AG);
  unsigned e = __hip_atomic_load(&ts->err, __ATOMIC_RELAXED, AG);
  if (!e) e = range_err(j.n, delta);
  if (!e && __hip_atomic_load(&ts->maxdeg, __ATOMIC_RELAXED, AG)) e = BLK_SKEW;
  __syncthreads();
  if (tid == 0) {
    sh.err |= e;
    sh.delta = delta;
    sh.n_active = n_active;
  }
  __syncthreads();
  if (sh.err) return;
  wake_sort(j, sh, sh.tlo, sh.thi, delta);
  if (tid < BLOCK_WCAP / 64) {
    u64 bits = 0;
    for (int b = 0; b < 64; ++b) {
      const int q = tid * 64 + b;
      bits |= (u64)(sh.woff[q + 1] > sh.woff[q]) << b;
    }
    if (bits) __hip_atomic_fetch_or(&ts->nz[tid], bits, __ATOMIC_RELAXED, AG);
  }
  team_barrier<true>(sh);
  if (tid < BLOCK_WCAP / 64) sh.nz[tid] = __hip_atomic_load(&ts->nz[tid], __ATOMIC_RELAXED, AG);
  __syncthreads();
}

// The rounds of a team: the same rounds and tail as block_rounds, with labels at device scope,
// wakes from the member's slice, expansion of the member's K-th of the frontier, appends to the
// shared queue, and one barrier per round (or seed, or sweep), which returns the next frontier's
// length.
__device__ __attribute__((noinline)) void team_rounds(const BlockJob& j, BlockShared& sh) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  const long long* __restrict__ shift = j.shift;
  u64* P = j.P;
  TeamSync* ts = sh.ts;
  const int tid = threadIdx.x;
  const int K = sh.tK, m = sh.tm, lo = sh.tlo, hi = sh.thi;
  const u64 delta = sh.delta, n_active = sh.n_active;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const int D = (int)(delta >> FIX);
  const u64 unit = (u64)1 << (FIX + B);
  const u64 mask = ((u64)1 << B) - 1;
  int* cur = j.q0;
  int* nxt = j.q1;
  unsigned nf = 0;
  u64 settled = 0, examined = 0;
  long long rounds = 0, sweeps = 0;
  int r = team_next_nonempty(sh, 0, D);
  bool tail = false;
  while (settled < n_active && r <= D + n && rounds <= (long long)D + n + 2) {
    u64* gcnt = &ts->qcnt[sh.epoch % 3];
    const TeamAppend app{&sh, nxt, gcnt};
    if (r <= D) {
      const int w0 = sh.woff[r], w1 = sh.woff[r + 1];
      for (int i0 = w0; i0 < w1; i0 += BT) {  // the same passes in every thread (app.step)
        const int i = i0 + tid;
        if (i < w1) {
          const u64 self = j.wk[lo + i];
          const int v = (int)(self & mask);
          if (wg_load(&P[v]) > self && lab_min<AG>(&P[v], self) == INF) app(v);
        }
        app.step();
      }
    }
    const unsigned e0 = (unsigned)((u64)nf * m / K), e1 = (unsigned)((u64)nf * (m + 1) / K);
    examined += expand_frontier<AG, false>(j, sh, cur, e0, e1, unit, 0, app);
    nf = team_round_end<false>(sh, nxt, gcnt);
    if (sh.err) break;
    settled += nf;
    ++rounds;
    int* t = cur;
    cur = nxt;
    nxt = t;
    if (nf) ++r;
    else r = team_next_nonempty(sh, r + 1, D);
    const u64 left = n_active - settled;
    if (j.tail_den > 0 && left > 0 && left * (u64)j.tail_den <= n_active && D - r > TAIL_MIN_LEFT) {
      tail = true;
      break;
    }
  }
  if (tail && !sh.err) {
    // seed over the member's slice (see block_rounds), then sweeps over the shared queue
    u64* gcnt = &ts->qcnt[sh.epoch % 3];
    const TeamAppend app{&sh, nxt, gcnt};
    const u64 prev_round = (u64)(r - 1);
    team_acquire();
    for (int v0 = lo; v0 < hi; v0 += BT) {  // the same passes in every thread (app.step)
      const int v = v0 + tid;
      const int a0 = v < hi ? rp[v] : 0, a1 = v < hi ? rp[v + 1] : 0;
      if (a1 > a0 && wg_load(&P[v]) == INF) {
        u64 best = ((delta - (u64)shift[v]) << B) | (u64)v;
        for (int a = a0; a < a1; ++a) {
          const int u = col[a];
          if ((unsigned)u >= (unsigned)n) {
            atomicOr(&sh.err, ERR_BAD_COL);
            break;
          }
          const u64 pu = wg_load(&P[u]);
          if (pu != INF && (pu >> (FIX + B)) == prev_round && pu + unit < best) best = pu + unit;
        }
        examined += (u64)(a1 - a0);
        lab_store<AG>(&P[v], best);
        j.wake[v] = -1;  // the stamp of the first sweep
        app(v);
      }
      app.step();
    }
    nf = team_round_end<true>(sh, nxt, gcnt);
    int* t = cur;
    cur = nxt;
    nxt = t;
    for (int k = 1; nf && !sh.err && sweeps <= n; ++k) {
      gcnt = &ts->qcnt[sh.epoch % 3];
      const unsigned e0 = (unsigned)((u64)nf * m / K), e1 = (unsigned)((u64)nf * (m + 1) / K);
      examined += expand_frontier<AG, true>(j, sh, cur, e0, e1, unit, -(k + 1), TeamAppend{&sh, nxt, gcnt});
      nf = team_round_end<false>(sh, nxt, gcnt);
      ++sweeps;
      t = cur;
      cur = nxt;
      nxt = t;
    }
    settled = n_active;
  }
  __syncthreads();
  examined = block_sum64(examined, sh);
  if (tid == 0) {
    sh.settled = settled;
    sh.examined = examined;
    sh.rounds = rounds;
    sh.sweeps = sweeps;
  }
  __syncthreads();
}

// Centres and cut of the member's slice, summed in the team's record; after a last barrier,
// member 0 writes the graph's result.
__device__ __attribute__((noinline)) void team_output(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  TeamSync* ts = sh.ts;
  const int tid = threadIdx.x;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const u64 mask = ((u64)1 << B) - 1;
  const unsigned e0 = sh.err | (sh.settled < sh.n_active ? ERR_WATCHDOG : 0u);
  u64 cut2 = 0, pieces = 0;
  team_acquire();
  if (!e0) output_slice(j, sh, sh.tlo, sh.thi, mask, &cut2, &pieces);
  cut2 = block_sum64(cut2, sh);
  pieces = block_sum64(pieces, sh);
  __syncthreads();
  if (tid == 0) {
    if (cut2) __hip_atomic_fetch_add(&ts->cut, cut2, __ATOMIC_RELAXED, AG);
    if (pieces) __hip_atomic_fetch_add(&ts->pieces, pieces, __ATOMIC_RELAXED, AG);
    if (sh.examined) __hip_atomic_fetch_add(&ts->examined, sh.examined, __ATOMIC_RELAXED, AG);
    if (e0 | sh.err) __hip_atomic_fetch_or(&ts->err, e0 | sh.err, __ATOMIC_RELAXED, AG);
  }
  team_barrier<true>(sh);
  if (tid == 0 && sh.tm == 0) {
    out->err = __hip_atomic_load(&ts->err, __ATOMIC_RELAXED, AG) | sh.err;
    out->cut_arcs = __hip_atomic_load(&ts->cut, __ATOMIC_RELAXED, AG);
    out->pieces = __hip_atomic_load(&ts->pieces, __ATOMIC_RELAXED, AG);
    out->examined = __hip_atomic_load(&ts->examined, __ATOMIC_RELAXED, AG);
    out->delta = sh.delta;
    out->n_active = sh.n_active;
    out->rounds = sh.rounds;
    out->sweeps = sh.sweeps;
  }
}

// Member m of the graph's team: the slice of 64-aligned vertices it owns, then the three phases.
__device__ void team_graph(const BlockJob& j, BlockShared& sh, BlockOut* out, int m) {
  const int n = j.n, K = j.team;
  const int chunk = (int)((((long long)n + K - 1) / K + 63) & ~63ll);
  if (threadIdx.x == 0) {
    sh.ts = j.sync;
    sh.tK = K;
    sh.tm = m;
    sh.tlo = (int)min((long long)n, (long long)m * chunk);
    sh.thi = (int)min((long long)n, (long long)sh.tlo + chunk);
    sh.epoch = 0;
    sh.tcount = 0;
  }
  __syncthreads();
  team_prepare(j, sh);
  if (sh.err) {
    if (threadIdx.x == 0 && m == 0) {
      out->err = sh.err;
      out->delta = sh.delta;
    }
    return;
  }
  team_rounds(j, sh);
  team_output(j, sh, out);
}

}  // namespace

// (BT, 4): four waves per SIMD, one workgroup per CU, up to 128 VGPRs (at 64, the bound that two
// workgroups per CU would need, the team and round loops spilled to scratch).
// With a job list each workgroup takes the next job of `order` (a graph, or one member of a
// graph's team) from the shared counter until none is left; without one, block b runs member b of
// the single graph.
// A team's members are consecutive jobs: a member that starts early waits at the team's first
// barrier for workgroups that finish their current job, which every resident workgroup does, so
// the team size must not exceed the resident workgroups (the host keeps it within the grid).
__global__ __launch_bounds__(BT, 4) void k_block_decompose(const BlockJob* __restrict__ jobs,
                                                           const TeamJob* __restrict__ order, int njobs,
                                                           unsigned* next_job, BlockOut* outs, BlockJob single,
                                                           int lds_bytes) {
  __shared__ BlockShared sh;
  for (;;) {
    int g = 0, m = (int)blockIdx.x;
    if (order) {
      if (threadIdx.x == 0) sh.job = (int)atomicAdd(next_job, 1u);
      __syncthreads();
      const int k = sh.job;
      __syncthreads();
      if (k >= njobs) return;
      g = order[k].g;
      m = order[k].m;
    }
    const BlockJob& j = order ? jobs[g] : single;
    const u64 t0 = wall_clock64();
    if (j.team > 1) team_graph(j, sh, &outs[g], m);
    else if (fix_lds_bytes(j.n, j.nnz) <= lds_bytes) block_graph_fix(j, sh, &outs[g]);
    else if (rounds_lds_bytes(j.n) <= lds_bytes) block_graph_lds(j, sh, &outs[g]);
    else block_graph(j, sh, &outs[g]);
    if (threadIdx.x == 0 && m == 0) {
      outs[g].t_begin = t0;
      outs[g].t_end = wall_clock64();
    }
    if (!order) {
      // one graph: member 0 announces the result once every write of its workgroup (centres,
      // labels, the result record) has completed; the other members' writes completed before
      // they arrived at the team's last barrier
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0 && m == 0) {
        __threadfence_system();
        __hip_atomic_store(&outs[0].ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      return;
    }
    __syncthreads();
  }
}

// Per-graph job descriptors of a batch in one offset CSR (graph g's rows at row_ptr[vo[g] + g]);
// team[2 g] = graph g's team size, team[2 g + 1] its TeamSync.
__global__ void k_block_jobs(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const int* col, const long long* shift, int* centre, u64* P, int* wq, int tail_den,
                             const int* team, TeamSync* sync, BlockJob* jobs) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
    BlockJob j;
    const long long v0 = vo[g];
    j.n = (int)(vo[g + 1] - v0);
    j.nnz = ao[g + 1] - ao[g];
    j.row_ptr = row_ptr + v0 + g;
    j.col = col + ao[g];
    j.shift = shift + v0;
    j.centre = centre + v0;
    j.P = P + v0;
    j.wk = (u64*)wq + v0;
    j.wake = (int*)(j.wk);
    j.q0 = wq + 2 * N + v0;
    j.q1 = wq + 3 * N + v0;
    j.tail_den = tail_den;
    j.team = team ? team[2 * g] : 1;
    j.sync = j.team > 1 ? sync + team[2 * g + 1] : nullptr;
    j.deg_cap = 0;
    jobs[g] = j;
  }
}

}  // namespace ldd
