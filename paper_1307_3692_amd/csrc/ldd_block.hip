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
// A graph too large for one workgroup to finish in step with the rest of a batch runs on a team
// of K workgroups (K <= TEAM_MAX, all resident at once): member m owns a slice of the vertices
// (its preparation, wake buckets, tail seed and output) and one K-th of every frontier; each
// member appends what it reaches to a segment of its own, and the members meet once per round
// at a barrier in device memory where they exchange their segment lengths and error bits, so
// the next frontier is the concatenation of the K segments.  The labels are then shared by
// several CUs, so their loads and atomics take device scope.
#include "ldd_block.h"

namespace ldd {

namespace {

constexpr int BT = 1024;         // threads per workgroup
constexpr int BNW = BT / WAVE;   // waves per workgroup
constexpr int WPT = BLOCK_WCAP / BT;  // wake buckets per thread in the scans

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
  int par;                   // exchange buffer in use
  unsigned tpre[TEAM_MAX + 1];  // current frontier: exclusive prefix of the members' segment lengths
  u64 tv[TEAM_MAX][4];       // the members' values of the last exchange
  u64 nz[BLOCK_WCAP / 64];   // non-empty wake buckets of the whole graph
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
// need workgroup scope alone (all waves of a workgroup share one CU and its vector L1); a team's
// labels are shared by its members' CUs and take device scope.
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
  for (int v = lo + tid; v < hi; v += BT)
    if (rp[v + 1] > rp[v]) atomicAdd(&sh.woff[(int)((delta - (u64)shift[v]) >> FIX)], 1);
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
  for (int v = lo + tid; v < hi; v += BT) {
    if (rp[v + 1] > rp[v]) {
      const int q = (int)((delta - (u64)shift[v]) >> FIX);
      j.wk[lo + atomicAdd(&sh.woff[q], 1)] = ((delta - (u64)shift[v]) << B) | (u64)v;
    }
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
                                             u64* dmax_out, u64* active_out) {
  const int n = j.n;
  const long long nnz = j.nnz;
  const int* __restrict__ rp = j.row_ptr;
  const long long* __restrict__ shift = j.shift;
  u64* P = j.P;
  const int tid = threadIdx.x;
  unsigned err = 0;
  u64 dmax = 0, active = 0;
  if (ends && n > 0 && (rp[0] != 0 || (long long)rp[n] != nnz) && tid == 0) err |= ERR_BAD_ROWPTR;
  for (int v = lo + tid; v < hi; v += BT) {
    const long long s = shift[v];
    if (s < 0 || s > (1ll << 52)) err |= ERR_BAD_SHIFT;
    const int a0 = rp[v], a1 = rp[v + 1];
    if (a1 < a0) err |= ERR_BAD_ROWPTR;
    active += a1 > a0;
    dmax = (u64)s > dmax ? (u64)s : dmax;
    P[v] = INF;
  }
  if (err) atomicOr(&sh.err, err);
  *dmax_out = block_max64(dmax, sh);
  *active_out = block_sum64(active, sh);
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
template <int SC, bool SWEEP>
__device__ __forceinline__ void relax_chunk(const BlockJob& j, BlockShared& sh, int* next, unsigned ne,
                                            unsigned total, int tag, unsigned* cnt) {
  constexpr int U = 1;
  const int n = j.n;
  const long long nnz = j.nnz;
  const int* __restrict__ col = j.col;
  u64* P = j.P;
  const int top = ne > 1 ? 1 << (31 - __builtin_clz(ne - 1)) : 0;
  for (unsigned base = threadIdx.x; base < total; base += U * BT) {
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
      pw[k] = ok ? lab_load<SC>(&P[w[k]]) : 0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (pw[k] > off[k]) {
        const u64 old = lab_min<SC>(&P[w[k]], off[k]);
        if (SWEEP) {
          if (old > off[k] && __hip_atomic_exchange(&j.wake[w[k]], tag, __ATOMIC_RELAXED, SC) != tag)
            append(cnt, next, w[k]);
        } else if (old == INF) {
          append(cnt, next, w[k]);
        }
      }
    }
  }
}

// Relax the arcs of frontier entries [e0, e1), staged in LDS a chunk of BT entries at a time (all
// threads call).  Alone (TEAM false) the frontier is cur[0 ...]; in a team it is the concatenation
// of the members' segments, member s's at cur + s n with length tpre[s + 1] - tpre[s].
template <int SC, bool SWEEP, bool TEAM>
__device__ __forceinline__ u64 expand_frontier(const BlockJob& j, BlockShared& sh, const int* cur, unsigned e0,
                                               unsigned e1, int* next, u64 unit, int tag, unsigned* cnt) {
  const int* __restrict__ rp = j.row_ptr;
  u64 examined = 0;
  for (unsigned c0 = e0; c0 < e1; c0 += BT) {
    const unsigned e = c0 + threadIdx.x;
    unsigned deg = 0;
    if (e < e1) {
      int u;
      if (TEAM) {
        int s = 0;
        while (s + 1 < sh.tK && sh.tpre[s + 1] <= e) ++s;
        u = cur[(long long)s * j.n + (e - sh.tpre[s])];
      } else {
        u = cur[e];
      }
      const int a0 = rp[u], a1 = rp[u + 1];
      deg = (unsigned)(a1 - a0);
      sh.first[threadIdx.x] = a0;
      sh.offer[threadIdx.x] = lab_load<SC>(&j.P[u]) + unit;
    }
    unsigned total;
    const unsigned ex = block_excl_scan(deg, sh, &total);
    sh.pre[threadIdx.x] = ex;
    __syncthreads();
    examined += threadIdx.x == 0 ? total : 0;
    relax_chunk<SC, SWEEP>(j, sh, next, e1 - c0 < (unsigned)BT ? e1 - c0 : (unsigned)BT, total, tag, cnt);
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
    examined += expand_frontier<WG, false, false>(j, sh, cur, 0, nf, next, unit, 0, cnt);
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
      examined += expand_frontier<WG, true, false>(j, sh, cur, 0, nf, next, unit, -(k + 1), cnt);
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
__device__ __attribute__((noinline)) void block_output(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  u64* P = j.P;
  const int tid = threadIdx.x;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const u64 mask = ((u64)1 << B) - 1;
  const unsigned e0 = sh.err | (sh.settled < sh.n_active ? ERR_WATCHDOG : 0u);
  u64 cut2 = 0, pieces = 0;
  if (!e0) {
    for (int v = tid; v < n; v += BT) {
      const u64 p = wg_load(&P[v]);
      const int c = p == INF ? v : (int)(p & mask);
      j.centre[v] = c;
      pieces += c == v;
      for (int a = rp[v]; a < rp[v + 1]; ++a) {
        const int w = col[a];
        if ((unsigned)w >= (unsigned)n) {  // arcs of the last frontier were not read by a round
          atomicOr(&sh.err, ERR_BAD_COL);
          break;
        }
        const u64 pw = wg_load(&P[w]);
        const int cw = pw == INF ? w : (int)(pw & mask);
        cut2 += cw != c;
      }
    }
  }
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

// ---- a team of workgroups on one graph ----------------------------------------------------

// The team's barrier, with an exchange: every member publishes four values (workgroup-uniform:
// thread 0's are taken), and after the barrier every member holds all members' values in sh.tv
// (all threads call).  The arrival counter only grows; the values are double-buffered, so a
// member that leaves one exchange cannot overwrite values another member has yet to read (that
// member must arrive at the next barrier first).  The release on arrival and the acquire after
// the wait make every write of the members before the barrier (labels, segments, stamps) visible
// after it.  A bounded wait raises ERR_BARRIER instead of hanging.
__device__ void team_exchange(BlockShared& sh, u64 a, u64 b, u64 c, u64 d) {
  __syncthreads();
  if (threadIdx.x == 0) {
    TeamSync* ts = sh.ts;
    u64* r = &ts->red[sh.par][sh.tm][0];
    __hip_atomic_store(r + 0, a, __ATOMIC_RELAXED, AG);
    __hip_atomic_store(r + 1, b, __ATOMIC_RELAXED, AG);
    __hip_atomic_store(r + 2, c, __ATOMIC_RELAXED, AG);
    __hip_atomic_store(r + 3, d, __ATOMIC_RELAXED, AG);
    const unsigned target = (sh.epoch + 1) * (unsigned)sh.tK;
    __hip_atomic_fetch_add(&ts->arrive, 1u, __ATOMIC_RELEASE, AG);
    unsigned spins = 0;
    while (__hip_atomic_load(&ts->arrive, __ATOMIC_RELAXED, AG) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 26)) {
        sh.err |= ERR_BARRIER;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if ((int)threadIdx.x < 4 * sh.tK)
    sh.tv[threadIdx.x >> 2][threadIdx.x & 3] =
        __hip_atomic_load(&sh.ts->red[sh.par][0][0] + threadIdx.x, __ATOMIC_RELAXED, AG);
  __syncthreads();
  if (threadIdx.x == 0) {
    sh.epoch += 1;
    sh.par ^= 1;
  }
  __syncthreads();
}

// After an exchange of (segment length, -, error bits, -): the exclusive prefix of the segment
// lengths in sh.tpre, their total (returned) and the OR of the error bits (all threads call;
// uniform results).
__device__ __forceinline__ unsigned team_counts(BlockShared& sh, unsigned* err) {
  unsigned tot = 0, e = 0;
  for (int k = 0; k < sh.tK; ++k) {
    if (threadIdx.x == 0) sh.tpre[k] = tot;
    tot += (unsigned)sh.tv[k][0];
    e |= (unsigned)sh.tv[k][2];
  }
  if (threadIdx.x == 0) sh.tpre[sh.tK] = tot;
  *err = e;
  __syncthreads();
  return tot;
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

// Team preparation: every member scans its slice (checks, labels INF, Delta and the vertices
// with arcs, combined by an exchange) and sorts its slice's wake buckets; the members' non-empty
// buckets are combined into sh.nz by a second barrier.
__device__ __attribute__((noinline)) void team_prepare(const BlockJob& j, BlockShared& sh) {
  const int tid = threadIdx.x;
  if (tid == 0) sh.err = 0;
  __syncthreads();
  u64 dmax, active;
  prepare_scan(j, sh, sh.tlo, sh.thi, sh.tm == 0, &dmax, &active);
  team_exchange(sh, active, dmax, sh.err, 0);
  u64 n_active = 0, delta = 0;
  unsigned e = 0;
  for (int k = 0; k < sh.tK; ++k) {
    n_active += sh.tv[k][0];
    delta = sh.tv[k][1] > delta ? sh.tv[k][1] : delta;
    e |= (unsigned)sh.tv[k][2];
  }
  if (!e) e = range_err(j.n, delta);
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
    __hip_atomic_store(&sh.ts->nz[sh.tm][tid], bits, __ATOMIC_RELAXED, AG);
  }
  team_exchange(sh, 0, 0, 0, 0);
  if (tid < BLOCK_WCAP / 64) {
    u64 bits = 0;
    for (int k = 0; k < sh.tK; ++k) bits |= __hip_atomic_load(&sh.ts->nz[k][tid], __ATOMIC_RELAXED, AG);
    sh.nz[tid] = bits;
  }
  __syncthreads();
}

// The rounds of a team: the same rounds and tail as block_rounds, with labels at device scope,
// wakes from the member's slice, expansion of the member's K-th of the frontier, appends to the
// member's segment, and one exchange per round (or seed, or sweep) for the segment lengths.
__device__ __attribute__((noinline)) void team_rounds(const BlockJob& j, BlockShared& sh) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  const long long* __restrict__ shift = j.shift;
  u64* P = j.P;
  const int tid = threadIdx.x;
  const int K = sh.tK, m = sh.tm, lo = sh.tlo, hi = sh.thi;
  const u64 delta = sh.delta, n_active = sh.n_active;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const int D = (int)(delta >> FIX);
  const u64 unit = (u64)1 << (FIX + B);
  const u64 mask = ((u64)1 << B) - 1;
  int* cur = j.tq;
  int* nxt = j.tq + (long long)K * n;
  unsigned nf = 0, e = 0;
  u64 settled = 0, examined = 0;
  long long rounds = 0, sweeps = 0;
  int r = team_next_nonempty(sh, 0, D);
  bool tail = false;
  while (settled < n_active && r <= D + n && rounds <= (long long)D + n + 2) {
    __syncthreads();
    if (tid == 0) sh.cnt = 0;
    __syncthreads();
    int* mine = nxt + (long long)m * n;
    if (r <= D) {
      const int w0 = sh.woff[r], w1 = sh.woff[r + 1];
      for (int i = w0 + tid; i < w1; i += BT) {
        const u64 self = j.wk[lo + i];
        const int v = (int)(self & mask);
        if (lab_load<AG>(&P[v]) > self && lab_min<AG>(&P[v], self) == INF) append(&sh.cnt, mine, v);
      }
    }
    const unsigned e0 = (unsigned)((u64)nf * m / K), e1 = (unsigned)((u64)nf * (m + 1) / K);
    examined += expand_frontier<AG, false, true>(j, sh, cur, e0, e1, mine, unit, 0, &sh.cnt);
    __syncthreads();
    team_exchange(sh, sh.cnt, 0, sh.err, 0);
    nf = team_counts(sh, &e);
    if (e) break;
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
  if (tail && !e) {
    // seed over the member's slice (see block_rounds), then sweeps over the team's segments
    __syncthreads();
    if (tid == 0) sh.cnt = 0;
    __syncthreads();
    int* mine = nxt + (long long)m * n;
    const u64 prev_round = (u64)(r - 1);
    for (int v = lo + tid; v < hi; v += BT) {
      const int a0 = rp[v], a1 = rp[v + 1];
      if (a1 == a0 || lab_load<AG>(&P[v]) != INF) continue;
      u64 best = ((delta - (u64)shift[v]) << B) | (u64)v;
      for (int a = a0; a < a1; ++a) {
        const int u = col[a];
        if ((unsigned)u >= (unsigned)n) {
          atomicOr(&sh.err, ERR_BAD_COL);
          break;
        }
        const u64 pu = lab_load<AG>(&P[u]);
        if (pu != INF && (pu >> (FIX + B)) == prev_round && pu + unit < best) best = pu + unit;
      }
      examined += (u64)(a1 - a0);
      lab_store<AG>(&P[v], best);
      j.wake[v] = -1;  // the stamp of the first sweep
      append(&sh.cnt, mine, v);
    }
    __syncthreads();
    team_exchange(sh, sh.cnt, 0, sh.err, 0);
    nf = team_counts(sh, &e);
    int* t = cur;
    cur = nxt;
    nxt = t;
    for (int k = 1; nf && !e && sweeps <= n; ++k) {
      __syncthreads();
      if (tid == 0) sh.cnt = 0;
      __syncthreads();
      mine = nxt + (long long)m * n;
      const unsigned e0 = (unsigned)((u64)nf * m / K), e1 = (unsigned)((u64)nf * (m + 1) / K);
      examined += expand_frontier<AG, true, true>(j, sh, cur, e0, e1, mine, unit, -(k + 1), &sh.cnt);
      __syncthreads();
      team_exchange(sh, sh.cnt, 0, sh.err, 0);
      nf = team_counts(sh, &e);
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
    sh.err |= e;
    sh.settled = settled;
    sh.examined = examined;
    sh.rounds = rounds;
    sh.sweeps = sweeps;
  }
  __syncthreads();
}

// Centres and cut of the member's slice, summed over the team by a last exchange; member 0
// writes the graph's result.
__device__ __attribute__((noinline)) void team_output(const BlockJob& j, BlockShared& sh, BlockOut* out) {
  const int n = j.n;
  const int* __restrict__ rp = j.row_ptr;
  const int* __restrict__ col = j.col;
  u64* P = j.P;
  const int tid = threadIdx.x;
  const int B = n > 1 ? 32 - __builtin_clz((unsigned)(n - 1)) : 1;
  const u64 mask = ((u64)1 << B) - 1;
  const unsigned e0 = sh.err | (sh.settled < sh.n_active ? ERR_WATCHDOG : 0u);
  u64 cut2 = 0, pieces = 0;
  if (!e0) {
    for (int v = sh.tlo + tid; v < sh.thi; v += BT) {
      const u64 p = lab_load<AG>(&P[v]);
      const int c = p == INF ? v : (int)(p & mask);
      j.centre[v] = c;
      pieces += c == v;
      for (int a = rp[v]; a < rp[v + 1]; ++a) {
        const int w = col[a];
        if ((unsigned)w >= (unsigned)n) {
          atomicOr(&sh.err, ERR_BAD_COL);
          break;
        }
        const u64 pw = lab_load<AG>(&P[w]);
        const int cw = pw == INF ? w : (int)(pw & mask);
        cut2 += cw != c;
      }
    }
  }
  cut2 = block_sum64(cut2, sh);
  pieces = block_sum64(pieces, sh);
  __syncthreads();
  team_exchange(sh, cut2, pieces, e0 | sh.err, sh.examined);
  if (tid == 0 && sh.tm == 0) {
    u64 c = 0, p = 0, x = 0;
    unsigned e = 0;
    for (int k = 0; k < sh.tK; ++k) {
      c += sh.tv[k][0];
      p += sh.tv[k][1];
      e |= (unsigned)sh.tv[k][2];
      x += sh.tv[k][3];
    }
    out->err = e | sh.err;
    out->cut_arcs = c;
    out->pieces = p;
    out->delta = sh.delta;
    out->n_active = sh.n_active;
    out->rounds = sh.rounds;
    out->sweeps = sh.sweeps;
    out->examined = x;
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
    sh.par = 0;
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

// (BT, 8): eight waves per SIMD, two workgroups per CU (at most 64 VGPRs).
// Each workgroup takes the next job of `order` (a graph, or one member of a graph's team) from
// the shared counter until none is left.
// A team's members are consecutive jobs: a member that starts early waits at the team's first
// barrier for workgroups that finish their current job, which every resident workgroup does, so
// the team size must not exceed the resident workgroups (the host keeps it within the grid).
__global__ __launch_bounds__(BT, 8) void k_block_decompose(const BlockJob* __restrict__ jobs,
                                                           const TeamJob* __restrict__ order, int njobs,
                                                           unsigned* next_job, BlockOut* outs) {
  __shared__ BlockShared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.job = (int)atomicAdd(next_job, 1u);
    __syncthreads();
    const int k = sh.job;
    __syncthreads();
    if (k >= njobs) return;
    const int g = order ? order[k].g : k;
    const int m = order ? order[k].m : 0;
    const u64 t0 = wall_clock64();
    if (jobs[g].team > 1) team_graph(jobs[g], sh, &outs[g], m);
    else block_graph(jobs[g], sh, &outs[g]);
    if (threadIdx.x == 0 && m == 0) {
      outs[g].t_begin = t0;
      outs[g].t_end = wall_clock64();
    }
    __syncthreads();
  }
}

// Per-graph job descriptors of a batch in one offset CSR (graph g's rows at row_ptr[vo[g] + g]);
// team[2 g] = graph g's team size, team[2 g + 1] its TeamSync, tq_off[g] its segments in tq.
__global__ void k_block_jobs(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const int* col, const long long* shift, int* centre, u64* P, int* wq, int tail_den,
                             const int* team, TeamSync* sync, int* tq, const long long* tq_off, BlockJob* jobs) {
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
    j.tq = j.team > 1 ? tq + tq_off[g] : nullptr;
    jobs[g] = j;
  }
}

}  // namespace ldd
