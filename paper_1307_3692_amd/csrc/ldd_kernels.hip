// HIP kernels of the exponential-shift low-diameter decomposition for gfx950.
//
// Pipeline for one graph (Sec. 5 of the paper: shortest paths from a super source whose
// arcs of length Delta - delta_u are added lazily, processed one integer distance at a time):
//   k_init          labels := INF, Delta := max shift (Algorithm 1 step 2), CSR bounds checks,
//                   per-block histogram of q = shift >> 20 and lists of the highest buckets
//   k_qbucket_scan  per bucket, offsets of the blocks' counts
//   k_qscan         bucket offsets and "next round that wakes anyone" links
//   k_place_window  the first window of buckets into the wake order (the round steps place
//                   lower buckets if the rounds reach them)
//   (shifts spanning QCAP units or more: k_wake_count / k_wake_scan / k_wake_scatter, a
//   counting sort by exact wake round w(u) = (Delta - shift_fix[u]) >> 20)
//   rounds          one step per round (ldd_rounds.hip): wake the round's vertices, expand
//                   F_{r-1} top-down (push) or bottom-up (pull), append first-reached vertices
//                   to F_r; a label-correcting tail once few vertices are left
//   k_finalize      centre = low B bits of the label (Algorithm 1 step 4)
//   k_cut           edges whose endpoints have different centres (Def. 1.1)
#include "ldd_device.h"
#include "ldd_kernels.h"

namespace ldd {

// ------------------------------------------------------------------------------------------
// prep
// ------------------------------------------------------------------------------------------
// Block-wide reductions for 256-thread blocks (one global atomic per block, not per wave:
// same-address atomics serialise at ~12 ns each).
// (any block size up to 1024 threads; red holds one entry per wave)
__device__ __forceinline__ u64 block_max(u64 v, u64* red) {
  v = wave_max_u64(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  u64 m = 0;
  for (unsigned w = 0; w < blockDim.x / WAVE; ++w) m = red[w] > m ? red[w] : m;
  return m;
}
__device__ __forceinline__ u64 block_sum(u64 v, u64* red) {
  v = wave_sum_u64(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  u64 t = 0;
  for (unsigned w = 0; w < blockDim.x / WAVE; ++w) t += red[w];
  return t;
}

// Pass A of the preparation.  Labels := INF, Delta := max shift (Algorithm 1 step 2),
// vertices with arcs, the highest-degree vertex, CSR and shift bounds checks -- and, since
// Delta is not known yet, a per-block LDS histogram of the integer part q = shift >> 20 of
// the vertices with arcs.  The wake round of u is D - q or D - q - 1 (D = Delta >> 20),
// depending on whether the fractional part of u's shift exceeds that of Delta, so q-buckets
// ordered by q give every round's wakers in two adjacent segments.
// Block b owns vertices [b n / G, (b+1) n / G); each wave takes 256 consecutive ones per
// pass (four per lane at stride 64, coalesced).  mat[q * G + b] = count of block b in bucket
// q for q <= qmax[b]; a q >= QCAP sets ctrl->wide and the sorted layout is not used.
//
// The first wake window.  Shifts are exponential, so the high buckets (the early rounds)
// hold few vertices and the low ones nearly all.  Each block lists the vertices of its
// highest buckets, as many whole buckets as fit in CAND entries, with their bucket:
// cand[b * CAND + i] = (q << 32) | v, bucket floor t_b.  Every block has listed all of its
// vertices in buckets >= place_lo = max_b t_b, so the preparation places exactly those
// buckets from the lists, without another pass over the shifts; the rest are placed by a
// round step only if the rounds get that far (isolated vertices are never placed: their label
// stays INF and the output maps it to the vertex itself).
constexpr int QL = 16384;  // vertices per block whose bucket is kept in LDS between the passes
constexpr unsigned short Q_NONE = 0xFFFF;

__global__ __launch_bounds__(1024, 8) void k_init(int n, long long nnz, const int* __restrict__ row_ptr,
                                              const long long* __restrict__ shift, u64* __restrict__ P,
                                              Ctrl* ctrl, unsigned* __restrict__ mat, int* __restrict__ qmax,
                                              u64* __restrict__ cand, unsigned* __restrict__ cand_cnt) {
  __shared__ unsigned h[QCAP];
  __shared__ unsigned short ql[QL];
  __shared__ u64 red[4][16];
  __shared__ int t_sh;
  __shared__ unsigned c_n;
  for (int i = threadIdx.x; i < QCAP; i += blockDim.x) h[i] = 0;
  if (threadIdx.x == 0) c_n = 0;
  __syncthreads();
  u64 mx = 0, hub = 0;
  unsigned active = 0, qm = 0, bad = 0, wide = 0;
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  const long long lo = (long long)n * blockIdx.x / gridDim.x, hi = (long long)n * (blockIdx.x + 1) / gridDim.x;
  for (long long base = lo + 256ll * wid; base < hi; base += 256ll * nw) {
    // all loads of the four vertices first (indices clamped into the block, so unconditional)
    long long sv[4];
    int av[4], bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long v = min(base + 64 * j + lane, hi - 1);
      sv[j] = shift[v];
      av[j] = row_ptr[v];
      bv[j] = row_ptr[v + 1];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long v = base + 64 * j + lane;
      if (v < hi) {
        const long long s = sv[j];
        const bool s_ok = s >= 0 && s <= (1ll << 52);
        if (!s_ok) bad |= ERR_BAD_SHIFT;
        else mx = (u64)s > mx ? (u64)s : mx;
        const int a = av[j], b = bv[j];
        if (a < 0 || b < a || (long long)b > nnz) bad |= ERR_BAD_ROWPTR;
        if (v == 0 && a != 0) bad |= ERR_BAD_ROWPTR;
        if (v == n - 1 && (long long)b != nnz) bad |= ERR_BAD_ROWPTR;
        active += (b > a);
        const u64 key = ((u64)(unsigned)(b - a) << 32) | (u64)v;  // degree, then id
        hub = key > hub ? key : hub;
        P[v] = INF;
        unsigned short qs = Q_NONE;
        if (b > a && s_ok) {
          const u64 q = (u64)s >> FIX;
          if (q < (u64)QCAP) {
            atomicAdd(&h[q], 1u);
            qm = (unsigned)q + 1 > qm ? (unsigned)q + 1 : qm;  // q + 1 so that 0 means "no vertex"
            qs = (unsigned short)q;
          } else {
            wide = 1;
          }
        }
        if (v - lo < QL) ql[v - lo] = qs;
      }
    }
  }
  mx = block_max(mx, red[0]);
  const u64 act = block_sum(active, red[1]);
  hub = block_max(hub, red[2]);
  qm = (unsigned)block_max(qm, red[3]);
  // bucket floor t_b: the lowest bucket such that buckets t_b .. qm - 1 hold at most CAND
  // vertices (wave 0 walks the histogram down from the top, 64 buckets at a time)
  if (wid == 0) {
    int t = 0;
    unsigned acc = 0;
    for (int top = (int)qm - 1; top >= 0; top -= WAVE) {
      const int q = top - (int)lane;
      const unsigned incl = acc + wave_incl_scan(q >= 0 ? h[q] : 0u);
      const u64 over = __ballot(incl > (unsigned)CAND);
      if (over) {  // wave-uniform
        t = top - (int)__builtin_ctzll(over) + 1;
        break;
      }
      acc = __shfl(incl, WAVE - 1, WAVE);
    }
    if (lane == 0) t_sh = t;
  }
  __syncthreads();
  const int tb = t_sh;
  u64* my_cand = cand + (size_t)blockIdx.x * CAND;
  auto list = [&](long long v, unsigned q) {
    if (q != Q_NONE && (int)q >= tb) {
      const unsigned idx = atomicAdd(&c_n, 1u);
      if (idx < (unsigned)CAND) my_cand[idx] = ((u64)q << 32) | (u64)v;
      else bad |= ERR_QUEUE;  // cannot happen: the buckets >= t_b hold at most CAND
    }
  };
  const long long hi_l = min(hi, lo + QL);
  for (long long v = lo + threadIdx.x; v < hi_l; v += blockDim.x) list(v, ql[v - lo]);
  for (long long v = hi_l + threadIdx.x; v < hi; v += blockDim.x) {  // blocks of more than QL vertices
    const long long s = shift[v];
    const bool keep = row_ptr[v + 1] > row_ptr[v] && s >= 0 && (u64)s < ((u64)QCAP << FIX);
    list(v, keep ? (unsigned)((u64)s >> FIX) : Q_NONE);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (mx) atomic_max_u64(&ctrl->delta, mx);
    if (act) atomic_add_u64(&ctrl->n_active, act);
    atomic_max_u64(&ctrl->hub, hub);
    qmax[blockIdx.x] = (int)qm - 1;
    cand_cnt[blockIdx.x] = c_n < (unsigned)CAND ? c_n : (unsigned)CAND;
    if (qm) __hip_atomic_fetch_max(&ctrl->place_lo, (unsigned)tb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (bad) atomic_or_u32(&ctrl->err, bad);
  if (wide) atomic_or_u32(&ctrl->wide, 1u);
  const unsigned G = gridDim.x;
  for (int q = threadIdx.x; q < (int)qm; q += blockDim.x) mat[(size_t)q * G + blockIdx.x] = h[q];
}

// The sorted (q-bucket) layout applies: valid input, every shift's integer part below QCAP.
// The kernels of that layout are enqueued before the host knows, and leave at once otherwise.
__device__ __forceinline__ bool qpath_ok(const Ctrl* ctrl) {
  return !(ctrl->err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) && !ctrl->wide &&
         (ctrl->delta >> FIX) < (u64)QCAP;
}

// One block per q-bucket (striding): exclusive scan of the per-block counts (in place) and
// the bucket's total.  G <= 1024 preparation blocks, at most four per thread.
__global__ __launch_bounds__(256) void k_qbucket_scan(int G, unsigned* __restrict__ mat, const int* __restrict__ qmax,
                                                      unsigned* __restrict__ tot, const Ctrl* __restrict__ ctrl) {
  __shared__ unsigned wsum[4];
  if (!qpath_ok(ctrl)) return;
  const int Qn = (int)(ctrl->delta >> FIX) + 1;
  const unsigned lane = lane_id(), wid = threadIdx.x / WAVE;
  const int per = (G + 255) / 256;
  const int b0 = (int)threadIdx.x * per;
  int qm[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) qm[i] = (i < per && b0 + i < G) ? qmax[b0 + i] : -1;
  for (int q = blockIdx.x; q < Qn; q += gridDim.x) {
    unsigned* row = mat + (size_t)q * G;
    unsigned x[4], sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[i] = q <= qm[i] ? row[b0 + i] : 0u;
      sum += x[i];
    }
    const unsigned incl = wave_incl_scan(sum);
    __syncthreads();  // the previous bucket's reads of wsum are done
    if (lane == WAVE - 1) wsum[wid] = incl;
    __syncthreads();
    unsigned acc = incl - sum, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (w < (int)wid) acc += wsum[w];
      total += wsum[w];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (q <= qm[i]) {
        row[b0 + i] = acc;
        acc += x[i];
      }
    if (threadIdx.x == 0) tot[q] = total;
  }
}

// One block: bucket offsets qoff[0..D+1] and, per round r (R = D + 1 rounds), the next round
// at or after r whose two q-buckets (D - r and D - r - 1) are not both empty.  Thread t takes
// a run of consecutive buckets (rounds); the runs' sums are combined by an exclusive prefix
// scan, their first non-empty rounds by a suffix minimum (wave shuffles, then across waves).
__global__ __launch_bounds__(1024) void k_qscan(const Ctrl* __restrict__ ctrl, const unsigned* __restrict__ tot,
                                                int* __restrict__ qoff, int* __restrict__ next_ne) {
  __shared__ unsigned w_sum[16];
  __shared__ int w_first[16];
  if (!qpath_ok(ctrl)) return;
  const int D = (int)(ctrl->delta >> FIX);
  const int Qn = D + 1, R = D + 1;
  const int t = threadIdx.x;
  const unsigned lane = lane_id(), wid = t / WAVE;
  const int per = (Qn + 1023) / 1024;
  const int lo = min(Qn, t * per), hi = min(Qn, lo + per);
  unsigned s = 0;
  int first = R;  // smallest round of this run that may wake someone
  for (int i = lo; i < hi; ++i) s += tot[i];
  for (int r = hi - 1; r >= lo; --r)
    if (tot[D - r] > 0 || (r < D && tot[D - r - 1] > 0)) first = r;
  const unsigned incl = wave_incl_scan(s);
  int suf = first;  // inclusive suffix minimum over the wave
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int y = __shfl_down(suf, o, WAVE);
    if (lane + (unsigned)o < (unsigned)WAVE) suf = y < suf ? y : suf;
  }
  if (lane == WAVE - 1) w_sum[wid] = incl;
  if (lane == 0) w_first[wid] = suf;
  __syncthreads();
  unsigned before = 0, total = 0;
  int after = R;
  for (int w = 0; w < 16; ++w) {
    if (w < (int)wid) before += w_sum[w];
    if (w > (int)wid) after = w_first[w] < after ? w_first[w] : after;
    total += w_sum[w];
  }
  const int next_in_wave = __shfl_down(suf, 1, WAVE);
  if (lane + 1 < (unsigned)WAVE) after = next_in_wave < after ? next_in_wave : after;
  unsigned acc = before + incl - s;
  for (int i = lo; i < hi; ++i) {
    qoff[i] = (int)acc;
    acc += tot[i];
  }
  int nx = after;
  for (int r = hi - 1; r >= lo; --r) {
    if (tot[D - r] > 0 || (r < D && tot[D - r - 1] > 0)) nx = r;
    next_ne[r] = nx;
  }
  if (t == 0) {
    qoff[Qn] = (int)total;
    next_ne[R] = R;
  }
}

// Places the first wake window, buckets [q_lo, D] (q_lo = place_lo), from the blocks'
// candidate lists.  A vertex's slot is its bucket's offset, plus the counts of the same bucket
// in earlier preparation blocks, plus its rank inside its own block (an LDS cursor per bucket).
__global__ __launch_bounds__(256) void k_place_window(const Ctrl* __restrict__ ctrl, const unsigned* __restrict__ mat,
                                                      const int* __restrict__ qmax, const int* __restrict__ qoff,
                                                      const u64* __restrict__ cand,
                                                      const unsigned* __restrict__ cand_cnt,
                                                      int* __restrict__ wake_ord) {
  __shared__ unsigned cur[QCAP];
  if (!qpath_ok(ctrl)) return;
  const int D = (int)(ctrl->delta >> FIX);
  const int q_lo = (int)ctrl->place_lo;
  if (q_lo > D) return;
  const unsigned G = gridDim.x;
  const int qm = min(qmax[blockIdx.x], D);
  for (int q = q_lo + (int)threadIdx.x; q <= qm; q += blockDim.x)
    cur[q - q_lo] = (unsigned)qoff[q] + mat[(size_t)q * G + blockIdx.x];
  __syncthreads();
  const unsigned cnt = cand_cnt[blockIdx.x];
  for (unsigned i = threadIdx.x; i < cnt; i += blockDim.x) {
    const u64 e = cand[(size_t)blockIdx.x * CAND + i];
    const int q = (int)(e >> 32);
    if (q >= q_lo && q <= qm) wake_ord[atomicAdd(&cur[q - q_lo], 1u)] = (int)(unsigned)e;
  }
}

// One block, after the preparation: decides whether the rounds run (ctrl->setup), writes the
// initial round state into both slots, clears the steps' queue counters and statistics, and
// writes the round kernels' argument block: the host's arguments completed with what only the
// device knows (Delta, the rounds bound, the vertices with arcs), first step 1.  When the rounds
// are not to run, both slots say "done" (enqueued steps return at once) and the report is written
// here.
__global__ void k_setup(RoundCtx c, LaunchBlock* lb, int qpath) {
  if (blockIdx.x != 0) return;
  for (int i = threadIdx.x; i < 3 * 16; i += blockDim.x) c.qcnt[i] = 0;
  for (int i = threadIdx.x; i < RT; i += blockDim.x) c.ex_part[i] = 0;
  if (threadIdx.x != 0) return;
  Ctrl* ctrl = c.ctrl;
  const u64 delta = ctrl->delta, n_active = ctrl->n_active;
  const u64 D = delta >> FIX;
  unsigned code = SETUP_OK;
  if (ctrl->err & (ERR_BAD_SHIFT | ERR_BAD_ROWPTR | ERR_BAD_COL)) code = SETUP_INVALID;
  else if (delta + ((u64)1 << FIX) >= ((u64)1 << (64 - c.B)) || D + 1 > ((u64)1 << 28)) code = SETUP_OVERFLOW;
  else if (qpath && (ctrl->wide || D >= (u64)QCAP)) code = SETUP_WIDE;
  else if (n_active == 0) code = SETUP_EMPTY;
  ctrl->setup = code;
  RoundState s0{};
  s0.seq = 0;
  s0.mode = code == SETUP_OK ? MODE_ROUNDS : MODE_DONE;
  s0.round = -1;
  s0.dir = DIR_TD;
  s0.unsettled_arcs = c.nnz;
  s0.tail_round = -1;
  s0.placed_lo = qpath ? (long long)(ctrl->place_lo < D + 1 ? ctrl->place_lo : D + 1) : 0;
  s0.flip = 0;
  c.st[0] = s0;
  s0.seq = -1;  // slot 1 stands for "step -1"
  c.st[1] = s0;
  c.delta = delta;
  c.R = code == SETUP_OK ? (int)(D + 1) : 0;
  c.n_active = n_active;
  lb->c = c;
  lb->kbase = 1;
  if (code != SETUP_OK && c.report) {
    Report* report = c.report;
    report->st = s0;
    report->delta = delta;
    report->n_active = n_active;
    report->err = ctrl->err;
    report->setup = code;
    __threadfence_system();  // the fields before the flag
    __hip_atomic_store(&report->ready, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Verification (proof of Theorem 1.1, Sec. 5): the largest distance from a vertex to its centre.
// A final label holds key(v) = Delta - shift[c] + 2^20 dist(c, v) and c = low B bits, so the
// distance is (key(v) - (Delta - shift[c])) >> 20 exactly; a label still INF (an isolated vertex,
// its own centre) has distance 0.  Block maxima are combined with one atomic per block into *out
// (cleared by the caller).
__global__ __launch_bounds__(256) void k_max_radius(int n, int B, const u64* __restrict__ P,
                                                    const long long* __restrict__ shift, u64 delta, u64* out) {
  __shared__ u64 red[256 / WAVE];
  u64 best = 0;
  const u64 mask = ((u64)1 << B) - 1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const u64 p = P[v];
    if (p == INF) continue;
    const u64 c = p & mask, key = p >> B;
    const u64 off = delta - (u64)shift[c];
    const u64 d = (key - off) >> FIX;
    best = d > best ? d : best;
  }
  best = wave_max_u64(best);
  if (lane_id() == 0) red[threadIdx.x / WAVE] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 m = 0;
    for (int w = 0; w < 256 / WAVE; ++w) m = red[w] > m ? red[w] : m;
    if (m) atomic_max_u64(out, m);
  }
}

// Single thread, after the cut: the output totals for the host.
__global__ void k_out_report(const Ctrl* ctrl, Report* report) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  report->cut_arcs = ctrl->cut_arcs;
  report->pieces = ctrl->pieces;
  report->unreached = ctrl->unreached;
  report->out_err = ctrl->err;
  __threadfence_system();
  __hip_atomic_store(&report->out_ready, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

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
// Centre of every vertex (Algorithm 1 step 4: the origin of its shortest path), plus one bit
// per vertex, "same centre as the highest-degree vertex" (piece H), and the list of vertices
// with arcs outside H together with the running prefix of their degrees.
//
// Every cut edge has an endpoint outside H, so the cut is found from those rows alone:
//   cut = #{arcs v->w : v not in H, w in H} + #{arcs v->w : v, w not in H, c(v) != c(w)} / 2
// (an edge with one endpoint in H is seen once; one with both outside is seen twice).  On
// graphs with one dominant piece that skips nearly every arc.
constexpr int FT = 512;      // threads per finalize block
constexpr int FBUF = 4096;   // LDS list buffer entries

// (FT, 6): at most 80 VGPRs, three 512-thread blocks per CU
__global__ __launch_bounds__(FT, 6) void k_finalize(int n, int B, const int* __restrict__ row_ptr,
                                                 const u64* __restrict__ P, int* __restrict__ centre,
                                                 u64* __restrict__ hub_bits, int* __restrict__ lv,
                                                 unsigned* __restrict__ la, Ctrl* ctrl) {
  __shared__ int b_vert[FBUF];
  __shared__ unsigned b_off[FBUF];
  __shared__ unsigned w_cnt[FT / WAVE], w_arcs[FT / WAVE];
  __shared__ unsigned b_n, b_arcs;
  __shared__ u64 b_base;
  __shared__ u64 red[2][FT / WAVE];
  // labels and rows are not to be trusted when the preparation refused the input; the list
  // stays empty and the cut kernel finds nothing to do
  if (ctrl->setup >= SETUP_INVALID) return;
  const u64 mask = ((u64)1 << B) - 1;
  const int hub = (int)(unsigned)ctrl->hub;
  // a label still INF belongs to an isolated vertex (never placed, never reached): its own centre
  const u64 p_hub = (hub >= 0 && hub < n) ? P[hub] : INF;
  const int hub_c = (hub >= 0 && hub < n) ? (p_hub == INF ? hub : (int)(p_hub & mask)) : -1;
  if (threadIdx.x == 0) {
    b_n = 0;
    b_arcs = 0;
  }
  u64 pieces = 0, unreached = 0;
  const unsigned wid = threadIdx.x / WAVE, lane = lane_id();
  // block chunk [lo, hi) of whole 64-vertex words; each wave takes 256 vertices per pass,
  // four per lane at stride 64, so that each ballot is one bitmap word
  const long long words = ((long long)n + 63) / 64;
  const long long lo = words * blockIdx.x / gridDim.x * 64, hi = min((long long)n, words * (blockIdx.x + 1) / gridDim.x * 64);
  for (long long base = lo; base < hi; base += 4 * FT) {
    bool want[4];
    unsigned deg[4];
    u64 pl[4];
    int a0[4], a1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // all loads first (indices clamped, so unconditional)
      const long long v = min(base + 256 * wid + 64 * j + lane, hi - 1);
      pl[j] = P[v];
      a0[j] = row_ptr[v];
      a1[j] = row_ptr[v + 1];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long v = base + 256 * wid + 64 * j + lane;
      bool in_hub = false;
      want[j] = false;
      deg[j] = 0;
      if (v < hi) {
        const u64 p = pl[j];
        const int cv = p == INF ? (int)v : (int)(p & mask);
        centre[v] = cv;
        pieces += (cv == (int)v);
        deg[j] = (unsigned)(a1[j] - a0[j]);
        unreached += (p == INF && deg[j] > 0);
        in_hub = cv == hub_c;
        want[j] = !in_hub && deg[j] > 0;
      }
      const u64 bits = __ballot(in_hub);
      const long long w0 = base + 256 * wid + 64 * j;
      if (lane == 0 && w0 < hi) hub_bits[w0 >> 6] = bits;
    }
    // a pass that lists nothing (most passes when one piece holds most rows) ends here
    if (!__syncthreads_or((int)(want[0] | want[1] | want[2] | want[3]))) continue;
    // list entries of this pass: per-wave counts over the four sub-tiles, then the block
    unsigned my_cnt[4], my_arcs[4], wc_tot = 0, wa_tot = 0;
    u64 m[4];
    unsigned incl[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      m[j] = __ballot(want[j]);
      incl[j] = wave_incl_scan(want[j] ? deg[j] : 0u);
      my_cnt[j] = wc_tot;   // entries of sub-tiles before j in this wave
      my_arcs[j] = wa_tot;
      wc_tot += (unsigned)__popcll(m[j]);
      wa_tot += __shfl(incl[j], WAVE - 1, WAVE);
    }
    if (lane == 0) {
      w_cnt[wid] = wc_tot;
      w_arcs[wid] = wa_tot;
    }
    __syncthreads();
    unsigned wc = 0, wa = 0, tc = 0, ta = 0;
    for (int w = 0; w < FT / WAVE; ++w) {
      if (w < (int)wid) {
        wc += w_cnt[w];
        wa += w_arcs[w];
      }
      tc += w_cnt[w];
      ta += w_arcs[w];
    }
    if (tc) {  // uniform
      if (b_n + tc > (unsigned)FBUF) {
        if (threadIdx.x == 0) b_base = atomic_add_u64(&ctrl->list_cnt, ((u64)b_n << 32) | b_arcs);
        __syncthreads();
        for (unsigned i = threadIdx.x; i < b_n; i += FT) {
          const unsigned idx = (unsigned)(b_base >> 32) + i;
          if (idx < (unsigned)n) {
            lv[idx] = b_vert[i];
            la[idx] = (unsigned)b_base + b_off[i];
          }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
          b_n = 0;
          b_arcs = 0;
        }
        __syncthreads();
      }
      const unsigned fill = b_n, fill_arcs = b_arcs;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (want[j]) {
          const unsigned idx = fill + wc + my_cnt[j] + rank_below(m[j]);
          b_vert[idx] = (int)(base + 256 * wid + 64 * j + lane);
          b_off[idx] = fill_arcs + wa + my_arcs[j] + incl[j] - deg[j];
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        b_n = fill + tc;
        b_arcs = fill_arcs + ta;
      }
    }
    __syncthreads();
  }
  if (b_n) {
    if (threadIdx.x == 0) b_base = atomic_add_u64(&ctrl->list_cnt, ((u64)b_n << 32) | b_arcs);
    __syncthreads();
    for (unsigned i = threadIdx.x; i < b_n; i += FT) {
      const unsigned idx = (unsigned)(b_base >> 32) + i;
      if (idx < (unsigned)n) {
        lv[idx] = b_vert[i];
        la[idx] = (unsigned)b_base + b_off[i];
      }
    }
  }
  pieces = wave_sum_u64(pieces);
  unreached = wave_sum_u64(unreached);
  __syncthreads();
  if (lane == 0) {
    red[0][wid] = pieces;
    red[1][wid] = unreached;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 p = 0, u = 0;
    for (int w = 0; w < FT / WAVE; ++w) {
      p += red[0][w];
      u += red[1][w];
    }
    if (p) atomic_add_u64(&ctrl->pieces, p);
    if (u) atomic_add_u64(&ctrl->unreached, u);
  }
}

__device__ __forceinline__ bool hub_bit(const u64* bits, int v) { return (bits[v >> 6] >> (v & 63)) & 1; }

// Per-graph cut totals (batch): lane contributions to graph g (g < 0: none), one atomic per
// wave when all of its contributions go to one graph.  Called by a converged wave.
__device__ __forceinline__ void cut_per_graph(u64* cut_g, int g, unsigned contrib) {
  const u64 any = __ballot(g >= 0);
  if (!any) return;
  const int leader = __ffsll((long long)any) - 1;
  const int g0 = __shfl(g, leader, WAVE);
  if (__all(g < 0 || g == g0)) {
    const u64 t = wave_sum_u64(g >= 0 ? contrib : 0);
    if ((int)lane_id() == leader) atomic_add_u64(&cut_g[g0], t);
  } else if (g >= 0) {
    atomic_add_u64(&cut_g[g], contrib);
  }
}

// Largest degree up to which the cut walks whole rows, one per thread, instead of splitting
// the listed rows' arcs evenly over the grid.
constexpr unsigned CUT_ROW_DEG = 64;

// Cut count over the rows outside H (see k_finalize).  When no degree exceeds CUT_ROW_DEG each
// thread walks whole rows (independent loads, no staging); otherwise the listed rows' arcs are
// split evenly over the grid and walked in tiles of 256 with the list entries staged in LDS.
__global__ __launch_bounds__(256) void k_cut(int n, const int* __restrict__ row_ptr, const int* __restrict__ col,
                                             const int* __restrict__ centre, const u64* __restrict__ hub_bits,
                                             const int* __restrict__ lv, const unsigned* __restrict__ la,
                                             Ctrl* ctrl, const int* __restrict__ gid, u64* __restrict__ cut_g) {
  constexpr int T = 256;
  __shared__ unsigned w_pre[T + 1];
  __shared__ int w_first[T + 1];
  __shared__ int w_c[T + 1];
  __shared__ unsigned s_start;
  __shared__ u64 red[16];
  const u64 lc = ctrl->list_cnt;
  const unsigned nl = min((unsigned)(lc >> 32), (unsigned)n), al = (unsigned)lc;
  const unsigned G = gridDim.x;
  const unsigned a_begin = (unsigned)(((u64)al * blockIdx.x) / G);
  const unsigned a_end = (unsigned)(((u64)al * (blockIdx.x + 1)) / G);
  u64 one_side = 0, both = 0;
  if ((unsigned)(ctrl->hub >> 32) <= CUT_ROW_DEG) {
    // every degree is small: rows one per thread, every row outside H (the listed rows)
    for (long long base = (long long)blockIdx.x * T; base < n; base += (long long)G * T) {
      const long long v = base + threadIdx.x;
      unsigned c1 = 0, c2 = 0;  // arcs to another piece outside H, arcs into H
      int g = -1;
      if (v < n && !hub_bit(hub_bits, (int)v)) {
        const int a0 = row_ptr[v], a1 = row_ptr[v + 1], cv = centre[v];
        // four arcs at a time: their column ids, then their hub bits and centres, so that
        // each group costs two dependent loads rather than each arc
        for (int a = a0; a < a1; a += 4) {
          int w[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) w[j] = a + j < a1 ? col[a + j] : -1;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool ok = (unsigned)w[j] < (unsigned)n;
            const u64 hb = ok ? hub_bits[w[j] >> 6] : 0;
            const int cw = ok ? centre[w[j]] : cv;
            if ((hb >> (w[j] & 63)) & 1) ++c2;
            else c1 += cw != cv ? 1u : 0u;
          }
        }
        if (cut_g && (c1 | c2)) g = gid[v];
      }
      one_side += c2;
      both += c1;
      if (cut_g) cut_per_graph(cut_g, g, 2 * c2 + c1);
    }
  } else if (a_begin < a_end) {
    if (threadIdx.x < WAVE) {
      const unsigned e = wave_search_le(la, nl, a_begin);
      if (threadIdx.x == 0) s_start = e;
    }
    __syncthreads();
    unsigned ent = s_start;
    for (unsigned tile = a_begin; tile < a_end; tile += T) {
      for (int kk = threadIdx.x; kk <= T; kk += T) {
        const unsigned e = ent + kk;
        if (e < nl) {
          const int v = lv[e];
          const bool ok = (unsigned)v < (unsigned)n;
          w_pre[kk] = la[e];
          w_first[kk] = ok ? row_ptr[v] : 0;
          w_c[kk] = ok ? centre[v] : -1;
        } else {
          w_pre[kk] = al;
          w_first[kk] = 0;
          w_c[kk] = -1;
        }
      }
      __syncthreads();
      const unsigned a = tile + threadIdx.x;
      unsigned contrib = 0;  // 2 per arc to H, 1 per two-sided cut arc
      int row = -1;
      if (a < a_end) {
        int lo = 0, hi = T;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_pre[mid] <= a) lo = mid;
          else hi = mid;
        }
        const unsigned j = a - w_pre[lo];
        if (j < w_pre[lo + 1] - w_pre[lo]) {
          const int w = col[(long long)w_first[lo] + j];
          if ((unsigned)w < (unsigned)n) {
            if (hub_bit(hub_bits, w)) contrib = 2;
            else contrib = centre[w] != w_c[lo] ? 1 : 0;
          }
          row = lv[ent + lo];
        }
      }
      if (contrib == 2) one_side += 1;
      else both += contrib;
      if (cut_g) cut_per_graph(cut_g, (contrib && row >= 0) ? gid[row] : -1, contrib);
      const unsigned next = tile + T;
      __syncthreads();
      if (threadIdx.x == 0) {
        int lo = 0, hi = T + 1;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (w_pre[mid] <= next) lo = mid;
          else hi = mid;
        }
        s_start = ent + lo;
      }
      __syncthreads();
      ent = s_start;
    }
  }
  // cut_arcs accumulates 2 per one-sided arc and 1 per two-sided arc: cut = cut_arcs / 2
  const u64 v = block_sum(2 * one_side + both, red);
  if (threadIdx.x == 0 && v) atomic_add_u64(&ctrl->cut_arcs, v);
}

// ------------------------------------------------------------------------------------------
// batch: the disjoint union of many graphs (packed CSR with local ids -> global ids)
// ------------------------------------------------------------------------------------------
// the last index g with off[g] <= x (graphs may be empty; the non-empty one containing x wins)
__device__ __forceinline__ int graph_of(const long long* __restrict__ off, int G, long long x) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The graph of positions that a thread visits in increasing order: one search for the first,
// then a walk over the offsets (amortised one comparison per position).
struct GraphCursor {
  int g = -1;
  long long next = 0;  // off[g + 1]
  __device__ __forceinline__ int at(const long long* __restrict__ off, int G, long long x) {
    if (g < 0) {
      g = graph_of(off, G, x);
      next = off[g + 1];
    }
    while (next <= x) next = off[++g + 1];
    return g;
  }
};

// Global row offsets and the graph of every vertex; per-graph max shift (one 128-byte line per
// graph, one atomic per wave when the wave lies in one graph); bounds checks of each graph.
__global__ __launch_bounds__(256) void k_batch_rows(int G, long long N, const long long* __restrict__ vo,
                                                    const long long* __restrict__ ao, const int* __restrict__ row_ptr,
                                                    const long long* __restrict__ shift, int* __restrict__ rp_out,
                                                    int* __restrict__ gid, u64* __restrict__ dg, Ctrl* ctrl) {
  unsigned bad = 0;
  const long long lo = N * blockIdx.x / gridDim.x, hi = N * (blockIdx.x + 1) / gridDim.x;
  GraphCursor cur;
  for (long long base = lo; base < hi; base += blockDim.x) {
    const long long v = base + threadIdx.x;
    int g = -1;
    u64 sv = 0;
    if (v < hi) {
      g = cur.at(vo, G, v);
      const long long lv = v - vo[g], ng = vo[g + 1] - vo[g], mg = ao[g + 1] - ao[g];
      const long long at = vo[g] + g + lv;
      const int a = row_ptr[at], b = row_ptr[at + 1];
      if (a < 0 || b < a || b > mg || (lv == 0 && a != 0) || (lv == ng - 1 && b != mg)) bad |= ERR_BAD_ROWPTR;
      rp_out[v] = (int)(ao[g] + a);
      if (v == N - 1) rp_out[N] = (int)ao[G];
      gid[v] = g;
      const long long s = shift[v];
      if (s < 0 || s > (1ll << 52)) bad |= ERR_BAD_SHIFT;
      else sv = (u64)s;
    }
    const u64 any = __ballot(g >= 0);
    if (any) {
      const int leader = __ffsll((long long)any) - 1;
      const int g0 = __shfl(g, leader, WAVE);
      if (__all(g < 0 || g == g0)) {
        const u64 m = wave_max_u64(sv);
        if ((int)lane_id() == leader) atomic_max_u64(&dg[(size_t)g0 * 16], m);
      } else if (g >= 0) {
        atomic_max_u64(&dg[(size_t)g * 16], sv);
      }
    }
  }
  if (bad) atomic_or_u32(&ctrl->err, bad);
}

// Column ids to global ids; out-of-range local ids are reported and replaced by the graph's
// first vertex so that no later access leaves the union.
__global__ __launch_bounds__(256) void k_batch_cols(int G, long long M, const long long* __restrict__ vo,
                                                    const long long* __restrict__ ao, const int* __restrict__ col,
                                                    int* __restrict__ col_out, Ctrl* ctrl) {
  unsigned bad = 0;
  const long long lo = M * blockIdx.x / gridDim.x, hi = M * (blockIdx.x + 1) / gridDim.x;
  GraphCursor cur;
  for (long long a = lo + threadIdx.x; a < hi; a += blockDim.x) {
    const int g = cur.at(ao, G, a);
    const int c = col[a];
    const long long ng = vo[g + 1] - vo[g];
    if (c < 0 || c >= ng) {
      bad = ERR_BAD_COL;
      col_out[a] = (int)vo[g];
    } else {
      col_out[a] = (int)(vo[g] + c);
    }
  }
  if (bad) atomic_or_u32(&ctrl->err, bad);
}

__global__ __launch_bounds__(1024) void k_batch_dmax(int G, u64* dg) {
  __shared__ u64 red[16];
  u64 m = 0;
  for (int g = threadIdx.x; g < G; g += blockDim.x) m = dg[(size_t)g * 16] > m ? dg[(size_t)g * 16] : m;
  m = block_max(m, red);
  if (threadIdx.x == 0) dg[(size_t)G * 16] = m;
}

// shift' = shift + (Delta_max - Delta_g): the union's offset Delta_max - shift' is Delta_g - shift
__global__ __launch_bounds__(256) void k_batch_shift(int G, long long N, const int* __restrict__ gid,
                                                     const long long* __restrict__ shift, const u64* __restrict__ dg,
                                                     long long* __restrict__ shift_out) {
  const u64 dmax = dg[(size_t)G * 16];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
    shift_out[v] = shift[v] + (long long)(dmax - dg[(size_t)gid[v] * 16]);
}

__global__ __launch_bounds__(256) void k_batch_localize(long long N, const int* __restrict__ gid,
                                                        const long long* __restrict__ vo, int* __restrict__ centre) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
    centre[v] -= (int)vo[gid[v]];
}

}  // namespace ldd
