// Kernel declarations, the argument block of the round kernels and the state they carry
// from one round to the next.
#pragma once
#include "ldd_device.h"

namespace ldd {

enum { DIR_TD = 1, DIR_BU = 2 };  // matches LDD_DIR_TOP_DOWN / LDD_DIR_BOTTOM_UP; 0 = auto
// MODE_PLACE: the step places the wake buckets [max(0, placed_lo - ABUF), placed_lo) that the
// next round needs (the preparation placed only the first window), then the rounds go on
enum { MODE_ROUNDS = 0, MODE_TAIL = 1, MODE_DONE = 2, MODE_PLACE = 3 };

constexpr int RT = 1024;    // threads per block of the round kernels (16 waves)
constexpr int ABUF = 4096;  // entries of a block's LDS append buffer

// State after round-kernel step k (k = 0 is the initial state written by the host).
// All fields are 64-bit so that the state can be copied field by field with coherent
// 64-bit loads and stores (kept in registers: no type punning, no scratch).
#define LDD_STATE_FIELDS(X)                                                                 \
  X(seq)            /* k */                                                                 \
  X(prev)           /* (count << 32 | arcs) of the queue step k consumes */                 \
  X(settled)        /* vertices with arcs settled by the rounds so far */                   \
  X(unsettled_arcs) /* arcs of vertices not settled by the rounds yet */                    \
  X(max_frontier)                                                                           \
  X(round)          /* rounds: the round step k processes; tail: the sweep index */         \
  X(mode)           /* MODE_* */                                                            \
  X(dir)            /* direction of the round step k processes */                           \
  X(rounds)         /* statistics */                                                        \
  X(td_rounds)                                                                              \
  X(bu_rounds)                                                                              \
  X(tail_iters)                                                                             \
  X(tail_round)     /* first round the tail replaced (-1: none) */                        \
  X(placed_lo)      /* wake buckets >= placed_lo are placed (q-layout) */                   \
  X(flip)           /* step k reads queue (k - 1 + flip) & 1 and writes (k + flip) & 1 */

struct RoundState {
#define LDD_DECL(f) long long f;
  LDD_STATE_FIELDS(LDD_DECL)
#undef LDD_DECL
};

// What the host reads at the end, in mapped host memory.  The step that finds the rounds done
// (or k_setup, when the rounds are not to run) writes the first part and then `ready`; the
// output pass writes the totals and then `out_ready`.
struct Report {
  RoundState st;
  u64 delta, n_active;
  unsigned err, setup;
  long long ready;
  u64 cut_arcs, pieces, unreached;
  unsigned out_err;
  long long out_ready;
  long long tail_hint;  // set by the step that starts the label-correcting tail
};

// Server mode: one admitted request per slot, in its own vertex range of the arena.
constexpr int MAX_SLOTS = 256;
// The request's CSR and shifts stay in the caller's device buffers (local ids); arena vertex
// vbeg + v is the request's vertex v.
struct SlotInfo {
  const int* rp;
  const int* col;
  const long long* shift;
  u64 delta;        // the request's max shift
  long long vbeg;   // first arena vertex of the slot
  long long r0;     // global round of the request's round 0
  long long nnz;
  int R;            // the request's rounds (its wake rounds are r0 .. r0 + R - 1)
  int wbase;        // its rows of wake_tab (bucket offsets, R + 1) and wake_cur (splits, R)
  int active;
  int n;            // the request's vertices
};
// Per-slot traversal state after step k (double-buffered by parity, like RoundState).
// A request runs rounds, then (once few of its vertices are left) one seed step and
// label-correcting sweeps, then is done: its labels are final.
enum { SM_ROUNDS = 0, SM_SEED = 1, SM_TAIL = 2, SM_DONE = 3 };
struct SlotState {
  long long ua;       // arcs of the request's vertices not settled yet
  long long dir;      // direction of the request's round in step k (DIR_TD / DIR_BU; 0 = TD)
  long long mode;     // SM_* in step k
  long long settled;  // vertices with arcs reached so far (rounds mode)
};
// Per-slot report the round step writes to mapped host memory: the step at whose start the
// request was found done (its labels final as of the step before).
struct SlotEnd {
  long long step;
};

// Everything a round step needs, passed by value.
struct RoundCtx {
  int n;
  int B;            // id bits
  int R;            // rounds bound: (Delta >> 20) + 1
  long long nnz;
  u64 delta;        // max shift
  u64 n_active;     // vertices with at least one arc
  const int* row_ptr;
  const int* col;
  const long long* shift;
  u64* P;           // labels
  int* qv[2];       // queues (double-buffered by step parity)
  unsigned* qa[2];  // arc prefix of each queue entry
  int* wake_ord;
  const int* wake_off;  // wake_q: q-bucket offsets [D + 2]; else round offsets [R + 1]
  const int* next_ne;
  int wake_q;           // 1: wake_ord is sorted by integer part of the shift (see k_init)
  int prep_blocks;      // wake_q: blocks of the preparation, whose per-bucket counts are
  const unsigned* mat;  //   mat[q * prep_blocks + b] (exclusive over blocks) for q <= qmax[b]
  const int* qmax;
  u64* qcnt;        // 3 counters, 16 u64 apart: step k appends to counter k % 3
  u64* lr_part;     // [2][G]: per-block minimum label written by a step (parity of k)
  unsigned* stamp;  // per vertex: last tail sweep that queued it, as stamp_base + sweep + 1
  unsigned stamp_base;  // every stamp left by earlier calls is <= stamp_base (no clearing per call)
  RoundState* st;   // [2]: state after step k lives in st[k & 1]
  Ctrl* ctrl;
  int dir_policy;   // 0 auto, DIR_TD, DIR_BU
  int td_to_bu;
  int bu_to_td;
  int tail_den;     // enter the tail once unsettled * tail_den <= n_active (0: never)
  int tail_min_left;  // ... and more than this many rounds remain
  Report* report;   // mapped host memory (may be null)
  u64* ex_part;     // [G]: arcs examined by each block over all steps (statistics)
  // server mode (k_round_step_srv): every step is the next global round for every slot; round
  // r's wakers are those of every slot's local round r - r0 in rounds mode; each slot has its
  // own mode and direction, and its frontier queued in its own vertex range of qv / qa
  const SlotInfo* slots;
  int nslots;
  const int* wake_tab;          // per slot: first wake_ord entry of each shift bucket q, then the total
  const u64* wake_cur;          // per slot: low half = end of bucket q's wakers of round D - q
  SlotState* sst;              // [2][MAX_SLOTS]
  u64* s_cnt;                  // [3][MAX_SLOTS]: (count << 32 | arcs) queued by step k, at k % 3
  u64* s_lr;                   // [3][MAX_SLOTS]: smallest label written by step k, at k % 3
  SlotEnd* s_end;              // [MAX_SLOTS], mapped host memory
  unsigned* slot_err;          // [MAX_SLOTS]: error bits of each request (a column id out of range)
};

// Arguments of graph-launched steps: step k = kbase + j of a chunk; k_advance moves kbase.
struct LaunchBlock {
  RoundCtx c;
  long long kbase;
};

__global__ void k_init(int n, long long nnz, const int* row_ptr, const long long* shift, u64* P, Ctrl* ctrl,
                       unsigned* mat, int* qmax, u64* cand, unsigned* cand_cnt);
__global__ void k_qbucket_scan(int G, unsigned* mat, const int* qmax, unsigned* tot, const Ctrl* ctrl);
__global__ void k_qscan(const Ctrl* ctrl, const unsigned* tot, int* qoff, int* next_ne);
__global__ void k_place_window(const Ctrl* ctrl, const unsigned* mat, const int* qmax, const int* qoff, const u64* cand,
                               const unsigned* cand_cnt, int* wake_ord);
__global__ void k_check_cols(int n, long long nnz, const int* col, Ctrl* ctrl);
__global__ void k_wake_count(int n, int B, const int* row_ptr, const long long* shift, const Ctrl* ctrl, u64* P,
                             unsigned* hist, int R, int use_lds);
__global__ void k_wake_scan(int R, const unsigned* hist, int* wake_off, int* cursor, int* next_ne);
__global__ void k_wake_scatter(int n, const int* row_ptr, const long long* shift, const Ctrl* ctrl, int* cursor,
                               int* wake_ord);
__global__ void k_fill_u64(u64* p, long long count, u64 value);
__global__ void k_round_step_lb(const LaunchBlock* lb, int j);
__global__ void k_round_step_srv(const LaunchBlock* lb, int j);
__global__ void k_advance(LaunchBlock* lb, int C);
__global__ void k_rounds_persistent(const LaunchBlock* lb);
__global__ void k_setup(RoundCtx c, LaunchBlock* lb, int qpath);
__global__ void k_out_report(const Ctrl* ctrl, Report* report);
__global__ void k_max_radius(int n, int B, const u64* P, const long long* shift, u64 delta, u64* out);
__global__ void k_finalize(int n, int B, const int* row_ptr, const u64* P, int* centre, u64* hub_bits, int* lv,
                           unsigned* la, Ctrl* ctrl);
__global__ void k_cut(int n, const int* row_ptr, const int* col, const int* centre, const u64* hub_bits, const int* lv,
                      const unsigned* la, Ctrl* ctrl, const int* gid, u64* cut_g);
// batch (disjoint union)
__global__ void k_batch_rows(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const long long* shift, int* rp_out, int* gid, u64* dg, Ctrl* ctrl);
__global__ void k_batch_cols(int G, long long M, const long long* vo, const long long* ao, const int* col, int* col_out,
                             Ctrl* ctrl);
__global__ void k_batch_dmax(int G, u64* dg);
__global__ void k_batch_shift(int G, long long N, const int* gid, const long long* shift, const u64* dg,
                              long long* shift_out);
__global__ void k_batch_localize(long long N, const int* gid, const long long* vo, int* centre);

}  // namespace ldd
