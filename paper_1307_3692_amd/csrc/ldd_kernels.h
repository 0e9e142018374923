// Kernel declarations, the argument block of the round kernels and the state they carry
// from one round to the next.
#pragma once
#include "ldd_device.h"

namespace ldd {

enum { DIR_TD = 1, DIR_BU = 2 };  // matches LDD_DIR_TOP_DOWN / LDD_DIR_BOTTOM_UP; 0 = auto
enum { MODE_ROUNDS = 0, MODE_TAIL = 1, MODE_DONE = 2 };

constexpr int RT = 1024;    // threads per block of the round kernels (16 waves)
constexpr int ABUF = 4096;  // entries of a block's LDS append buffer

// State after round-kernel step k (k = 0 is the initial state written by the host).
struct RoundState {
  u64 seq;             // k
  u64 prev;            // (count << 32 | arcs) of the queue step k consumes
  u64 settled;         // vertices with arcs settled by the rounds so far
  u64 unsettled_arcs;  // arcs of vertices not settled by the rounds yet
  u64 max_frontier;
  int round;           // rounds: the round step k processes; tail: the sweep index
  int mode;            // MODE_*
  int dir;             // direction of the round step k processes
  int rounds;          // statistics
  int td_rounds;
  int bu_rounds;
  int tail_iters;
  int tail_round;      // first round the tail replaced (-1: none)
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
  const int* wake_ord;
  const int* wake_off;
  const int* next_ne;
  u64* qcnt;        // 3 counters, 16 u64 apart: step k appends to counter k % 3
  u64* lr_part;     // [2][G]: per-block minimum label written by a step (parity of k)
  unsigned* stamp;  // per vertex: last tail sweep that queued it
  RoundState* st;   // [2]: state after step k lives in st[k & 1]
  Ctrl* ctrl;
  int dir_policy;   // 0 auto, DIR_TD, DIR_BU
  int td_to_bu;
  int bu_to_td;
  int tail_den;     // enter the tail once unsettled * tail_den <= n_active (0: never)
  int tail_min_left;  // ... and more than this many rounds remain
};

__global__ void k_init(int n, long long nnz, const int* row_ptr, const long long* shift, u64* P, Ctrl* ctrl);
__global__ void k_check_cols(int n, long long nnz, const int* col, Ctrl* ctrl);
__global__ void k_wake_count(int n, int B, const int* row_ptr, const long long* shift, const Ctrl* ctrl, u64* P,
                             unsigned* hist, int R, int use_lds);
__global__ void k_wake_scan(int R, const unsigned* hist, int* wake_off, int* cursor, int* next_ne);
__global__ void k_wake_scatter(int n, const int* row_ptr, const long long* shift, const Ctrl* ctrl, int* cursor,
                               int* wake_ord);
__global__ void k_fill_u64(u64* p, long long count, u64 value);
__global__ void k_round_step(RoundCtx c, int k);
__global__ void k_rounds_persistent(RoundCtx c);
__global__ void k_finalize(int n, int B, const u64* P, int* centre, Ctrl* ctrl);
__global__ void k_cut(int n, long long nnz, const int* row_ptr, const int* col, const int* centre, Ctrl* ctrl);

}  // namespace ldd
