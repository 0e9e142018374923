// The workgroup-owned engine (one workgroup, or a team of a few workgroups, runs every round of
// one graph): job and result records and the kernels.
#pragma once
#include "ldd_device.h"

namespace ldd {

// wake buckets a workgroup sorts in LDS: graphs whose shifts span this many units of distance
// or more (floor(Delta / 2^20) >= BLOCK_WCAP) are left to the multi-block engine
constexpr int BLOCK_WCAP = 4096;

// error bits of a workgroup job beyond ERR_*: the labels would not fit 64 bits; the shift range
// needs more wake buckets than the workgroup sorts
enum : unsigned { BLK_OVERFLOW = 64u, BLK_WIDE = 128u };

// A large graph of a batch runs on a team of K <= TEAM_MAX workgroups that meet at a barrier
// once per round.  Per team, in device memory, zeroed before the launch: the barrier's arrival
// counter, each member's values for the round's exchange (double-buffered), and each member's
// non-empty wake buckets.
constexpr int TEAM_MAX = 16;

struct TeamSync {
  alignas(128) unsigned arrive;
  alignas(128) u64 red[2][TEAM_MAX][4];
  u64 nz[TEAM_MAX][BLOCK_WCAP / 64];
};

struct BlockJob {
  int n;
  long long nnz;
  const int* row_ptr;    // [n + 1]
  const int* col;        // [nnz], local ids
  const long long* shift;
  int* centre;           // OUT [n]
  u64* P;                // workspace [n]: labels
  u64* wk;               // workspace [n]: own labels of the vertices with arcs, by wake round
  int* wake;             // the first 4n bytes of wk: the tail's sweep stamps (once no wake is left)
  int* q0;               // workspace [n]: frontier queues
  int* q1;
  int tail_den;          // label-correcting tail once unreached * tail_den <= vertices with arcs (0: never)
  int team;              // workgroups on this graph (1: alone)
  TeamSync* sync;        // team > 1: the team's barrier and exchange area
  int* tq;               // team > 1: workspace [2 * team * n]: two sets of per-member frontier segments
};

struct BlockOut {
  unsigned err;
  u64 cut_arcs;   // arcs whose ends have different centres (twice the cut)
  u64 pieces;
  u64 delta;
  u64 n_active;
  long long rounds;
  long long sweeps;  // label-correcting sweeps of the tail (0: the rounds ran to the end)
  u64 examined;   // arcs read by the rounds, the seed and the sweeps
  u64 t_begin;    // device wall clock (constant-rate counter) when the workgroup took the graph
  u64 t_end;      // ... and when it finished it
};

// One job of the kernel's list: graph g, member m of its team.
struct TeamJob {
  int g, m;
};

__global__ void k_block_decompose(const BlockJob* jobs, const TeamJob* order, int njobs, unsigned* next_job, BlockOut* outs);
__global__ void k_block_jobs(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const int* col, const long long* shift, int* centre, u64* P, int* wq, int tail_den,
                             const int* team, TeamSync* sync, int* tq, const long long* tq_off, BlockJob* jobs);

}  // namespace ldd
