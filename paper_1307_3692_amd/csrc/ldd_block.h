// The workgroup-owned engine (one workgroup, or a team of a few workgroups, runs every round of
// one graph): job and result records and the kernels.
#pragma once
#include "ldd_device.h"

namespace ldd {

// wake buckets a workgroup sorts in LDS: graphs whose shifts span this many units of distance
// or more (floor(Delta / 2^20) >= BLOCK_WCAP) are left to the multi-block engine
constexpr int BLOCK_WCAP = 4096;

// Dynamic LDS a launch of the workgroup engine may give each workgroup for a small graph run alone:
// when its labels and CSR fit (8 B per vertex, 4 B per row offset and per arc) the whole
// decomposition is a label-correcting iteration in LDS (block_graph_fix); else, when its labels,
// wake order and queues fit (24 B per vertex), the rounds run on them in LDS (block_graph_lds).
// Either way its labels are copied to the graph's label array at the end.
constexpr int BLOCK_LDS_BYTES = 116 * 1024;
__host__ __device__ constexpr long long fix_lds_bytes(long long n, long long nnz) { return 12 * n + 4 * nnz + 4; }
__host__ __device__ constexpr long long rounds_lds_bytes(long long n) { return 24 * n; }

// error bits of a workgroup job beyond ERR_*: the labels would not fit 64 bits; the shift range
// needs more wake buckets than the workgroup sorts; a team was asked to refuse a graph with a
// vertex of more than deg_cap arcs, and it has one
enum : unsigned { BLK_OVERFLOW = 64u, BLK_WIDE = 128u, BLK_SKEW = 256u };

// A graph too large for one workgroup runs on a team of K workgroups (all resident at once) that
// meet at a barrier in device memory once per round.  Per team, in device memory, zeroed before
// the launch: the barrier's words (below), the OR of the members' error bits, the append counters
// of the shared frontier queue, the preparation's and the output's sums, the largest degree found
// above deg_cap (0: none), and the OR of the members' non-empty wake buckets.  Its size does not
// depend on K.  A batch gives a team at most TEAM_MAX workgroups; one graph alone may take every
// resident workgroup.
constexpr int TEAM_MAX = 16;

constexpr int TEAM_GROUP = 16;   // barrier arrivals are counted per group of 16 members, then per group
constexpr int TEAM_GROUPS = 32;  // a team has at most TEAM_GROUP * TEAM_GROUPS = 512 members

struct TeamLine {
  alignas(128) u64 v;
};

// Barrier k of a team uses the words of slot k % 3; member 0 clears slot (k + 1) % 3 before it
// arrives at barrier k.  An arrival adds (1 << 42) | (error ? 1 << 32 : 0) | (its appends) to its
// group's word, the group's last arrival adds the group's sums (one arrival) to the team's word,
// and the team's last arrival publishes the step's queue length with the barrier's number in gen.
struct TeamSync {
  TeamLine gw[3][TEAM_GROUPS];  // per step slot: the groups' arrivals, errors and appends
  TeamLine tw[3];               // per step slot: the team's (arrivals are groups)
  alignas(128) u64 gen;         // (queue length, or 0xffffffff after an error) << 32 | barriers passed
  alignas(128) unsigned err;    // OR of every member's error bits
  alignas(128) u64 qcnt[3];     // per step slot: the shared queue's reservations
  alignas(128) u64 delta;
  alignas(128) u64 active;
  alignas(128) u64 cut, pieces, examined;
  alignas(128) u64 maxdeg;
  alignas(128) u64 nz[BLOCK_WCAP / 64];
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
  TeamSync* sync;        // team > 1: the team's barrier and counters
  int deg_cap;           // team > 1: refuse (BLK_SKEW) a graph with a vertex of more arcs (0: never)
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
  unsigned ready; // one graph without a job list: set last, at system scope (the host waits for it)
};

// One job of the kernel's list: graph g, member m of its team.
struct TeamJob {
  int g, m;
};

// order != NULL: workgroups take jobs (order[k], njobs of them) from *next_job; order == NULL: one
// job per workgroup, member blockIdx.x of the graph `single`.  lds_bytes: the launch's dynamic LDS
// per workgroup (0: none).
__global__ void k_block_decompose(const BlockJob* jobs, const TeamJob* order, int njobs, unsigned* next_job, BlockOut* outs,
                                  BlockJob single, int lds_bytes);
__global__ void k_block_jobs(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const int* col, const long long* shift, int* centre, u64* P, int* wq, int tail_den,
                             const int* team, TeamSync* sync, BlockJob* jobs);

}  // namespace ldd
