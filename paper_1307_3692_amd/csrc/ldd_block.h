// The workgroup-owned engine (one workgroup runs every round of one graph): job and result
// records and the kernels.
#pragma once
#include "ldd_device.h"

namespace ldd {

// wake buckets a workgroup sorts in LDS: graphs whose shifts span this many units of distance
// or more (floor(Delta / 2^20) >= BLOCK_WCAP) are left to the multi-block engine
constexpr int BLOCK_WCAP = 4096;

// error bits of a workgroup job beyond ERR_*: the labels would not fit 64 bits; the shift range
// needs more wake buckets than the workgroup sorts
enum : unsigned { BLK_OVERFLOW = 64u, BLK_WIDE = 128u };

struct BlockJob {
  int n;
  long long nnz;
  const int* row_ptr;    // [n + 1]
  const int* col;        // [nnz], local ids
  const long long* shift;
  int* centre;           // OUT [n]
  u64* P;                // workspace [n]: labels
  int* wake;             // workspace [n]: vertices with arcs by wake round
  int* q0;               // workspace [n]: frontier queues
  int* q1;
  int tail_den;          // label-correcting tail once unreached * tail_den <= vertices with arcs (0: never)
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

__global__ void k_block_decompose(const BlockJob* jobs, const int* order, int njobs, unsigned* next_job, BlockOut* outs);
__global__ void k_block_jobs(int G, long long N, const long long* vo, const long long* ao, const int* row_ptr,
                             const int* col, const long long* shift, int* centre, u64* P, int* wq, int tail_den,
                             BlockJob* jobs);

}  // namespace ldd
