// Batched decomposition of many independent graphs packed into one offset CSR.
#include <hip/hip_runtime.h>

#include "../../include/ldd.h"
#include "ldd_internal.h"

ldd_status ldd_batch_union(int32_t G, const int64_t* vtx_off, const int64_t* arc_off, const int32_t* row_ptr,
                           const int32_t* col_idx, const int64_t* shift_fix, int32_t* centre, int64_t* cut_edges,
                           const ldd_options* opt, void* hip_stream);
ldd_status ldd_batch_workgroup(int32_t G, const int64_t* vtx_off, const int64_t* arc_off, const int32_t* row_ptr,
                               const int32_t* col_idx, const int64_t* shift_fix, int32_t* centre, int64_t* cut_edges,
                               const ldd_options* opt, void* hip_stream);
ldd_status ldd_batch_sequential(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off,
                                const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                                int32_t* centre, int64_t* cut_edges, const ldd_options* opt, void* hip_stream);

extern "C" ldd_status ldd_decompose_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off,
                                          const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                                          int32_t* centre, int64_t* cut_edges, const ldd_options* opt,
                                          void* hip_stream) {
  if (num_graphs < 0 || (num_graphs > 0 && (!vtx_off || !arc_off))) {
    ldd_set_error("bad batch descriptors");
    return LDD_ERR_INVALID_ARG;
  }
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (vtx_off[g + 1] < vtx_off[g] || arc_off[g + 1] < arc_off[g] || vtx_off[g + 1] - vtx_off[g] > INT32_MAX ||
        arc_off[g + 1] - arc_off[g] >= (1ll << 31)) {
      ldd_set_error("graph %d: offsets not monotone or too large", g);
      return LDD_ERR_INVALID_ARG;
    }
  }
  const int mode = opt ? opt->batch_mode : LDD_BATCH_AUTO;
  if (mode < LDD_BATCH_AUTO || mode > LDD_BATCH_WORKGROUP) {
    ldd_set_error("bad batch_mode %d", mode);
    return LDD_ERR_INVALID_ARG;
  }
  if (mode == LDD_BATCH_SEQUENTIAL)
    return ldd_batch_sequential(num_graphs, vtx_off, arc_off, row_ptr, col_idx, shift_fix, centre, cut_edges, opt,
                                hip_stream);
  if (mode == LDD_BATCH_UNION)
    return ldd_batch_union(num_graphs, vtx_off, arc_off, row_ptr, col_idx, shift_fix, centre, cut_edges, opt,
                           hip_stream);
  return ldd_batch_workgroup(num_graphs, vtx_off, arc_off, row_ptr, col_idx, shift_fix, centre, cut_edges, opt,
                             hip_stream);
}
