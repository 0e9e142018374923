// Autotuning of the engine and its mapping: the engine (one graph: launch, persistent, a team of
// workgroups, or one workgroup; a batch: workgroup engine or disjoint union), the grid size, the top-down /
// bottom-up switching thresholds, the tail threshold and, for the workgroup batch engine, the
// arcs per team member, searched one knob at a time (coordinate descent) by timing whole
// decompositions of the caller's inputs with HIP events.  Every candidate computes the
// same result (the labels are the unique lexicographic minimum whatever the schedule), so
// tuning trades nothing but time.  Results are cached per workload signature, in the process and
// optionally in a text file (one line per signature).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ldd.h"
#include "ldd_internal.h"

namespace {

struct Knobs {
  int mode;  // one graph: LDD_ENGINE_*; a batch: LDD_BATCH_*
  int blocks, td_to_bu, bu_to_td, tail, team_arcs;
};

// the workgroup engine and its teams take no direction thresholds (they run top-down only)
bool workgroup_mode(int G, const Knobs& k) {
  return G == 1 ? (k.mode == LDD_ENGINE_WORKGROUP || k.mode == LDD_ENGINE_TEAM)
                : (k.mode == LDD_BATCH_AUTO || k.mode == LDD_BATCH_WORKGROUP);
}

std::mutex g_mu;
std::map<std::string, std::pair<Knobs, float>> g_cache;

std::string signature(int G, long long n, long long nnz, int dev) {
  hipDeviceProp_t p{};
  (void)hipGetDeviceProperties(&p, dev);
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/cu%d/G%d/n%lld/nnz%lld", p.gcnArchName, p.multiProcessorCount, G, n, nnz);
  return buf;
}

bool file_lookup(const char* path, const std::string& key, Knobs* k, float* ms) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char name[300];
    Knobs x{};
    float t = 0;
    if (sscanf(line, "%299s %d %d %d %d %d %d %f", name, &x.mode, &x.blocks, &x.td_to_bu, &x.bu_to_td, &x.tail,
               &x.team_arcs, &t) == 8 &&
        key == name) {
      *k = x;  // the last line for a signature wins
      *ms = t;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void file_store(const char* path, const std::string& key, const Knobs& k, float ms) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %d %d %d %.4f\n", key.c_str(), k.mode, k.blocks, k.td_to_bu, k.bu_to_td, k.tail,
          k.team_arcs, ms);
  fclose(f);
}

ldd_options to_options(const ldd_options* base, int G, const Knobs& k) {
  ldd_options o{};
  if (base) o = *base;
  if (G == 1) o.engine = k.mode;
  else o.batch_mode = k.mode;
  o.team_arcs = k.team_arcs;
  o.blocks = k.blocks;
  o.td_to_bu = k.td_to_bu;
  o.bu_to_td = k.bu_to_td;
  o.tail_vertices = k.tail;
  return o;
}

}  // namespace

extern "C" ldd_status ldd_tune(int32_t num_graphs, const int64_t* vtx_off, const int64_t* arc_off,
                               const int32_t* row_ptr, const int32_t* col_idx, const int64_t* shift_fix,
                               int32_t* centre, const ldd_options* base, const char* cache_path,
                               ldd_options* best, ldd_tune_report* report, void* hip_stream) {
  if (num_graphs < 1 || !vtx_off || !arc_off || !best || !centre || !shift_fix || !row_ptr) {
    ldd_set_error("bad tuning arguments");
    return LDD_ERR_INVALID_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    ldd_set_error("no HIP device");
    return LDD_ERR_HIP;
  }
  int ncu = 0;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const long long n = vtx_off[num_graphs], nnz = arc_off[num_graphs];
  const std::string key = signature(num_graphs, n, nnz, dev);
  ldd_tune_report rep{};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    Knobs k{};
    float ms = 0;
    bool hit = false;
    if (it != g_cache.end()) {
      k = it->second.first;
      ms = it->second.second;
      hit = true;
    } else if (file_lookup(cache_path, key, &k, &ms)) {
      g_cache[key] = {k, ms};
      hit = true;
    }
    if (hit) {
      *best = to_options(base, num_graphs, k);
      rep.best_ms = ms;
      rep.from_cache = 1;
      if (report) *report = rep;
      return LDD_OK;
    }
  }
  const hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    ldd_set_error("event creation failed");
    return LDD_ERR_HIP;
  }
  ldd_status failure = LDD_OK;
  // one timed decomposition (median of three) with the given knobs
  auto measure = [&](const Knobs& k) -> float {
    const ldd_options o = to_options(base, num_graphs, k);
    float t[3];
    for (int i = 0; i < 3; ++i) {
      ldd_status s;
      (void)hipEventRecord(e0, st);
      if (num_graphs == 1) {
        ldd_csr g{(int32_t)n, (int64_t)nnz, row_ptr, col_idx};
        s = ldd_decompose(&g, shift_fix, 1.0, centre, nullptr, &o, nullptr, hip_stream);
      } else {
        s = ldd_decompose_batch(num_graphs, vtx_off, arc_off, row_ptr, col_idx, shift_fix, centre, nullptr, &o,
                                hip_stream);
      }
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      if (s != LDD_OK) {
        failure = s;
        return 1e30f;
      }
      (void)hipEventElapsedTime(&t[i], e0, e1);
      ++rep.runs;
    }
    std::sort(t, t + 3);
    return t[1];
  };
  const int mode0 = num_graphs == 1 ? (base ? base->engine : 0) : (base ? base->batch_mode : 0);
  const int blocks0 = num_graphs > 1 && (mode0 == LDD_BATCH_AUTO || mode0 == LDD_BATCH_WORKGROUP) ? ncu : 2 * ncu;
  Knobs cur{mode0,
            base && base->blocks ? base->blocks : blocks0,
            base && base->td_to_bu ? base->td_to_bu : 14,
            base && base->bu_to_td ? base->bu_to_td : 24,
            base && base->tail_vertices ? base->tail_vertices : 32,
            base ? base->team_arcs : 0};
  (void)measure(cur);  // warm-up (workspace growth, code loading)
  if (failure != LDD_OK) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return failure;
  }
  float cur_ms = measure(cur);
  rep.default_ms = cur_ms;
  // engines: one graph tries the workgroup engine only when it is small enough that one
  // workgroup could compete (at most 2^22 arcs); a batch tries both batch engines
  std::vector<int> modes;
  if (num_graphs == 1) {
    modes = {LDD_ENGINE_LAUNCH, LDD_ENGINE_PERSISTENT, LDD_ENGINE_TEAM};
    if (nnz <= (1ll << 22)) modes.push_back(LDD_ENGINE_WORKGROUP);
  } else {
    modes = {LDD_BATCH_WORKGROUP, LDD_BATCH_UNION};
  }
  // fewer than one per CU too: smaller teams, and persistent grids whose barriers cost less
  const std::vector<int> blocks = {std::max(1, ncu / 4), std::max(1, ncu / 2), std::max(1, 3 * ncu / 4), ncu,
                                   2 * ncu, 3 * ncu, 4 * ncu};
  const std::vector<int> td_to_bu = {6, 10, 14, 20, 30};
  const std::vector<int> bu_to_td = {12, 24, 48};
  const std::vector<int> tail = {16, 32, 64, 128, 256, -1};
  const std::vector<int> team = {-1, 1 << 16, 1 << 17, 1 << 18, 1 << 19, 0};
  constexpr int KNOBS = 6;
  for (int round = 0; round < 2 && failure == LDD_OK; ++round) {
    bool moved = false;
    for (int knob = 0; knob < KNOBS && failure == LDD_OK; ++knob) {
      const bool wg = workgroup_mode(num_graphs, cur);
      if ((knob == 2 || knob == 3) && wg) continue;        // no direction switching to tune
      if (knob == 5 && (!wg || num_graphs == 1)) continue;  // teams: the workgroup batch engine only
      const std::vector<int>& cand = knob == 0 ? modes : knob == 1 ? blocks : knob == 2 ? td_to_bu
                                   : knob == 3 ? bu_to_td : knob == 4 ? tail : team;
      for (int v : cand) {
        Knobs k = cur;
        int* field = knob == 0 ? &k.mode : knob == 1 ? &k.blocks : knob == 2 ? &k.td_to_bu : knob == 3 ? &k.bu_to_td
                   : knob == 4 ? &k.tail : &k.team_arcs;
        if (*field == v || (knob == 1 && v > 1024)) continue;
        *field = v;
        const float t = measure(k);
        if (t < cur_ms * 0.98f) {  // a clear win only
          cur = k;
          cur_ms = t;
          moved = true;
        }
      }
    }
    if (!moved) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (failure != LDD_OK) return failure;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = {cur, cur_ms};
    file_store(cache_path, key, cur, cur_ms);
  }
  *best = to_options(base, num_graphs, cur);
  rep.best_ms = cur_ms;
  if (report) *report = rep;
  return LDD_OK;
}
