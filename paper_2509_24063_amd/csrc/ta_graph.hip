// ta_graph.hip -- one exchange iteration as a unit: run it, capture it in a
// HIP graph, and tune its launch shapes.
//
// An iteration is the four batched calls over every partition and segment
// (select, serialize, encode, decode), each a fixed sequence of grid-stride
// kernels whose sizes live on the device.  Captured once, it replays as one
// graph launch per iteration; a caller that alternates two reference
// buffers captures two graphs (A -> B and B -> A).
//
// ta_tune times the iteration under candidate grids for each kernel family
// (coordinate descent over 1, 2, 4, 8, 16 blocks per compute unit) and keeps
// the fastest; results are cached per device and workload shape in a text
// file: one line "arch cus key g_select g_serialize g_encode g_decode".
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ta_internal.hpp"
#include "ta_scratch.hpp"

using namespace ta;

struct ta_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

ta_status run(ta_ctx* c, const ta_iteration* it, void* stream) {
  ta_status st = ta_select_aura(c, it->agents, it->P, it->part_off, it->boxes, it->w, it->ndirs, it->idx,
                                it->idx_cap, it->seg_off, stream);
  if (st) return st;
  const int64_t nseg = (int64_t)it->P * it->ndirs;
  st = ta_serialize(c, it->agents, it->idx, it->seg_off, nseg, it->idx_cap, it->msgs, it->msgs_cap, it->msg_off,
                    it->msg_keys, it->msg_keys ? it->keys_cap : 0, stream);
  if (st) return st;
  const ta_keys tk{it->msg_keys, it->ref_keys, it->newref_keys, it->newref_keys ? it->keys_cap : 0};
  const bool tx_keys = it->msg_keys || it->ref_keys || it->newref_keys;
  st = ta_delta_encode(c, nseg, it->msgs, it->msgs_cap, it->msg_off, it->ref, it->ref_len, it->ref_off, it->pred,
                       it->hist_in, it->hist_out, it->enc, it->enc_cap, it->enc_off, it->newref, it->newref_cap,
                       it->newref_off, it->modes, tx_keys ? &tk : nullptr, stream);
  if (st) return st;
  if (!it->rx_out) return TA_OK;
  const ta_keys rk{nullptr, it->rx_ref_keys, it->rx_out_keys, it->rx_out_keys ? it->keys_cap : 0};
  const bool rx_keys = it->rx_ref_keys || it->rx_out_keys;
  return ta_delta_decode(c, nseg, it->enc, it->enc_cap, it->enc_off, it->rx_ref, it->rx_ref_len, it->rx_ref_off,
                         it->pred, it->rx_hist_in, it->rx_hist_out, it->rx_out, it->rx_out_cap, it->rx_out_off,
                         rx_keys ? &rk : nullptr, stream);
}

// Size the scratch memory for every call of the iteration (so that a
// capture allocates nothing).
ta_status presize(ta_ctx* c, const ta_iteration* it) {
  const int64_t nseg = (int64_t)it->P * it->ndirs;
  int64_t tiles = 0, t;
  size_t need = select_scratch(it->agents->n, it->P, it->ndirs, &t);
  tiles = std::max(tiles, t);
  need = std::max(need, serialize_scratch(nseg, it->idx_cap, &t));
  tiles = std::max(tiles, t);
  need = std::max(need, encode_scratch(nseg, it->msgs_cap, it->ref_len, c->rec_cap, it->pred != nullptr, &t));
  tiles = std::max(tiles, t);
  if (it->rx_out) {
    need = std::max(need, decode_scratch(nseg, it->enc_cap, it->rx_ref_len, it->rx_out_cap, c->rec_cap, it->pred != nullptr,
                                          &t));
    tiles = std::max(tiles, t);
  }
  return ensure_scratch(c, need, tiles);
}

bool valid(const ta_ctx* c, const ta_iteration* it) {
  return c && it && it->agents && it->P >= 1 && (it->ndirs == 6 || it->ndirs == 26);
}

std::string arch_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  for (auto& ch : s)
    if (ch == ' ') ch = '_';
  return s;
}

std::string shape_key(const ta_iteration* it) {
  auto lg = [](int64_t v) { return v > 0 ? (int)ceil(log2((double)v)) : 0; };
  char buf[160];
  snprintf(buf, sizeof buf, "P%d_d%d_n%d_m%d_r%d_p%d", it->P, it->ndirs, lg(it->agents->n), lg(it->msgs_cap),
           lg(it->ref_len), it->pred ? 1 : 0);
  return buf;
}

bool cache_read(const char* path, const std::string& arch, int cus, const std::string& key, int* g) {
  if (!path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char a[128], k[160];
  int cu, v[N_FAMILIES];
  bool found = false;
  while (fscanf(f, "%127s %d %159s %d %d %d %d", a, &cu, k, &v[0], &v[1], &v[2], &v[3]) == 7) {
    if (arch == a && cu == cus && key == k) {
      bool ok = true;
      for (int i = 0; i < N_FAMILIES; ++i) ok = ok && v[i] >= 1 && v[i] <= (1 << 20);
      if (ok) {
        for (int i = 0; i < N_FAMILIES; ++i) g[i] = v[i];
        found = true;  // the last matching line wins
      }
    }
  }
  fclose(f);
  return found;
}

void cache_append(const char* path, const std::string& arch, int cus, const std::string& key, const int* g) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %s %d %d %d %d\n", arch.c_str(), cus, key.c_str(), g[0], g[1], g[2], g[3]);
  fclose(f);
}

// Median of `reps` timed runs (after one warm-up run), in milliseconds.
ta_status time_iteration(ta_ctx* c, const ta_iteration* it, hipStream_t s, int reps, double* ms) {
  hipEvent_t a, b;
  TA_HIP(hipEventCreate(&a));
  TA_HIP(hipEventCreate(&b));
  std::vector<double> v;
  ta_status st = run(c, it, s);
  for (int r = 0; r < reps && !st; ++r) {
    if (hipEventRecord(a, s) != hipSuccess) st = TA_ERR_HIP;
    if (!st) st = run(c, it, s);
    if (!st && hipEventRecord(b, s) != hipSuccess) st = TA_ERR_HIP;
    if (!st && hipEventSynchronize(b) != hipSuccess) st = TA_ERR_HIP;
    float t = 0;
    if (!st && hipEventElapsedTime(&t, a, b) != hipSuccess) st = TA_ERR_HIP;
    v.push_back(t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st;
  std::sort(v.begin(), v.end());
  *ms = v[v.size() / 2];
  return TA_OK;
}

}  // namespace

extern "C" ta_status ta_iteration_run(ta_ctx* c, const ta_iteration* it, void* stream) {
  if (!valid(c, it)) return TA_ERR_INVALID;
  return run(c, it, stream);
}

extern "C" ta_status ta_graph_capture(ta_ctx* c, const ta_iteration* it, void* stream, ta_graph** out) {
  if (!valid(c, it) || !out || !stream) return TA_ERR_INVALID;
  ta_status st = presize(c, it);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const std::string timed = c->timed;
  c->timed.clear();  // no timing events inside a graph
  c->capturing = true;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->capturing = false;
    c->timed = timed;
    return TA_ERR_HIP;
  }
  st = run(c, it, stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  c->capturing = false;
  c->timed = timed;
  if (!st && e != hipSuccess) st = TA_ERR_HIP;
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return TA_ERR_HIP;
  }
  // upload now, so that the first launch costs what every launch costs
  if (hipGraphUpload(x, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return TA_ERR_HIP;
  }
  ta_graph* r = new ta_graph();
  r->graph = g;
  r->exec = x;
  *out = r;
  return TA_OK;
}

extern "C" ta_status ta_graph_launch(ta_graph* g, void* stream) {
  if (!g) return TA_ERR_INVALID;
  TA_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return TA_OK;
}

extern "C" void ta_graph_free(ta_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

extern "C" ta_status ta_get_grids(ta_ctx* c, int32_t* grids) {
  if (!c || !grids) return TA_ERR_INVALID;
  for (int f = 0; f < N_FAMILIES; ++f) grids[f] = c->fam_grid[f];
  return TA_OK;
}

extern "C" ta_status ta_set_grids(ta_ctx* c, const int32_t* grids) {
  if (!c) return TA_ERR_INVALID;
  if (grids)
    for (int f = 0; f < N_FAMILIES; ++f)
      if (grids[f] < 1 || grids[f] > (1 << 20)) return TA_ERR_INVALID;
  for (int f = 0; f < N_FAMILIES; ++f) c->fam_grid[f] = grids ? grids[f] : c->grid_default;
  return TA_OK;
}

extern "C" ta_status ta_tune(ta_ctx* c, const ta_iteration* it, const char* cache_path, int32_t reps, void* stream,
                             int32_t* from_cache) {
  if (!valid(c, it) || reps < 1) return TA_ERR_INVALID;
  const std::string arch = arch_name(c->device), key = shape_key(it);
  int g[N_FAMILIES];
  if (from_cache) *from_cache = 0;
  if (cache_read(cache_path, arch, c->cus, key, g)) {
    for (int f = 0; f < N_FAMILIES; ++f) c->fam_grid[f] = g[f];
    if (from_cache) *from_cache = 1;
    return TA_OK;
  }
  ta_status st = presize(c, it);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const std::string timed = c->timed;
  c->timed.clear();
  double best;
  st = time_iteration(c, it, s, reps, &best);
  const int mult[] = {1, 2, 4, 8, 16};
  for (int f = 0; f < N_FAMILIES && !st; ++f) {
    int keep = c->fam_grid[f];
    for (int m : mult) {
      const int cand = m * c->cus;
      if (cand == keep) continue;
      c->fam_grid[f] = cand;
      double ms;
      st = time_iteration(c, it, s, reps, &ms);
      if (st) break;
      if (ms < best) {
        best = ms;
        keep = cand;
      }
    }
    c->fam_grid[f] = keep;
  }
  c->timed = timed;
  if (st) return st;
  cache_append(cache_path, arch, c->cus, key, c->fam_grid);
  return TA_OK;
}
