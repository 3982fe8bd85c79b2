// tune.hip -- launch-option autotuner for the tracing kernel (host code).
//
// The options it tunes only change how work is scheduled on the GPU
// (occupancy target, when a wave handles events, work items per atomic,
// block size, record layout), never which paths are traced, so any choice
// renders the same image up to FP32 summation order.  Candidates are timed
// on probe renders of the caller's own frame at a few samples per pixel;
// coordinate descent keeps the count of probes small.  Results can be kept
// in a small JSON file, one object per workload key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

namespace tv {

int render_grid(const tet_grid*, const tet_camera*, const tet_medium*, const tet_light*, int32_t, uint64_t,
                const tet_render_opts*, float*, int32_t, hipStream_t, tet_render_stats*);

namespace {

// A candidate replaces the current choice only when its probe is faster by
// more than this fraction: smaller differences are within the probes' noise.
constexpr double kMinGain = 0.005;

const char* kFields[5] = {"waves_per_simd", "event_wait", "batch_items", "block_size", "record_layout"};

int32_t* field(tet_render_opts& o, int i) {
  switch (i) {
    case 0: return &o.waves_per_simd;
    case 1: return &o.event_wait;
    case 2: return &o.batch_items;
    case 3: return &o.block_size;
    default: return &o.record_layout;
  }
}

std::string workload_key(const tet_grid* g, const tet_camera* cam, const tet_render_opts& o) {
  int dev = 0;
  hipDeviceProp_t p;
  std::string arch = "gpu";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
    arch = p.gcnArchName;
    cus = p.multiProcessorCount;
  }
  for (char& c : arch)
    if (c == '"' || c == '\\') c = '_';
  int lg = 0;
  while ((1ll << (lg + 1)) <= g->n) lg++;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s/%dcu/tets2^%d/%dx%d/b%d/t%d", arch.c_str(), cus, lg, cam->width, cam->height,
           o.max_bounces, o.transmittance);
  return buf;
}

// The cache file: {"key": {"waves_per_simd": 5, ..., "ms": 1.5}, ...}; a
// small reader for exactly this shape.
struct Entry {
  int32_t v[5];
  double ms;
};

std::mutex g_file_mu;

std::map<std::string, Entry> read_cache(const char* path) {
  std::map<std::string, Entry> out;
  std::ifstream f(path);
  if (!f) return out;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  auto next_string = [&](size_t from, std::string& str) -> size_t {
    size_t a = s.find('"', from);
    if (a == std::string::npos) return std::string::npos;
    size_t b = s.find('"', a + 1);
    if (b == std::string::npos) return std::string::npos;
    str = s.substr(a + 1, b - a - 1);
    return b + 1;
  };
  while (true) {
    std::string key;
    size_t k = next_string(i, key);
    if (k == std::string::npos) break;
    size_t ob = s.find('{', k), cb = s.find('}', k);
    if (ob == std::string::npos || cb == std::string::npos || cb < ob) break;
    std::string body = s.substr(ob + 1, cb - ob - 1);
    Entry e;
    bool ok = true;
    for (int f = 0; f < 5 && ok; f++) {
      size_t at = body.find(std::string("\"") + kFields[f] + "\"");
      if (at == std::string::npos) {
        ok = false;
        break;
      }
      size_t colon = body.find(':', at);
      e.v[f] = (int32_t)strtol(body.c_str() + colon + 1, nullptr, 10);
    }
    size_t at = body.find("\"ms\"");
    e.ms = at == std::string::npos ? 0.0 : strtod(body.c_str() + body.find(':', at) + 1, nullptr);
    if (ok) out[key] = e;
    i = cb + 1;
  }
  return out;
}

bool write_cache(const char* path, const std::map<std::string, Entry>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t k = 0;
  for (const auto& kv : m) {
    fprintf(f, "  \"%s\": {", kv.first.c_str());
    for (int i = 0; i < 5; i++) fprintf(f, "\"%s\": %d, ", kFields[i], kv.second.v[i]);
    fprintf(f, "\"ms\": %.4f}%s\n", kv.second.ms, ++k < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

int autotune(const tet_grid* g, const tet_camera* cam, const tet_medium* med, const tet_light* light,
             const tet_autotune_opts* ao_in, tet_render_opts* inout, hipStream_t st, double* best_ms) {
  if (!g || !cam || !med || !light || !inout) return fail(TET_ERR_INVALID_ARG, "tet_autotune: NULL argument");
  if (inout->nrc) return fail(TET_ERR_INVALID_ARG, "tet_autotune: tune without a radiance cache");
  tet_autotune_opts ao;
  if (ao_in) ao = *ao_in;
  else tet_autotune_opts_defaults(&ao);
  if (ao.probe_spp < 1 || ao.probe_spp > 1024 || ao.probe_repeats < 1 || ao.probe_repeats > 16)
    return fail(TET_ERR_INVALID_ARG, "tet_autotune: bad probe options");
  if (int rc = check_camera(cam)) return rc;
  tet_render_opts base = *inout;
  base.samples_per_item = 1;
  const std::string key = workload_key(g, cam, base);
  if (ao.cache_path) {
    std::lock_guard<std::mutex> lk(g_file_mu);
    auto m = read_cache(ao.cache_path);
    auto it = m.find(key);
    if (it != m.end()) {
      *inout = base;
      for (int i = 0; i < 5; i++) *field(*inout, i) = it->second.v[i];
      if (best_ms) *best_ms = it->second.ms;
      return TET_OK;
    }
  }
  // candidate values per option (record layouts only those the grid has)
  std::vector<std::vector<int32_t>> cand = {{4, 5, 6}, {16, 32, 48}, {32, 64, 128}, {128, 256}, {48}};
  if (g->rec32) cand[4] = {32, 48};
  tet_render_opts cur = base;
  if (!cur.waves_per_simd) cur.waves_per_simd = 5;
  if (!cur.event_wait) cur.event_wait = 32;
  if (!cur.batch_items) cur.batch_items = 64;
  if (!cur.block_size) cur.block_size = 256;
  if (!cur.record_layout) cur.record_layout = g->rec32 ? 32 : 48;
  const size_t img = (size_t)cam->width * cam->height * 3 * sizeof(float);
  float* out = (float*)dev_alloc(img);
  if (!out) return fail(TET_ERR_OUT_OF_MEMORY, "tet_autotune: image");
  struct Free {
    void* p;
    ~Free() { dev_free(p); }
  } f_{out};
  std::map<std::vector<int32_t>, double> seen;
  auto probe = [&](const tet_render_opts& o, double* ms) -> int {
    std::vector<int32_t> k;
    for (int i = 0; i < 5; i++) k.push_back(*field(const_cast<tet_render_opts&>(o), i));
    auto it = seen.find(k);
    if (it != seen.end()) {
      *ms = it->second;
      return TET_OK;
    }
    double best = 1e300;
    for (int r = 0; r < ao.probe_repeats; r++) {
      tet_render_stats s;
      if (int rc = render_grid(g, cam, med, light, ao.probe_spp, 0x7E57ull + (uint64_t)r, &o, out, 1, st, &s))
        return rc;
      best = std::min(best, s.trace_ms);
    }
    seen[k] = best;
    *ms = best;
    return TET_OK;
  };
  {  // warm-up (first-launch costs), not recorded: the defaults are timed warm like every other candidate
    tet_render_stats s;
    if (int rc = render_grid(g, cam, med, light, ao.probe_spp, 0x7E57ull, &cur, out, 1, st, &s)) return rc;
  }
  double cur_ms = 0.0;
  if (int rc = probe(cur, &cur_ms)) return rc;
  for (int sweep = 0; sweep < 2; sweep++) {
    bool changed = false;
    for (int i = 0; i < 5; i++) {
      for (int32_t v : cand[i]) {
        if (v == *field(cur, i)) continue;
        tet_render_opts t = cur;
        *field(t, i) = v;
        double ms = 0.0;
        if (int rc = probe(t, &ms)) return rc;
        if (ms < cur_ms * (1.0 - kMinGain)) {
          cur = t;
          cur_ms = ms;
          changed = true;
        }
      }
    }
    if (!changed) break;
  }
  *inout = cur;
  if (best_ms) *best_ms = cur_ms;
  if (ao.cache_path) {
    std::lock_guard<std::mutex> lk(g_file_mu);
    auto m = read_cache(ao.cache_path);
    Entry e;
    for (int i = 0; i < 5; i++) e.v[i] = *field(cur, i);
    e.ms = cur_ms;
    m[key] = e;
    if (!write_cache(ao.cache_path, m)) return fail(TET_ERR_INVALID_ARG, "tet_autotune: cannot write the cache file");
  }
  return TET_OK;
}

}  // namespace tv
