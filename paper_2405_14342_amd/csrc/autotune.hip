// Tile-shape autotuner (rogs_autotune).  The tile shape is a free parameter
// of the implementation: the per-pixel rule (q32 <= q_cut, Sec. 3.3.1 with a
// 3-sigma cut) does not depend on it, so every shape renders the same values;
// it only changes how many (surfel, tile) pairs are emitted and sorted and how
// much of each wave's work is rejected.  The tuner times the batch's
// projection, binning, forward and backward compositing for every supported
// shape and keeps the fastest, optionally through a small JSON cache.
#include <stdio.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "rogs_internal.h"

namespace {

struct Shape { int tw, th; };

std::vector<Shape> candidate_shapes() {
  std::vector<Shape> v;
  for (int tw : {4, 8, 16, 32, 64})
    for (int area : {64, 128, 256})
      if (area % tw == 0) v.push_back({tw, area / tw});
  return v;
}

std::string workload_key(const rogs_surfels* s, const rogs_camera* cams, int n_views) {
  std::string k = "n=" + std::to_string(s->n) + ";C=" + std::to_string(s->n_sem) + ";views=";
  char buf[96];
  for (int v = 0; v < n_views; ++v) {
    snprintf(buf, sizeof(buf), "%s%dx%d/m%d/f%.6g", v ? "," : "", cams[v].w, cams[v].h,
             cams[v].model, (double)cams[v].fx);
    k += buf;
  }
  return k;
}

// The cache file holds one JSON object with one entry per line:
//   {
//   "<key>": {"tile_w": 16, "tile_h": 4, "ms": 1.234},
//   ...
//   }
// Only files in this form (as written here) are read; anything else is an
// error, so a foreign file is never overwritten.
bool read_cache(const char* path, std::map<std::string, std::string>* out, bool* exists) {
  *exists = false;
  FILE* f = fopen(path, "rb");
  if (!f) return true;
  *exists = true;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  fclose(f);
  size_t pos = 0;
  bool opened = false, closed = false;
  while (pos < text.size()) {
    size_t e = text.find('\n', pos);
    if (e == std::string::npos) e = text.size();
    std::string line = text.substr(pos, e - pos);
    pos = e + 1;
    while (!line.empty() && (line.back() == '\r' || line.back() == ' ' || line.back() == ','))
      line.pop_back();
    if (line.empty()) continue;
    if (line == "{") { if (opened) return false; opened = true; continue; }
    if (line == "}") { closed = true; continue; }
    if (!opened || closed || line[0] != '"') return false;
    const size_t q = line.find("\": {");
    if (q == std::string::npos || line.back() != '}') return false;
    (*out)[line.substr(1, q - 1)] = line.substr(q + 3);
  }
  return !*exists || text.empty() || (opened && closed);
}

bool parse_entry(const std::string& obj, int* tw, int* th, double* ms) {
  return sscanf(obj.c_str(), "{\"tile_w\": %d, \"tile_h\": %d, \"ms\": %lf", tw, th, ms) == 3;
}

bool write_cache(const char* path, const std::map<std::string, std::string>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f, "\"%s\": %s%s\n", kv.first.c_str(), kv.second.c_str(),
            ++i < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  if (fclose(f) != 0) return false;
  return rename(tmp.c_str(), path) == 0;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
  hipError_t alloc(size_t bytes) {
    if (p) { (void)hipFree(p); p = nullptr; }
    return hipMalloc(&p, std::max<size_t>(bytes, 256));
  }
};

}  // namespace

extern "C" int rogs_autotune(rogs_ctx* c, const rogs_surfels* s, const rogs_camera* cams,
                             int32_t n_views, rogs_render_opts* opts, const char* cache_json,
                             int32_t reps, float* ms_out, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (!s || !cams || !opts || n_views < 1)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: null argument or no views");
  if (reps < 1) return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: reps must be >= 1");
  size_t probe = 0;
  int r = rogs_workspace_size(s, cams, n_views, opts, 1, 0, &probe);
  if (r != ROGS_OK) return rogs::ctx_fail(c, r, "rogs_autotune: invalid surfels, views or options");
  const std::string key = workload_key(s, cams, n_views);
  std::map<std::string, std::string> cache;
  if (cache_json) {
    bool exists = false;
    if (!read_cache(cache_json, &cache, &exists))
      return rogs::ctx_fail(c, ROGS_EINVAL, std::string("rogs_autotune: ") + cache_json +
                                                " is not a cache file written by rogs_autotune");
    auto it = cache.find(key);
    int tw = 0, th = 0;
    double ms = 0.0;
    if (it != cache.end() && parse_entry(it->second, &tw, &th, &ms)) {
      rogs_render_opts o = *opts;
      o.tile_w = tw;
      o.tile_h = th;
      if (rogs_workspace_size(s, cams, n_views, &o, 1, 0, &probe) == ROGS_OK) {
        *opts = o;
        if (ms_out) *ms_out = (float)ms;
        return ROGS_OK;
      }
    }
  }

  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t total_pix = 0;
  for (int v = 0; v < n_views; ++v) total_pix += (int64_t)cams[v].w * cams[v].h;
  const int64_t nout = (5 + (int64_t)s->n_sem) * total_pix;
  DevBuf out, g, grads, ws;
  hipError_t e = out.alloc(4 * (size_t)nout);
  if (e == hipSuccess) e = g.alloc(4 * (size_t)nout);
  if (e == hipSuccess) e = grads.alloc(4 * (size_t)(11 + s->n_sem) * s->n);
  if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: hipMalloc failed");
  struct Drain {                    // runs before the buffers above are freed
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{st};
  // dL/d(out) = 1 in every channel: all of the backward's terms are live
  rogs::fill_u32(static_cast<uint32_t*>(g.p), 0x3f800000u, nout, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: hipEventCreate failed");

  std::string table;
  double best_ms = 1e30;
  Shape best{opts->tile_w, opts->tile_h};
  int status = ROGS_OK;
  for (const Shape sh : candidate_shapes()) {
    rogs_render_opts o = *opts;
    o.tile_w = sh.tw;
    o.tile_h = sh.th;
    if (rogs_workspace_size(s, cams, n_views, &o, 1, 0, &probe) != ROGS_OK) continue;
    // size the capacities with one counted run, then time device-count runs
    int64_t cap = std::max<int64_t>(1 << 16, total_pix / 4), scap = 0;
    for (int attempt = 0; attempt < 6; ++attempt) {
      size_t bytes = 0;
      status = rogs_workspace_size(s, cams, n_views, &o, cap, scap, &bytes);
      if (status == ROGS_OK && hipSuccess != ws.alloc(bytes)) status = ROGS_EHIP;
      if (status == ROGS_OK)
        status = rogs_project(c, s, cams, n_views, &o, ws.p, bytes, cap, scap, stream);
      int64_t n = 0;
      if (status == ROGS_OK) status = rogs_bin_sort(c, ws.p, &n, ROGS_SYNC_COUNT, stream);
      if (status == ROGS_ECAPACITY) {
        int64_t stats[6];
        if (rogs_batch_stats(c, ws.p, stats, stream) != ROGS_OK) break;
        cap = (int64_t)(stats[0] * 1.1) + 4096;
        scap = std::min<int64_t>(cap, (int64_t)(stats[2] * 1.1) + 4096);
        continue;
      }
      if (status == ROGS_OK) {
        int64_t stats[6];
        status = rogs_batch_stats(c, ws.p, stats, stream);
        if (status == ROGS_OK) {
          cap = (int64_t)(stats[0] * 1.1) + 4096;
          scap = std::min<int64_t>(cap, (int64_t)(stats[2] * 1.1) + 4096);
          status = rogs_workspace_size(s, cams, n_views, &o, cap, scap, &bytes);
          if (status == ROGS_OK && hipSuccess != ws.alloc(bytes)) status = ROGS_EHIP;
        }
      }
      break;
    }
    if (status != ROGS_OK) break;
    size_t bytes = 0;
    (void)rogs_workspace_size(s, cams, n_views, &o, cap, scap, &bytes);
    double total_ms = 0.0;
    for (int rep = 0; rep <= reps && status == ROGS_OK; ++rep) {
      if (rep == 1) e = hipEventRecord(e0, st);     // rep 0 is the warm-up
      status = rogs_project(c, s, cams, n_views, &o, ws.p, bytes, cap, scap, stream);
      if (status == ROGS_OK) status = rogs_bin_sort(c, ws.p, nullptr, 0u, stream);
      if (status == ROGS_OK)
        status = rogs_render_fwd(c, s, ws.p, static_cast<float*>(out.p), ROGS_CH_ALL, stream);
      if (status == ROGS_OK)
        status = rogs_render_bwd(c, s, ws.p, static_cast<const float*>(out.p),
                                 static_cast<const float*>(g.p), static_cast<float*>(grads.p), 0u,
                                 stream);
    }
    if (status != ROGS_OK) break;
    e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { status = rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: timing failed"); break; }
    int32_t ovf = 0;
    status = rogs_pair_count(c, ws.p, nullptr, &ovf, stream);
    if (status != ROGS_OK) break;
    if (ovf) continue;                       // counts grew between runs: not a valid timing
    total_ms = ms / reps;
    char buf[64];
    snprintf(buf, sizeof(buf), "%s\"%dx%d\": %.4f", table.empty() ? "" : ", ", sh.tw, sh.th,
             total_ms);
    table += buf;
    if (total_ms < best_ms) {
      best_ms = total_ms;
      best = sh;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != ROGS_OK) return status;
  if (best_ms >= 1e30) return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: no tile shape ran");
  opts->tile_w = best.tw;
  opts->tile_h = best.th;
  if (ms_out) *ms_out = (float)best_ms;
  if (cache_json) {
    char buf[128];
    snprintf(buf, sizeof(buf), "{\"tile_w\": %d, \"tile_h\": %d, \"ms\": %.4f, \"shapes\": {",
             best.tw, best.th, best_ms);
    cache[key] = std::string(buf) + table + "}}";
    if (!write_cache(cache_json, cache))
      return rogs::ctx_fail(c, ROGS_EINVAL, std::string("rogs_autotune: cannot write ") + cache_json);
  }
  return ROGS_OK;
}
