// Launch-configuration autotuner (rogs_autotune).  The tile shape (and with
// it the pixels per lane), the LDS staging depth and the per-view tile shapes
// are free parameters of the implementation: the per-pixel rule (q32 <= q_cut,
// Sec. 3.3.1 with a 3-sigma cut) does not depend on them, so every choice
// renders the same values; they change how many (surfel, tile) pairs are
// emitted and sorted, how much of each wave's work is rejected and how many
// waves a compute unit holds.  The tuner times the batch's projection,
// binning, forward and backward compositing over a coordinate descent of
// these parameters and keeps the fastest, optionally through a JSON cache.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "rogs_internal.h"

namespace {

struct Shape { int tw, th; };

// One launch configuration: the options' tile shape, the staging depth and
// the rogs_camera.tile code of every view (0 = the options' shape).
struct Config {
  int tw, th, stage;
  std::vector<int32_t> vt;
};

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
//   "<key>": {"tile_w": 16, "tile_h": 4, "stage": 32, "ms": 1.234, "views": [0, ...], ...},
//   ...
//   }
// where "views" lists the rogs_camera.tile code of every view.
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

bool parse_entry(const std::string& obj, int n_views, int* tw, int* th, int* stage, double* ms,
                 std::vector<int32_t>* vt) {
  if (sscanf(obj.c_str(), "{\"tile_w\": %d, \"tile_h\": %d, \"stage\": %d, \"ms\": %lf", tw, th,
             stage, ms) != 4)
    return false;
  size_t p = obj.find("\"views\": [");
  if (p == std::string::npos) return false;
  p += 10;
  vt->clear();
  for (int v = 0; v < n_views; ++v) {
    char* end = nullptr;
    const long x = strtol(obj.c_str() + p, &end, 10);
    if (end == obj.c_str() + p) return false;
    vt->push_back((int32_t)x);
    p = (size_t)(end - obj.c_str());
    if (p < obj.size() && obj[p] == ',') ++p;
  }
  return p < obj.size() && obj[p] == ']';
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

// Times configurations on one workload with the buffers it needs.  Render
// mode: project + bin/sort + forward + backward.  Step mode: one fused
// training step on copies of the caller's state, restored before each
// configuration.
struct Timer {
  rogs_ctx* c = nullptr;
  const rogs_surfels* s = nullptr;
  const rogs_tune_step* step = nullptr;
  std::vector<rogs_camera> cams;
  int n_views = 0;
  rogs_render_opts base{};
  void* stream = nullptr;
  hipStream_t st = nullptr;
  int reps = 1;
  int64_t total_pix = 0;
  DevBuf out, g, grads, ws;
  DevBuf cp, cm, cv, cs, ca, ce, cme, cve, cde, css;   // step mode: state copies
  rogs_train_state ts{};
  rogs_targets tg{};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::string table;

  ~Timer() {
    (void)hipStreamSynchronize(st);      // before the buffers are freed
    if (step) rogs::ctx_fused_forget(c);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }

  int setup() {
    hipError_t e = hipSuccess;
    if (!step) {
      const int64_t nout = (5 + (int64_t)s->n_sem) * total_pix;
      e = out.alloc(4 * (size_t)nout);
      if (e == hipSuccess) e = g.alloc(4 * (size_t)nout);
      if (e == hipSuccess) e = grads.alloc(4 * (size_t)(11 + s->n_sem) * s->n);
      if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: hipMalloc failed");
      // dL/d(out) = 1 in every channel: all of the backward's terms are live
      rogs::fill_u32(static_cast<uint32_t*>(g.p), 0x3f800000u, nout, st);
    } else {
      const rogs_train_state& u = *step->state;
      const size_t N = (size_t)u.n, K = 11 + (size_t)u.n_sem, V = (size_t)n_views;
      e = cp.alloc(4 * K * N);
      if (e == hipSuccess) e = cm.alloc(4 * K * N);
      if (e == hipSuccess) e = cv.alloc(4 * K * N);
      if (e == hipSuccess) e = cs.alloc(4 * 2 * N);
      if (e == hipSuccess) e = ca.alloc(4 * N);
      if (e == hipSuccess) e = ce.alloc(4 * 2 * V);
      if (e == hipSuccess) e = cme.alloc(4 * 2 * V);
      if (e == hipSuccess) e = cve.alloc(4 * 2 * V);
      if (e == hipSuccess) e = cde.alloc(4 * 2 * V);
      if (e == hipSuccess) e = css.alloc(64);
      if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: hipMalloc failed");
      ts = u;
      ts.params = static_cast<float*>(cp.p);
      ts.m = static_cast<float*>(cm.p);
      ts.v = static_cast<float*>(cv.p);
      ts.s_act = static_cast<float*>(cs.p);
      ts.alpha_act = static_cast<float*>(ca.p);
      ts.exposure = static_cast<float*>(ce.p);
      ts.m_exp = static_cast<float*>(cme.p);
      ts.v_exp = static_cast<float*>(cve.p);
      ts.d_exposure = static_cast<float*>(cde.p);
      ts.grads = nullptr;
      ts.step_state = css.p;
      tg = *step->targets;
      tg.exposure = ts.exposure;
      // steps of the caller still in flight are waited for (and forgotten)
      rogs::ctx_fused_forget(c);
    }
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: hipEventCreate failed");
    return ROGS_OK;
  }

  // step mode: the copies take the caller's state again
  int restore() {
    const rogs_train_state& u = *step->state;
    const size_t N = (size_t)u.n, K = 11 + (size_t)u.n_sem, V = (size_t)n_views;
    const struct { void* d; const void* s; size_t b; } cps[] = {
        {ts.params, u.params, 4 * K * N}, {ts.m, u.m, 4 * K * N}, {ts.v, u.v, 4 * K * N},
        {ts.s_act, u.s_act, 4 * 2 * N}, {ts.alpha_act, u.alpha_act, 4 * N},
        {ts.exposure, u.exposure, 4 * 2 * V}, {ts.m_exp, u.m_exp, 4 * 2 * V},
        {ts.v_exp, u.v_exp, 4 * 2 * V}, {ts.step_state, u.step_state, 64}};
    for (const auto& k : cps) {
      hipError_t e = hipMemcpyAsync(k.d, k.s, k.b, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: state copy failed");
    }
    return ROGS_OK;
  }

  rogs_render_opts opts_of(const Config& k) {
    rogs_render_opts o = base;
    o.tile_w = k.tw;
    o.tile_h = k.th;
    o.stage = k.stage;
    for (int v = 0; v < n_views; ++v) cams[v].tile = k.vt[v];
    return o;
  }

  int size_ws(const rogs_render_opts& o, int64_t cap, int64_t scap, size_t* bytes) {
    return step ? rogs_fused_workspace_size(&ts, cams.data(), n_views, &o, cap, scap, bytes)
                : rogs_workspace_size(s, cams.data(), n_views, &o, cap, scap, bytes);
  }

  // One run of the configuration (project + sort + forward + backward, or
  // one eager fused step).
  int once(const rogs_render_opts& o, size_t bytes, int64_t cap, int64_t scap) {
    if (step)
      return rogs_step_fused(c, &ts, cams.data(), n_views, &o, &tg, step->optim, ws.p, bytes, cap,
                             scap, ROGS_FUSED_EAGER, stream);
    int status = rogs_project(c, s, cams.data(), n_views, &o, ws.p, bytes, cap, scap, stream);
    if (status == ROGS_OK) status = rogs_bin_sort(c, ws.p, nullptr, 0u, stream);
    if (status == ROGS_OK)
      status = rogs_render_fwd(c, s, ws.p, static_cast<float*>(out.p), ROGS_CH_ALL, stream);
    if (status == ROGS_OK)
      status = rogs_render_bwd(c, s, ws.p, static_cast<const float*>(out.p),
                               static_cast<const float*>(g.p), static_cast<float*>(grads.p), 0u,
                               stream);
    return status;
  }

  // Pairs and visible slots of the last run; *ovf when it overflowed.
  int counts(int64_t* pairs, int64_t* visible, int32_t* ovf) {
    int64_t stats[8];
    int status = step ? rogs_fused_status(c, stats, nullptr) : rogs_batch_stats(c, ws.p, stats, stream);
    if (status != ROGS_OK) return status;
    *pairs = stats[0];
    *visible = stats[2];
    *ovf = step ? (int32_t)stats[1] : 0;
    return ROGS_OK;
  }

  // Time per run of configuration k in *ms; *ms < 0 when k is not valid for
  // the workload or its counts changed between runs.  Returns a status.
  int run(const Config& k, const char* label, double* ms) {
    *ms = -1.0;
    const rogs_render_opts o = opts_of(k);
    size_t bytes = 0;
    if (size_ws(o, 1, 0, &bytes) != ROGS_OK) return ROGS_OK;
    // size the capacities with one counted run, then time device-count runs
    int64_t cap = std::max<int64_t>(1 << 16, total_pix / 4), scap = 0;
    int status = step ? restore() : ROGS_OK;
    bool sized = false;
    for (int attempt = 0; attempt < 6 && status == ROGS_OK && !sized; ++attempt) {
      status = size_ws(o, cap, scap, &bytes);
      if (status == ROGS_OK && hipSuccess != ws.alloc(bytes)) status = ROGS_EHIP;
      if (status != ROGS_OK) break;
      int32_t ovf = 0;
      int64_t pairs = 0, visible = 0;
      if (step) {
        status = once(o, bytes, cap, scap);
        if (status == ROGS_OK) status = counts(&pairs, &visible, &ovf);
      } else {
        status = rogs_project(c, s, cams.data(), n_views, &o, ws.p, bytes, cap, scap, stream);
        int64_t n = 0;
        if (status == ROGS_OK) status = rogs_bin_sort(c, ws.p, &n, ROGS_SYNC_COUNT, stream);
        if (status == ROGS_ECAPACITY) {
          ovf = 1;
          status = ROGS_OK;
        }
        if (status == ROGS_OK) {
          int32_t unused = 0;
          status = counts(&pairs, &visible, &unused);
        }
      }
      if (status != ROGS_OK) break;
      cap = (int64_t)(pairs * 1.1) + 4096;
      scap = std::min<int64_t>(cap, (int64_t)(visible * 1.1) + 4096);
      sized = !ovf;
    }
    if (status != ROGS_OK) return status;
    if (!sized) return ROGS_OK;
    status = size_ws(o, cap, scap, &bytes);
    if (status == ROGS_OK && hipSuccess != ws.alloc(bytes)) status = ROGS_EHIP;
    if (status == ROGS_OK && step) status = restore();
    if (status != ROGS_OK) return status;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep <= reps && status == ROGS_OK; ++rep) {
      if (rep == 1) e = hipEventRecord(e0, st);     // rep 0 is the warm-up
      status = once(o, bytes, cap, scap);
    }
    if (status != ROGS_OK) return status;
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return rogs::ctx_fail(c, ROGS_EHIP, "rogs_autotune: timing failed");
    int32_t ovf = 0;
    if (step) {
      int64_t pairs = 0, visible = 0;
      status = counts(&pairs, &visible, &ovf);
    } else {
      status = rogs_pair_count(c, ws.p, nullptr, &ovf, stream);
    }
    if (status != ROGS_OK) return status;
    if (ovf) return ROGS_OK;                 // counts grew between runs: not a valid timing
    *ms = (double)t / reps;
    char buf[96];
    snprintf(buf, sizeof(buf), "%s\"%s\": %.4f", table.empty() ? "" : ", ", label, *ms);
    table += buf;
    return ROGS_OK;
  }
};

int32_t tile_code(int tw, int th) { return (int32_t)((uint32_t)tw | ((uint32_t)th << 16)); }

}  // namespace

extern "C" int rogs_autotune(rogs_ctx* c, const rogs_surfels* s, const rogs_camera* cams,
                             int32_t n_views, rogs_render_opts* opts, int32_t* view_tiles,
                             const rogs_tune_step* step, const char* cache_json, int32_t reps,
                             float* ms_out, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (!s || !cams || !opts || n_views < 1)
    return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: null argument or no views");
  if (reps < 1) return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: reps must be >= 1");
  if (step) {
    const rogs_train_state* u = step->state;
    if (!u || !step->targets || !step->optim || !u->params || !u->m || !u->v || !u->s_act ||
        !u->alpha_act || !u->exposure || !u->m_exp || !u->v_exp || !u->step_state)
      return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: incomplete step description");
    if (u->n != s->n || u->n_sem != s->n_sem)
      return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: surfels and training state differ");
  }
  std::vector<rogs_camera> cv(cams, cams + n_views);
  for (auto& k : cv) k.tile = 0;               // the cameras' own codes are ignored
  size_t probe = 0;
  int r = rogs_workspace_size(s, cv.data(), n_views, opts, 1, 0, &probe);
  if (r != ROGS_OK) return rogs::ctx_fail(c, r, "rogs_autotune: invalid surfels, views or options");
  auto finish = [&](const Config& k, double ms) {
    opts->tile_w = k.tw;
    opts->tile_h = k.th;
    opts->stage = k.stage;
    if (view_tiles)
      for (int v = 0; v < n_views; ++v) view_tiles[v] = k.vt[v];
    if (ms_out) *ms_out = (float)ms;
  };
  const std::string key = (step ? "step;" : "render;") + workload_key(s, cams, n_views);
  std::map<std::string, std::string> cache;
  if (cache_json) {
    bool exists = false;
    if (!read_cache(cache_json, &cache, &exists))
      return rogs::ctx_fail(c, ROGS_EINVAL, std::string("rogs_autotune: ") + cache_json +
                                                " is not a cache file written by rogs_autotune");
    auto it = cache.find(key);
    Config k;
    double ms = 0.0;
    if (it != cache.end() && parse_entry(it->second, n_views, &k.tw, &k.th, &k.stage, &ms, &k.vt)) {
      rogs_render_opts o = *opts;
      o.tile_w = k.tw;
      o.tile_h = k.th;
      o.stage = k.stage;
      std::vector<rogs_camera> ck = cv;
      for (int v = 0; v < n_views; ++v) ck[v].tile = k.vt[v];
      if (rogs_workspace_size(s, ck.data(), n_views, &o, 1, 0, &probe) == ROGS_OK) {
        finish(k, ms);
        return ROGS_OK;
      }
    }
  }

  Timer T;
  T.c = c;
  T.s = s;
  T.step = step;
  T.cams = cv;
  T.n_views = n_views;
  T.base = *opts;
  T.stream = stream;
  T.st = static_cast<hipStream_t>(stream);
  T.reps = reps;
  for (int v = 0; v < n_views; ++v) T.total_pix += (int64_t)cams[v].w * cams[v].h;
  r = T.setup();
  if (r != ROGS_OK) return r;

  // (1) every shape, all views alike, staging depth 32
  Config best{opts->tile_w, opts->tile_h, 32, std::vector<int32_t>(n_views, 0)};
  double best_ms = 1e30;
  char label[96];
  for (const Shape sh : candidate_shapes()) {
    Config k{sh.tw, sh.th, 32, std::vector<int32_t>(n_views, 0)};
    snprintf(label, sizeof(label), "%dx%d/s32", sh.tw, sh.th);
    double ms = 0.0;
    r = T.run(k, label, &ms);
    if (r != ROGS_OK) return r;
    if (ms >= 0.0 && ms < best_ms) {
      best_ms = ms;
      best = k;
    }
  }
  if (best_ms >= 1e30) return rogs::ctx_fail(c, ROGS_EINVAL, "rogs_autotune: no tile shape ran");
  // a later step replaces the choice only when it is faster by more than the
  // timing noise
  const double kGain = 0.99;
  // (2) staging depth at that shape
  for (int stage : {16, 64}) {
    Config k = best;
    k.stage = stage;
    snprintf(label, sizeof(label), "%dx%d/s%d", k.tw, k.th, stage);
    double ms = 0.0;
    r = T.run(k, label, &ms);
    if (r != ROGS_OK) return r;
    if (ms >= 0.0 && ms < kGain * best_ms) {
      best_ms = ms;
      best = k;
    }
  }
  // (3) resolution classes (equal w, h and model), each in turn over the
  // other shapes of the same area
  std::vector<int> cls(n_views, -1);
  std::vector<int> first;                     // first view of each class
  for (int v = 0; v < n_views; ++v) {
    for (size_t q = 0; q < first.size() && cls[v] < 0; ++q) {
      const rogs_camera& a = cams[first[q]];
      if (a.w == cams[v].w && a.h == cams[v].h && a.model == cams[v].model) cls[v] = (int)q;
    }
    if (cls[v] < 0) {
      cls[v] = (int)first.size();
      first.push_back(v);
    }
  }
  const int area = best.tw * best.th;
  std::vector<Shape> cls_shape(first.size(), Shape{best.tw, best.th});
  if (first.size() > 1) {
    for (size_t q = 0; q < first.size(); ++q) {
      const Shape start = cls_shape[q];
      for (int tw : {4, 8, 16, 32, 64}) {
        const int th = area / tw;
        if (th < 1 || (tw == start.tw && th == start.th)) continue;
        Config k = best;
        for (int v = 0; v < n_views; ++v)
          if (cls[v] == (int)q) k.vt[v] = (tw == best.tw && th == best.th) ? 0 : tile_code(tw, th);
        const rogs_camera& a = cams[first[q]];
        snprintf(label, sizeof(label), "%dx%d/m%d:%dx%d", a.w, a.h, a.model, tw, th);
        double ms = 0.0;
        r = T.run(k, label, &ms);
        if (r != ROGS_OK) return r;
        if (ms >= 0.0 && ms < kGain * best_ms) {
          best_ms = ms;
          best = k;
          cls_shape[q] = Shape{tw, th};
        }
      }
    }
  }
  finish(best, best_ms);
  if (cache_json) {
    std::string e;
    char buf[160];
    snprintf(buf, sizeof(buf), "{\"tile_w\": %d, \"tile_h\": %d, \"stage\": %d, \"ms\": %.4f, \"views\": [",
             best.tw, best.th, best.stage, best_ms);
    e = buf;
    for (int v = 0; v < n_views; ++v) e += (v ? ", " : "") + std::to_string(best.vt[v]);
    e += "], \"classes\": {";
    for (size_t q = 0; q < first.size(); ++q) {
      const rogs_camera& a = cams[first[q]];
      snprintf(buf, sizeof(buf), "%s\"%dx%d/m%d\": \"%dx%d\"", q ? ", " : "", a.w, a.h, a.model,
               cls_shape[q].tw, cls_shape[q].th);
      e += buf;
    }
    e += "}, \"timed\": {" + T.table + "}}";
    cache[key] = e;
    if (!write_cache(cache_json, cache))
      return rogs::ctx_fail(c, ROGS_EINVAL, std::string("rogs_autotune: cannot write ") + cache_json);
  }
  return ROGS_OK;
}
