// Host side of the C ABI declared in include/rogs.h: argument validation,
// workspace layout, view-table upload and the launch sequence of each entry
// point.  No device memory is allocated here; the caller owns all of it.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rogs_internal.h"

using rogs::Layout;
using rogs::ViewDev;

struct rogs_ctx {
  std::string err;
  bool have_batch = false;
  bool sorted = false;
  // per-view channel sets for the next rogs_project (render server); the
  // batch's views had sets of their own; the last forward wrote every plane
  // and the backward's per-pixel state
  std::vector<uint32_t> view_ch;
  bool batch_view_ch = false;
  bool fwd_full = false;
  Layout L;
  void* ws = nullptr;
  int64_t n_pairs_host = -1;
  void* stage = nullptr;          // pinned staging for the view table upload
  size_t stage_bytes = 0;
  hipEvent_t stage_evt = nullptr;
  bool stage_pending = false;
  uint32_t* readback = nullptr;   // pinned, for pair-count read-back
  int64_t last_visible = 0;
  // kernel timing (rogs_prof_enable): events bracketing each launch group
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int group; hipEvent_t a, b; };
  std::vector<Rec> recs;
  int open_group = -1;
  hipEvent_t open_ev = nullptr;
  double prof_ms[ROGS_PROF_GROUPS] = {};
  int64_t prof_n[ROGS_PROF_GROUPS] = {};
  // fused step: the captured graph and what it was captured for
  struct Fused {
    bool valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Layout L;
    int alt = 0;
    void* ws = nullptr;
    hipStream_t st = nullptr;
    uint32_t flags = 0;
    rogs_train_state ts{};
    rogs_targets tg{};
    rogs_optim opt{};
    rogs_render_opts opts{};
    std::vector<int32_t> sizes;         // w, h, model and tile code of every view
    // two steps in flight: step k uses buffer k & 1, and step k + 2 waits for it
    void* stage[2] = {nullptr, nullptr}; // pinned: view table + first-block table
    size_t stage_bytes = 0;
    uint32_t* status[2] = {nullptr, nullptr};   // pinned: misc[4] + StepState
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    int64_t launched = 0;                // steps launched so far
    int last = 0;                        // buffer of the last launched step
    hipStream_t cap_stream = nullptr;    // capture happens here (the null stream cannot be captured)
    hipStream_t side = nullptr;          // the long lists' depth sort, beside the short ones
    hipEvent_t fork = nullptr, join = nullptr;
  } fz;
};

namespace {

int fail(rogs_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(rogs_ctx* c, hipError_t e, const char* where) {
  return fail(c, ROGS_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int check_launch(rogs_ctx* c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, where);
  return ROGS_OK;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

bool is_fin(float x) { return isfinite(x); }

}  // namespace

namespace rogs {

int ctx_fail(rogs_ctx* c, int code, const std::string& msg) { return fail(c, code, msg); }

// Tile shape of a view: the options' (tw, th) unless camera.tile gives its
// own, tile_w | tile_h << 16 with tile_w dividing 64 and the same area.
bool view_shape(const rogs_camera& c, int tw, int th, int* vtw, int* vth) {
  if (c.tile == 0) {
    *vtw = tw;
    *vth = th;
    return true;
  }
  const uint32_t code = (uint32_t)c.tile;
  const int w = (int)(code & 0xffffu), h = (int)(code >> 16);
  if (w < 1 || w > 64 || (64 % w) != 0 || h < 1 || w * h != tw * th) return false;
  *vtw = w;
  *vth = h;
  return true;
}

int make_layout(const rogs_surfels* s, const rogs_camera* cams, int n_views,
                const rogs_render_opts* opts, int64_t cap, int64_t scap, Layout* L,
                const char** why, bool fused) {
  *why = nullptr;
  if (!s || !cams || !opts || !L) { *why = "null argument"; return ROGS_EINVAL; }
  if (s->n < 1) { *why = "surfel count must be >= 1"; return ROGS_EINVAL; }
  if (!sem_supported(s->n_sem)) { *why = "n_sem must be 1..8 or 16"; return ROGS_EINVAL; }
  if (n_views < 1 || n_views > kMaxViews) { *why = "n_views out of range"; return ROGS_EINVAL; }
  if (cap < 0 || cap >= (int64_t(1) << 31)) { *why = "pair_capacity must be in [0, 2^31)"; return ROGS_EINVAL; }
  if (scap < 0) { *why = "slot_capacity must be >= 0"; return ROGS_EINVAL; }
  if (scap == 0 || scap > cap) scap = cap;
  const int tw = opts->tile_w, th = opts->tile_h;
  if (tw < 1 || tw > 64 || (64 % tw) != 0 || th < 1 || tw * th < 64 || tw * th > 256 ||
      ((tw * th) & (tw * th - 1)) != 0) {
    *why = "tile shape: tile_w must divide 64 and tile_w*tile_h must be 64, 128 or 256";
    return ROGS_EINVAL;
  }
  if (!(opts->eps2d >= 0.0f) || !is_fin(opts->eps2d) || !(opts->q_cut > 0.0f) ||
      !is_fin(opts->q_cut) || !(opts->alpha_max > 0.0f && opts->alpha_max < 1.0f) ||
      !(opts->t_eps >= 0.0f && opts->t_eps < 1.0f)) {
    *why = "render options out of range";
    return ROGS_EINVAL;
  }
  if (opts->stage != 0 && opts->stage != 16 && opts->stage != 32 && opts->stage != 64) {
    *why = "stage must be 0, 16, 32 or 64";
    return ROGS_EINVAL;
  }
  Layout l;
  l.N = s->n;
  l.C = s->n_sem;
  l.V = n_views;
  l.tw = tw;
  l.th = th;
  l.ppl = tw * th / 64;
  l.stage = opts->stage ? opts->stage : 32;
  l.FS = feat_stride(l.C);
  l.GS = grad_stride(l.C);
  l.nb = (l.N + kProjBlock - 1) / kProjBlock;
  l.eps2d = opts->eps2d;
  l.q_cut = opts->q_cut;
  l.alpha_max = opts->alpha_max;
  l.t_eps = opts->t_eps;
  l.cap = cap;
  l.scap = scap;
  int64_t loss_blocks = 0;
  for (int v = 0; v < n_views; ++v) {
    const rogs_camera& c = cams[v];
    if (c.w < 1 || c.h < 1 || c.w > 16384 || c.h > 16384) { *why = "camera size out of range"; return ROGS_EINVAL; }
    if (c.model != ROGS_PINHOLE && c.model != ROGS_ORTHO) { *why = "unknown camera model"; return ROGS_EINVAL; }
    int vtw = tw, vth = th;
    if (!view_shape(c, tw, th, &vtw, &vth)) {
      *why = "camera.tile: tile_w must divide 64 and tile_w*tile_h must equal the options' area";
      return ROGS_EINVAL;
    }
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !is_fin(c.fx) || !is_fin(c.fy) || !is_fin(c.cx) ||
        !is_fin(c.cy) || !is_fin(c.z_near)) {
      *why = "camera intrinsics must be finite with fx, fy > 0";
      return ROGS_EINVAL;
    }
    for (int k = 0; k < 9; ++k) if (!is_fin(c.R_cw[k])) { *why = "camera pose not finite"; return ROGS_EINVAL; }
    for (int k = 0; k < 3; ++k) if (!is_fin(c.t_cw[k])) { *why = "camera pose not finite"; return ROGS_EINVAL; }
    const int64_t np = (int64_t)c.w * c.h;
    l.total_pix += np;
    l.max_view_pix = std::max(l.max_view_pix, np);
    const int64_t vt = (int64_t)((c.w + vtw - 1) / vtw) * ((c.h + vth - 1) / vth);
    l.total_tiles += vt;
    l.max_view_tiles = std::max(l.max_view_tiles, vt);
    loss_blocks += (np + 255) / 256;
  }
  if (l.total_tiles >= (int64_t(1) << 31) || l.total_pix >= (int64_t(1) << 40)) {
    *why = "batch too large";
    return ROGS_EINVAL;
  }
  l.slots = (int64_t)l.V * l.N;
  if (l.slots >= (int64_t(1) << 32)) { *why = "n_views * n must be < 2^32"; return ROGS_EINVAL; }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 1)); return r; };
  // the view table and the loss first-block table are contiguous, as in the
  // host stage, so one copy uploads both
  l.o_views = take(sizeof(ViewDev) * l.V + sizeof(int64_t) * (l.V + 1) +
                   sizeof(float) * 3 * loss_blocks);
  l.o_lpart = l.o_views + sizeof(ViewDev) * l.V;
  l.o_misc = take(sizeof(uint32_t) * kMiscCount);
  l.o_mcount = take(sizeof(uint32_t) * 2 * l.V);   // mask counts, then per-view loss sums
  l.o_cnt = take(4 * (size_t)l.slots);
  l.o_rec = take(32 * (size_t)l.slots);
  l.o_rect = take(8 * (size_t)l.slots);
  l.o_rspan = take(2 * kSpanRows * (size_t)l.slots);
  l.o_feat = take(4 * (size_t)l.N * l.FS);
  l.o_part = take(4 * (size_t)l.V * l.nb);
  l.o_partv = take(4 * (size_t)l.V * l.nb);
  l.o_parttmp = take(4 * 2 * scan_tmp_words((int64_t)l.V * l.nb));   // one sums table each
  l.o_keys = take(4 * (size_t)cap);          // tile of each pair
  l.o_keys2 = take(4 * (size_t)cap);         // alternate keys of the pair sort
  l.o_vals = take(4 * (size_t)cap);
  l.o_vals2 = take(4 * (size_t)cap);
  l.o_pslot = take(4 * (size_t)cap);
  l.o_spair = take(4 * (size_t)cap);
  l.o_pdep = take(4 * (size_t)cap);
  l.o_tcnt = take(4 * (size_t)l.total_tiles);
  l.o_tstart = take(4 * (size_t)l.total_tiles);
  l.o_tscan = take(4 * ((size_t)rogs::kTPart * ((l.total_tiles + rogs::kTileBlk - 1) / rogs::kTileBlk) +
                         rogs::kTPart));                          // tile layout partials
  l.o_bstart = take(4 * ((size_t)cap / rogs::kEmitPairs + 2));   // first slot of each emission block
  l.o_sval = take(4 * (size_t)scap);
  l.o_scnt = take(4 * (size_t)scap);
  l.o_soff = take(4 * (size_t)scap);
  l.o_ssum = take(4 * (size_t)l.GS * scap);
  l.o_long = take(4 * (size_t)scap);
  l.o_pos = take(4 * (size_t)l.slots);
  l.o_ranges = take(8 * (size_t)l.total_tiles);
  l.o_tinfo = take(16 * (size_t)l.total_tiles);
  l.o_tfin = take(4 * (size_t)l.total_pix);
  l.o_nlast = take(4 * (size_t)l.total_pix);
  l.o_drel = take(8 * (size_t)l.total_pix);
  l.o_gpair = take(4 * (size_t)cap * l.GS);
  l.o_histtmp = take(4 * 16);                  // tiles per launch-order bucket
  if (fused) {
    l.o_tpart = take(4 * 3 * (size_t)l.total_tiles);
    l.o_dzr = take(4 * (size_t)l.N);                          // grid-side dL/dz
    l.o_regpart = take(4 * (size_t)rogs::elev_reg_blocks(l.N));
    l.o_regtot = take(4);
    l.o_status = take(sizeof(uint32_t) * 4 + sizeof(StepState));   // misc[0..3] + step state
    l.o_mpart = take(4 * (size_t)l.V * rogs::mask_chunks(l));        // mask counts per chunk
  }
  l.total = o;
  *L = l;
  return ROGS_OK;
}

void ctx_fused_forget(rogs_ctx* c) {
  auto& F = c->fz;
  for (int k = 0; k < 2; ++k) {
    if (F.pending[k]) (void)hipEventSynchronize(F.done[k]);
    F.pending[k] = false;
  }
  if (F.exec) (void)hipGraphExecDestroy(F.exec);
  if (F.graph) (void)hipGraphDestroy(F.graph);
  F.exec = nullptr;
  F.graph = nullptr;
  F.valid = false;
  F.launched = 0;
}

int ctx_set_view_channels(rogs_ctx* c, const uint32_t* ch, int n) {
  if (!c || n < 0 || (n > 0 && !ch)) return ROGS_EINVAL;
  c->view_ch.assign(ch, ch + n);
  // elevation is formed from depth and alpha
  for (uint32_t& k : c->view_ch)
    if (k & ROGS_CH_ELEV) k |= ROGS_CH_D | ROGS_CH_A;
  return ROGS_OK;
}

}  // namespace rogs

namespace {

// Writes the device view table and the per-view first loss-block table of a
// batch into host memory at dst (sizeof(ViewDev) * V + 8 * (V + 1) bytes).
void fill_view_table(const Layout& L, const rogs_camera* cams, void* dst,
                     const uint32_t* ch = nullptr) {
  const size_t vbytes = sizeof(ViewDev) * L.V;
  ViewDev* vt = static_cast<ViewDev*>(dst);
  int64_t* fb = reinterpret_cast<int64_t*>(static_cast<char*>(dst) + vbytes);
  int64_t pix = 0, tiles = 0, blk = 0;
  for (int v = 0; v < L.V; ++v) {
    const rogs_camera& k = cams[v];
    ViewDev d;
    memset(&d, 0, sizeof(d));
    d.pix_off = pix;
    for (int j = 0; j < 9; ++j) d.R[j] = k.R_cw[j];
    for (int j = 0; j < 3; ++j) d.t[j] = k.t_cw[j];
    d.fx = k.fx; d.fy = k.fy; d.cx = k.cx; d.cy = k.cy;
    d.znear = k.z_near;
    d.o[0] = k.cull_o[0]; d.o[1] = k.cull_o[1];
    d.ex[0] = k.cull_ex[0]; d.ex[1] = k.cull_ex[1];
    d.ez[0] = k.cull_ez[0]; d.ez[1] = k.cull_ez[1];
    d.lat = k.cull_lat; d.fwd = k.cull_fwd;
    d.w = k.w; d.h = k.h; d.model = k.model;
    int vtw = L.tw, vth = L.th;
    (void)rogs::view_shape(k, L.tw, L.th, &vtw, &vth);     // validated by make_layout
    d.tw = (int16_t)vtw;
    d.th = (int16_t)vth;
    // the contract's clamp limits, rounded as the device rounded them in
    // binary64, and the exact reciprocals of the tile sides
    d.limx = (0.65 * (double)k.w) / (double)k.fx;
    d.limy = (0.65 * (double)k.h) / (double)k.fy;
    d.itw = 1.0 / (double)vtw;
    d.ith = 1.0 / (double)vth;
    d.tiles_x = (k.w + vtw - 1) / vtw;
    d.tiles_y = (k.h + vth - 1) / vth;
    d.tile_off = (int32_t)tiles;
    d.ch = ch ? ch[v] : (uint32_t)ROGS_CH_ALL;
    vt[v] = d;
    fb[v] = blk;
    pix += (int64_t)k.w * k.h;
    tiles += (int64_t)d.tiles_x * d.tiles_y;
    blk += ((int64_t)k.w * k.h + 255) / 256;
  }
  fb[L.V] = blk;
}

int upload_views(rogs_ctx* c, const Layout& L, const rogs_camera* cams, void* ws, hipStream_t st) {
  const size_t vbytes = sizeof(ViewDev) * L.V;
  const size_t fbytes = sizeof(int64_t) * (L.V + 1);
  const size_t need = vbytes + fbytes;
  if (c->stage_pending) {
    hipError_t e = hipEventSynchronize(c->stage_evt);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    c->stage_pending = false;
  }
  if (c->stage_bytes < need) {
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    hipError_t e = hipHostMalloc(&c->stage, need, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc");
    c->stage_bytes = need;
  }
  const bool own = c->view_ch.size() == (size_t)L.V;
  fill_view_table(L, cams, c->stage, own ? c->view_ch.data() : nullptr);
  c->batch_view_ch = own;
  c->view_ch.clear();
  hipError_t e = hipMemcpyAsync(rogs::at<void>(ws, L.o_views), c->stage, vbytes + fbytes,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(c->stage_evt, st);
  if (e != hipSuccess) return hip_fail(c, e, "view table upload");
  c->stage_pending = true;
  return ROGS_OK;
}

const char* kProfNames[ROGS_PROF_GROUPS] = {"project",    "scan",       "emit",
                                            "sort",       "ranges",     "render_fwd",
                                            "loss",       "render_bwd", "proj_bwd",
                                            "adam",       "fused_graph", "render_step"};

hipEvent_t prof_event(rogs_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// Brackets the launches between prof_begin and prof_end with two events on
// the launch stream (no-op unless timing is enabled).
void prof_begin(rogs_ctx* c, int group, hipStream_t st) {
  if (!c->prof) return;
  hipEvent_t e = prof_event(c);
  if (!e) return;
  (void)hipEventRecord(e, st);
  c->open_group = group;
  c->open_ev = e;
}

void prof_end(rogs_ctx* c, hipStream_t st) {
  if (!c->prof || c->open_group < 0) return;
  hipEvent_t e = prof_event(c);
  if (!e) return;
  (void)hipEventRecord(e, st);
  c->recs.push_back({c->open_group, c->open_ev, e});
  c->open_group = -1;
}

// Folds finished records into the per-group totals (waits for them).
int prof_collect(rogs_ctx* c) {
  for (const auto& r : c->recs) {
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_prof_read");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_prof_read");
    c->prof_ms[r.group] += ms;
    c->prof_n[r.group] += 1;
  }
  c->recs.clear();
  c->ev_used = 0;
  return ROGS_OK;
}

int need_batch(rogs_ctx* c, void* ws, bool sorted) {
  if (!c) return ROGS_EINVAL;
  if (!c->have_batch) return fail(c, ROGS_ESTATE, "no batch: call rogs_project first");
  if (ws != c->ws) return fail(c, ROGS_EINVAL, "workspace differs from the one given to rogs_project");
  if (sorted && !c->sorted) return fail(c, ROGS_ESTATE, "pairs not sorted: call rogs_bin_sort first");
  return ROGS_OK;
}

// Range check of the optimiser settings; the reason, or nullptr when valid.
const char* check_optim(const rogs_optim* o) {
  if (!(o->beta1 >= 0.0f && o->beta1 < 1.0f) || !(o->beta2 >= 0.0f && o->beta2 < 1.0f) ||
      !(o->eps > 0.0f) || o->total_steps < 0 || !is_fin(o->z_start) || !is_fin(o->z_end) ||
      (o->total_steps > 0 && !(o->z_start > 0.0f && o->z_end > 0.0f)))
    return "optimizer settings out of range";
  return nullptr;
}

int check_surfels(rogs_ctx* c, const rogs_surfels* s, const Layout& L) {
  if (!s) return fail(c, ROGS_EINVAL, "surfels is null");
  if (s->n != L.N || s->n_sem != L.C) return fail(c, ROGS_EINVAL, "surfels differ from the batch (n or n_sem)");
  if (!s->x || !s->y || !s->z || !s->q || !s->s || !s->alpha || !s->rgb || !s->sem)
    return fail(c, ROGS_EINVAL, "a surfel array pointer is null");
  return ROGS_OK;
}

}  // namespace

extern "C" {

int rogs_create(rogs_ctx** ctx) {
  if (!ctx) return ROGS_EINVAL;
  *ctx = nullptr;
  rogs_ctx* c = new (std::nothrow) rogs_ctx();
  if (!c) return ROGS_ENOMEM;
  hipError_t e = hipEventCreateWithFlags(&c->stage_evt, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->readback, 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (c->stage_evt) (void)hipEventDestroy(c->stage_evt);
    delete c;
    return ROGS_EHIP;
  }
  *ctx = c;
  return ROGS_OK;
}

void rogs_destroy(rogs_ctx* c) {
  if (!c) return;
  for (int k = 0; k < 2; ++k)
    if (c->fz.pending[k]) (void)hipEventSynchronize(c->fz.done[k]);
  if (c->fz.exec) (void)hipGraphExecDestroy(c->fz.exec);
  if (c->fz.graph) (void)hipGraphDestroy(c->fz.graph);
  for (int k = 0; k < 2; ++k) {
    if (c->fz.stage[k]) (void)hipHostFree(c->fz.stage[k]);
    if (c->fz.status[k]) (void)hipHostFree(c->fz.status[k]);
    if (c->fz.done[k]) (void)hipEventDestroy(c->fz.done[k]);
  }
  if (c->fz.cap_stream) (void)hipStreamDestroy(c->fz.cap_stream);
  if (c->fz.side) (void)hipStreamDestroy(c->fz.side);
  if (c->fz.fork) (void)hipEventDestroy(c->fz.fork);
  if (c->fz.join) (void)hipEventDestroy(c->fz.join);
  if (!c->recs.empty()) (void)hipEventSynchronize(c->recs.back().b);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->stage_pending) (void)hipEventSynchronize(c->stage_evt);
  if (c->stage) (void)hipHostFree(c->stage);
  if (c->readback) (void)hipHostFree(c->readback);
  if (c->stage_evt) (void)hipEventDestroy(c->stage_evt);
  delete c;
}

const char* rogs_last_error(const rogs_ctx* c) { return c ? c->err.c_str() : "null context"; }

void rogs_default_opts(rogs_render_opts* o) {
  if (!o) return;
  o->tile_w = 16;
  o->tile_h = 16;
  o->eps2d = 0.3f;
  o->q_cut = 9.0f;
  o->alpha_max = 0.99f;
  o->t_eps = 1e-6f;
  o->stage = 32;
}

int rogs_workspace_size(const rogs_surfels* s, const rogs_camera* cams, int32_t n_views,
                        const rogs_render_opts* opts, int64_t pair_capacity, int64_t slot_capacity,
                        size_t* bytes) {
  if (!bytes) return ROGS_EINVAL;
  Layout L;
  const char* why = nullptr;
  int r = rogs::make_layout(s, cams, n_views, opts, pair_capacity, slot_capacity, &L, &why);
  if (r != ROGS_OK) return r;
  *bytes = L.total;
  return ROGS_OK;
}

int rogs_project(rogs_ctx* c, const rogs_surfels* s, const rogs_camera* cams, int32_t n_views,
                 const rogs_render_opts* opts, void* ws, size_t ws_bytes, int64_t pair_capacity,
                 int64_t slot_capacity, void* stream) {
  if (!c) return ROGS_EINVAL;
  Layout L;
  const char* why = nullptr;
  int r = rogs::make_layout(s, cams, n_views, opts, pair_capacity, slot_capacity, &L, &why);
  if (r != ROGS_OK) return fail(c, r, why ? why : "invalid argument");
  r = check_surfels(c, s, L);
  if (r != ROGS_OK) return r;
  if (!ws) return fail(c, ROGS_EINVAL, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, ROGS_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(c, ROGS_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  hipStream_t st = static_cast<hipStream_t>(stream);
  c->have_batch = false;
  c->sorted = false;
  c->fwd_full = false;
  r = upload_views(c, L, cams, ws, st);
  if (r != ROGS_OK) return r;
  prof_begin(c, 0, st);
  rogs::launch_project(L, ws, s, true, st);
  prof_end(c, st);
  prof_begin(c, 1, st);
  rogs::launch_scan_part(L, ws, st);
  prof_end(c, st);
  r = check_launch(c, "rogs_project");
  if (r != ROGS_OK) return r;
  c->L = L;
  c->ws = ws;
  c->have_batch = true;
  c->n_pairs_host = -1;
  return ROGS_OK;
}

int rogs_pair_count(rogs_ctx* c, void* ws, int64_t* n_pairs, int32_t* overflow, void* stream) {
  int r = need_batch(c, ws, false);
  if (r != ROGS_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(c->readback, rogs::at<void>(ws, c->L.o_misc), 16,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_pair_count");
  if (n_pairs) *n_pairs = (int64_t)c->readback[rogs::kMiscPairs];
  if (overflow) *overflow = (int32_t)c->readback[rogs::kMiscOverflow];
  c->last_visible = (int64_t)c->readback[rogs::kMiscVisible];
  return ROGS_OK;
}

int rogs_batch_stats(rogs_ctx* c, void* ws, int64_t* stats, void* stream) {
  if (!stats) return fail(c, ROGS_EINVAL, "stats is null");
  int64_t n = 0;
  int32_t ovf = 0;
  int r = rogs_pair_count(c, ws, &n, &ovf, stream);
  if (r != ROGS_OK) return r;
  stats[0] = n;
  stats[1] = ovf;
  stats[2] = c->last_visible;
  stats[3] = c->L.total_pix;
  stats[4] = c->L.total_tiles;
  stats[5] = c->L.slots;
  return ROGS_OK;
}

int rogs_prof_enable(rogs_ctx* c, int32_t on) {
  if (!c) return ROGS_EINVAL;
  if (!on && c->prof) {
    int r = prof_collect(c);
    if (r != ROGS_OK) return r;
  }
  c->prof = on != 0;
  return ROGS_OK;
}

int rogs_prof_read(rogs_ctx* c, double* ms, int64_t* launches, int32_t n) {
  if (!c || !ms || !launches || n < ROGS_PROF_GROUPS) return c ? fail(c, ROGS_EINVAL, "bad arguments") : ROGS_EINVAL;
  int r = prof_collect(c);
  if (r != ROGS_OK) return r;
  for (int k = 0; k < ROGS_PROF_GROUPS; ++k) {
    ms[k] = c->prof_ms[k];
    launches[k] = c->prof_n[k];
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return ROGS_OK;
}

const char* rogs_prof_name(int32_t group) {
  return (group >= 0 && group < ROGS_PROF_GROUPS) ? kProfNames[group] : "";
}

int rogs_bin_sort(rogs_ctx* c, void* ws, int64_t* n_pairs_out, uint32_t flags, void* stream) {
  int r = need_batch(c, ws, false);
  if (r != ROGS_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int64_t n_host = -1, n_vis = -1;
  if (flags & ROGS_SYNC_COUNT) {
    int32_t ovf = 0;
    r = rogs_pair_count(c, ws, &n_host, &ovf, stream);
    if (r != ROGS_OK) return r;
    n_vis = c->last_visible;
    if (n_pairs_out) *n_pairs_out = n_host;
    if (n_host > c->L.cap || n_vis > c->L.scap)
      return fail(c, ROGS_ECAPACITY, "capacity (" + std::to_string(c->L.cap) + " pairs, " +
                                         std::to_string(c->L.scap) + " slots) too small for " +
                                         std::to_string(n_host) + " pairs, " +
                                         std::to_string(n_vis) + " slots");
  } else if (n_pairs_out) {
    *n_pairs_out = -1;
  }
  Layout& L = c->L;
  prof_begin(c, 3, st);
  rogs::launch_binning(L, ws, n_host, n_vis, st);
  prof_end(c, st);
  prof_begin(c, 4, st);
  (void)rogs::launch_ranges(L, ws, st);
  prof_end(c, st);
  r = check_launch(c, "rogs_bin_sort");
  if (r != ROGS_OK) return r;
  c->sorted = true;
  c->n_pairs_host = n_host;
  return ROGS_OK;
}

int rogs_render_fwd(rogs_ctx* c, const rogs_surfels* s, void* ws, float* out_images,
                    uint32_t channel_mask, void* stream) {
  int r = need_batch(c, ws, true);
  if (r != ROGS_OK) return r;
  r = check_surfels(c, s, c->L);
  if (r != ROGS_OK) return r;
  if (!out_images) return fail(c, ROGS_EINVAL, "out_images is null");
  if (channel_mask == 0u || (channel_mask & ~(uint32_t)ROGS_CH_ALL) != 0u)
    return fail(c, ROGS_EINVAL, "channel_mask must be a non-empty OR of ROGS_CH_* bits");
  // elevation is formed from depth and alpha
  uint32_t mask = channel_mask;
  if (mask & ROGS_CH_ELEV) mask |= ROGS_CH_D | ROGS_CH_A;
  constexpr uint32_t kPlanes = ROGS_CH_RGB | ROGS_CH_SEM | ROGS_CH_D | ROGS_CH_A;
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_begin(c, 5, st);
  int rr = rogs::launch_render_fwd(c->L, ws, s, out_images, mask, st);
  c->fwd_full = (mask & kPlanes) == kPlanes && !c->batch_view_ch;
  prof_end(c, st);
  if (rr != 0) return fail(c, ROGS_EINVAL, "unsupported n_sem / tile shape");
  return check_launch(c, "rogs_render_fwd");
}

int rogs_debug_work(rogs_ctx* c, void* ws, int64_t* evaluated, int64_t* contributing,
                    void* stream) {
  int r = need_batch(c, ws, true);
  if (r != ROGS_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t* misc = rogs::at<uint32_t>(ws, c->L.o_misc);
  rogs::fill_u32(misc + rogs::kMiscWork, 0u, 4, st);
  rogs::launch_count_work(c->L, ws, reinterpret_cast<unsigned long long*>(misc + rogs::kMiscWork),
                          st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->readback, misc + rogs::kMiscWork, 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_debug_work");
  const unsigned long long* w = reinterpret_cast<const unsigned long long*>(c->readback);
  if (evaluated) *evaluated = (int64_t)w[0];
  if (contributing) *contributing = (int64_t)w[1];
  return ROGS_OK;
}

int rogs_loss(rogs_ctx* c, void* ws, const float* out_images, const rogs_targets* t,
              float* dL_dout, float* loss_out, float* d_exposure, void* stream) {
  int r = need_batch(c, ws, true);
  if (r != ROGS_OK) return r;
  if (!out_images || !t || !dL_dout) return fail(c, ROGS_EINVAL, "null argument");
  if (!t->rgb || !t->label || !t->mask || !t->exposure)
    return fail(c, ROGS_EINVAL, "a target array pointer is null");
  if (!is_fin(t->lambda_c) || !is_fin(t->lambda_s) || !is_fin(t->view_scale))
    return fail(c, ROGS_EINVAL, "loss weights must be finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_begin(c, 6, st);
  rogs::launch_loss(c->L, ws, out_images, t, dL_dout, loss_out, d_exposure, st);
  prof_end(c, st);
  return check_launch(c, "rogs_loss");
}

int rogs_render_bwd(rogs_ctx* c, const rogs_surfels* s, void* ws, const float* out_images,
                    const float* dL_dout, float* grads, uint32_t flags, void* stream) {
  int r = need_batch(c, ws, true);
  if (r != ROGS_OK) return r;
  r = check_surfels(c, s, c->L);
  if (r != ROGS_OK) return r;
  if (!out_images || !dL_dout || !grads) return fail(c, ROGS_EINVAL, "null argument");
  if (!c->fwd_full)
    return fail(c, ROGS_ESTATE,
                "rogs_render_bwd needs a rogs_render_fwd of every plane (RGB, SEM, D, A) first");
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_begin(c, 7, st);
  int rr = rogs::launch_render_bwd(c->L, ws, s, out_images, dL_dout, st);
  prof_end(c, st);
  if (rr != 0) return fail(c, ROGS_EINVAL, "unsupported n_sem / tile shape");
  prof_begin(c, 8, st);
  rogs::launch_slot_sums(c->L, ws, st);
  rogs::launch_proj_bwd(c->L, ws, s, grads, (flags & ROGS_ACCUMULATE) != 0, st);
  prof_end(c, st);
  return check_launch(c, "rogs_render_bwd");
}

int rogs_adam_step(rogs_ctx* c, int32_t n, int32_t n_sem, float* params, const float* grads,
                   float* m, float* v, float* s_act, float* alpha_act, const rogs_optim* optim,
                   int64_t step, float* exposure, const float* d_exposure, float* m_exp,
                   float* v_exp, int32_t n_views, void* stream) {
  if (!c) return ROGS_EINVAL;
  if (n < 1) return fail(c, ROGS_EINVAL, "n must be >= 1");
  if (!rogs::sem_supported(n_sem)) return fail(c, ROGS_EINVAL, "n_sem must be 1..8 or 16");
  if (!params || !grads || !m || !v || !s_act || !alpha_act || !optim)
    return fail(c, ROGS_EINVAL, "null argument");
  if (step < 1) return fail(c, ROGS_EINVAL, "step must be >= 1");
  const char* why = check_optim(optim);
  if (why) return fail(c, ROGS_EINVAL, why);
  if (exposure && (!d_exposure || !m_exp || !v_exp || n_views < 1))
    return fail(c, ROGS_EINVAL, "exposure group needs gradients, moments and n_views >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  prof_begin(c, 9, st);
  rogs::launch_adam(n, n_sem, params, grads, m, v, s_act, alpha_act, *optim, step, exposure,
                    d_exposure, m_exp, v_exp, n_views, st);
  prof_end(c, st);
  return check_launch(c, "rogs_adam_step");
}

int rogs_debug_pairs(rogs_ctx* c, void* ws, uint64_t* keys, int32_t* surfel_ids, int32_t* views,
                     int64_t cap, uint32_t* ranges, int64_t n_tiles, void* stream) {
  int r = need_batch(c, ws, true);
  if (r != ROGS_OK) return r;
  const Layout& L = c->L;
  int64_t P = 0;
  int32_t ovf = 0;
  r = rogs_pair_count(c, ws, &P, &ovf, stream);
  if (r != ROGS_OK) return r;
  if (P > L.cap) P = L.cap;
  if (cap < P || !keys || !surfel_ids || !views) return fail(c, ROGS_EINVAL, "output capacity too small");
  if (ranges && n_tiles < L.total_tiles) return fail(c, ROGS_EINVAL, "ranges capacity too small");
  std::vector<uint32_t> tiles(P), vals(P), pslot(P), rg(2 * (size_t)L.total_tiles);
  std::vector<float> rec(8 * (size_t)L.slots);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(rg.data(), rogs::at<void>(ws, L.o_ranges), 8 * L.total_tiles,
                                hipMemcpyDeviceToHost, st);
  if (P > 0) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(vals.data(), rogs::at<void>(ws, L.o_vals), 4 * P, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(pslot.data(), rogs::at<void>(ws, L.o_pslot), 4 * P, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(rec.data(), rogs::at<void>(ws, L.o_rec), 32 * (size_t)L.slots,
                         hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_debug_pairs");
  if (ranges) memcpy(ranges, rg.data(), 8 * (size_t)L.total_tiles);
  // tile of each sorted position, from the ranges (they partition [0, P))
  for (int64_t t = 0; t < L.total_tiles; ++t)
    for (uint32_t k = rg[2 * t]; k < rg[2 * t + 1] && (int64_t)k < P; ++k) tiles[k] = (uint32_t)t;
  for (int64_t k = 0; k < P; ++k) {
    const uint32_t sl = pslot[vals[k]];
    surfel_ids[k] = (int32_t)(sl % (uint32_t)L.N);
    views[k] = (int32_t)(sl / (uint32_t)L.N);
    uint32_t db;
    memcpy(&db, &rec[8 * (size_t)sl + 7], 4);
    keys[k] = ((uint64_t)tiles[k] << 32) | db;
  }
  return ROGS_OK;
}

int rogs_debug_records(rogs_ctx* c, void* ws, float* rec, int32_t* rect, uint32_t* count,
                       void* stream) {
  int r = need_batch(c, ws, false);
  if (r != ROGS_OK) return r;
  if (!rec || !rect || !count) return fail(c, ROGS_EINVAL, "null argument");
  const Layout& L = c->L;
  const size_t S = (size_t)L.slots;
  std::vector<uint32_t> rc(2 * S);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(rec, rogs::at<void>(ws, L.o_rec), 32 * S, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rc.data(), rogs::at<void>(ws, L.o_rect), 8 * S, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(count, rogs::at<void>(ws, L.o_cnt), 4 * S, hipMemcpyDeviceToHost, st);
  // the scanned visible counts per (view, projection block) and their total:
  // a block with no visible slot in a view writes no counts
  const size_t nparts = (size_t)L.V * L.nb;
  std::vector<uint32_t> partv(nparts + 1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(partv.data(), rogs::at<void>(ws, L.o_partv), 4 * nparts,
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(partv.data() + nparts, rogs::at<uint32_t>(ws, L.o_misc) + rogs::kMiscVisible,
                       4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_debug_records");
  for (size_t k = 0; k < S; ++k) {
    const size_t pb = (k / (size_t)L.N) * (size_t)L.nb + (k % (size_t)L.N) / rogs::kProjBlock;
    if (partv[pb + 1] == partv[pb]) count[k] = 0;
    if (count[k] == 0) {   // culled slots keep no record
      for (int j = 0; j < 8; ++j) rec[8 * k + j] = 0.0f;
      for (int j = 0; j < 4; ++j) rect[4 * k + j] = 0;
      continue;
    }
    rect[4 * k + 0] = (int32_t)(rc[2 * k] & 0xffff);
    rect[4 * k + 1] = (int32_t)(rc[2 * k] >> 16);
    rect[4 * k + 2] = (int32_t)(rc[2 * k + 1] & 0xffff);
    rect[4 * k + 3] = (int32_t)(rc[2 * k + 1] >> 16);
  }
  return ROGS_OK;
}

// ------------------------------------------------------------ fused step

namespace {

bool same_bytes(const void* a, const void* b, size_t n) { return memcmp(a, b, n) == 0; }

rogs_surfels fused_surfels(const rogs_train_state* t) {
  rogs_surfels s;
  const size_t N = (size_t)t->n;
  s.n = t->n;
  s.n_sem = t->n_sem;
  s.x = t->x;
  s.y = t->y;
  s.z = t->params;
  s.q = t->params + N;
  s.s = t->s_act;
  s.alpha = t->alpha_act;
  s.rgb = t->params + 8 * N;
  s.sem = t->params + 11 * N;
  return s;
}

int check_fused_args(rogs_ctx* c, const rogs_train_state* t, const rogs_targets* tg,
                     const rogs_optim* o) {
  if (!t || !tg || !o) return fail(c, ROGS_EINVAL, "null argument");
  if (!t->x || !t->y || !t->params || !t->m || !t->v || !t->s_act || !t->alpha_act ||
      !t->exposure || !t->m_exp || !t->v_exp || !t->d_exposure || !t->step_state)
    return fail(c, ROGS_EINVAL, "a training-state pointer is null");
  if (reinterpret_cast<uintptr_t>(t->step_state) % 16 != 0)
    return fail(c, ROGS_EINVAL, "step_state must be 16-byte aligned");
  if (!tg->rgb || !tg->label || !tg->mask || tg->exposure != t->exposure)
    return fail(c, ROGS_EINVAL, "targets incomplete, or targets.exposure differs from the state's");
  if ((tg->nbr && !is_fin(tg->lambda_smooth)) || (tg->zbar && !is_fin(tg->lambda_z)))
    return fail(c, ROGS_EINVAL, "grid-side loss weights must be finite");
  const char* why = check_optim(o);
  if (why) return fail(c, ROGS_EINVAL, why);
  return ROGS_OK;
}

rogs::AdamArgs fused_adam_args(const rogs_optim* o, const Layout& L, void* ws, const void* state) {
  rogs::AdamArgs aa{};
  aa.lr = o->lr;
  aa.b1 = o->beta1;
  aa.b2 = o->beta2;
  aa.eps = o->eps;
  aa.z_start = o->z_start;
  aa.z_end = o->z_end;
  aa.total_steps = o->total_steps;
  aa.step = 0;
  aa.state = static_cast<const rogs::StepState*>(state);
  aa.misc = rogs::at<const uint32_t>(ws, L.o_misc);
  return aa;
}

// The whole step on one stream; captured once into a graph or run eagerly.
// Returns the sort's buffer parity.
int fused_sequence(rogs_ctx* c, Layout& L, const rogs_train_state* t, const rogs_targets* tg,
                   const rogs_optim* o, void* ws, hipStream_t st) {
  rogs_surfels s = fused_surfels(t);
  prof_begin(c, 0, st);
  // the same launch counts the loss mask per view and clears the tile counters
  rogs::launch_project(L, ws, &s, true, st, tg->mask);
  prof_end(c, st);
  prof_begin(c, 1, st);
  rogs::launch_scan_part(L, ws, st, true);
  prof_end(c, st);
  prof_begin(c, 3, st);
  rogs::launch_binning(L, ws, -1, -1, st, true);
  prof_end(c, st);
  prof_begin(c, 4, st);
  hipError_t e = rogs::launch_ranges(L, ws, st, c->fz.side, c->fz.fork, c->fz.join);
  prof_end(c, st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused: depth sort streams");
  rogs::FusedLoss fl;
  fl.tgt = tg->rgb;
  fl.label = tg->label;
  fl.mask = tg->mask;
  fl.expo = tg->exposure;
  fl.mcount = rogs::at<const uint32_t>(ws, L.o_mcount);
  fl.lam_c = tg->lambda_c;
  fl.lam_s = tg->lambda_s;
  fl.scale = tg->view_scale;
  fl.part = rogs::at<float>(ws, L.o_tpart);
  prof_begin(c, 11, st);
  int r = rogs::launch_render_step(L, ws, fl, st);
  prof_end(c, st);
  if (r != 0) return fail(c, ROGS_EINVAL, "unsupported n_sem / tile shape");
  rogs::AdamArgs aa = fused_adam_args(o, L, ws, t->step_state);
  prof_begin(c, 6, st);
  // per-view loss sums, dL/d(a, b) and the exposure's Adam step
  rogs::launch_loss_tiles(L, ws, t->d_exposure, t->exposure, t->m_exp, t->v_exp, aa, st);
  prof_end(c, st);
  prof_begin(c, 8, st);
  // grid-side terms (Eq. 10, 11) from the heights before the update
  const bool reg = tg->nbr || tg->zbar;
  if (reg)
    rogs::launch_elev_reg(L.N, t->params, tg->nbr, tg->lambda_smooth, tg->zbar, tg->lambda_z,
                          rogs::at<float>(ws, L.o_dzr), nullptr, rogs::at<float>(ws, L.o_regpart),
                          rogs::at<float>(ws, L.o_regtot), false, st);
  rogs::launch_slot_sums(L, ws, st, false);      // misc's long-slot count is still zero
  rogs::launch_proj_bwd_adam(L, ws, t->x, t->y, t->params, t->m, t->v, t->s_act, t->alpha_act,
                             t->grads, aa, nullptr, nullptr, nullptr, nullptr,
                             reg ? rogs::at<const float>(ws, L.o_dzr) : nullptr, st);
  prof_end(c, st);
  rogs::launch_step_end(L, ws, static_cast<rogs::StepState*>(t->step_state), aa,
                        reg ? rogs::at<const float>(ws, L.o_regtot) : nullptr, st);
  return ROGS_OK;
}

}  // namespace

int rogs_fused_workspace_size(const rogs_train_state* t, const rogs_camera* cams, int32_t n_views,
                              const rogs_render_opts* opts, int64_t pair_capacity,
                              int64_t slot_capacity, size_t* bytes) {
  if (!t || !bytes) return ROGS_EINVAL;
  rogs_surfels s = fused_surfels(t);
  Layout L;
  const char* why = nullptr;
  int r = rogs::make_layout(&s, cams, n_views, opts, pair_capacity, slot_capacity, &L, &why, true);
  if (r != ROGS_OK) return r;
  *bytes = L.total;
  return ROGS_OK;
}

int rogs_step_fused(rogs_ctx* c, const rogs_train_state* t, const rogs_camera* cams,
                    int32_t n_views, const rogs_render_opts* opts, const rogs_targets* tg,
                    const rogs_optim* o, void* ws, size_t ws_bytes, int64_t pair_capacity,
                    int64_t slot_capacity, uint32_t flags, void* stream) {
  if (!c) return ROGS_EINVAL;
  int r = check_fused_args(c, t, tg, o);
  if (r != ROGS_OK) return r;
  rogs_surfels s = fused_surfels(t);
  Layout L;
  const char* why = nullptr;
  r = rogs::make_layout(&s, cams, n_views, opts, pair_capacity, slot_capacity, &L, &why, true);
  if (r != ROGS_OK) return fail(c, r, why ? why : "invalid argument");
  if (!ws) return fail(c, ROGS_EINVAL, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(c, ROGS_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(c, ROGS_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto& F = c->fz;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    if (F.done[k]) continue;
    e = hipEventCreateWithFlags(&F.done[k], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&F.status[k], 128, hipHostMallocDefault);
    if (e == hipSuccess) memset(F.status[k], 0, 128);
  }
  if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused setup");
  // this step's buffers were last used two steps ago: that step must have
  // finished before its status is read and its pinned camera table is
  // rewritten (the step launched last may still be queued)
  const int p = (int)(F.launched & 1);
  if (F.pending[p]) {
    e = hipEventSynchronize(F.done[p]);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused");
    F.pending[p] = false;
    if (F.status[p][rogs::kMiscOverflow])
      return fail(c, ROGS_ECAPACITY, "an earlier fused step overflowed the pair capacity (" +
                                         std::to_string(F.status[p][rogs::kMiscPairs]) +
                                         " pairs) and was skipped");
  }
  std::vector<int32_t> sizes;
  for (int v = 0; v < n_views; ++v) {
    sizes.push_back(cams[v].w);
    sizes.push_back(cams[v].h);
    sizes.push_back(cams[v].model);
    sizes.push_back(cams[v].tile);
  }
  const bool eager = (flags & ROGS_FUSED_EAGER) != 0;
  const bool same = F.valid && F.ws == ws && F.st == st && F.flags == flags &&
                    same_bytes(&F.ts, t, sizeof(*t)) && same_bytes(&F.tg, tg, sizeof(*tg)) &&
                    same_bytes(&F.opt, o, sizeof(*o)) && same_bytes(&F.opts, opts, sizeof(*opts)) &&
                    F.sizes == sizes && F.L.total == L.total && F.L.cap == L.cap &&
                    F.L.scap == L.scap;
  const size_t need = sizeof(ViewDev) * L.V + sizeof(int64_t) * (L.V + 1);
  if (!same) {
    if (F.exec) (void)hipGraphExecDestroy(F.exec);
    if (F.graph) (void)hipGraphDestroy(F.graph);
    F.exec = nullptr;
    F.graph = nullptr;
    F.valid = false;
    if (F.stage_bytes < need) {
      // both stages may be read by queued copies
      for (int k = 0; k < 2; ++k) {
        if (F.pending[k]) {
          e = hipEventSynchronize(F.done[k]);
          if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused");
        }
      }
      for (int k = 0; k < 2; ++k) {
        if (F.stage[k]) (void)hipHostFree(F.stage[k]);
        F.stage[k] = nullptr;
      }
      F.stage_bytes = 0;
      for (int k = 0; k < 2; ++k) {
        e = hipHostMalloc(&F.stage[k], need, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(c, e, "hipHostMalloc");
      }
      F.stage_bytes = need;
    }
  }
  fill_view_table(L, cams, F.stage[p]);
  {
    const size_t vbytes = sizeof(ViewDev) * L.V, fbytes = sizeof(int64_t) * (L.V + 1);
    e = hipMemcpyAsync(rogs::at<void>(ws, L.o_views), F.stage[p], vbytes + fbytes,
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused: camera table");
  }
  if (!F.side) {
    e = hipStreamCreateWithFlags(&F.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&F.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&F.join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused: side stream");
  }
  if (eager) {
    Layout Lr = L;
    r = fused_sequence(c, Lr, t, tg, o, ws, st);
    if (r != ROGS_OK) return r;
    r = check_launch(c, "rogs_step_fused");
    if (r != ROGS_OK) return r;
    F.L = Lr;
  } else {
    if (!same) {
      Layout Lr = L;
      if (!F.cap_stream) {
        e = hipStreamCreateWithFlags(&F.cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
      }
      // captured work touches the workspace: let earlier work on st finish first
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      e = hipStreamBeginCapture(F.cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
      const bool prof = c->prof;
      c->prof = false;                 // no timing events inside the graph
      r = fused_sequence(c, Lr, t, tg, o, ws, F.cap_stream);
      c->prof = prof;
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(F.cap_stream, &g);
      if (r != ROGS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
      }
      if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
      e = hipGraphInstantiate(&F.exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(c, e, "hipGraphInstantiate");
      }
      F.graph = g;
      F.L = Lr;
    }
    prof_begin(c, 10, st);
    e = hipGraphLaunch(F.exec, st);
    prof_end(c, st);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
  }
  F.valid = true;
  F.ws = ws;
  F.st = st;
  F.flags = flags;
  F.ts = *t;
  F.tg = *tg;
  F.opt = *o;
  F.opts = *opts;
  F.sizes = sizes;
  // the step's last kernel left misc[0..3] and the step state side by side
  e = hipMemcpyAsync(F.status[p], rogs::at<void>(ws, F.L.o_status),
                     16 + sizeof(rogs::StepState), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(F.done[p], st);
  if (e != hipSuccess) return hip_fail(c, e, "rogs_step_fused: status");
  F.pending[p] = true;
  F.last = p;
  F.launched += 1;
  // the batch state of the plain entry points no longer describes the workspace
  if (c->ws == ws) {
    c->have_batch = false;
    c->sorted = false;
  }
  return ROGS_OK;
}

int rogs_fused_status(rogs_ctx* c, int64_t* stats, float* loss) {
  if (!c) return ROGS_EINVAL;
  if (!stats) return fail(c, ROGS_EINVAL, "stats is null");
  auto& F = c->fz;
  if (F.launched == 0) return fail(c, ROGS_ESTATE, "no fused step has run");
  // both steps in flight are waited for and seen: the next step call does
  // not report them again
  for (int k = 0; k < 2; ++k) {
    if (!F.pending[k]) continue;
    hipError_t e = hipEventSynchronize(F.done[k]);
    if (e != hipSuccess) return hip_fail(c, e, "rogs_fused_status");
    F.pending[k] = false;
  }
  const uint32_t* stt = F.status[F.last];
  const rogs::StepState* ss = reinterpret_cast<const rogs::StepState*>(
      reinterpret_cast<const char*>(stt) + 16);
  stats[0] = stt[rogs::kMiscPairs];
  stats[1] = stt[rogs::kMiscOverflow];
  stats[2] = stt[rogs::kMiscVisible];
  stats[3] = ss->step;
  stats[4] = ss->skipped;
  stats[5] = F.L.total_pix;
  stats[6] = F.L.total_tiles;
  stats[7] = F.L.slots;
  if (loss) *loss = ss->loss;
  return ROGS_OK;
}

}  // extern "C"
