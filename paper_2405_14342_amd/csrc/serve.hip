// Continuous-batching render server over a resident surfel map.
//
// Requests (one view each, a channel set and a caller-owned device output
// buffer) are queued by rogs_serve_submit from any thread.  The server runs
// `lanes` worker threads; each owns a library context, a stream and an equal
// share of the arena.  Whenever a lane is idle it takes every queued request
// that fits (up to max_views views and its arena share), so requests that
// arrive while other batches are on the GPU start on a free lane and their
// work overlaps on the device.  A lane renders its requests as one batch
// (rogs_project + rogs_bin_sort with the pair count on the device +
// rogs_render_fwd into its arena share, each view compositing only the planes
// its request asked for), copies each request's channels into its buffer, and
// waits for the batch.  If the batch overflowed the pair
// capacity that the arena allows, it is split in two and both halves run
// again; a single view that does not fit fails with ROGS_ECAPACITY.  Each
// view is rendered independently of the others in its batch (per-view tile
// lists and compositing), so a request's output does not depend on what it
// was batched with.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rogs_internal.h"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Copies the requested planes of one rendered view (5 + C planes: R G B,
// sem, D, A) into the request's buffer, in the order RGB, SEM, D, A, ELEV.
// ELEV = elev_ref - D / A where A > 0, NaN where nothing was composited.
__global__ __launch_bounds__(256) void k_serve_extract(const float* __restrict__ img, int64_t npix,
                                                       int C, uint32_t ch, float elev_ref,
                                                       float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  int o = 0;
  if (ch & ROGS_CH_RGB)
    for (int c = 0; c < 3; ++c) out[(o++) * npix + p] = img[c * npix + p];
  if (ch & ROGS_CH_SEM)
    for (int c = 0; c < C; ++c) out[(o++) * npix + p] = img[(3 + c) * npix + p];
  const float D = img[(3 + C) * npix + p], A = img[(4 + C) * npix + p];
  if (ch & ROGS_CH_D) out[(o++) * npix + p] = D;
  if (ch & ROGS_CH_A) out[(o++) * npix + p] = A;
  if (ch & ROGS_CH_ELEV)
    out[(o++) * npix + p] = (A > 0.0f) ? elev_ref - D / A : __int_as_float(0x7fc00000);
}

struct Item {
  uint64_t ticket;
  rogs_request req;
  int64_t t_arrive;
};

}  // namespace

struct ServeLane {
  uint8_t* arena = nullptr;       // this lane's share of the arena
  size_t arena_bytes = 0;
  rogs_ctx* ctx = nullptr;        // owned by the lane's thread
  hipStream_t st = nullptr;
  std::thread thread;
  int init_status = ROGS_OK;
  bool ready = false;
};

struct rogs_server {
  int device = 0;
  rogs_surfels map{};
  rogs_render_opts opts{};
  size_t lane_bytes = 0;
  int max_views = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Item> queue;
  std::unordered_map<uint64_t, rogs_result> results;   // pending (status NOT_READY) or done
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<ServeLane> lanes;
  int64_t stats[8] = {};          // batches, views, splits, max batch, capacity failures,
                                  // -, -, most batches on the GPU at once
  int64_t busy = 0;
};

namespace {

size_t image_bytes(const rogs_server* s, int64_t pix) {
  return ((size_t)(5 + s->map.n_sem) * (size_t)pix * 4 + 255) / 256 * 256;
}

// Largest pair capacity whose workspace fits `room` bytes (0 if none).
int64_t fit_capacity(const rogs_server* s, const std::vector<rogs_camera>& cams, size_t room) {
  size_t b0 = 0, b1 = 0;
  if (rogs_workspace_size(&s->map, cams.data(), (int)cams.size(), &s->opts, 0, 0, &b0) != ROGS_OK ||
      b0 > room)
    return 0;
  int64_t lo = 0, hi = (int64_t(1) << 31) - 1;
  if (rogs_workspace_size(&s->map, cams.data(), (int)cams.size(), &s->opts, hi, 0, &b1) == ROGS_OK &&
      b1 <= room)
    return hi;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    size_t b = 0;
    if (rogs_workspace_size(&s->map, cams.data(), (int)cams.size(), &s->opts, mid, 0, &b) ==
            ROGS_OK && b <= room)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Renders one batch on a lane; returns false if it overflowed and must be split.
bool run_batch(rogs_server* s, ServeLane& ln, std::vector<Item>& batch) {
  std::vector<rogs_camera> cams;
  int64_t pix = 0;
  for (const Item& it : batch) {
    cams.push_back(it.req.cam);
    pix += (int64_t)it.req.cam.w * it.req.cam.h;
  }
  const size_t img = image_bytes(s, pix);
  const int64_t t_start = now_ns();
  auto finish = [&](int status) {
    const int64_t t = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    for (const Item& it : batch) {
      rogs_result& r = s->results[it.ticket];
      r.status = status;
      r.batch_views = (int32_t)batch.size();
      r.t_arrive_ns = it.t_arrive;
      r.t_start_ns = t_start;
      r.t_done_ns = t;
    }
  };
  const int64_t cap = img < ln.arena_bytes ? fit_capacity(s, cams, ln.arena_bytes - img) : 0;
  if (cap <= 0) {
    if (batch.size() > 1) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stats[2] += 1;
      return false;
    }
    finish(ROGS_ECAPACITY);
    return true;
  }
  size_t wsb = 0;
  (void)rogs_workspace_size(&s->map, cams.data(), (int)cams.size(), &s->opts, cap, 0, &wsb);
  void* ws = ln.arena;
  float* images = reinterpret_cast<float*>(ln.arena + wsb);
  // each view composites only the planes its request asked for
  std::vector<uint32_t> chans;
  for (const Item& it : batch) chans.push_back(it.req.channels);
  int r = rogs::ctx_set_view_channels(ln.ctx, chans.data(), (int)chans.size());
  if (r == ROGS_OK)
    r = rogs_project(ln.ctx, &s->map, cams.data(), (int)cams.size(), &s->opts, ws, wsb, cap, 0,
                     ln.st);
  if (r == ROGS_OK) r = rogs_bin_sort(ln.ctx, ws, nullptr, 0u, ln.st);
  if (r == ROGS_OK) r = rogs_render_fwd(ln.ctx, &s->map, ws, images, ROGS_CH_ALL, ln.st);
  int64_t off = 0;
  const int C = s->map.n_sem;
  for (size_t k = 0; k < batch.size() && r == ROGS_OK; ++k) {
    const rogs_request& q = batch[k].req;
    const int64_t np = (int64_t)q.cam.w * q.cam.h;
    hipLaunchKernelGGL(k_serve_extract, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, ln.st,
                       images + (5 + C) * off, np, C, q.channels, q.elev_ref, q.out);
    off += np;
  }
  if (r == ROGS_OK && hipGetLastError() != hipSuccess) r = ROGS_EHIP;
  int64_t n = 0;
  int32_t ovf = 0;
  if (r == ROGS_OK) r = rogs_pair_count(ln.ctx, ws, &n, &ovf, ln.st);   // waits for the batch
  if (r == ROGS_OK && ovf) {
    if (batch.size() > 1) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stats[2] += 1;
      return false;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[4] += 1;
    r = ROGS_ECAPACITY;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[0] += 1;
    s->stats[1] += (int64_t)batch.size();
    if ((int64_t)batch.size() > s->stats[3]) s->stats[3] = (int64_t)batch.size();
  }
  finish(r);
  return true;
}

void worker_main(rogs_server* s, int lane) {
  ServeLane& ln = s->lanes[lane];
  int r = hipSetDevice(s->device) == hipSuccess ? ROGS_OK : ROGS_EHIP;
  if (r == ROGS_OK) r = rogs_create(&ln.ctx);
  if (r == ROGS_OK && hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking) != hipSuccess)
    r = ROGS_EHIP;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ln.init_status = r;
    ln.ready = true;
  }
  s->cv.notify_all();
  if (r != ROGS_OK) return;
  std::vector<Item> batch;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
      if (s->queue.empty()) break;                 // stop requested and drained
      // continuous batching: everything queued now, up to max_views views
      // whose images leave room for a workspace in this lane's arena share
      int64_t pix = 0;
      batch.clear();
      while (!s->queue.empty() && (int)batch.size() < s->max_views) {
        const Item& it = s->queue.front();
        const int64_t np = (int64_t)it.req.cam.w * it.req.cam.h;
        if (!batch.empty() && image_bytes(s, pix + np) * 2 > ln.arena_bytes) break;
        pix += np;
        batch.push_back(it);
        s->queue.pop_front();
      }
      s->busy += 1;
      if (s->busy > s->stats[7]) s->stats[7] = s->busy;
    }
    // split until every part fits; parts keep the arrival order
    std::deque<std::vector<Item>> work;
    work.push_back(batch);
    while (!work.empty()) {
      std::vector<Item> b = std::move(work.front());
      work.pop_front();
      if (run_batch(s, ln, b)) continue;
      const size_t h = b.size() / 2;
      work.push_front(std::vector<Item>(b.begin() + h, b.end()));
      work.push_front(std::vector<Item>(b.begin(), b.begin() + h));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->busy -= 1;
  }
}

void stop_lanes(rogs_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (ServeLane& ln : s->lanes) {
    if (ln.thread.joinable()) ln.thread.join();
    if (ln.st) (void)hipStreamDestroy(ln.st);
    rogs_destroy(ln.ctx);
    ln.st = nullptr;
    ln.ctx = nullptr;
  }
}

}  // namespace

extern "C" {

int rogs_server_create(rogs_server** out, const rogs_surfels* map, const rogs_render_opts* opts,
                       void* arena, size_t arena_bytes, int32_t max_views, int32_t lanes,
                       int32_t device) {
  if (!out) return ROGS_EINVAL;
  *out = nullptr;
  if (!map || !opts || !arena || max_views < 1 || max_views > 256 || lanes < 1 || lanes > 8 ||
      device < 0)
    return ROGS_EINVAL;
  if (reinterpret_cast<uintptr_t>(arena) % 256 != 0) return ROGS_EINVAL;
  if (!map->x || !map->y || !map->z || !map->q || !map->s || !map->alpha || !map->rgb || !map->sem)
    return ROGS_EINVAL;
  rogs_camera probe{};
  probe.w = probe.h = 8;
  probe.fx = probe.fy = 1.0f;
  probe.R_cw[0] = probe.R_cw[4] = probe.R_cw[8] = 1.0f;
  size_t b = 0;
  if (rogs_workspace_size(map, &probe, 1, opts, 0, 0, &b) != ROGS_OK) return ROGS_EINVAL;
  rogs_server* s = new (std::nothrow) rogs_server();
  if (!s) return ROGS_ENOMEM;
  s->device = device;
  s->map = *map;
  s->opts = *opts;
  s->max_views = max_views;
  s->lane_bytes = arena_bytes / (size_t)lanes / 256 * 256;
  s->lanes.resize((size_t)lanes);
  for (int k = 0; k < lanes; ++k) {
    s->lanes[k].arena = static_cast<uint8_t*>(arena) + (size_t)k * s->lane_bytes;
    s->lanes[k].arena_bytes = s->lane_bytes;
  }
  int r = ROGS_OK;
  for (int k = 0; k < lanes; ++k) s->lanes[k].thread = std::thread(worker_main, s, k);
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] {
      for (const ServeLane& ln : s->lanes) if (!ln.ready) return false;
      return true;
    });
    for (const ServeLane& ln : s->lanes) if (ln.init_status != ROGS_OK) r = ln.init_status;
  }
  if (r != ROGS_OK) {
    stop_lanes(s);
    delete s;
    return r;
  }
  *out = s;
  return ROGS_OK;
}

int rogs_serve_submit(rogs_server* s, const rogs_request* req, uint64_t* ticket) {
  if (!s || !req || !ticket) return ROGS_EINVAL;
  *ticket = 0;
  if (!req->out || req->channels == 0 || (req->channels & ~ROGS_CH_ALL) != 0) return ROGS_EINVAL;
  size_t b = 0;
  if (rogs_workspace_size(&s->map, &req->cam, 1, &s->opts, 0, 0, &b) != ROGS_OK) return ROGS_EINVAL;
  // admission: the view's images and a minimal workspace must fit the arena
  if (image_bytes(s, (int64_t)req->cam.w * req->cam.h) + b > s->lane_bytes) return ROGS_EREJECT;
  const int64_t t = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return ROGS_ESTATE;
    if (s->queue.size() >= 65536) return ROGS_EREJECT;
    const uint64_t id = s->next_ticket++;
    rogs_result pending{};
    pending.status = ROGS_NOT_READY;
    pending.t_arrive_ns = t;
    s->results[id] = pending;
    s->queue.push_back(Item{id, *req, t});
    *ticket = id;
  }
  s->cv.notify_all();
  return ROGS_OK;
}

int rogs_serve_poll(rogs_server* s, uint64_t ticket, rogs_result* res) {
  if (!s || !res) return ROGS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return ROGS_EINVAL;
  *res = it->second;
  if (it->second.status == ROGS_NOT_READY) return ROGS_NOT_READY;
  s->results.erase(it);
  return ROGS_OK;
}

int rogs_server_stats(rogs_server* s, int64_t* stats) {
  if (!s || !stats) return ROGS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  for (int k = 0; k < 5; ++k) stats[k] = s->stats[k];
  stats[5] = (int64_t)s->queue.size();
  stats[6] = s->stats[7];
  return ROGS_OK;
}

void rogs_server_destroy(rogs_server* s) {
  if (!s) return;
  stop_lanes(s);
  delete s;
}

}  // extern "C"
