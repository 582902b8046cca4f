// The serving runtime under host sanitizers (test infrastructure, built by
// the package's build step with AddressSanitizer and UndefinedBehaviorSanitizer
// on host code only): a server over a small synthetic map, requests of three
// sizes and four channel sets submitted from two threads and polled to
// completion, the argument errors, the statistics and shutdown.  Exits 0 and
// prints "serve sanitizer run: ok" when every request completed without error.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "../include/rogs.h"

#define CHECK(x)                                                              \
  do {                                                                        \
    if (!(x)) {                                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__);          \
      exit(1);                                                                \
    }                                                                         \
  } while (0)

static float* dev_copy(const std::vector<float>& h) {
  float* d = nullptr;
  CHECK(hipMalloc(&d, h.size() * sizeof(float)) == hipSuccess);
  CHECK(hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess);
  return d;
}

int main() {
  // 64 x 64 surfels on a 0.1 m grid, flat, facing up, C = 4 classes
  const int G = 64, N = G * G, C = 4;
  std::vector<float> x(N), y(N), z(N), q(4 * N, 0.0f), s(2 * N, 0.06f), al(N, 0.9f), rgb(3 * N),
      sem(C * N);
  for (int i = 0; i < N; ++i) {
    x[i] = 0.1f * (float)(i % G);
    y[i] = 0.1f * (float)(i / G);
    z[i] = 0.02f * std::sin(0.3f * x[i]);
    q[i] = 1.0f;                                   // w first
    for (int c = 0; c < 3; ++c) rgb[c * N + i] = (float)((i * (c + 3)) % 17) / 16.0f;
    for (int c = 0; c < C; ++c) sem[c * N + i] = (float)(((i + c) % 5) - 2);
  }
  rogs_surfels map{N, C, dev_copy(x), dev_copy(y), dev_copy(z), dev_copy(q), dev_copy(s),
                   dev_copy(al), dev_copy(rgb), dev_copy(sem)};
  rogs_render_opts opts;
  rogs_default_opts(&opts);
  opts.tile_w = 16;
  opts.tile_h = 4;
  const size_t arena_bytes = size_t(256) << 20;
  void* arena = nullptr;
  CHECK(hipMalloc(&arena, arena_bytes) == hipSuccess);
  rogs_server* srv = nullptr;
  CHECK(rogs_server_create(&srv, &map, &opts, arena, arena_bytes, 8, 2, 0) == ROGS_OK);

  // output buffers: the largest request has all planes of a 128 x 128 view
  const int kReq = 96;
  const size_t max_floats = (size_t)(5 + C + 1) * 128 * 128;
  std::vector<float*> out(kReq, nullptr);
  for (auto& o : out) CHECK(hipMalloc(&o, max_floats * sizeof(float)) == hipSuccess);
  const uint32_t sets[4] = {ROGS_CH_RGB, ROGS_CH_RGB | ROGS_CH_SEM, ROGS_CH_ALL,
                            ROGS_CH_ELEV | ROGS_CH_SEM};
  const int sizes[3] = {64, 100, 128};
  std::vector<uint64_t> ticket(kReq, 0);
  std::atomic<int> failed{0};
  auto submit = [&](int t0) {
    for (int k = t0; k < kReq; k += 2) {
      const int px = sizes[k % 3];
      rogs_request r{};
      // top-down orthographic chunk over the grid, 0.05 m per pixel, 5 m up
      rogs_bev_camera(0.0, 0.0, 128, 128, 0.05f, 0, 0, px, px, 5.0f, &r.cam);
      r.channels = sets[k % 4];
      r.elev_ref = 5.0f;
      r.out = out[k];
      if (rogs_serve_submit(srv, &r, &ticket[k]) != ROGS_OK) failed++;
    }
  };
  std::thread a(submit, 0), b(submit, 1);
  a.join();
  b.join();
  CHECK(failed.load() == 0);
  // argument errors: no channel, no buffer, a bad camera
  {
    rogs_request r{};
    rogs_bev_camera(0.0, 0.0, 64, 64, 0.05f, 0, 0, 64, 64, 5.0f, &r.cam);
    r.out = out[0];
    uint64_t t = 0;
    CHECK(rogs_serve_submit(srv, &r, &t) == ROGS_EINVAL);
    r.channels = ROGS_CH_RGB;
    r.out = nullptr;
    CHECK(rogs_serve_submit(srv, &r, &t) == ROGS_EINVAL);
    r.out = out[0];
    r.cam.w = 0;
    CHECK(rogs_serve_submit(srv, &r, &t) == ROGS_EINVAL);
  }
  int done = 0;
  std::vector<bool> finished(kReq, false);
  for (int spin = 0; done < kReq && spin < 200000; ++spin) {
    for (int k = 0; k < kReq; ++k) {
      if (finished[k]) continue;
      rogs_result res{};
      const int r = rogs_serve_poll(srv, ticket[k], &res);
      if (r == ROGS_NOT_READY) continue;
      CHECK(r == ROGS_OK);
      CHECK(res.status == ROGS_OK);
      CHECK(res.batch_views >= 1 && res.t_done_ns >= res.t_start_ns);
      finished[k] = true;
      ++done;
    }
    if (done < kReq) std::this_thread::yield();
  }
  CHECK(done == kReq);
  rogs_result res{};
  CHECK(rogs_serve_poll(srv, ticket[0], &res) == ROGS_EINVAL);   // ticket released
  int64_t st[7];
  CHECK(rogs_server_stats(srv, st) == ROGS_OK);
  CHECK(st[1] == kReq && st[4] == 0);
  // one more request queued at shutdown is rendered by destroy
  {
    rogs_request r{};
    rogs_bev_camera(0.0, 0.0, 64, 64, 0.05f, 0, 0, 64, 64, 5.0f, &r.cam);
    r.channels = ROGS_CH_RGB;
    r.out = out[0];
    uint64_t t = 0;
    CHECK(rogs_serve_submit(srv, &r, &t) == ROGS_OK);
  }
  rogs_server_destroy(srv);
  CHECK(hipDeviceSynchronize() == hipSuccess);
  for (auto o : out) CHECK(hipFree(o) == hipSuccess);
  CHECK(hipFree(arena) == hipSuccess);
  for (const void* p : {(const void*)map.x, (const void*)map.y, (const void*)map.z,
                        (const void*)map.q, (const void*)map.s, (const void*)map.alpha,
                        (const void*)map.rgb, (const void*)map.sem})
    CHECK(hipFree(const_cast<void*>(p)) == hipSuccess);
  printf("serve sanitizer run: ok (%d requests, %lld batches, largest %lld views)\n", kReq,
         (long long)st[0], (long long)st[3]);
  return 0;
}
