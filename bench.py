#!/usr/bin/env python3
"""Benchmark of the surfel-splatting training step on one MI355X.

A step is the whole hot path over one batch: cull + EWA projection, tile-key
emission with per-tile counting + placement + ranges, forward compositing, L1
+ cross-entropy loss seed, backward compositing, projection adjoint, and the
Adam update.

Default workload: the batched step of 800,000 surfels (2000 x 400 grid at
0.1 m along a curved trajectory, 8 semantic classes) seen by 24 views (4
frames of a six-camera rig: front/back 1600 x 900, sides 1280 x 720).  The
headline is the fused step (loss fused into the forward, Adam into the
projection adjoint, the whole step one replayed hipGraph).  On the same
workload it also times the same kernels launched one by one (each bracketed
by HIP events: the per-kernel breakdown), the batched path (all views in one
launch sequence) and the plain path (one launch sequence per view with a host
read-back of the pair count).  Extra keys: the fused step on the 3M-surfel,
6 x 1920 x 1080, C = 16 workload, the grid-side loss terms, serving, and the
FP64 oracle on a stated subset of the views at all host threads and at one.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak (packed FP32)
VALU_NOPK_TFLOPS = 78.6    # FP32 FMA without packed-FP32 ops: 256 CU x 64 lanes x 2 x 2.4 GHz


def algorithmic_bytes(kernel: str, st, stats, C: int, fused: bool) -> float:
    """Compulsory HBM bytes of one launch group of one step.
    P pairs, S visible (view, surfel) slots, X pixels, N surfels, V views."""
    N, V = st.N, st.V
    P, S, X, slots = stats["pairs"], stats["visible"], stats["pixels"], stats["slots"]
    FS = ((4 + C) + 3) // 4 * 4
    K = 11 + C
    if kernel == "project":
        return N * (40 + 4 * FS) + slots * 4 + S * 40
    if kernel == "sort":
        # compaction (slot, count, position of each visible slot) + emission
        # offsets + one tile key, rank, slot and depth key per pair + the
        # per-tile counters and their scan + placement (key and rank read,
        # emission index written per pair)
        return slots * 4 + S * 12 + S * 8 + P * 16 + stats["tiles"] * 12 + P * 12
    if kernel == "ranges":
        # tile ranges from the counters and their scan, the launch order and
        # the per-tile work items, then the depth order inside each tile
        # (emission index, slot and depth key read, emission index and slot
        # written per pair)
        return stats["tiles"] * (16 + 36) + P * 20
    if kernel == "render_step":
        # fused forward + loss + backward of a tile: targets (12 B colour,
        # label, mask) in, the work item of each tile (16 B), the slot and
        # emission index of each pair and the records of the listed slots in,
        # one gradient record per pair and the per-tile loss partials out
        return X * 14 + P * (8 + 4 * (10 + C)) + S * (32 + 4 * FS) + stats["tiles"] * 28
    if kernel == "render_fwd":
        return X * ((5 + C) * 4 + 8) + P * 8 + S * (32 + 4 * FS)
    if kernel == "loss":
        if fused:   # mask count + per-view sums of the per-tile partials
            return X * 1 + stats["tiles"] * 12
        return X * ((3 + C) * 4 + 14 + 1 + (5 + C) * 4)
    if kernel == "render_bwd":
        return X * ((5 + C) * 4 + (4 + C) * 4 + 8) + P * (8 + 4 * (10 + C)) + S * (32 + 4 * FS)
    if kernel == "proj_bwd":
        base = slots * 4 + S * 4 + P * 4 * (10 + C) + N * (40 + 4 * K)
        if fused:   # + Adam: p, m, v read and written, s and alpha refreshed
            return base - N * 4 * K + N * (K * 4 * 6 + 2 * 3 * 4)
        return base
    if kernel == "adam":
        return N * (K * 4 * 7 + 2 * 3 * 4) + V * 2 * 4 * 7
    return 0.0


def compositing_flops(kernel: str, n_eval: int, n_contrib: int, C: int, fused: bool) -> float:
    """Issued arithmetic of the compositing kernels (FMA = 2 FLOPs), a
    diagnostic.  Per evaluated (pixel, list entry): the pixel offsets and the
    3-sigma quadratic form, 14.  Per contributing entry, forward: exp, clamp,
    weight, 4 + C accumulations, transmittance update and test, 9 + 2 (4 + C).
    Backward: the same alpha and weight plus the (3 + C)-channel dot product,
    the (3 + C) feature gradients, the suffix/alpha adjoint and the five
    moments of dL/dq over the pixel offsets, 31 + 4 (3 + C) without the depth
    and alpha loss terms (fused loss), +7 with them."""
    if kernel == "render_fwd":
        return 14.0 * n_eval + (9 + 2 * (4 + C)) * n_contrib
    if kernel == "render_bwd":
        return 14.0 * n_eval + (31 + 4 * (3 + C) + (0 if fused else 7)) * n_contrib
    if kernel == "render_step":
        return (compositing_flops("render_fwd", n_eval, n_contrib, C, True) +
                compositing_flops("render_bwd", n_eval, n_contrib, C, True))
    return 0.0


def algorithmic_flops(n_contrib: int, C: int) -> float:
    """Algorithmic work of forward + backward compositing: per contributing
    (pixel, surfel) entry 17 + 2 (4 + C) FLOPs forward (q 6, exp 2, clamp 2,
    transmittance and weight 3, 2 per accumulated channel) and 35 + 5 (4 + C)
    backward; 136 at C = 8.  Entries that are evaluated but rejected by the
    3-sigma test are tiling overhead and are not counted."""
    return float((17 + 2 * (4 + C) + 35 + 5 * (4 + C)) * n_contrib)


def profiled_traffic(kernel: str, workload: str, tile: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_tile{tile}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


def tile_choice(st) -> dict:
    """The launch configuration a TrainState runs: the options' tile shape and
    LDS staging depth, and the tile shape of every resolution class."""
    o = st.opts
    classes = {}
    for c in st.cams:
        t = getattr(c, "tile", 0)
        shape = (t & 0xFFFF, t >> 16) if t else (o.tile_w, o.tile_h)
        classes[f"{c.w}x{c.h}/m{c.model}"] = f"{shape[0]}x{shape[1]}"
    return {"tile": f"{o.tile_w}x{o.tile_h}", "stage": o.stage or 32, "classes": classes}


def tile_label(choice: dict) -> str:
    """Short name of a launch configuration (profile summaries are keyed by it)."""
    parts = [choice["tile"] + (f"s{choice['stage']}" if choice["stage"] != 32 else "")]
    parts += sorted(f"{k.split('/')[0]}-{v}" for k, v in choice["classes"].items()
                    if v != choice["tile"])
    return "_".join(parts)


def make_state(scene, tile: str, cache):
    """TrainState in a fixed tile shape 'WxH', or 'auto' (rogs_autotune over
    fused training steps: tile shape, staging depth and a shape per
    resolution class)."""
    from paper_2405_14342_amd import binding as B
    from paper_2405_14342_amd.pipeline import TrainState
    if tile == "auto":
        import tempfile
        tmp = None
        if cache is None:            # tune on this run; the file only carries the table out
            tmp = tempfile.mkdtemp()
            cache = os.path.join(tmp, "autotune.json")
        st = TrainState(scene, device="cuda:0", opts="auto", autotune_cache=cache)
        entries = json.load(open(cache))
        # the entry of this workload: every configuration timed and the choice
        key = [k for k in entries if k.startswith("step;") and f"n={scene.n};" in k]
        st.autotune_entry = entries[key[0]] if len(key) == 1 else None
        if tmp is not None:
            os.remove(cache)
            os.rmdir(tmp)
        print(f"[bench] {scene.name}: autotuned {tile_choice(st)} "
              f"({st.autotune_ms:.3f} ms per eager fused step)", file=sys.stderr, flush=True)
        return st
    tw, th = (int(t) for t in tile.split("x"))
    return TrainState(scene, device="cuda:0", opts=B.make_opts(tile_w=tw, tile_h=th))


def cpu_baseline(scene, views, threads: int, budget_s: float = 10.0):
    """The FP64 oracle's training step restricted to the given views (forward,
    loss and backward of those views, then the Sec. 4.2 optimiser on every
    row of every surfel), on `threads` host threads; repeated until budget_s
    is used.  Rate = pixels of those views per second."""
    import numpy as np
    import oracle

    oracle.set_threads(threads)
    prm = oracle.Params.from_scene(scene)
    cams = [scene.cams[v] for v in views]
    tgts = [scene.targets[v] for v in views]
    N, C = scene.n, scene.n_sem
    raw = np.concatenate([scene.z[None], scene.q, scene.log_s, scene.logit_a[None], scene.rgb,
                          scene.sem]).astype(np.float64)
    m, v = np.zeros_like(raw), np.zeros_like(raw)
    rates = oracle.paper_rates(scene.extent, 1)
    npx = sum(c.w * c.h for c in cams)
    t0 = time.perf_counter()
    reps = 0
    while True:
        L, g, dexp, _ = oracle.loss_and_grads(prm, cams, tgts)
        G = np.concatenate([g[:N][None], g[N:5 * N].reshape(4, N), g[5 * N:7 * N].reshape(2, N),
                            g[7 * N:8 * N][None], g[8 * N:11 * N].reshape(3, N),
                            g[11 * N:].reshape(C, N)])
        oracle.adam_raw(raw, G, m, v, rates, reps + 1)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 20:
            break
    desc = ", ".join(f"view {k} ({scene.cams[k].w}x{scene.cams[k].h})" for k in views)
    return {"value": round(npx * reps / el / 1e6, 3), "unit": "Mpixel/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} FP64 oracle step(s) on {len(views)} of the {scene.n_views} views "
                      f"({desc}; {npx} px each step: forward, loss, backward, then Adam on all "
                      f"{11 + C} rows of the {N} surfels), {el:.1f} s"}


def grid_terms_bench(st, scene, run, steps: int, n_points: int = 1_000_000):
    """The fused step with the grid-side terms of Eq. 12 switched on
    (elevation smoothness over the four grid neighbours, lambda 1, and the
    LiDAR elevation loss, lambda 0.02, on synthetic road returns), the
    one-off LiDAR target lookup, and the meshgrid layout + pose-based
    initialisation of the 3M-surfel road (1 km of poses every 0.5 m)."""
    import torch
    from paper_2405_14342_amd import binding as B
    from paper_2405_14342_amd import synth

    pts = torch.as_tensor(synth.lidar_points(scene.trajectory, n_points, 4242), device=st.dev)
    zbar = torch.empty(st.N, dtype=torch.float32, device=st.dev)
    scr0 = torch.empty(B.lidar_scratch_bytes(st.N, n_points), dtype=torch.uint8, device=st.dev)
    # points, targets and scratch resident in HBM: the timed call is the lookup
    st.rg.lidar_targets(st.x, st.y, pts[0], pts[1], pts[2], zbar, scratch=scr0)   # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.rg.lidar_targets(st.x, st.y, pts[0], pts[1], pts[2], zbar, scratch=scr0)
    torch.cuda.synchronize()
    t_nn = (time.perf_counter() - t0) * 1e3
    del scr0
    st.set_grid_terms(synth.grid_neighbours(*scene.grid_shape), zbar, lambda_smooth=1.0,
                      lambda_z=0.02)
    run("fused", 2)
    ms, _, _ = run("fused", steps)
    st.set_grid_terms(None, None)
    # meshgrid layout of the 1 km road: raster bounding box of the poses + 16 m
    traj = synth.Trajectory(1000.0, 3000)
    poses = synth.vehicle_poses(traj, 0.5)
    h = 0.1
    lo = poses[:, :2].min(0) - 16.0
    hi = poses[:, :2].max(0) + 16.0
    W, H = int((hi[0] - lo[0]) / h) + 1, int((hi[1] - lo[1]) / h) + 1
    pd = torch.as_tensor(poses, device=st.dev)
    st.rg.meshgrid_layout(pd, float(lo[0]), float(lo[1]), h, W, H, 150)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = st.rg.meshgrid_layout(pd, float(lo[0]), float(lo[1]), h, W, H, 150)
    torch.cuda.synchronize()
    t_lay = (time.perf_counter() - t0) * 1e3
    # LiDAR targets of the laid-out 1 km road (about 3M surfels) from 1M
    # returns along the same trajectory
    pts1k = torch.as_tensor(synth.lidar_points(traj, n_points, 4243), device=st.dev)
    n3 = int(out["n"])
    xg, yg = out["x"][:n3], out["y"][:n3]
    z3 = torch.empty(n3, dtype=torch.float32, device=st.dev)
    scr = torch.empty(B.lidar_scratch_bytes(n3, n_points), dtype=torch.uint8, device=st.dev)
    st.rg.lidar_targets(xg, yg, pts1k[0], pts1k[1], pts1k[2], z3, scratch=scr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.rg.lidar_targets(xg, yg, pts1k[0], pts1k[1], pts1k[2], z3, scratch=scr)
    torch.cuda.synchronize()
    t_nn3 = (time.perf_counter() - t0) * 1e3
    return {"ms_per_step": round(ms, 4), "value": round(scene.npix / (ms * 1e-3) / 1e6, 2),
            "unit": "Mpixel/s", "lambda_smooth": 1.0, "lambda_z": 0.02,
            "lidar_points": n_points, "lidar_targets_ms": round(t_nn, 3),
            "lidar_targets_3M": {"surfels": n3, "points": n_points, "ms": round(t_nn3, 3)},
            "layout": {"poses": int(poses.shape[0]), "raster": f"{W}x{H}", "radius_px": 150,
                       "surfels": out["n"], "ms": round(t_lay, 3)}}


def bev_bench(surf, sc, opts, m_per_px: float = 0.05, chunk_px: int = 2000):
    """Top-down export of the whole 3M-surfel map at 0.05 m/px in 2000 x 2000
    orthographic chunks, stitched, with colour and elevation planes."""
    import numpy as np
    import torch
    from paper_2405_14342_amd import binding as B

    x0, y0 = float(np.floor(sc.x.min())) - 1.0, float(np.floor(sc.y.min())) - 1.0
    W = int(np.ceil((float(sc.x.max()) + 1.0 - x0) / m_per_px))
    H = int(np.ceil((float(sc.y.max()) + 1.0 - y0) / m_per_px))
    height = float(sc.z.max()) + 50.0
    ch = B.CH_RGB | B.CH_ELEV
    out = torch.empty((4, H, W), dtype=torch.float32, device="cuda:0")
    rg = B.Rogs()
    cap = rg.bev_export(surf, opts, x0, y0, W, H, m_per_px, chunk_px, height, ch, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = rg.bev_export(surf, opts, x0, y0, W, H, m_per_px, chunk_px, height, ch, out,
                          pair_capacity=int(cap * 1.1) + 4096)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    chunks = ((W + chunk_px - 1) // chunk_px) * ((H + chunk_px - 1) // chunk_px)
    return {"image": f"{W}x{H}", "m_per_px": m_per_px, "chunk_px": chunk_px, "chunks": chunks,
            "planes": "RGB+ELEV", "ms": round(ms, 2),
            "Mpixel_per_s": round(W * H / (ms * 1e-3) / 1e6, 1), "max_chunk_pairs": worst}


def c4_bench(steps: int, warmup: int, tile: str, cache):
    """The fused step (graph) on the 3M-surfel, C = 16 map seen by six
    1920 x 1080 cameras (per-view culling), in the given tile configuration."""
    import torch
    from paper_2405_14342_amd import synth

    sc = synth.config4()
    st = make_state(sc, tile, cache)
    total = warmup + steps + 1
    st.step_fused(total_steps=total)
    st.fit_fused_capacity()
    for _ in range(max(0, warmup - 1)):
        st.step_fused(total_steps=total, check=False)
    torch.cuda.synchronize()
    skipped0 = st.fused_status()["skipped"]
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step_fused(total_steps=total, check=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, steps)
    fst = st.fused_status()
    if fst["overflow"] or fst["skipped"] != skipped0:
        raise RuntimeError("C4: pair capacity overflow during the timed steps")
    out = {"workload": sc.name, "surfels": sc.n, "views": sc.n_views, "sem_classes": sc.n_sem,
           "pixels_per_step": sc.npix, "path": "fused (hipGraph)", "tile": tile,
           "tile_choice": tile_choice(st), "autotune": getattr(st, "autotune_entry", None),
           "ms_per_step": round(ms, 4), "value": round(sc.npix / (ms * 1e-3) / 1e6, 2),
           "unit": "Mpixel/s", "pairs": fst["pairs"], "visible_slots": fst["visible"]}
    del st
    torch.cuda.empty_cache()
    return out


def serve_bench(seconds: float, warmup_s: float = 1.0, rates=(200.0, 8000.0),
                max_views: int = 16, lanes: int = 2, buffers: int = 128):
    """Serving workload: the 3M-surfel, C = 16 map resident on the GPU,
    Poisson arrivals of single-view requests (four pinhole sizes and a 512 x
    512 top-down orthographic view; channel sets RGB / RGB+SEM / RGB+SEM+D+A,
    ELEV+SEM for the top-down view), served by the library's
    continuous-batching server: one run per offered rate (the paper-derived
    200 req/s, then 8000 req/s, more than the server can render).  Latency =
    completion - submit, measured by the server on the steady clock; requests
    arriving during the first warmup_s seconds are not counted; a request
    that finds all `buffers` output buffers in use is dropped and counted."""
    import numpy as np
    import torch
    from paper_2405_14342_amd import binding as B
    from paper_2405_14342_amd import synth

    sc = synth.config4(with_targets=False)
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")
    dev = dict(x=f(sc.x), y=f(sc.y), z=f(sc.z), q=f(sc.q), s=f(sc.s), alpha=f(sc.alpha),
               rgb=f(sc.rgb), sem=f(sc.sem))
    surf = B.Surfels(sc.n, sc.n_sem, *(dev[k].data_ptr() for k in
                                       ("x", "y", "z", "q", "s", "alpha", "rgb", "sem")))
    C = sc.n_sem
    kinds = {"rgb": B.CH_RGB, "rgb_sem": B.CH_RGB | B.CH_SEM,
             "rgb_sem_d_a": B.CH_RGB | B.CH_SEM | B.CH_D | B.CH_A,
             "elev_sem": B.CH_ELEV | B.CH_SEM}
    max_floats = max(B.channel_planes(ch, C) for ch in kinds.values()) * 1920 * 1080
    pool = [torch.empty(max_floats, dtype=torch.float32, device="cuda:0") for _ in range(buffers)]
    arena = torch.empty(8 << 30, dtype=torch.uint8, device="cuda:0")
    opts = B.make_opts(tile_w=16, tile_h=4)
    srv = B.Server(surf, opts, arena, max_views=max_views, lanes=lanes, keep=(dev, sc))
    runs = []
    for k, rate in enumerate(rates):
        sched = synth.serve_schedule(sc.trajectory, rate, warmup_s + seconds, seed=5000 + k)
        # one request of every class first, so the timed run starts warm
        for cls_req in sched[:8]:
            srv.wait(srv.submit(cls_req.cam, kinds[cls_req.kind], pool[0], cls_req.elev_ref))
        s0 = srv.stats()
        free = list(range(len(pool)))
        live = {}                      # ticket -> (buffer index, request)
        done = []
        dropped = 0

        def collect(block: bool):
            for tk in list(live):
                r = srv.wait(tk) if block else srv.poll(tk)
                if r is not None:
                    b, rq = live.pop(tk)
                    free.append(b)
                    done.append((rq, r))

        t0 = time.perf_counter()
        for rq in sched:
            while True:
                collect(False)
                now = time.perf_counter() - t0
                if now >= rq.t:
                    break
                if rq.t - now > 0.0005:
                    time.sleep(0.0002)
            if not free:
                dropped += 1
                continue
            b = free.pop()
            live[srv.submit(rq.cam, kinds[rq.kind], pool[b], rq.elev_ref)] = (b, rq)
        collect(True)
        st = srv.stats()
        ok = [(rq, r) for rq, r in done if r["status"] == B.OK and rq.t >= warmup_s]
        lat = np.array([(r["t_done_ns"] - r["t_arrive_ns"]) * 1e-6 for _, r in ok])
        t_first = min(r["t_arrive_ns"] for _, r in ok)
        t_last = max(r["t_done_ns"] for _, r in ok)
        span = (t_last - t_first) * 1e-9
        px = sum(rq.cam.w * rq.cam.h for rq, _ in ok)
        nb = st["batches"] - s0["batches"]
        runs.append({
            "workload": "C5: 3M-surfel C=16 map, Poisson %.0f req/s offered, %.0f s (+%.0f s "
                        "warm-up)" % (rate, seconds, warmup_s),
            "offered_req_per_s": rate,
            "renders_per_s": round(len(ok) / span, 2), "Mpixel_per_s": round(px / span / 1e6, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "requests": len(ok), "failed": sum(1 for _, r in done if r["status"] != B.OK),
            "dropped_no_buffer": dropped, "batches": nb,
            "mean_batch_views": round((st["views"] - s0["views"]) / max(1, nb), 2),
            "max_batch_views": st["max_batch"], "lanes": lanes, "buffers": buffers,
            "max_batches_in_flight": st["max_in_flight"], "tile": "16x4"})
        print(f"[bench] serve {rate:.0f} req/s offered: {runs[-1]['renders_per_s']} renders/s, "
              f"p50 {runs[-1]['p50_ms']} ms, p99 {runs[-1]['p99_ms']} ms, mean batch "
              f"{runs[-1]['mean_batch_views']}", file=sys.stderr, flush=True)
    srv.close()
    del arena, pool
    torch.cuda.empty_cache()
    out = dict(runs[0])
    out["saturated"] = runs[1] if len(runs) > 1 else None
    out["bev_export"] = bev_bench(surf, sc, opts)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=3, help="1..4: workload (default 3)")
    ap.add_argument("--no-c4", action="store_true",
                    help="skip the fused step on the 3M-surfel, 6 x 1920 x 1080 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--tile", default="auto",
                    help="tile shape WxH, or 'auto' (default: rogs_autotune chooses the tile "
                         "shape, the LDS staging depth and a shape per resolution class)")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON cache file of rogs_autotune (default: tune on every run)")
    ap.add_argument("--no-grid-terms", action="store_true",
                    help="skip the step with the smoothness and LiDAR losses")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the timed serving run (0 = skip)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a 256 MiB device copy (known bytes) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_14342_amd import synth
    from paper_2405_14342_amd.pipeline import TrainState

    torch.cuda.set_device(0)
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    scene = synth.CONFIGS[args.config]()
    C = scene.n_sem
    total_steps = args.warmup + args.steps
    st = make_state(scene, args.tile, args.autotune_cache)
    choice = tile_choice(st)
    print(f"[bench] {scene.name}: {scene.n} surfels, {scene.n_views} views, "
          f"{scene.npix} px/step", file=sys.stderr, flush=True)

    def run(path, steps, profile=False):
        if path == "fused":
            fn = lambda total_steps: st.step_fused(total_steps=total_steps, check=False)
        elif path == "fused_eager":
            fn = lambda total_steps: st.step_fused(total_steps=total_steps, eager=True, check=False)
        else:
            fn = st.step_batched if path == "batched" else st.step_plain
        torch.cuda.synchronize()
        if profile:
            st.rg.prof_enable(True)
            st.rg.prof_read()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fn(total_steps=total_steps)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = None
        if profile:
            prof = st.rg.prof_read()
            st.rg.prof_enable(False)
        n = max(steps, 1)
        return wall * 1e3 / n, e0.elapsed_time(e1) / n, prof

    # headline: the fused step, captured once as a graph and replayed; after
    # the first step the capacities are fitted to the measured counts (+10 %)
    run("fused", 1)
    st.fit_fused_capacity()
    run("fused", max(0, args.warmup - 1))
    print("[bench] warmup done", file=sys.stderr, flush=True)
    skipped0 = st.fused_status()["skipped"]
    ms_f, ev_f, _ = run("fused", args.steps)
    fst = st.fused_status()
    if fst["overflow"] or fst["skipped"] != skipped0:
        raise RuntimeError("pair capacity overflow during the timed steps (steps skipped)")
    stats = {k: fst[k] for k in ("pairs", "visible", "pixels", "tiles", "slots")}
    print(f"[bench] fused (graph): {ms_f:.3f} ms/step, pairs {stats['pairs']}", file=sys.stderr,
          flush=True)
    # the same kernels launched one by one, each bracketed by HIP events
    run("fused_eager", 1)
    ms_fe, _, prof = run("fused_eager", args.steps, profile=True)
    print(f"[bench] fused (eager, timed kernels): {ms_fe:.3f} ms/step", file=sys.stderr, flush=True)
    ms_b = None
    if not args.no_batched:
        run("batched", 1)
        ms_b, _, _ = run("batched", args.steps)
        print(f"[bench] batched: {ms_b:.3f} ms/step", file=sys.stderr, flush=True)
    plain = None
    if not args.no_plain:
        run("plain", 1)
        ms_p, ev_p, _ = run("plain", args.steps)
        plain = {"ms_per_step": round(ms_p, 4),
                 "value": round(scene.npix / (ms_p * 1e-3) / 1e6, 2)}
        print(f"[bench] plain: {ms_p:.3f} ms/step", file=sys.stderr, flush=True)

    kernels = {}
    for name, (ms, n) in prof.items():
        if n == 0 or name == "fused_graph":
            continue
        per = ms / args.steps
        b = algorithmic_bytes(name, st, stats, C, fused=True)
        kernels[name] = {"ms_per_step": round(per, 4), "launches_per_step": n // args.steps,
                         "alg_GBs": round(b / (per * 1e-3) / 1e9, 1) if per > 0 else None}
    # work counts of this workload: one batched forward of the same surfels
    ws_b, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    st.rg.render_fwd(st.surfels(), ws_b, st.out)
    n_eval, n_contrib = st.rg.debug_work(ws_b)
    flops = {k: compositing_flops(k, n_eval, n_contrib, C, fused=True)
             for k in ("render_step",)}
    for k, f in flops.items():
        if k in kernels and kernels[k]["ms_per_step"] > 0:
            kernels[k]["alg_TFLOPs"] = round(f / (kernels[k]["ms_per_step"] * 1e-3) / 1e12, 2)
    # roofline of the dominant single kernel (the fused step's compositing:
    # forward, loss and backward of a tile): algorithmic FLOPs (per
    # contributing entry) per launch over its average launch duration, timed
    # with HIP events on its launch stream, against the published FP32 peak
    dom = "render_step"
    dom_ms = prof[dom][0] / prof[dom][1]          # average duration of one launch
    per_launch = prof[dom][1] / args.steps
    dom_flops = algorithmic_flops(n_contrib, C)    # one launch covers the whole step
    dom_bytes = algorithmic_bytes(dom, st, stats, C, True) / per_launch
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    issued = flops[dom] / per_launch
    roofline = {"kernel": dom, "bound": "alu", "achieved": round(achieved, 2),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": profiled_traffic(dom, scene.name, tile_label(choice)),
                "avg_launch_ms": round(dom_ms, 4), "alg_flops_per_launch": int(dom_flops),
                "flops_per_contributing_entry": int(algorithmic_flops(1, C)),
                "alg_bytes_per_launch": int(dom_bytes),
                "hbm_achieved_GBs": round(dom_bytes / (dom_ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(dom_bytes / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "evaluated_entries": n_eval, "contributing_entries": n_contrib,
                "peak_no_packed_fp32": VALU_NOPK_TFLOPS,
                "frac_no_packed_fp32": round(achieved / VALU_NOPK_TFLOPS, 4),
                "issued_flops_per_launch": int(issued),
                "issued_TFLOPs": round(issued / (dom_ms * 1e-3) / 1e12, 2),
                "peak_note": "157.3 TFLOP/s published FP32 vector peak (packed FP32); this build "
                             "issues no packed FP32, whose ceiling is 256 CU x 64 lanes x 2 FLOP "
                             "x 2.4 GHz = 78.6"}

    value = scene.npix / (ms_f * 1e-3) / 1e6
    line = {
        "metric": "fwd+bwd Mpixel/s per train step (fused vs plain); serve renders/s + p50/p99",
        "value": round(value, 2), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_f, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded surfel grid, cameras and random targets)",
        "config": {"workload": scene.name, "surfels": scene.n, "views": scene.n_views,
                   "tile": args.tile, "tile_choice": choice,
                   "autotune_ms": (round(st.autotune_ms, 4) if args.tile == "auto" else None),
                   "autotune": getattr(st, "autotune_entry", None),
                   "pixels_per_step": scene.npix, "sem_classes": C,
                   "path": "fused (hipGraph)", "pairs": stats["pairs"],
                   "visible_slots": stats["visible"]},
        "fused_eager_ms_per_step": round(ms_fe, 4),
        "batched": ({"ms_per_step": round(ms_b, 4),
                     "value": round(scene.npix / (ms_b * 1e-3) / 1e6, 2)} if ms_b else None),
        "plain": plain,
        "speedup_vs_plain": round(plain["ms_per_step"] / ms_f, 3) if plain else None,
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_grid_terms and hasattr(scene, "trajectory"):
        line["grid_terms"] = grid_terms_bench(st, scene, run, args.steps)
        g = line["grid_terms"]
        print(f"[bench] fused step with smoothness + LiDAR loss: {g['ms_per_step']} ms/step; "
              f"LiDAR targets {g['lidar_targets_ms']} ms; meshgrid layout {g['layout']['ms']} ms",
              file=sys.stderr, flush=True)
    del st, ws_b
    torch.cuda.empty_cache()
    if not args.no_c4 and args.config != 4:
        line["c4"] = c4_bench(args.steps, args.warmup, args.tile, args.autotune_cache)
        print(f"[bench] C4 fused: {line['c4']['ms_per_step']} ms/step, "
              f"{line['c4']['value']} Mpixel/s", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        print("[bench] serving (3M-surfel map, Poisson 200 and 8000 req/s offered)...",
              file=sys.stderr, flush=True)
        line["serve"] = serve_bench(args.serve_seconds)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)...", file=sys.stderr, flush=True)
        # the host's CPU share: OMP_NUM_THREADS where set, else the affinity mask
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        # a bounded sample: the first two views (one front, one side camera
        # at C3) of the same workload
        views = list(range(min(2, scene.n_views)))
        line["cpu_baseline"] = cpu_baseline(scene, views, threads)
        line["cpu_baseline_1_thread"] = cpu_baseline(scene, views, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
