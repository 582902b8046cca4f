"""Continuous-batching render server (rogs_server_*): outputs equal the direct
batched render bitwise, a request renders the same alone and mixed into a
batch, overflowing batches are split, admission and argument errors."""
import math
import time

import numpy as np
import pytest
import torch

from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth
from paper_2405_14342_amd.pipeline import TrainState

pytestmark = pytest.mark.gpu
ALL = B.CH_RGB | B.CH_SEM | B.CH_D | B.CH_A | B.CH_ELEV


def _scene():
    sc = synth.mini_strip()
    c = sc.cams[0]
    p = -np.asarray(c.R_cw, np.float64).T @ np.asarray(c.t_cw, np.float64)
    extra = [synth.pinhole_camera((p[0] + 1.0, p[1] + 0.3, p[2]), 0.2, math.radians(-15.0),
                                  96, 64, 80.0),
             synth.ortho_bev_camera((p[0] + 3.0, p[1]), 12.0, 80, 64, m_per_px=0.05)]
    sc.cams = list(sc.cams) + extra
    sc.targets = synth._targets(sc.cams, sc.n_sem, 4242, 1.0)
    return sc


def _server(st, arena_bytes=512 << 20, max_views=16, lanes=2):
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    keep = (st.params, st.s_act, st.alpha_act, st.x, st.y)
    return B.Server(st.surfels(), st.opts, arena, max_views=max_views, lanes=lanes, keep=keep)


def _direct(st):
    ws, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    st.rg.render_fwd(st.surfels(), ws, st.out)
    torch.cuda.synchronize()
    return [st.image(v).clone() for v in range(st.V)]


def _expected(img, channels, C, elev_ref):
    planes = []
    if channels & B.CH_RGB:
        planes += [img[0:3]]
    if channels & B.CH_SEM:
        planes += [img[3:3 + C]]
    D, A = img[3 + C:4 + C], img[4 + C:5 + C]
    if channels & B.CH_D:
        planes += [D]
    if channels & B.CH_A:
        planes += [A]
    if channels & B.CH_ELEV:
        planes += [torch.where(A > 0, elev_ref - D / A, torch.full_like(A, float("nan")))]
    return torch.cat(planes)


def _out(cam, channels, C):
    return torch.full((B.channel_planes(channels, C), cam.h, cam.w), -7.0, device="cuda")


def test_served_views_equal_direct_render():
    sc = _scene()
    st = TrainState(sc)
    ref = _direct(st)
    srv = _server(st)
    try:
        chans = [ALL, B.CH_RGB, B.CH_SEM | B.CH_D, B.CH_ELEV | B.CH_A]
        outs, tickets = [], []
        for v, cam in enumerate(sc.cams):
            ch = chans[v % len(chans)]
            o = _out(cam, ch, sc.n_sem)
            outs.append((o, ch))
            tickets.append(srv.submit(cam, ch, o, elev_ref=2.5))
        for v, t in enumerate(tickets):
            r = srv.wait(t)
            assert r["status"] == B.OK
            assert r["t_arrive_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
            o, ch = outs[v]
            exp = _expected(ref[v], ch, sc.n_sem, 2.5)
            assert torch.equal(torch.nan_to_num(o, nan=-1.0), torch.nan_to_num(exp, nan=-1.0)), v
        with pytest.raises(B.RogsError, match="EINVAL"):
            srv.poll(tickets[0])                       # released
    finally:
        srv.close()


def test_request_renders_the_same_alone_and_batched():
    sc = _scene()
    st = TrainState(sc)
    srv = _server(st)
    try:
        cam = sc.cams[1]
        alone = _out(cam, ALL, sc.n_sem)
        r = srv.wait(srv.submit(cam, ALL, alone, elev_ref=1.0))
        assert r["status"] == B.OK and r["batch_views"] == 1
        seen_batched = False
        for _ in range(8):
            # a burst: whatever is queued when a lane frees up is one batch
            others = [(c, _out(c, ALL, sc.n_sem)) for c in sc.cams]
            mixed = _out(cam, ALL, sc.n_sem)
            ts = [srv.submit(c, ALL, o) for c, o in others]
            tr = srv.submit(cam, ALL, mixed, elev_ref=1.0)
            res = [srv.wait(t) for t in ts]
            rr = srv.wait(tr)
            assert rr["status"] == B.OK and all(x["status"] == B.OK for x in res)
            assert torch.equal(torch.nan_to_num(mixed, nan=-1.0), torch.nan_to_num(alone, nan=-1.0))
            if rr["batch_views"] > 1:
                seen_batched = True
                break
        assert seen_batched and srv.stats()["max_batch"] > 1
    finally:
        srv.close()


def test_batches_overlap_on_two_lanes():
    sc = _scene()
    st = TrainState(sc)
    srv = _server(st, arena_bytes=4 << 30, lanes=2)
    try:
        cam = sc.cams[1]
        alone = _out(cam, ALL, sc.n_sem)
        srv.wait(srv.submit(cam, ALL, alone))
        # a request long enough that the small one, submitted at most a
        # millisecond later, starts while it still runs
        big = synth.pinhole_camera((0.0, 0.0, 1.5), 0.0, math.radians(-10.0), 6144, 3072, 4350.0)
        ob = _out(big, B.CH_RGB, sc.n_sem)
        seen = False
        spans = []
        for k in range(10):
            tb = srv.submit(big, B.CH_RGB, ob)
            time.sleep(0.0001 * k)
            mixed = _out(cam, ALL, sc.n_sem)
            tr = srv.submit(cam, ALL, mixed)
            rb, rr = srv.wait(tb), srv.wait(tr)
            assert rb["status"] == B.OK and rr["status"] == B.OK
            assert torch.equal(torch.nan_to_num(mixed, nan=-1.0), torch.nan_to_num(alone, nan=-1.0))
            spans.append(tuple((r[key] - rb["t_start_ns"]) // 1000 for r in (rb, rr)
                               for key in ("t_start_ns", "t_done_ns")))
            if rr["t_start_ns"] < rb["t_done_ns"] and rb["t_start_ns"] < rr["t_done_ns"]:
                seen = True
                break
        # spans: (big start, big done, small start, small done) in us
        assert seen and srv.stats()["max_in_flight"] == 2, (spans, srv.stats())
    finally:
        srv.close()


def _image_bytes(pix, C):
    return ((5 + C) * pix * 4 + 255) // 256 * 256


def test_overflowing_batch_is_split():
    # large footprints: many pairs per pixel, so the workspace rather than the
    # images decides what fits
    sc = _scene()
    sc.s = sc.s * np.float32(8.0)
    sc.log_s = sc.log_s + np.float32(math.log(8.0))
    st = TrainState(sc)
    ref = _direct(st)
    surf = st.surfels()
    n_all = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")[1]
    pix = sum(c.w * c.h for c in sc.cams)
    img_all = _image_bytes(pix, sc.n_sem)
    # room for half of the batch's pairs: the whole batch is admitted (its
    # images take at most half the arena) but overflows, every view alone fits
    arena = (img_all + B.workspace_size(surf, sc.cams, st.opts, n_all // 2)) // 256 * 256
    assert 2 * img_all <= arena
    for c in sc.cams:
        n_v = st.project_and_sort([c], "cap_view", "_ws_view")[1]
        assert _image_bytes(c.w * c.h, sc.n_sem) + B.workspace_size(surf, [c], st.opts, n_v) <= arena
    srv = _server(st, arena_bytes=arena, lanes=1)
    try:
        # two rounds: the worker may take the first request of a round alone,
        # but the second round queues up while the first renders, so some
        # batch holds more than half of the pairs and must be split
        outs = [[_out(c, B.CH_RGB, sc.n_sem) for c in sc.cams] for _ in range(2)]
        ts = [srv.submit(c, B.CH_RGB, o) for rnd in outs for c, o in zip(sc.cams, rnd)]
        res = [srv.wait(t) for t in ts]
        assert all(r["status"] == B.OK for r in res), res
        for rnd in outs:
            for v in range(len(sc.cams)):
                assert torch.equal(rnd[v], ref[v][0:3])
        s = srv.stats()
        assert s["views"] == 2 * len(sc.cams) and s["splits"] >= 1, s
    finally:
        srv.close()


def test_admission_and_argument_errors():
    sc = _scene()
    st = TrainState(sc)
    srv = _server(st, arena_bytes=2 << 20)
    try:
        big = synth.pinhole_camera((0.0, 0.0, 1.5), 0.0, 0.0, 1920, 1080, 1371.02)
        with pytest.raises(B.RogsError, match="EREJECT"):
            srv.submit(big, B.CH_RGB, _out(big, B.CH_RGB, sc.n_sem))
        with pytest.raises(B.RogsError, match="EINVAL"):
            srv.submit(sc.cams[0], 0, _out(sc.cams[0], B.CH_RGB, sc.n_sem))
        with pytest.raises(B.RogsError, match="EINVAL"):
            srv.submit(sc.cams[0], 64, _out(sc.cams[0], B.CH_RGB, sc.n_sem))
        with pytest.raises(B.RogsError, match="EINVAL"):
            srv.poll(123456)
    finally:
        srv.close()


def test_destroy_drains_queue():
    sc = _scene()
    st = TrainState(sc)
    ref = _direct(st)
    srv = _server(st)
    outs = [_out(c, B.CH_A, sc.n_sem) for c in sc.cams]
    for c, o in zip(sc.cams, outs):
        srv.submit(c, B.CH_A, o)
    srv.close()
    torch.cuda.synchronize()
    for v in range(len(sc.cams)):
        assert torch.equal(outs[v][0], ref[v][4 + sc.n_sem])
