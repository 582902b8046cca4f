"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (from the key contract and the stated tolerances):
  * projection records, culling, tile rectangles, sort keys, surfel order and
    per-tile ranges: bit-exact;
  * rendered R, G, B, semantic logits and alpha: |delta| <= 1e-5; depth:
    |delta| <= 1e-5 * max(1, D);
  * gradients, per parameter tensor: max |delta| <= 1e-4 * max |g_ref|, and
    |delta| <= 1e-4 |g_ref| elementwise where |g_ref| >= 1e-2 max |g_ref|.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth
from paper_2405_14342_amd.pipeline import TrainState, n_out

pytestmark = pytest.mark.gpu

ROWS = {"z": slice(0, 1), "q": slice(1, 5), "s": slice(5, 7), "alpha": slice(7, 8),
        "rgb": slice(8, 11), "sem": slice(11, None)}


def oopts(o: B.RenderOpts) -> oracle.Opts:
    return oracle.Opts(o.tile_w, o.tile_h, o.eps2d, o.q_cut, o.alpha_max, o.t_eps)


def make_scene(name):
    if name == "c1":
        return synth.config1(mask_keep=0.9)
    if name == "tiny2":
        return synth.tiny_scene(n_views=2)
    if name == "mini":
        return synth.mini_strip()
    if name == "mini16":
        return synth.mini_strip(n_along=160, n_across=40, n_sem=16, w=200, h=120, cfg_index=8)
    if name == "big":
        # large footprints: 76 of the 100 slots cover more than 32 tiles of
        # 16 x 16 (summed by a wave), 28 more than 64, up to all 120
        sc = synth.tiny_scene(nx=10, ny=10, n_sem=3, w=192, h=160, f=140.0, seed=21)
        sc.s[:] = sc.s * np.float32(5.0)
        sc.log_s[:] = np.log(sc.s.astype(np.float64)).astype(np.float32)
        return sc
    if name == "ortho":
        sc = synth.mini_strip(n_along=120, n_across=50, n_sem=4, cfg_index=9)
        c = sc.cams[0]
        p = -np.asarray(c.R_cw, np.float64).T @ np.asarray(c.t_cw, np.float64)
        sc.cams = [synth.ortho_bev_camera((p[0], p[1]), 20.0, 200, 136, m_per_px=0.05)]
        sc.targets = synth._targets(sc.cams, sc.n_sem, 9000, 0.9)
        return sc
    if name == "flat":
        # one height for every surfel under a top-down orthographic camera:
        # all centre depths are equal, so each tile's order rests on the
        # tie rule alone (ascending surfel id)
        sc = make_scene("ortho")
        sc.z[:] = np.float32(np.median(sc.z))
        return sc
    if name == "stack":
        # 6400 surfels squeezed into a 8 cm square: one tile's list holds all
        # of them (ranked through global memory), neighbours hold hundreds
        # to thousands (sorted in LDS), the rest a few (sorted in one wave)
        sc = synth.tiny_scene(nx=80, ny=80, n_sem=2, w=64, h=48, f=60.0, seed=33)
        sc.x[:] = (1.0 + 0.001 * (sc.x - sc.x.min()) / synth.SPACING).astype(np.float32)
        sc.y[:] = (0.001 * (sc.y - sc.y.mean()) / synth.SPACING).astype(np.float32)
        return sc
    raise KeyError(name)


SCENES = ["c1", "tiny2", "mini", "mini16", "ortho", "big"]


@pytest.fixture(scope="module")
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    B.load_library()
    return torch.device("cuda")


def batched_state(sc, opts=None):
    st = TrainState(sc, opts=opts)
    ws, n = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    return st, ws, n


@pytest.mark.parametrize("name", SCENES)
def test_projection_records_bitexact(gpu, name):
    sc = make_scene(name)
    st, ws, n = batched_state(sc)
    rec, rect, cnt = st.rg.debug_records(ws, st.V, st.N)
    prm = oracle.Params.from_scene(sc)
    for v, cam in enumerate(sc.cams):
        vis, orec, orect = oracle.contract(prm, cam, oopts(st.opts))
        _, oids, _ = oracle.tile_lists(prm, cam, oopts(st.opts))
        ocnt = np.bincount(oids, minlength=sc.n)
        # pairs per surfel: the tiles its row spans reach (zero off the view)
        np.testing.assert_array_equal(cnt[v], np.where(vis, ocnt, 0))
        assert vis.sum() > 0 and (ocnt > 0).sum() > 0
        vis = vis & (ocnt > 0)                   # slots without pairs keep no record
        g = rec[v][vis].view(np.uint32)          # u_hi v_hi u_lo v_lo A B C t_z
        o = orec[vis].view(np.uint32)
        bad = np.nonzero((g != o).any(axis=1))[0]
        assert bad.size == 0, (v, bad[:5], rec[v][vis][bad[:3]], orec[vis][bad[:3]])
        np.testing.assert_array_equal(rect[v][vis], orect[vis])
        r = orect[vis]
        assert np.all(cnt[v][vis] <= (r[:, 1] - r[:, 0]) * (r[:, 3] - r[:, 2]))


@pytest.mark.parametrize("name", SCENES + ["stack", "flat"])
def test_keys_order_ranges_bitexact(gpu, name):
    sc = make_scene(name)
    st, ws, n = batched_state(sc)
    prm = oracle.Params.from_scene(sc)
    ok, oi, ov, orr = [], [], [], []
    tile_off, pair_off = 0, 0
    for v, cam in enumerate(sc.cams):
        k, i, r = oracle.tile_lists(prm, cam, oopts(st.opts))
        ok.append(k + (np.uint64(tile_off) << np.uint64(32)))
        oi.append(i)
        ov.append(np.full(len(i), v, np.int32))
        orr.append(r + pair_off)
        tile_off += r.shape[0]
        pair_off += len(k)
    okeys, oids, oviews, oranges = (np.concatenate(a) for a in (ok, oi, ov, orr))
    assert n == len(okeys) > 0
    keys, ids, views, ranges = st.rg.debug_pairs(ws, n, tile_off)
    np.testing.assert_array_equal(keys[:n], okeys)
    np.testing.assert_array_equal(ids[:n], oids)
    np.testing.assert_array_equal(views[:n], oviews)
    # empty tiles: the oracle writes (p, p), the library (0, 0)
    empty = oranges[:, 0] == oranges[:, 1]
    np.testing.assert_array_equal(ranges[~empty].astype(np.int64), oranges[~empty])
    assert np.all(ranges[empty] == 0)


def fwd_compare(sc, st, opts=None, views=None):
    prm = oracle.Params.from_scene(sc)
    o = oopts(st.opts)
    out = st.out.cpu().numpy()
    NO = n_out(sc.n_sem)
    worst = 0.0
    for v, cam in enumerate(sc.cams):
        if views is not None and v not in views:
            continue
        ref, tf, nl = oracle.render_fwd(prm, cam, o)
        g = out[NO * st.pix_off[v]: NO * st.pix_off[v + 1]].reshape(NO, -1)
        d = np.abs(g - ref)
        col = np.r_[0:NO - 2, NO - 1]
        assert d[col].max() <= 1e-5, (v, d[col].max())
        assert np.all(d[NO - 2] <= 1e-5 * np.maximum(1.0, np.abs(ref[NO - 2])))
        worst = max(worst, d[col].max())
        assert ref[-1].max() > 0.5
    return worst


@pytest.mark.parametrize("name", SCENES + ["stack", "flat"])
def test_forward_matches_oracle(gpu, name):
    sc = make_scene(name)
    st = TrainState(sc)
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    fwd_compare(sc, st)


def grads_compare(g_gpu, ref_flat, n, C, tol=1e-4):
    ref = oracle.split_grads(ref_flat, n, C)
    for name, sl in ROWS.items():
        a = g_gpu[sl].reshape(ref[name].shape) if ref[name].ndim > 1 else g_gpu[sl].reshape(-1)
        r = ref[name]
        mx = np.abs(r).max()
        if mx == 0.0:            # e.g. dL/dz under a top-down orthographic camera
            assert np.abs(a).max() == 0.0, name
            continue
        d = np.abs(a - r)
        assert d.max() <= tol * mx, (name, d.max() / mx)
        big = np.abs(r) >= 1e-2 * mx
        rel = d[big] / np.abs(r[big])
        assert rel.max() <= tol, (name, rel.max(), np.argmax(rel))


@pytest.mark.parametrize("name", SCENES)
def test_loss_and_gradients_match_oracle(gpu, name):
    sc = make_scene(name)
    st = TrainState(sc)
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    prm = oracle.Params.from_scene(sc)
    L, gref, dexp, fwd = oracle.loss_and_grads(prm, sc.cams, sc.targets, opts=oopts(st.opts))
    assert abs(st.loss.item() - L) <= 1e-5 * max(1.0, abs(L))
    grads_compare(st.grads.cpu().numpy(), gref, sc.n, sc.n_sem)
    np.testing.assert_allclose(st.d_exp.cpu().numpy(), dexp, rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("name", ["c1", "mini"])
def test_plain_path_equals_batched_bitwise(gpu, name):
    sc = make_scene(name)
    a = TrainState(sc)
    a.step_plain(adam=False)
    b = TrainState(sc)
    b.step_batched(adam=False)
    torch.cuda.synchronize()
    assert torch.equal(a.out, b.out)
    assert torch.equal(a.G, b.G)
    assert torch.equal(a.grads, b.grads)
    assert torch.allclose(a.d_exp, b.d_exp, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("tile", [(32, 8), (8, 8), (64, 4), (16, 8), (4, 16)])
def test_tile_shape_does_not_change_results(gpu, tile):
    sc = make_scene("mini")
    a = TrainState(sc)
    a.step_batched(adam=False)
    b = TrainState(sc, opts=B.make_opts(tile_w=tile[0], tile_h=tile[1]))
    b.step_batched(adam=False)
    torch.cuda.synchronize()
    assert torch.equal(a.out, b.out)          # same per-pixel operations in the same order
    g1, g2 = a.grads.cpu().numpy(), b.grads.cpu().numpy()
    # gradients are summed over tiles in a different grouping
    for name, sl in ROWS.items():
        mx = np.abs(g1[sl]).max()
        assert np.abs(g1[sl] - g2[sl]).max() <= 1e-5 * mx


def test_adam_matches_oracle(gpu):
    sc = make_scene("tiny2")
    st = TrainState(sc)
    rng = np.random.default_rng(12)
    K, N = st.K, st.N
    lr = B.LR(2e-3, 1e-3, 1e-3, 1e-3, 8e-3, 0.1, 1e-3)
    p = st.params.cpu().numpy().astype(np.float64)
    s_act = st.s_act.cpu().numpy().astype(np.float64)
    a_act = st.alpha_act.cpu().numpy().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lrs = [lr.z] + [lr.q] * 4 + [lr.s] * 2 + [lr.alpha] + [lr.rgb] * 3 + [lr.sem] * (K - 11)
    for step in range(1, 4):
        g = rng.normal(size=(K, N)).astype(np.float32)
        st.grads.copy_(torch.as_tensor(g))
        st.step_count = step
        st.d_exp.copy_(torch.as_tensor(rng.normal(size=(st.V, 2)).astype(np.float32)))
        dexp = st.d_exp.cpu().numpy().astype(np.float64)
        st.adam(lr)
        # oracle: chain rule to the raw parameters (s = exp(l), alpha = sigmoid(o)), then Adam
        graw = g.astype(np.float64).copy()
        graw[5:7] *= s_act
        graw[7] *= a_act * (1.0 - a_act)
        for r in range(K):
            pr, mr, vr = p[r].copy(), m[r].copy(), v[r].copy()
            oracle.adam(pr, np.ascontiguousarray(graw[r]), mr, vr, lrs[r], step)
            p[r], m[r], v[r] = pr, mr, vr
        s_act = np.exp(p[5:7])
        a_act = 1.0 / (1.0 + np.exp(-p[7]))
        torch.cuda.synchronize()
        np.testing.assert_allclose(st.params.cpu().numpy(), p, rtol=1e-6, atol=2e-6)
        np.testing.assert_allclose(st.m.cpu().numpy(), m, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(st.v.cpu().numpy(), v, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(st.s_act.cpu().numpy(), s_act, rtol=1e-6)
        np.testing.assert_allclose(st.alpha_act.cpu().numpy(), a_act, rtol=1e-6)
        # s_act / alpha_act on the GPU side are FP32 refreshes of the same raw values
        s_act = st.s_act.cpu().numpy().astype(np.float64)
        a_act = st.alpha_act.cpu().numpy().astype(np.float64)


def test_capacity_error_reports_needed_pairs(gpu):
    sc = make_scene("c1")
    st = TrainState(sc, pair_capacity=64)
    ws = st._workspace(st.cams, 64, "_ws_batch")
    st.rg.project(st.surfels(), st.cams, st.opts, ws, 64)
    r = st.rg.bin_sort(ws, B.SYNC_COUNT, raise_on_capacity=False)
    assert r < 0
    need = -r - 1
    prm = oracle.Params.from_scene(sc)
    k, _, _ = oracle.tile_lists(prm, sc.cams[0], oopts(st.opts))
    assert need == len(k)
    n, ovf = st.rg.pair_count(ws)
    assert n == need and ovf == 1
    with pytest.raises(B.RogsError) as e:
        st.rg.render_fwd(st.surfels(), ws, st.out)
    assert e.value.code == B.ESTATE


def test_nothing_visible(gpu):
    sc = make_scene("c1")
    # turn the camera around: everything is behind it
    c = sc.cams[0]
    sc.cams = [synth.pinhole_camera((-1.0, 0.0, 1.5), np.pi, np.radians(-10.0), 160, 90, 120.0)]
    st = TrainState(sc)
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    n, _ = st.rg.pair_count(st._ws_batch)
    assert n == 0
    assert float(st.out.abs().max()) == 0.0
    assert float(st.grads.abs().max()) == 0.0


def test_invalid_calls_raise(gpu):
    sc = make_scene("c1")
    st = TrainState(sc)
    ws = st._workspace(st.cams, 1000, "_ws_batch")
    with pytest.raises(B.RogsError) as e:
        st.rg.bin_sort(ws)
    assert e.value.code == B.ESTATE
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.RogsError) as e:
        st.rg.project(st.surfels(), st.cams, st.opts, small, 1000)
    assert e.value.code == B.ENOMEM
    bad = st.surfels()
    bad.n_sem = 9
    with pytest.raises(B.RogsError) as e:
        st.rg.project(bad, st.cams, st.opts, ws, 1000)
    assert e.value.code == B.EINVAL


# ------------------------------------------------------------------ fused step

def _snapshot(st):
    return {k: getattr(st, k).detach().cpu().clone() for k in
            ("params", "m", "v", "s_act", "alpha_act", "exposure", "m_exp", "v_exp")}


@pytest.mark.parametrize("name,eager", [("c1", True), ("c1", False), ("mini", False),
                                        ("mini16", False)])
def test_fused_step_equals_batched_plus_adam(gpu, name, eager):
    sc = make_scene(name)
    a = TrainState(sc)
    a.step_batched(total_steps=5)
    b = TrainState(sc)
    b.step_fused(total_steps=5, eager=eager, grads_out=True)
    torch.cuda.synchronize()
    sa, sb = _snapshot(a), _snapshot(b)
    # surfel parameters and moments: same per-pixel loss seed and the same
    # gradient records, so the same bits
    for k in ("params", "m", "v", "s_act", "alpha_act"):
        assert torch.equal(sa[k], sb[k]), k
    assert torch.equal(a.grads.cpu(), b.grads.cpu())
    # the per-view sums of dL/d(a, b) and of the loss group pixels differently
    np.testing.assert_allclose(b.d_exp.cpu().numpy(), a.d_exp.cpu().numpy(), rtol=1e-5, atol=1e-7)
    for k in ("exposure", "m_exp", "v_exp"):
        np.testing.assert_allclose(sb[k].numpy(), sa[k].numpy(), rtol=1e-4, atol=1e-9)
    stf = b.fused_status()
    assert stf["step"] == 1 and stf["skipped"] == 0 and stf["overflow"] == 0
    assert abs(stf["loss"] - a.loss.item()) <= 1e-5 * abs(a.loss.item())


def test_fused_graph_replays_match_eager(gpu):
    sc = make_scene("mini")
    a = TrainState(sc)
    b = TrainState(sc)
    for _ in range(3):
        a.step_fused(total_steps=3, eager=True)
        b.step_fused(total_steps=3, eager=False, check=False)
        torch.cuda.synchronize()          # eager work between the replays
        assert torch.equal(a.params, b.params)
    sa, sb = a.fused_status(), b.fused_status()
    assert sa["step"] == sb["step"] == 3
    for k in ("params", "m", "v", "s_act", "alpha_act"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def test_fused_overflow_skips_update_and_recovers(gpu):
    sc = make_scene("c1")
    st = TrainState(sc, pair_capacity=256)
    before = st.params.clone()
    ts = st.train_state()
    from paper_2405_14342_amd.pipeline import paper_optim
    optim = paper_optim(sc.extent, 1)
    size = B.fused_workspace_size(ts, st.cams, st.opts, 256)
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    # two steps in flight: the second call launches while the first may run,
    # the third waits for the first, sees its overflow and launches nothing
    for _ in range(2):
        r = st.rg.step_fused(ts, st.cams, st.opts, st.targets(0, st.V), optim, ws, 256,
                             raise_on_capacity=False)
        assert r == B.OK
    r = st.rg.step_fused(ts, st.cams, st.opts, st.targets(0, st.V), optim, ws, 256,
                         raise_on_capacity=False)
    assert r == B.ECAPACITY
    s1 = st.rg.fused_status()
    assert s1["overflow"] == 1 and s1["step"] == 0 and s1["skipped"] == 2
    assert s1["pairs"] > 256
    assert torch.equal(st.params, before)             # no update on overflow
    st.cap_fused = 256
    st.step_fused(total_steps=1)                      # grows and runs the step
    s2 = st.fused_status()
    assert s2["step"] == 1 and s2["overflow"] == 0
    assert not torch.equal(st.params, before)


@pytest.mark.parametrize("name", ["c1", "tiny2"])
def test_work_counts_match_oracle_lists(gpu, name):
    """rogs_debug_work against a count over the oracle's tile lists: per pixel,
    the entries up to its termination (n_last of the oracle's forward) and
    those passing the binary32 3-sigma test."""
    sc = make_scene(name)
    st = TrainState(sc)
    ws, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    st.rg.render_fwd(st.surfels(), ws, st.out)
    ev, co = st.rg.debug_work(ws)
    prm = oracle.Params.from_scene(sc)
    o = oopts(st.opts)
    e_ref = k_ref = 0
    for cam in sc.cams:
        _, rec, _ = oracle.contract(prm, cam, o)
        keys, ids, ranges = oracle.tile_lists(prm, cam, o)
        _, _, nl = oracle.render_fwd(prm, cam, o)
        tx = (cam.w + o.tile_w - 1) // o.tile_w
        for py in range(cam.h):
            for px in range(cam.w):
                t = (py // o.tile_h) * tx + px // o.tile_w
                a, b = ranges[t]
                n = int(nl[py * cam.w + px])
                lst = ids[a:a + n]
                e_ref += len(lst)
                q = oracle.q32(rec[lst], [px], [py])[:, 0] if len(lst) else np.zeros(0)
                k_ref += int((q <= np.float32(o.q_cut)).sum())
    assert (ev, co) == (e_ref, k_ref)
