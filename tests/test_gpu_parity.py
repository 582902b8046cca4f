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
from paper_2405_14342_amd.pipeline import TrainState, n_out, paper_optim
from parity_util import ROWS, grads_compare, oracle_work_counts

pytestmark = pytest.mark.gpu


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
    if name == "clamp":
        # opacities 0.995-0.999: alpha g passes the clamp 0.99 near the centres
        return synth.clamp_scene()
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


def test_projection_records_after_workspace_reuse(gpu):
    # a second batch on the same workspace with the views in reverse order:
    # projection blocks that a view of the first batch reached and the same
    # view slot of the second culls whole keep the first batch's per-slot
    # values in memory, and must still report no pairs
    sc = make_scene("mini")
    assert len(sc.cams) > 1 and sc.n > 4 * 256
    st, ws, _ = batched_state(sc)
    cams = list(reversed(st.cams))
    ws2, _ = st.project_and_sort(cams, "cap_batch", "_ws_batch")
    assert ws2.data_ptr() == ws.data_ptr()
    _, _, cnt = st.rg.debug_records(ws2, st.V, st.N)
    prm = oracle.Params.from_scene(sc)
    stale = 0
    for v, cam in enumerate(reversed(sc.cams)):
        vis, _, _ = oracle.contract(prm, cam, oopts(st.opts))
        _, oids, _ = oracle.tile_lists(prm, cam, oopts(st.opts))
        ocnt = np.bincount(oids, minlength=sc.n)
        np.testing.assert_array_equal(cnt[v], np.where(vis, ocnt, 0))
        # blocks culled here whose surfels the first batch's view v reached
        vis1, _, _ = oracle.contract(prm, sc.cams[v], oopts(st.opts))
        b2 = np.zeros(-(-sc.n // 256) * 256, bool)
        b2[:sc.n] = vis
        culled = ~b2.reshape(-1, 256).any(1)
        b1 = np.zeros_like(b2)
        b1[:sc.n] = vis1
        stale += int((culled & b1.reshape(-1, 256).any(1)).sum())
    assert stale > 0


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


def exposure_for(sc, seed=31):
    """Per-view exposure (a, b) of Eq. 7: a in [-0.2, 0.2], b in [-0.05, 0.05]."""
    rng = np.random.default_rng(seed)
    V = len(sc.cams)
    return np.stack([rng.uniform(-0.2, 0.2, V), rng.uniform(-0.05, 0.05, V)], 1).astype(np.float32)


@pytest.mark.parametrize("name", SCENES + ["clamp"])
@pytest.mark.parametrize("expo", [False, True])
def test_loss_and_gradients_match_oracle(gpu, name, expo):
    sc = make_scene(name)
    st = TrainState(sc)
    e = exposure_for(sc) if expo else np.zeros((len(sc.cams), 2), np.float32)
    st.exposure.copy_(torch.as_tensor(e))
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    prm = oracle.Params.from_scene(sc)
    L, gref, dexp, fwd = oracle.loss_and_grads(prm, sc.cams, sc.targets, exposure=e,
                                               opts=oopts(st.opts))
    assert abs(st.loss.item() - L) <= 1e-5 * max(1.0, abs(L))
    if name == "clamp":
        # pixels whose alpha g lies within 1e-4 of the clamp may take either
        # branch in FP32: the full loss seed weighs them, so only the values
        # are compared here (gradients: test_clamp_scene_gradients)
        return
    grads_compare(st.grads.cpu().numpy(), gref, sc.n, sc.n_sem)
    np.testing.assert_allclose(st.d_exp.cpu().numpy(), dexp, rtol=1e-4, atol=1e-6)


def test_clamp_scene_gradients(gpu):
    """Forward and adjoint where alpha g passes alpha_max = 0.99 (Eq. 6 with
    the opacity clamp): dL/d(image) is random except at pixels within 1e-4 of
    the clamp's kink, where FP32 and FP64 may choose different branches."""
    sc = make_scene("clamp")
    st = TrainState(sc)
    ws, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    surf = st.surfels()
    st.rg.render_fwd(surf, ws, st.out)
    torch.cuda.synchronize()
    fwd_compare(sc, st)
    prm = oracle.Params.from_scene(sc)
    o = oopts(st.opts)
    cam = sc.cams[0]
    gg = oracle.geo64(prm, cam, o)
    vis, _, _ = oracle.contract(prm, cam, o)
    ys, xs = np.mgrid[0:cam.h, 0:cam.w]
    pxc, pyc = xs.reshape(-1) + 0.5, ys.reshape(-1) + 0.5
    margin = np.full(pxc.size, np.inf)
    clamped = 0
    for i in np.nonzero(vis)[0]:
        u, v, A, Bc, Cc, _ = gg[i]
        dx, dy = pxc - u, pyc - v
        q = A * dx * dx + Cc * dy * dy + 2.0 * Bc * dx * dy
        ag = prm.alpha[i] * np.exp(-0.5 * q)
        inside = q <= o.q_cut
        margin = np.where(inside, np.minimum(margin, np.abs(ag - o.alpha_max)), margin)
        clamped += int((inside & (ag > o.alpha_max) & (margin >= 1e-4)).sum())
    assert clamped >= 30
    NO = n_out(sc.n_sem)
    G = np.random.default_rng(8).normal(size=(NO, cam.w * cam.h)).astype(np.float32)
    G[:, margin < 1e-4] = 0.0
    _, tf, nl = oracle.render_fwd(prm, cam, o)
    ref = oracle.render_bwd(prm, cam, G.astype(np.float64), tf, nl, o)
    grads = torch.empty((st.K, st.N), dtype=torch.float32, device="cuda")
    st.rg.render_bwd(surf, ws, st.out, torch.as_tensor(G.reshape(-1), device="cuda"), grads, 0)
    grads_compare(grads.cpu().numpy(), ref, sc.n, sc.n_sem)


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


def ulp32(a):
    return np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)


@pytest.mark.parametrize("total", [3, 0])
def test_adam_matches_oracle(gpu, total):
    """rogs_adam_step against the oracle's optimiser (Sec. 4.2: chain rule
    through exp / sigmoid, per-group rates, the height rate from 1.6e-4 to
    1.6e-6 of the scene size over `total` steps, t = 0, 1/2, 1; total = 0: a
    constant height rate), on seeded gradients; both start from the same FP32
    values and run three steps on their own."""
    sc = make_scene("tiny2")
    st = TrainState(sc)
    rng = np.random.default_rng(12)
    K, N, V = st.K, st.N, st.V
    optim = paper_optim(sc.extent, total)
    if total == 0:
        optim.lr.z = 2e-3
    rates = oracle.Rates(optim.lr.z, optim.lr.q, optim.lr.s, optim.lr.alpha, optim.lr.rgb,
                         optim.lr.sem, optim.lr.exposure, optim.z_start, optim.z_end, total)
    p = st.params.cpu().numpy().astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    e = rng.normal(0.0, 0.1, (V, 2)).astype(np.float32)
    st.exposure.copy_(torch.as_tensor(e))
    e = e.astype(np.float64)
    me, ve = np.zeros_like(e), np.zeros_like(e)
    for step in range(1, 4):
        g = rng.normal(size=(K, N)).astype(np.float32)
        ge = rng.normal(size=(V, 2)).astype(np.float32)
        st.grads.copy_(torch.as_tensor(g))
        st.d_exp.copy_(torch.as_tensor(ge))
        st.step_count = step
        p_before = p.copy()
        st.adam(optim)
        # the library reads beta1, beta2 and eps as binary32 (1 - 0.999f is
        # 1.3e-5 away from 1e-3): the oracle gets the same values
        s_act, a_act = oracle.adam_raw(p, g.astype(np.float64), m, v, rates, step,
                                       b1=float(np.float32(optim.beta1)),
                                       b2=float(np.float32(optim.beta2)),
                                       eps=float(np.float32(optim.eps)), exposure=e,
                                       d_exposure=ge.astype(np.float64), m_exp=me, v_exp=ve)
        torch.cuda.synchronize()
        got = st.params.cpu().numpy()
        # each step rounds the FP32 parameters once; the update itself is
        # computed to ~1e-6 relative
        tol = 4 * step * ulp32(p) + 1e-5 * np.abs(p - p_before)
        assert np.all(np.abs(got - p) <= tol), (step, np.max(np.abs(got - p) - tol))
        np.testing.assert_allclose(st.m.cpu().numpy(), m, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(st.v.cpu().numpy(), v, rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(st.s_act.cpu().numpy(), s_act, rtol=2e-6)
        np.testing.assert_allclose(st.alpha_act.cpu().numpy(), a_act, rtol=2e-6)
        np.testing.assert_allclose(st.exposure.cpu().numpy(), e, rtol=0, atol=4e-7)
        # the height row moved by its scheduled rate (Adam's first step moves
        # every entry by the rate: |m / sqrt(v)| = 1)
        if step == 1:
            np.testing.assert_allclose(np.abs(got[0] - p_before[0]), oracle.z_rate(rates, 1),
                                       rtol=1e-4)


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


def test_fused_three_steps_match_oracle(gpu):
    """Three fused steps (loss, adjoint and the Sec. 4.2 optimiser with the
    height schedule over the three steps, exposure non-zero) against three
    steps of the oracle run on its own from the same FP32 start.  Adam moves a
    parameter by about its rate per step whatever the gradient's size, and by
    less where gradients change sign; so every entry must stay within
    2 rates * steps of the oracle, and entries whose oracle gradient was large
    at every step (|g| >= 1e-2 max |g| of its tensor, where the GPU gradient
    is within 1e-4) within 1e-3 of a rate per step (plus FP32 rounding)."""
    sc = make_scene("c1")
    total = 3
    st = TrainState(sc)
    e32 = exposure_for(sc)
    st.exposure.copy_(torch.as_tensor(e32))
    optim = paper_optim(sc.extent, total)
    rates = oracle.Rates(optim.lr.z, optim.lr.q, optim.lr.s, optim.lr.alpha, optim.lr.rgb,
                         optim.lr.sem, optim.lr.exposure, optim.z_start, optim.z_end, total)
    o = oopts(st.opts)
    K, N = st.K, st.N
    # oracle state: FP64 raw block and activated values
    p = st.params.cpu().numpy().astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    s_act, a_act = sc.s.astype(np.float64), sc.alpha.astype(np.float64)
    e = e32.astype(np.float64)
    me, ve = np.zeros_like(e), np.zeros_like(e)
    rowrate = np.array([0.0] + [rates.q] * 4 + [rates.s] * 2 + [rates.alpha] + [rates.rgb] * 3 +
                       [rates.sem] * (K - 11))
    steady = np.ones((K, N), bool)
    for step in range(1, total + 1):
        prm = oracle.Params(N, sc.n_sem, sc.x.astype(np.float64), sc.y.astype(np.float64),
                            p[0].copy(), p[1:5].copy(), s_act.copy(), a_act.copy(),
                            p[8:11].copy(), p[11:].copy())
        L, gref, dexp, _ = oracle.loss_and_grads(prm, sc.cams, sc.targets, exposure=e, opts=o)
        G = np.concatenate([gref[:N][None], gref[N:5 * N].reshape(4, N),
                            gref[5 * N:7 * N].reshape(2, N), gref[7 * N:8 * N][None],
                            gref[8 * N:11 * N].reshape(3, N),
                            gref[11 * N:].reshape(sc.n_sem, N)])
        for sl in ROWS.values():
            mx = np.abs(G[sl]).max()
            steady[sl] &= np.abs(G[sl]) >= 1e-2 * mx
        st.step_fused(total_steps=total, grads_out=True)
        torch.cuda.synchronize()
        grads_compare(st.grads.cpu().numpy(), gref, N, sc.n_sem)
        np.testing.assert_allclose(st.d_exp.cpu().numpy(), dexp, rtol=1e-4, atol=1e-6)
        assert abs(st.fused_status()["loss"] - L) <= 1e-5 * max(1.0, abs(L))
        s_act, a_act = oracle.adam_raw(p, G, m, v, rates, step, b1=float(np.float32(0.9)),
                                       b2=float(np.float32(0.999)), eps=float(np.float32(1e-8)),
                                       exposure=e, d_exposure=dexp, m_exp=me, v_exp=ve)
        rowrate[0] = max(rowrate[0], oracle.z_rate(rates, 1))
        got = st.params.cpu().numpy()
        d = np.abs(got - p)
        assert np.all(d <= 2.0 * step * rowrate[:, None] + 4 * step * ulp32(p))
        tol = 1e-3 * step * rowrate[:, None] + 4 * step * ulp32(p)
        assert steady.sum() > 0.05 * steady.size
        assert np.all(d[steady] <= tol[steady]), (step, np.max(d[steady] - tol[steady]))
        np.testing.assert_allclose(st.exposure.cpu().numpy(), e, rtol=0,
                                   atol=1e-3 * rates.exposure * step + 4e-7)
    assert st.fused_status()["step"] == total


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


@pytest.mark.parametrize("name,stage", [("mini", 32), ("mini16", 16), ("mini16", 32),
                                        ("mini16", 64)])
def test_fused_step_one_pixel_per_lane_equals_batched(gpu, name, stage):
    # 16 x 4 tiles (one pixel per lane): where the fused step keeps the
    # forward's footprint weights of each list's first 16 entries for its
    # backward (up to 8 classes at 32-entry staging; 16 classes at every
    # staging depth), they must be the bits the batched backward recomputes
    sc = make_scene(name)
    a = TrainState(sc, opts=B.make_opts(tile_w=16, tile_h=4, stage=stage))
    a.step_batched(total_steps=5)
    b = TrainState(sc, opts=B.make_opts(tile_w=16, tile_h=4, stage=stage))
    b.step_fused(total_steps=5, grads_out=True)
    torch.cuda.synchronize()
    sa, sb = _snapshot(a), _snapshot(b)
    for k in ("params", "m", "v", "s_act", "alpha_act"):
        assert torch.equal(sa[k], sb[k]), k
    assert torch.equal(a.grads.cpu(), b.grads.cpu())


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
    assert (ev, co) == oracle_work_counts(prm, sc.cams, oopts(st.opts))


@pytest.mark.parametrize("name", ["mini16", "c1"])
def test_channel_masks_render_only_selected_planes(gpu, name):
    """rogs_render_fwd with a channel set: the selected planes are bitwise
    those of an all-plane render, the others are left as they were; ELEV
    selects depth and alpha; the backward needs an all-plane forward."""
    sc = make_scene(name)
    st = TrainState(sc)
    ws, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    surf = st.surfels()
    st.rg.render_fwd(surf, ws, st.out)
    full = st.out.clone()
    C, NO = sc.n_sem, n_out(sc.n_sem)
    planes = {B.CH_RGB: [0, 1, 2], B.CH_SEM: list(range(3, 3 + C)), B.CH_D: [3 + C],
              B.CH_A: [4 + C], B.CH_ELEV: [3 + C, 4 + C]}
    sentinel = -12345.0
    for mask in (B.CH_RGB, B.CH_SEM, B.CH_RGB | B.CH_SEM, B.CH_D | B.CH_A, B.CH_ELEV,
                 B.CH_ELEV | B.CH_SEM, B.CH_A):
        st.out.fill_(sentinel)
        st.rg.render_fwd(surf, ws, st.out, channels=mask)
        torch.cuda.synchronize()
        sel = sorted({p for bit, ps in planes.items() if mask & bit for p in ps})
        for v in range(st.V):
            got, ref = st.image(v), full[NO * st.pix_off[v]: NO * st.pix_off[v + 1]].view(
                NO, sc.cams[v].h, sc.cams[v].w)
            for p in range(NO):
                if p in sel:
                    assert torch.equal(got[p], ref[p]), (mask, v, p)
                else:
                    assert bool((got[p] == sentinel).all()), (mask, v, p)
        with pytest.raises(B.RogsError) as e:
            st.rg.render_bwd(surf, ws, st.out, st.G, st.grads, 0)
        assert e.value.code == B.ESTATE
    with pytest.raises(B.RogsError) as e:
        st.rg.render_fwd(surf, ws, st.out, channels=0)
    assert e.value.code == B.EINVAL
    # an all-plane forward again allows the backward
    st.rg.render_fwd(surf, ws, st.out)
    st.rg.render_bwd(surf, ws, st.out, st.G, st.grads, 0)


@pytest.mark.parametrize("fused", [True, False])
def test_checkpoint_resume_is_bitwise(gpu, tmp_path, fused):
    """Two steps, checkpoint, a third step; a fresh state loaded from the
    checkpoint takes the same third step: parameters, moments, activated
    copies, exposure and the device step state are identical."""
    sc = make_scene("c1")
    total = 3
    a = TrainState(sc)
    a.exposure.copy_(torch.as_tensor(exposure_for(sc)))
    step = (lambda s: s.step_fused(total_steps=total)) if fused else \
        (lambda s: s.step_batched(total_steps=total))
    for _ in range(2):
        step(a)
    path = str(tmp_path / "ckpt.npz")
    a.save_checkpoint(path)
    step(a)
    b = TrainState(sc)
    b.load_checkpoint(path)
    step(b)
    torch.cuda.synchronize()
    for k in ("params", "m", "v", "s_act", "alpha_act", "exposure", "m_exp", "v_exp"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    if fused:       # the fused step counts its steps on the device
        assert torch.equal(a.step_state, b.step_state)
        assert b.fused_status()["step"] == total
    else:
        assert a.step_count == b.step_count == total
    other = TrainState(make_scene("tiny2"))
    with pytest.raises(ValueError):
        other.load_checkpoint(path)
