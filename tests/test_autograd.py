"""torch.autograd wrapper (RenderFn): forward equals the batched path bitwise,
backward equals the FP64 oracle's adjoint (pinned by finite differences) for
an arbitrary dL/d(image), including the depth and alpha channels."""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth
from paper_2405_14342_amd.autograd import RenderFn, render, split_views
from paper_2405_14342_amd.pipeline import TrainState

ROWS = {"z": slice(0, 1), "q": slice(1, 5), "s": slice(5, 7), "alpha": slice(7, 8),
        "rgb": slice(8, 11), "sem": slice(11, None)}


def _inputs(sc, dev="cuda"):
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    return dict(z=f(sc.z), q=f(sc.q), s=f(sc.s), alpha=f(sc.alpha), rgb=f(sc.rgb), sem=f(sc.sem),
                x=f(sc.x), y=f(sc.y))


def test_cpu_tensors_are_rejected():
    sc = synth.tiny_scene()
    t = _inputs(sc, dev="cpu")
    with pytest.raises(TypeError, match="CUDA"):
        render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"], sc.cams)


@pytest.mark.gpu
def test_forward_equals_batched_path():
    sc = synth.mini_strip()
    t = _inputs(sc)
    out = render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"], sc.cams)
    st = TrainState(sc)
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    assert torch.equal(out, st.out)
    views = split_views(out, sc.cams, sc.n_sem)
    assert torch.equal(views[0], st.image(0))


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["tiny2", "mini"])
def test_backward_matches_oracle_adjoint(name):
    sc = synth.tiny_scene(n_views=2) if name == "tiny2" else synth.mini_strip()
    t = _inputs(sc)
    for k in ("z", "q", "s", "alpha", "rgb", "sem"):
        t[k].requires_grad_(True)
    out = render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"], sc.cams)
    rng = np.random.default_rng(77)
    W = rng.normal(0.0, 1.0, out.numel()).astype(np.float32)
    (out * torch.as_tensor(W, device="cuda")).sum().backward()
    got = torch.cat([t["z"].grad[None], t["q"].grad, t["s"].grad, t["alpha"].grad[None],
                     t["rgb"].grad, t["sem"].grad]).cpu().numpy()
    prm = oracle.Params.from_scene(sc)
    ref = np.zeros((11 + sc.n_sem) * sc.n, np.float64)
    o = 0
    for cam in sc.cams:
        npx = cam.w * cam.h
        G = W[o:o + (5 + sc.n_sem) * npx].reshape(5 + sc.n_sem, npx).astype(np.float64)
        o += (5 + sc.n_sem) * npx
        fo, tf, nl = oracle.render_fwd(prm, cam)
        oracle.render_bwd(prm, cam, G, tf, nl, grads=ref)
    r = oracle.split_grads(ref, sc.n, sc.n_sem)
    for nm, sl in ROWS.items():
        a = got[sl].reshape(r[nm].shape) if r[nm].ndim > 1 else got[sl].reshape(-1)
        mx = np.abs(r[nm]).max()
        d = np.abs(a - r[nm])
        assert d.max() <= 1e-4 * mx, (nm, d.max() / mx)
        big = np.abs(r[nm]) >= 1e-2 * mx
        assert (d[big] / np.abs(r[nm][big])).max() <= 1e-4, nm


@pytest.mark.gpu
def test_two_renders_alive_before_backward():
    sc = synth.tiny_scene(n_views=2)
    t = _inputs(sc)
    t["rgb"].requires_grad_(True)
    a = render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"], sc.cams[:1])
    b = render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"], sc.cams)
    (a.sum() + b.sum()).backward()
    g_both = t["rgb"].grad.clone()
    t["rgb"].grad = None
    render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"],
           sc.cams[:1]).sum().backward()
    g_a = t["rgb"].grad.clone()
    t["rgb"].grad = None
    render(t["z"], t["q"], t["s"], t["alpha"], t["rgb"], t["sem"], t["x"], t["y"],
           sc.cams).sum().backward()
    g_b = t["rgb"].grad.clone()
    torch.testing.assert_close(g_both, g_a + g_b, rtol=1e-6, atol=1e-7)
