"""The termination threshold t_eps of the front-to-back walk (Eq. 6: a pixel
stops after the list entry that takes its transmittance below t_eps): at 0
no pixel stops; at 0.01 and 0.2 many do, at 0.2 mostly after their first
entries that reach them.  Images, loss and gradients match the oracle run
with the same threshold, the entries every pixel visits (its n_last, summed
over the batch) match the oracle's, and the fused step equals the batched
step plus Adam bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd.pipeline import TrainState
from parity_util import grads_compare, oracle_work_counts
from test_gpu_parity import fwd_compare, make_scene, oopts

pytestmark = pytest.mark.gpu
TEPS = [0.0, 1e-2, 0.2]


def opts(teps):
    return B.make_opts(tile_w=16, tile_h=4, t_eps=teps)


@pytest.mark.parametrize("teps", TEPS)
@pytest.mark.parametrize("name", ["c1", "mini"])
def test_images_loss_gradients(name, teps):
    sc = make_scene(name)
    st = TrainState(sc, opts=opts(teps))
    st.step_batched(adam=False)
    torch.cuda.synchronize()
    fwd_compare(sc, st)
    prm = oracle.Params.from_scene(sc)
    L, gref, _, _ = oracle.loss_and_grads(prm, sc.cams, sc.targets, opts=oopts(st.opts))
    assert abs(st.loss.item() - L) <= 1e-5 * max(1.0, abs(L))
    grads_compare(st.grads.cpu().numpy(), gref, sc.n, sc.n_sem)


@pytest.mark.parametrize("teps", TEPS)
def test_entries_visited(teps):
    sc = make_scene("c1")
    st = TrainState(sc, opts=opts(teps))
    ws, _ = st.project_and_sort(st.cams, "cap_batch", "_ws_batch")
    st.rg.render_fwd(st.surfels(), ws, st.out)
    ev, co = st.rg.debug_work(ws)
    ref = oracle_work_counts(oracle.Params.from_scene(sc), sc.cams, oopts(st.opts))
    assert (ev, co) == ref
    if teps == 0.2:
        # the threshold cuts the walk short for most pixels
        e0, _ = oracle_work_counts(oracle.Params.from_scene(sc), sc.cams,
                                   oopts(opts(0.0)))
        assert ev < 0.8 * e0, (ev, e0)


def _snapshot(st):
    return {k: getattr(st, k).detach().cpu().clone() for k in
            ("params", "m", "v", "s_act", "alpha_act")}


@pytest.mark.parametrize("teps", TEPS)
def test_fused_equals_batched(teps):
    sc = make_scene("mini")
    a = TrainState(sc, opts=opts(teps))
    a.step_batched(total_steps=5)
    b = TrainState(sc, opts=opts(teps))
    b.step_fused(total_steps=5, grads_out=True)
    torch.cuda.synchronize()
    sa, sb = _snapshot(a), _snapshot(b)
    for k in sa:
        assert torch.equal(sa[k], sb[k]), k
    assert torch.equal(a.grads.cpu(), b.grads.cpu())
