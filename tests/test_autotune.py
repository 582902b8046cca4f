"""rogs_autotune: a descent over the tile shape (all views alike), the LDS
staging depth and a tile shape per resolution class; the result is kept in a
JSON cache keyed by the workload, returned from the cache without timing,
foreign files are refused; a tuned TrainState renders the same images as the
default configuration."""
import json
import os

import pytest
import torch

from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth
from paper_2405_14342_amd.pipeline import TrainState, paper_optim

SHAPES = {(tw, a // tw) for tw in (4, 8, 16, 32, 64) for a in (64, 128, 256) if a % tw == 0}
MIXED = [(320, 180), (256, 144), (256, 144), (320, 180), (256, 144), (256, 144)]
pytestmark = pytest.mark.gpu


def _check_codes(o, cams, tiles):
    area = o.tile_w * o.tile_h
    for c, t in zip(cams, tiles):
        if t:
            tw, th = t & 0xFFFF, t >> 16
            assert tw * th == area and 64 % tw == 0 and (tw, th) != (o.tile_w, o.tile_h)


def test_autotune_chooses_and_caches(tmp_path):
    sc = synth.mini_strip()
    st = TrainState(sc)
    path = str(tmp_path / "tiles.json")
    o, ms, tiles = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2)
    assert (o.tile_w, o.tile_h) in SHAPES and o.stage in (16, 32, 64) and ms > 0.0
    assert tiles == [0] * len(st.cams)              # one resolution class
    data = json.load(open(path))
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert (entry["tile_w"], entry["tile_h"], entry["stage"]) == (o.tile_w, o.tile_h, o.stage)
    assert entry["views"] == tiles
    assert entry["classes"] == {"320x180/m0": f"{o.tile_w}x{o.tile_h}"}
    timed = entry["timed"]
    # every shape at depth 32, then the other depths at the best shape
    assert {k for k in timed if k.endswith("/s32")} >= {f"{w}x{h}/s32" for w, h in SHAPES}
    assert len(timed) == len(SHAPES) + 2
    best32 = min(v for k, v in timed.items() if k.endswith("/s32"))
    assert entry["ms"] <= best32 + 1e-3
    assert any(abs(v - entry["ms"]) <= 1e-3 for v in timed.values())
    # cached: same answer, the stored time, file unchanged
    before = open(path).read()
    o2, ms2, tiles2 = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2)
    assert (o2.tile_w, o2.tile_h, o2.stage) == (o.tile_w, o.tile_h, o.stage)
    assert tiles2 == tiles
    assert ms2 == pytest.approx(entry["ms"], abs=1e-3)
    assert open(path).read() == before
    # a second workload is added next to the first
    sc2 = synth.tiny_scene(n_views=2)
    st2 = TrainState(sc2)
    st2.rg.autotune(st2.surfels(), st2.cams, cache_json=path, reps=1)
    assert len(json.load(open(path))) == 2


def test_autotune_resolution_classes(tmp_path):
    sc = synth.mini_strip(sides=MIXED)
    st = TrainState(sc)
    path = str(tmp_path / "tiles.json")
    o, ms, tiles = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2)
    _check_codes(o, st.cams, tiles)
    entry = next(iter(json.load(open(path)).values()))
    assert set(entry["classes"]) == {"320x180/m0", "256x144/m0"}
    # views of one class share their code, and the class table says which
    for c, t in zip(st.cams, tiles):
        shape = f"{t & 0xFFFF}x{t >> 16}" if t else f"{o.tile_w}x{o.tile_h}"
        assert entry["classes"][f"{c.w}x{c.h}/m0"] == shape
    # the class step tried the other shapes of the chosen area for each class
    area = o.tile_w * o.tile_h
    per_class = [k for k in entry["timed"] if ":" in k]
    n_alt = sum(1 for tw in (4, 8, 16, 32, 64) if area // tw >= 1) - 1
    assert len(per_class) == 2 * n_alt


def test_autotune_refuses_foreign_file(tmp_path):
    sc = synth.tiny_scene()
    st = TrainState(sc)
    path = str(tmp_path / "other.json")
    with open(path, "w") as f:
        f.write('{"something": [1, 2, 3]}\n')
    with pytest.raises(B.RogsError, match="EINVAL"):
        st.rg.autotune(st.surfels(), st.cams, cache_json=path)
    assert open(path).read() == '{"something": [1, 2, 3]}\n'


def test_tuned_state_renders_like_default(tmp_path):
    sc = synth.mini_strip(sides=MIXED)
    a = TrainState(sc, opts="auto", autotune_cache=str(tmp_path / "t.json"))
    b = TrainState(sc)
    a.step_batched(adam=False)
    b.step_batched(adam=False)
    torch.cuda.synchronize()
    assert torch.equal(a.out, b.out)
    assert os.path.exists(str(tmp_path / "t.json"))
    # the fused step runs in the tuned configuration too
    a.step_fused(total_steps=2)
    torch.cuda.synchronize()
    assert a.fused_status()["overflow"] == 0


def test_step_mode_reads_the_state_only(tmp_path):
    """Timing fused steps runs them on copies: the caller's parameters,
    moments, exposure and step count are unchanged, and its own fused steps
    go on afterwards from where they were."""
    sc = synth.mini_strip(sides=MIXED)
    st = TrainState(sc)
    st.step_fused(total_steps=5)
    torch.cuda.synchronize()
    names = ("params", "m", "v", "s_act", "alpha_act", "exposure", "m_exp", "v_exp", "step_state")
    snap = {k: getattr(st, k).clone() for k in names}
    path = str(tmp_path / "tiles.json")
    step = (st.train_state(), st.targets(0, st.V), paper_optim(sc.extent, 5))
    o, ms, tiles = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2, step=step)
    torch.cuda.synchronize()
    for k in names:
        assert torch.equal(snap[k], getattr(st, k)), k
    _check_codes(o, st.cams, tiles)
    key, entry = next(iter(json.load(open(path)).items()))
    assert key.startswith("step;") and entry["views"] == tiles
    st.step_fused(total_steps=5)
    assert st.fused_status()["step"] == 2
