"""rogs_autotune: picks a supported tile shape, keeps it in a JSON cache keyed
by the workload, returns cached entries without timing, refuses foreign
files; a tuned TrainState renders the same images as the default shape."""
import json
import os

import pytest
import torch

from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth
from paper_2405_14342_amd.pipeline import TrainState

SHAPES = {(tw, a // tw) for tw in (4, 8, 16, 32, 64) for a in (64, 128, 256) if a % tw == 0}
pytestmark = pytest.mark.gpu


def test_autotune_chooses_and_caches(tmp_path):
    sc = synth.mini_strip()
    st = TrainState(sc)
    path = str(tmp_path / "tiles.json")
    o, ms = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2)
    assert (o.tile_w, o.tile_h) in SHAPES and ms > 0.0
    data = json.load(open(path))
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert (entry["tile_w"], entry["tile_h"]) == (o.tile_w, o.tile_h)
    assert len(entry["shapes"]) == len(SHAPES)
    assert min(entry["shapes"].values()) == pytest.approx(entry["ms"], abs=1e-3)
    # cached: same answer, the stored time, file unchanged
    before = open(path).read()
    o2, ms2 = st.rg.autotune(st.surfels(), st.cams, cache_json=path, reps=2)
    assert (o2.tile_w, o2.tile_h) == (o.tile_w, o.tile_h)
    assert ms2 == pytest.approx(entry["ms"], abs=1e-3)
    assert open(path).read() == before
    # a second workload is added next to the first
    sc2 = synth.tiny_scene(n_views=2)
    st2 = TrainState(sc2)
    st2.rg.autotune(st2.surfels(), st2.cams, cache_json=path, reps=1)
    assert len(json.load(open(path))) == 2


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
    sc = synth.mini_strip()
    a = TrainState(sc, opts="auto", autotune_cache=str(tmp_path / "t.json"))
    b = TrainState(sc)
    a.step_batched(adam=False)
    b.step_batched(adam=False)
    torch.cuda.synchronize()
    assert torch.equal(a.out, b.out)
    assert os.path.exists(str(tmp_path / "t.json"))
