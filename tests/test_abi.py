"""The C-ABI library loads, exports every symbol include/rogs.h declares, and
its host-only entry points validate their arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2405_14342_amd import binding as B
from paper_2405_14342_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rogs.h")).read()
    return sorted(set(re.findall(r"ROGS_API\s+[\w\s\*]*?\b(rogs_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_symbols()
    assert len(decl) >= 14
    assert sorted(B.EXPORTED) == decl


def test_library_exports_every_declared_symbol():
    L = B.load_library()
    for name in declared_symbols():
        assert hasattr(L, name), name
    # internal C++ symbols stay hidden
    out = os.popen(f"nm -D --defined-only {B.LIB_PATH}").read()
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    assert {s for s in exported if s.startswith("rogs_")} == set(declared_symbols())
    assert not any(s.startswith("_ZN4rogs") for s in exported)


def test_struct_sizes_match_header():
    # rogs_camera: 4 ints + 4 + 9 + 3 + 1 + 6 + 2 floats
    assert ctypes.sizeof(B.Camera) == 4 * (4 + 4 + 9 + 3 + 1 + 6 + 2)
    assert ctypes.sizeof(B.RenderOpts) == 28
    assert ctypes.sizeof(B.Surfels) == 8 + 8 * 8
    # 4 pointers, 3 floats (+4 padding), 2 pointers, 2 floats
    assert ctypes.sizeof(B.Targets) == 4 * 8 + 3 * 4 + 4 + 2 * 8 + 2 * 4
    assert ctypes.sizeof(B.Pose) == 12 * 4
    assert ctypes.sizeof(B.LR) == 7 * 4
    # rogs_request: camera, channels, elev_ref, then the 8-byte-aligned pointer
    assert ctypes.sizeof(B.Request) == 136 and B.Request.out.offset == 128
    assert ctypes.sizeof(B.Result) == 32


def _surf(n=100, C=8):
    return B.Surfels(n, C, 8, 8, 8, 8, 8, 8, 8, 8)


def test_default_opts():
    o = B.default_opts()
    assert (o.tile_w, o.tile_h) == (16, 16)
    assert abs(o.eps2d - 0.3) < 1e-7 and o.q_cut == 9.0
    assert abs(o.alpha_max - 0.99) < 1e-7 and abs(o.t_eps - 1e-6) < 1e-12


def test_workspace_size_grows_with_capacity_and_views():
    sc = synth.config1()
    s = _surf(sc.n, 8)
    o = B.make_opts()
    a = B.workspace_size(s, sc.cams, o, 1000)
    b = B.workspace_size(s, sc.cams, o, 100000)
    c = B.workspace_size(s, sc.cams * 3, o, 100000)
    d = B.workspace_size(s, sc.cams, o, 100000, 2000)
    assert 0 < a < d < b < c
    # per pair: keys (4 + 8), vals x2, emission slot, gradient record (C = 8 -> 20 floats)
    assert d - a >= (100000 - 1000) * (4 + 8 + 4 * 3 + 4 * 20)


@pytest.mark.parametrize("bad", ["n", "sem", "views", "cap", "tile", "tile2", "eps", "amax",
                                 "cam_w", "cam_model", "cam_tile", "cam_tile2", "cam_fx", "cam_nan",
                                 "stage"])
def test_workspace_size_rejects_invalid(bad):
    sc = synth.config1()
    cams = [B.make_camera(c) for c in sc.cams]
    s = _surf(sc.n, 8)
    o = B.make_opts()
    nv, cap = 1, 1000
    if bad == "n":
        s.n = 0
    elif bad == "sem":
        s.n_sem = 11
    elif bad == "views":
        nv = 0
    elif bad == "cap":
        cap = 1 << 31
    elif bad == "tile":
        o.tile_w, o.tile_h = 12, 16
    elif bad == "tile2":
        o.tile_w, o.tile_h = 16, 32
    elif bad == "eps":
        o.eps2d = float("nan")
    elif bad == "amax":
        o.alpha_max = 1.0
    elif bad == "cam_w":
        cams[0].w = 0
    elif bad == "cam_model":
        cams[0].model = 7
    elif bad == "cam_tile":          # area differs from the options' 16 x 16
        cams[0].tile = B.tile_code(16, 4)
    elif bad == "cam_tile2":         # tile_w must divide 64
        cams[0].tile = B.tile_code(12, 16)
    elif bad == "stage":
        o.stage = 48
    elif bad == "cam_fx":
        cams[0].fx = -1.0
    elif bad == "cam_nan":
        cams[0].R_cw[4] = float("nan")
    L = B.load_library()
    arr = B.camera_array(cams)
    out = ctypes.c_size_t(0)
    r = L.rogs_workspace_size(ctypes.byref(s), arr, nv, ctypes.byref(o), cap, 0, ctypes.byref(out))
    assert r == B.EINVAL


def test_workspace_size_null_arguments():
    L = B.load_library()
    out = ctypes.c_size_t(0)
    o = B.make_opts()
    assert L.rogs_workspace_size(None, None, 1, ctypes.byref(o), 10, 0, ctypes.byref(out)) == B.EINVAL
    assert L.rogs_workspace_size(ctypes.byref(_surf()), B.camera_array(synth.config1().cams), 1,
                                 ctypes.byref(o), 10, 0, None) == B.EINVAL
    assert L.rogs_workspace_size(ctypes.byref(_surf()), B.camera_array(synth.config1().cams), 1,
                                 ctypes.byref(o), 10, -1, ctypes.byref(out)) == B.EINVAL


def test_null_context_is_rejected():
    L = B.load_library()
    assert L.rogs_create(None) == B.EINVAL
    assert L.rogs_last_error(None) == b"null context"
    L.rogs_destroy(None)


def test_per_view_tile_and_stage_accepted():
    """A view's own tile shape of the options' area, and every staging depth,
    are valid; the per-tile arrays follow the view's own tile count."""
    sc = synth.config1()
    s = _surf(sc.n, 8)
    L = B.load_library()
    sizes = {}
    for code in (0, B.tile_code(64, 4), B.tile_code(4, 64), B.tile_code(32, 8)):
        cams = [B.make_camera(c) for c in sc.cams]
        cams[0].tile = code
        for stage in (0, 16, 32, 64):
            o = B.make_opts(stage=stage)
            out = ctypes.c_size_t(0)
            r = L.rogs_workspace_size(ctypes.byref(s), B.camera_array(cams), 1, ctypes.byref(o),
                                      1000, 0, ctypes.byref(out))
            assert r == B.OK, (code, stage)
            sizes.setdefault(code, set()).add(out.value)
    # the staging depth changes no buffer; a 16 x 16 code equals the default
    assert all(len(v) == 1 for v in sizes.values())
    w, h = sc.cams[0].w, sc.cams[0].h
    tiles = lambda tw, th: -(-w // tw) * -(-h // th)
    if tiles(64, 4) != tiles(16, 16):
        assert sizes[B.tile_code(64, 4)] != sizes[0]
