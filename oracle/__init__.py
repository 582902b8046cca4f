"""FP64 CPU oracle for meshgrid-surfel splatting (RoGs, arXiv 2405.14342).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it; the two meet only in the
seeded input generator (``paper_2405_14342_amd.synth``), which holds none of
the method's arithmetic.

The C++ core (``rogs_oracle.cpp``) follows the paper step by step:
Eq. 2 (covariance with s_z = 0), Eq. 5 (EWA projection; orthographic J),
the ascending-depth sort and Eq. 6 (alpha compositing of RGB, semantics,
depth and alpha), Eq. 7 (exposure), Eq. 8/9/12 (masked L1 + CE), and Adam
(Sec. 4.2).  Discrete decisions (cull, tile rectangles, per-pixel 3-sigma
test, depth order) are taken with the key contract that the library
documents (FP64 projection rounded to an FP32 record, FP32 per-pixel test);
every value is computed in FP64.

Parity status of each function (what pins it) is listed in the test files
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rogs_oracle.cpp")
_SRC_GRID = os.path.join(_HERE, "rogs_oracle_grid.cpp")
_LIB = os.path.join(_HERE, "_rogs_oracle.so")
_lib = None

CMD = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
       "-fPIC", "-shared", _SRC, _SRC_GRID, "-o", _LIB]


def _stale() -> bool:
    return not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                           for f in (_SRC, _SRC_GRID))


def build(force: bool = True) -> str:
    """Compile the oracle shared library with g++ (always, when force)."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        cmd = CMD[:-1] + [tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I, I64, D = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        _lib.orc_contract.argtypes = [I, I, P, P, P, P, P, P, P, P]
        _lib.orc_contract.restype = I
        _lib.orc_geo64.argtypes = [I, I, P, P, P, P, P, P]
        _lib.orc_geo64_adjoint.argtypes = [I, I, P, P, P, P, P, I, P, P]
        _lib.orc_tile_lists.argtypes = [I, I, P, P, P, P, P, I64, P, P, P]
        _lib.orc_tile_lists.restype = I64
        _lib.orc_render_fwd.argtypes = [I, I, P, P, P, P, P, P, I64, P, P, P]
        _lib.orc_render_bwd.argtypes = [I, I, P, P, P, P, P, P, I64, P, P, P, P]
        _lib.orc_loss.argtypes = [I, I64, P, P, P, P, I64, D, D, D, D, D, P, P]
        _lib.orc_loss.restype = D
        _lib.orc_adam.argtypes = [I64, P, P, P, P, D, D, D, D, I64]
        _lib.orc_num_threads.restype = I
        _lib.orc_set_threads.argtypes = [I]
        _lib.orc_z_rate.argtypes = [D, D, D, I64, I64]
        _lib.orc_z_rate.restype = D
        _lib.orc_adam_raw.argtypes = [I, I, P, P, P, P, P, D, D, I64, I64, D, D, D, P, P, I, P, P,
                                      P, P]
        _lib.orc_row_spans.argtypes = [P, I, I, I, I, ctypes.c_float, I, I, I, I, P, P]
        _lib.orc_q32.argtypes = [I, P, I, P, P, P]
        _lib.orc_smooth.argtypes = [I64, P, P, D, P]
        _lib.orc_smooth.restype = D
        _lib.orc_lidar_loss.argtypes = [I64, P, P, D, P]
        _lib.orc_lidar_loss.restype = D
        _lib.orc_lidar_nn.argtypes = [I64, P, P, I64, P, P, P]
        _lib.orc_pose_pixels.argtypes = [I, P, D, D, ctypes.c_float, P]
        _lib.orc_layout_mask.argtypes = [I, I, I, P, I, P]
        _lib.orc_layout_mask.restype = I64
        _lib.orc_layout_build.argtypes = [I, I, P, D, D, ctypes.c_float, I, P, I64, P, P, P, P,
                                          P, P]
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Opts:
    """Render options (the library's defaults)."""
    tile_w: int = 16
    tile_h: int = 16
    eps2d: float = 0.3      # EWA screen-space low-pass added to Sigma' (px^2)
    q_cut: float = 9.0      # per-pixel Mahalanobis cut (3 sigma)
    alpha_max: float = 0.99
    t_eps: float = 1e-6     # stop once transmittance falls below this

    def arrays(self):
        return (np.array([self.tile_w, self.tile_h], np.int32),
                np.array([self.eps2d, self.q_cut, self.alpha_max, self.t_eps], np.float32))


def pack_camera(cam) -> np.ndarray:
    """Flat 28-float camera record read by the C++ oracle."""
    c = np.zeros(28, np.float32)
    c[0], c[1], c[2] = cam.w, cam.h, cam.model
    c[3], c[4], c[5], c[6] = cam.fx, cam.fy, cam.cx, cam.cy
    c[7:16] = np.asarray(cam.R_cw, np.float32).reshape(9)
    c[16:19] = np.asarray(cam.t_cw, np.float32)
    c[19] = cam.z_near
    c[20:22] = cam.cull_o
    c[22:24] = cam.cull_ex
    c[24:26] = cam.cull_ez
    c[26], c[27] = cam.cull_lat, cam.cull_fwd
    return c


class Params:
    """Surfel parameters as the oracle consumes them.

    ``f32`` holds the FP32 decision inputs (x, y, z, q, s); the FP64 arrays
    hold the values.  ``Params.from_scene`` promotes the scene's FP32 bits;
    finite-difference tests edit only the FP64 arrays (decisions frozen).
    """

    def __init__(self, n, C, x, y, z, q, s, alpha, rgb, sem, f32=None):
        self.n, self.C = n, C
        self.x, self.y, self.z = x, y, z
        self.q, self.s, self.alpha, self.rgb, self.sem = q, s, alpha, rgb, sem
        if f32 is None:
            f32 = np.concatenate([np.asarray(a, np.float32).reshape(-1) for a in (x, y, z, q, s)])
        self.f32 = np.ascontiguousarray(f32, np.float32)

    @classmethod
    def from_scene(cls, sc):
        d = lambda a: np.array(a, np.float64)
        return cls(sc.n, sc.n_sem, d(sc.x), d(sc.y), d(sc.z), d(sc.q), d(sc.s), d(sc.alpha),
                   d(sc.rgb), d(sc.sem))

    def copy(self):
        c = lambda a: a.copy()
        return Params(self.n, self.C, c(self.x), c(self.y), c(self.z), c(self.q), c(self.s),
                      c(self.alpha), c(self.rgb), c(self.sem), f32=self.f32.copy())

    def f64(self) -> np.ndarray:
        return np.ascontiguousarray(np.concatenate(
            [a.reshape(-1) for a in (self.x, self.y, self.z, self.q, self.s, self.alpha,
                                     self.rgb, self.sem)]), np.float64)


GRAD_NAMES = ("z", "q", "s", "alpha", "rgb", "sem")


def split_grads(g: np.ndarray, n: int, C: int):
    """Split the flat gradient block into named arrays (views)."""
    return {"z": g[:n], "q": g[n:5 * n].reshape(4, n), "s": g[5 * n:7 * n].reshape(2, n),
            "alpha": g[7 * n:8 * n], "rgb": g[8 * n:11 * n].reshape(3, n),
            "sem": g[11 * n:(11 + C) * n].reshape(C, n)}


def contract(prm: Params, cam, opts: Opts = Opts()):
    """Key contract of one view: (vis[n] bool, rec[n,8] = u_hi v_hi u_lo v_lo A B C t_z
    (binary32), rect[n,4] = x0 x1 y0 y1)."""
    L = _load()
    io, fo = opts.arrays()
    f64 = prm.f64()
    rec = np.zeros((prm.n, 8), np.float32)
    rect = np.zeros((prm.n, 4), np.int32)
    vis = np.zeros(prm.n, np.uint8)
    L.orc_contract(prm.n, prm.C, _p(prm.f32), _p(f64), _p(pack_camera(cam)), _p(io), _p(fo),
                   _p(rec), _p(rect), _p(vis))
    return vis.astype(bool), rec, rect


def geo64(prm: Params, cam, opts: Opts = Opts()) -> np.ndarray:
    """FP64 projected values (u v A B C t_z) of every surfel, [n, 6]."""
    L = _load()
    io, fo = opts.arrays()
    out = np.zeros((prm.n, 6), np.float64)
    L.orc_geo64(prm.n, prm.C, _p(prm.f32), _p(prm.f64()), _p(pack_camera(cam)), _p(io), _p(fo),
                _p(out))
    return out


def geo64_adjoint(prm: Params, cam, i: int, dgeo, opts: Opts = Opts()) -> np.ndarray:
    """dL/d(z, q0..q3, sx, sy) of surfel i for dL/d(u v A B C t_z) = dgeo."""
    L = _load()
    io, fo = opts.arrays()
    dg = np.ascontiguousarray(dgeo, np.float64)
    out = np.zeros(7, np.float64)
    L.orc_geo64_adjoint(prm.n, prm.C, _p(prm.f32), _p(prm.f64()), _p(pack_camera(cam)), _p(io),
                        _p(fo), i, _p(dg), _p(out))
    return out


def tile_lists(prm: Params, cam, opts: Opts = Opts()):
    """Brute-force tile lists of one view: (keys u64[P], ids i32[P], ranges i32[T,2])."""
    L = _load()
    io, fo = opts.arrays()
    f64, cp = prm.f64(), pack_camera(cam)
    tx = (cam.w + opts.tile_w - 1) // opts.tile_w
    ty = (cam.h + opts.tile_h - 1) // opts.tile_h
    ranges = np.zeros((tx * ty, 2), np.int32)
    P = L.orc_tile_lists(prm.n, prm.C, _p(prm.f32), _p(f64), _p(cp), _p(io), _p(fo), 0, None,
                         None, _p(ranges))
    keys = np.zeros(max(P, 1), np.uint64)
    ids = np.zeros(max(P, 1), np.int32)
    L.orc_tile_lists(prm.n, prm.C, _p(prm.f32), _p(f64), _p(cp), _p(io), _p(fo), P, _p(keys),
                     _p(ids), _p(ranges))
    return keys[:P], ids[:P], ranges


def render_fwd(prm: Params, cam, opts: Opts = Opts(), pix: Optional[np.ndarray] = None):
    """Forward render (Eq. 6) of one view at all pixels or at the linear pixel
    indices ``pix``.  Returns (out[(5+C), npix], tfinal[npix], nlast[npix])."""
    L = _load()
    io, fo = opts.arrays()
    npix = cam.w * cam.h if pix is None else len(pix)
    pix = None if pix is None else np.ascontiguousarray(pix, np.int32)
    out = np.zeros((5 + prm.C, npix), np.float64)
    tf = np.zeros(npix, np.float64)
    nl = np.zeros(npix, np.int32)
    L.orc_render_fwd(prm.n, prm.C, _p(prm.f32), _p(prm.f64()), _p(pack_camera(cam)), _p(io),
                     _p(fo), _p(pix), npix, _p(out), _p(tf), _p(nl))
    return out, tf, nl


def render_bwd(prm: Params, cam, G, tfinal, nlast, opts: Opts = Opts(),
               pix: Optional[np.ndarray] = None, grads: Optional[np.ndarray] = None):
    """Adjoint of :func:`render_fwd`: given dL/d(outputs) ``G`` and the
    forward's T_final and n_last at the same pixels, accumulates dL/d(z q s
    alpha rgb sem) into ``grads`` (flat FP64 block, see :func:`split_grads`)
    and returns it."""
    L = _load()
    io, fo = opts.arrays()
    npix = cam.w * cam.h if pix is None else len(pix)
    pix = None if pix is None else np.ascontiguousarray(pix, np.int32)
    if grads is None:
        grads = np.zeros((11 + prm.C) * prm.n, np.float64)
    c = lambda a, t: np.ascontiguousarray(a, t)
    L.orc_render_bwd(prm.n, prm.C, _p(prm.f32), _p(prm.f64()), _p(pack_camera(cam)), _p(io),
                     _p(fo), _p(pix), npix, _p(c(G, np.float64)), _p(c(tfinal, np.float64)),
                     _p(c(nlast, np.int32)), _p(grads))
    return grads


def loss(C: int, out, tgt_rgb, label, mask, mcount: int, exp_a=0.0, exp_b=0.0,
         lam_c=1.0, lam_s=0.06, scale=1.0):
    """Eq. 7-9 and 12 at the given pixels.  Returns (loss, G[(5+C), npix], dexp[2])."""
    L = _load()
    npix = out.shape[1]
    G = np.zeros((5 + C, npix), np.float64)
    dexp = np.zeros(2, np.float64)
    c = lambda a, t: np.ascontiguousarray(a, t)
    val = L.orc_loss(C, npix, _p(c(out, np.float64)), _p(c(tgt_rgb, np.float32).reshape(3, npix)),
                     _p(c(label, np.uint8).reshape(-1)), _p(c(mask, np.uint8).reshape(-1)),
                     int(mcount), exp_a, exp_b, lam_c, lam_s, scale, _p(G), _p(dexp))
    return float(val), G, dexp


def adam(p, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """In-place FP64 Adam on contiguous float64 arrays p, m, v with gradient g."""
    L = _load()
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    L.orc_adam(p.size, _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, int(step))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (OpenMP)."""
    _load().orc_set_threads(int(n))


# Sec. 4.2: learning rates of the parameter groups; the height rate is
# proportional to the scene size and falls from 1.6e-4 to 1.6e-6 of it.
RATE_Q = RATE_S = RATE_ALPHA = 1e-4
RATE_RGB, RATE_SEM, RATE_EXPOSURE = 8e-3, 0.1, 1e-3
RATE_Z_START, RATE_Z_END = 1.6e-4, 1.6e-6


@dataclass
class Rates:
    """Per-group Adam rates; z_start / z_end: the height schedule (used when
    total_steps > 0), z: the constant height rate otherwise."""
    z: float
    q: float
    s: float
    alpha: float
    rgb: float
    sem: float
    exposure: float
    z_start: float = 0.0
    z_end: float = 0.0
    total_steps: int = 0

    def array(self):
        return np.array([self.z, self.q, self.s, self.alpha, self.rgb, self.sem, self.exposure],
                        np.float64)


def paper_rates(extent: float, total_steps: int) -> Rates:
    """The rates of Sec. 4.2 for a scene whose size (grid bounding-box
    diagonal, metres) is ``extent``, over a run of ``total_steps`` steps."""
    z0, z1 = RATE_Z_START * extent, RATE_Z_END * extent
    return Rates(z0, RATE_Q, RATE_S, RATE_ALPHA, RATE_RGB, RATE_SEM, RATE_EXPOSURE, z0, z1,
                 int(total_steps))


def z_rate(rates: Rates, step: int) -> float:
    """The height learning rate of step ``step`` (1-based) under ``rates``."""
    return float(_load().orc_z_rate(rates.z, rates.z_start, rates.z_end, int(rates.total_steps),
                                    int(step)))


def adam_raw(params, grads_act, m, v, rates: Rates, step: int, b1=0.9, b2=0.999, eps=1e-8,
             exposure=None, d_exposure=None, m_exp=None, v_exp=None):
    """One Adam step (Sec. 4.2) on the raw block params[11 + C][n] (rows z,
    q0..q3, log s_x, log s_y, logit alpha, rgb, sem), in place, from the
    gradients w.r.t. the activated values the renderer reads (chained here
    through exp and sigmoid), with per-group rates and the height schedule.
    Optionally steps the per-view exposure [V, 2] too.  Returns the refreshed
    activated (s[2][n], alpha[n])."""
    L = _load()
    for a in (params, grads_act, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == params.shape
    K, n = params.shape
    C = K - 11
    s_act = np.zeros((2, n), np.float64)
    a_act = np.zeros(n, np.float64)
    nv = 0
    if exposure is not None:
        for a in (exposure, d_exposure, m_exp, v_exp):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        nv = exposure.shape[0]
    L.orc_adam_raw(n, C, _p(params), _p(grads_act), _p(m), _p(v), _p(rates.array()),
                   rates.z_start, rates.z_end, int(rates.total_steps), int(step), b1, b2, eps,
                   _p(s_act), _p(a_act), nv, _p(exposure), _p(d_exposure), _p(m_exp), _p(v_exp))
    return s_act, a_act


# ------------------------------------------------------------ whole step

def forward_views(prm: Params, cams: Sequence, opts: Opts = Opts()):
    """Render every view; returns a list of (out, tfinal, nlast)."""
    return [render_fwd(prm, c, opts) for c in cams]


def loss_and_grads(prm: Params, cams: Sequence, targets: Sequence, exposure=None,
                   opts: Opts = Opts(), lam_c=1.0, lam_s=0.06, fwd=None):
    """Total loss (Eq. 12 with lambda_smooth = lambda_z = 0, averaged over
    views) and FP64 gradients w.r.t. the activated render parameters and the
    per-view exposure (a, b).  Returns (loss, grads_flat, dexp[V,2], fwd)."""
    V = len(cams)
    exposure = np.zeros((V, 2)) if exposure is None else np.asarray(exposure, np.float64)
    fwd = fwd or forward_views(prm, cams, opts)
    grads = np.zeros((11 + prm.C) * prm.n, np.float64)
    dexp = np.zeros((V, 2), np.float64)
    total = 0.0
    for v, (c, t) in enumerate(zip(cams, targets)):
        out, tf, nl = fwd[v]
        mc = int(t.mask.sum())
        l, G, de = loss(prm.C, out, t.rgb.reshape(3, -1), t.label, t.mask, mc,
                        exposure[v, 0], exposure[v, 1], lam_c, lam_s, 1.0 / V)
        total += l
        dexp[v] = de
        render_bwd(prm, c, G, tf, nl, opts, grads=grads)
    return total, grads, dexp, fwd


# ------------------------------------------------------ grid-side terms

def smooth_loss(z, nbr, lam: float = 1.0):
    """Eq. 10 (K = 4 neighbours from the table nbr[4][n]): (lambda * L, dL/dz)."""
    z = np.ascontiguousarray(z, np.float64)
    nbr = np.ascontiguousarray(nbr, np.int32)
    dz = np.zeros_like(z)
    val = _load().orc_smooth(z.size, _p(z), _p(nbr), float(lam), _p(dz))
    return float(val), dz


def lidar_loss(z, zbar, lam: float = 1.0):
    """Eq. 11: (lambda * L_z, dL/dz)."""
    z = np.ascontiguousarray(z, np.float64)
    zbar = np.ascontiguousarray(zbar, np.float64)
    dz = np.zeros_like(z)
    val = _load().orc_lidar_loss(z.size, _p(z), _p(zbar), float(lam), _p(dz))
    return float(val), dz


def lidar_nn(x, y, px, py) -> np.ndarray:
    """Index of the nearest point in the xy-plane (brute force, ties to the lower index)."""
    c = lambda a: np.ascontiguousarray(a, np.float32)
    x, y, px, py = c(x), c(y), c(px), c(py)
    idx = np.zeros(x.size, np.int32)
    _load().orc_lidar_nn(x.size, _p(x), _p(y), px.size, _p(px), _p(py), _p(idx))
    return idx


def meshgrid_layout(poses, x0: float, y0: float, h: float, W: int, H: int, radius_px: int):
    """Road mask, surfel grid, neighbour table and pose-based initialisation.

    poses: float32 [P, 12] = x, y, z, R row-major.  Returns a dict with mask
    [H, W], idx [H, W], x, y, z (float32), q [4, n] (float64), nbr [4, n]."""
    L = _load()
    poses = np.ascontiguousarray(poses, np.float32)
    P = poses.shape[0]
    pix = np.zeros((P, 2), np.int32)
    L.orc_pose_pixels(P, _p(poses), float(x0), float(y0), float(h), _p(pix))
    mask = np.zeros((H, W), np.uint8)
    n = L.orc_layout_mask(W, H, P, _p(pix), int(radius_px), _p(mask))
    idx = np.zeros((H, W), np.int32)
    x = np.zeros(n, np.float32)
    y = np.zeros(n, np.float32)
    z = np.zeros(n, np.float32)
    q = np.zeros((4, n), np.float64)
    nbr = np.zeros((4, n), np.int32)
    L.orc_layout_build(W, H, _p(mask), float(x0), float(y0), float(h), P, _p(poses), n, _p(idx),
                       _p(x), _p(y), _p(z), _p(q), _p(nbr))
    return dict(mask=mask, idx=idx, x=x, y=y, z=z, q=q, nbr=nbr, pose_pixels=pix)


def row_spans(rec7, rect, q_cut: float, tw: int, th: int, W: int, H: int):
    """Tight per-row tile spans of one binary32 record (u_hi v_hi u_lo v_lo A B
    C) inside its rectangle (x0, x1, y0, y1): arrays lo, hi per row."""
    rec7 = np.ascontiguousarray(rec7, np.float32)
    x0, x1, y0, y1 = (int(t) for t in rect)
    lo = np.zeros(max(y1 - y0, 1), np.int32)
    hi = np.zeros(max(y1 - y0, 1), np.int32)
    _load().orc_row_spans(_p(rec7), x0, x1, y0, y1, float(q_cut), int(tw), int(th), int(W), int(H),
                          _p(lo), _p(hi))
    return lo[:y1 - y0], hi[:y1 - y0]


def q32(rec7, px, py):
    """The binary32 per-pixel test value of records rec7 [n, 7] (u_hi v_hi
    u_lo v_lo A B C) at integer pixels (px, py): array [n, npix]."""
    rec7 = np.ascontiguousarray(np.atleast_2d(rec7)[:, :7], np.float32)
    px = np.ascontiguousarray(px, np.int32).reshape(-1)
    py = np.ascontiguousarray(py, np.int32).reshape(-1)
    q = np.zeros((rec7.shape[0], px.size), np.float32)
    _load().orc_q32(rec7.shape[0], _p(rec7), px.size, _p(px), _p(py), _p(q))
    return q
