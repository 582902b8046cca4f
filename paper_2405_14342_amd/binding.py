"""ctypes binding of librogs (see include/rogs.h).

Argument marshalling only: every step of the splatting path runs inside the
HIP library.  Each method of :class:`Rogs` wraps the C entry point of the same
name (``Rogs.project`` -> ``rogs_project`` ...), takes torch device tensors
for the device pointers and raises :class:`RogsError` on a non-zero status.
The library must have been built (``paper_2405_14342_amd.build``); there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librogs.so")

OK, NOT_READY, EINVAL, ENOMEM, ECAPACITY, EHIP, EREJECT, ESTATE = 0, 1, -1, -2, -3, -4, -5, -6
SYNC_COUNT, ACCUMULATE = 1, 2
PINHOLE, ORTHO = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_READY", -1: "EINVAL", -2: "ENOMEM", -3: "ECAPACITY",
                -4: "EHIP", -5: "EREJECT", -6: "ESTATE"}

EXPORTED = ("rogs_create", "rogs_destroy", "rogs_last_error", "rogs_default_opts",
            "rogs_workspace_size", "rogs_project", "rogs_bin_sort", "rogs_pair_count",
            "rogs_render_fwd", "rogs_loss", "rogs_render_bwd", "rogs_adam_step",
            "rogs_debug_pairs", "rogs_debug_records", "rogs_batch_stats", "rogs_prof_enable",
            "rogs_prof_read", "rogs_prof_name", "rogs_fused_workspace_size", "rogs_step_fused",
            "rogs_fused_status", "rogs_autotune", "rogs_server_create", "rogs_serve_submit",
            "rogs_serve_poll", "rogs_server_stats", "rogs_server_destroy", "rogs_debug_work",
            "rogs_elev_scratch_bytes", "rogs_elev_loss", "rogs_elev_loss_static",
            "rogs_lidar_scratch_bytes", "rogs_lidar_targets",
            "rogs_meshgrid_scratch_bytes", "rogs_meshgrid_layout", "rogs_bev_camera",
            "rogs_bev_workspace_size", "rogs_bev_export")
PROF_GROUPS = 12
FUSED_EAGER = 4


class RogsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p


class Surfels(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_sem", ctypes.c_int32), ("x", _vp), ("y", _vp),
                ("z", _vp), ("q", _vp), ("s", _vp), ("alpha", _vp), ("rgb", _vp), ("sem", _vp)]


class Camera(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32), ("model", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("R_cw", ctypes.c_float * 9),
                ("t_cw", ctypes.c_float * 3), ("z_near", ctypes.c_float),
                ("cull_o", ctypes.c_float * 2), ("cull_ex", ctypes.c_float * 2),
                ("cull_ez", ctypes.c_float * 2), ("cull_lat", ctypes.c_float),
                ("cull_fwd", ctypes.c_float)]


class Request(ctypes.Structure):
    _fields_ = [("cam", Camera), ("channels", ctypes.c_uint32), ("elev_ref", ctypes.c_float),
                ("out", _vp)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_views", ctypes.c_int32),
                ("t_arrive_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


CH_RGB, CH_SEM, CH_D, CH_A, CH_ELEV = 1, 2, 4, 8, 16
CH_ALL = CH_RGB | CH_SEM | CH_D | CH_A | CH_ELEV


def channel_planes(channels: int, C: int) -> int:
    return (3 * bool(channels & CH_RGB) + C * bool(channels & CH_SEM) + bool(channels & CH_D)
            + bool(channels & CH_A) + bool(channels & CH_ELEV))


class RenderOpts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("eps2d", ctypes.c_float),
                ("q_cut", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_eps", ctypes.c_float),
                ("stage", ctypes.c_int32)]


class Targets(ctypes.Structure):
    _fields_ = [("rgb", _vp), ("label", _vp), ("mask", _vp), ("exposure", _vp),
                ("lambda_c", ctypes.c_float), ("lambda_s", ctypes.c_float),
                ("view_scale", ctypes.c_float), ("nbr", _vp), ("zbar", _vp),
                ("lambda_smooth", ctypes.c_float), ("lambda_z", ctypes.c_float)]


class Pose(ctypes.Structure):
    _fields_ = [("x", ctypes.c_float), ("y", ctypes.c_float), ("z", ctypes.c_float),
                ("R", ctypes.c_float * 9)]


class LR(ctypes.Structure):
    _fields_ = [("z", ctypes.c_float), ("q", ctypes.c_float), ("s", ctypes.c_float),
                ("alpha", ctypes.c_float), ("rgb", ctypes.c_float), ("sem", ctypes.c_float),
                ("exposure", ctypes.c_float)]


class TrainStateC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_sem", ctypes.c_int32), ("x", _vp), ("y", _vp),
                ("params", _vp), ("m", _vp), ("v", _vp), ("s_act", _vp), ("alpha_act", _vp),
                ("exposure", _vp), ("m_exp", _vp), ("v_exp", _vp), ("d_exposure", _vp),
                ("grads", _vp), ("step_state", _vp)]


class Optim(ctypes.Structure):
    _fields_ = [("lr", LR), ("z_start", ctypes.c_float), ("z_end", ctypes.c_float),
                ("total_steps", ctypes.c_int64), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class TuneStep(ctypes.Structure):
    _fields_ = [("state", ctypes.POINTER(TrainStateC)), ("targets", ctypes.POINTER(Targets)),
                ("optim", ctypes.POINTER(Optim))]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librogs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"librogs.so not found at {path}: run paper_2405_14342_amd/build.py")
        L = ctypes.CDLL(path)
        P, I32, I64, U32, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
        sig = {
            "rogs_create": ([ctypes.POINTER(P)], I32),
            "rogs_destroy": ([P], None),
            "rogs_last_error": ([P], ctypes.c_char_p),
            "rogs_default_opts": ([ctypes.POINTER(RenderOpts)], None),
            "rogs_workspace_size": ([ctypes.POINTER(Surfels), ctypes.POINTER(Camera), I32,
                                     ctypes.POINTER(RenderOpts), I64, I64,
                                     ctypes.POINTER(ctypes.c_size_t)], I32),
            "rogs_project": ([P, ctypes.POINTER(Surfels), ctypes.POINTER(Camera), I32,
                              ctypes.POINTER(RenderOpts), P, ctypes.c_size_t, I64, I64, P], I32),
            "rogs_bin_sort": ([P, P, ctypes.POINTER(I64), U32, P], I32),
            "rogs_pair_count": ([P, P, ctypes.POINTER(I64), ctypes.POINTER(I32), P], I32),
            "rogs_render_fwd": ([P, ctypes.POINTER(Surfels), P, P, ctypes.c_uint32, P], I32),
            "rogs_loss": ([P, P, P, ctypes.POINTER(Targets), P, P, P, P], I32),
            "rogs_render_bwd": ([P, ctypes.POINTER(Surfels), P, P, P, P, U32, P], I32),
            "rogs_adam_step": ([P, I32, I32, P, P, P, P, P, P, ctypes.POINTER(Optim), I64,
                                P, P, P, P, I32, P], I32),
            "rogs_debug_pairs": ([P, P, P, P, P, I64, P, I64, P], I32),
            "rogs_debug_records": ([P, P, P, P, P, P], I32),
            "rogs_batch_stats": ([P, P, P, P], I32),
            "rogs_prof_enable": ([P, I32], I32),
            "rogs_prof_read": ([P, P, P, I32], I32),
            "rogs_prof_name": ([I32], ctypes.c_char_p),
            "rogs_fused_workspace_size": ([ctypes.POINTER(TrainStateC), ctypes.POINTER(Camera), I32,
                                           ctypes.POINTER(RenderOpts), I64, I64,
                                           ctypes.POINTER(ctypes.c_size_t)], I32),
            "rogs_step_fused": ([P, ctypes.POINTER(TrainStateC), ctypes.POINTER(Camera), I32,
                                 ctypes.POINTER(RenderOpts), ctypes.POINTER(Targets),
                                 ctypes.POINTER(Optim), P, ctypes.c_size_t, I64, I64, U32, P], I32),
            "rogs_fused_status": ([P, P, P], I32),
            "rogs_server_create": ([ctypes.POINTER(P), ctypes.POINTER(Surfels),
                                    ctypes.POINTER(RenderOpts), P, ctypes.c_size_t, I32, I32, I32],
                                   I32),
            "rogs_serve_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)],
                                  I32),
            "rogs_serve_poll": ([P, ctypes.c_uint64, ctypes.POINTER(Result)], I32),
            "rogs_server_stats": ([P, P], I32),
            "rogs_debug_work": ([P, P, ctypes.POINTER(I64), ctypes.POINTER(I64), P], I32),
            "rogs_bev_camera": ([ctypes.c_double, ctypes.c_double, I32, I32, F, I32, I32, I32, I32,
                                 F, ctypes.POINTER(Camera)], None),
            "rogs_bev_workspace_size": ([ctypes.POINTER(Surfels), I32, ctypes.POINTER(RenderOpts),
                                         I64, ctypes.POINTER(ctypes.c_size_t)], I32),
            "rogs_bev_export": ([P, ctypes.POINTER(Surfels), ctypes.POINTER(RenderOpts),
                                 ctypes.c_double, ctypes.c_double, I32, I32, F, I32, F, U32, P, P,
                                 ctypes.c_size_t, I64, ctypes.POINTER(I64), P], I32),
            "rogs_elev_scratch_bytes": ([I32], ctypes.c_size_t),
            "rogs_elev_loss": ([P, I32, P, P, F, P, F, P, P, P, ctypes.c_size_t, P], I32),
            "rogs_elev_loss_static": ([P, I32, P, P, F, P, F, P, P, P], I32),
            "rogs_lidar_scratch_bytes": ([I32, I32], ctypes.c_size_t),
            "rogs_lidar_targets": ([P, I32, P, P, I32, P, P, P, P, P, P, ctypes.c_size_t, P], I32),
            "rogs_meshgrid_scratch_bytes": ([I32, I32, I32], ctypes.c_size_t),
            "rogs_meshgrid_layout": ([P, P, I32, ctypes.c_double, ctypes.c_double, F, I32, I32, I32,
                                      P, I64, P, P, P, P, P, ctypes.POINTER(I64), P,
                                      ctypes.c_size_t, P], I32),
            "rogs_server_destroy": ([P], None),
            "rogs_autotune": ([P, ctypes.POINTER(Surfels), ctypes.POINTER(Camera), I32,
                               ctypes.POINTER(RenderOpts), ctypes.POINTER(I32),
                               ctypes.POINTER(TuneStep), ctypes.c_char_p, I32,
                               ctypes.POINTER(ctypes.c_float), P], I32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def ptr(t) -> Optional[int]:
    """Device (or host) address of a tensor / array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def make_camera(cam) -> Camera:
    """rogs_camera from a camera description with the fields of synth.Camera."""
    c = Camera()
    c.w, c.h, c.model = int(cam.w), int(cam.h), int(cam.model)
    c.tile = int(getattr(cam, "tile", 0))
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R_cw, np.float32).reshape(9)
    t = np.asarray(cam.t_cw, np.float32).reshape(3)
    for k in range(9):
        c.R_cw[k] = float(R[k])
    for k in range(3):
        c.t_cw[k] = float(t[k])
    c.z_near = float(cam.z_near)
    for k in range(2):
        c.cull_o[k] = float(cam.cull_o[k])
        c.cull_ex[k] = float(cam.cull_ex[k])
        c.cull_ez[k] = float(cam.cull_ez[k])
    c.cull_lat, c.cull_fwd = float(cam.cull_lat), float(cam.cull_fwd)
    return c


def camera_array(cams: Sequence) -> ctypes.Array:
    arr = (Camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = c if isinstance(c, Camera) else make_camera(c)
    return arr


def default_opts() -> RenderOpts:
    o = RenderOpts()
    load_library().rogs_default_opts(ctypes.byref(o))
    return o


def make_opts(tile_w=16, tile_h=16, eps2d=0.3, q_cut=9.0, alpha_max=0.99, t_eps=1e-6,
              stage=32) -> RenderOpts:
    return RenderOpts(tile_w, tile_h, eps2d, q_cut, alpha_max, t_eps, stage)


def tile_code(tile_w: int, tile_h: int) -> int:
    """rogs_camera.tile value giving a view its own tile shape."""
    return int(tile_w) | int(tile_h) << 16


def fused_workspace_size(ts: TrainStateC, cams, opts: RenderOpts, pair_capacity: int,
                         slot_capacity: int = 0) -> int:
    """rogs_fused_workspace_size (host-only)."""
    L = load_library()
    arr = camera_array(cams)
    out = ctypes.c_size_t(0)
    r = L.rogs_fused_workspace_size(ctypes.byref(ts), arr, len(cams), ctypes.byref(opts),
                                    int(pair_capacity), int(slot_capacity), ctypes.byref(out))
    if r != OK:
        raise RogsError(r, "rogs_fused_workspace_size rejected its arguments")
    return int(out.value)


def bev_camera(x0, y0, W, H, m_per_px, ox, oy, cw, ch, height) -> Camera:
    cam = Camera()
    load_library().rogs_bev_camera(float(x0), float(y0), int(W), int(H), float(m_per_px), int(ox),
                                   int(oy), int(cw), int(ch), float(height), ctypes.byref(cam))
    return cam


def elev_scratch_bytes(n: int) -> int:
    return int(load_library().rogs_elev_scratch_bytes(int(n)))


def lidar_scratch_bytes(n: int, m: int) -> int:
    return int(load_library().rogs_lidar_scratch_bytes(int(n), int(m)))


def workspace_size(surf: Surfels, cams, opts: RenderOpts, pair_capacity: int,
                   slot_capacity: int = 0) -> int:
    """rogs_workspace_size (host-only)."""
    L = load_library()
    arr = camera_array(cams)
    out = ctypes.c_size_t(0)
    r = L.rogs_workspace_size(ctypes.byref(surf), arr, len(cams), ctypes.byref(opts),
                              int(pair_capacity), int(slot_capacity), ctypes.byref(out))
    if r != OK:
        raise RogsError(r, "rogs_workspace_size rejected its arguments")
    return int(out.value)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream


class Rogs:
    """One librogs context (rogs_create / rogs_destroy)."""

    def __init__(self):
        self.L = load_library()
        h = ctypes.c_void_p()
        r = self.L.rogs_create(ctypes.byref(h))
        if r != OK:
            raise RogsError(r, "rogs_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.rogs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, r: int, what: str):
        if r != OK:
            msg = self.L.rogs_last_error(self.h)
            raise RogsError(r, f"{what}: {msg.decode() if msg else ''}")

    def last_error(self) -> str:
        m = self.L.rogs_last_error(self.h)
        return m.decode() if m else ""

    # --- entry points -------------------------------------------------
    def project(self, surf: Surfels, cams, opts: RenderOpts, ws, pair_capacity: int,
                slot_capacity: int = 0, stream=None):
        arr = camera_array(cams)
        self._check(self.L.rogs_project(self.h, ctypes.byref(surf), arr, len(cams), ctypes.byref(opts),
                                        ptr(ws), ws.numel() * ws.element_size(), int(pair_capacity),
                                        int(slot_capacity), _stream(stream)), "rogs_project")

    def bin_sort(self, ws, flags: int = SYNC_COUNT, stream=None, raise_on_capacity=True) -> int:
        n = ctypes.c_int64(-1)
        r = self.L.rogs_bin_sort(self.h, ptr(ws), ctypes.byref(n), flags, _stream(stream))
        if r == ECAPACITY and not raise_on_capacity:
            return -int(n.value) - 1
        self._check(r, "rogs_bin_sort")
        return int(n.value)

    def pair_count(self, ws, stream=None):
        n, o = ctypes.c_int64(0), ctypes.c_int32(0)
        self._check(self.L.rogs_pair_count(self.h, ptr(ws), ctypes.byref(n), ctypes.byref(o),
                                           _stream(stream)), "rogs_pair_count")
        return int(n.value), int(o.value)

    def render_fwd(self, surf: Surfels, ws, out, stream=None, channels: int = None):
        """rogs_render_fwd; channels: OR of CH_* (default: every plane)."""
        ch = CH_ALL if channels is None else int(channels)
        self._check(self.L.rogs_render_fwd(self.h, ctypes.byref(surf), ptr(ws), ptr(out), ch,
                                           _stream(stream)), "rogs_render_fwd")

    def loss(self, ws, out, targets: Targets, dL_dout, loss_out, d_exposure, stream=None):
        self._check(self.L.rogs_loss(self.h, ptr(ws), ptr(out), ctypes.byref(targets), ptr(dL_dout),
                                     ptr(loss_out), ptr(d_exposure), _stream(stream)), "rogs_loss")

    def render_bwd(self, surf: Surfels, ws, out, dL_dout, grads, flags: int = 0, stream=None):
        self._check(self.L.rogs_render_bwd(self.h, ctypes.byref(surf), ptr(ws), ptr(out),
                                           ptr(dL_dout), ptr(grads), flags, _stream(stream)),
                    "rogs_render_bwd")

    def adam_step(self, n, n_sem, params, grads, m, v, s_act, alpha_act, optim: "Optim", step,
                  exposure=None, d_exposure=None, m_exp=None, v_exp=None, n_views=0, stream=None):
        self._check(self.L.rogs_adam_step(self.h, int(n), int(n_sem), ptr(params), ptr(grads), ptr(m),
                                          ptr(v), ptr(s_act), ptr(alpha_act), ctypes.byref(optim),
                                          int(step), ptr(exposure), ptr(d_exposure), ptr(m_exp),
                                          ptr(v_exp), int(n_views), _stream(stream)),
                    "rogs_adam_step")

    def batch_stats(self, ws, stream=None) -> dict:
        st = np.zeros(6, np.int64)
        self._check(self.L.rogs_batch_stats(self.h, ptr(ws), st.ctypes.data, _stream(stream)),
                    "rogs_batch_stats")
        return dict(pairs=int(st[0]), overflow=int(st[1]), visible=int(st[2]), pixels=int(st[3]),
                    tiles=int(st[4]), slots=int(st[5]))

    def prof_enable(self, on: bool = True):
        self._check(self.L.rogs_prof_enable(self.h, 1 if on else 0), "rogs_prof_enable")

    def prof_read(self) -> dict:
        ms = np.zeros(PROF_GROUPS, np.float64)
        n = np.zeros(PROF_GROUPS, np.int64)
        self._check(self.L.rogs_prof_read(self.h, ms.ctypes.data, n.ctypes.data, PROF_GROUPS),
                    "rogs_prof_read")
        return {self.L.rogs_prof_name(k).decode(): (float(ms[k]), int(n[k]))
                for k in range(PROF_GROUPS)}

    def step_fused(self, ts: "TrainStateC", cams, opts: RenderOpts, targets: Targets,
                   optim: Optim, ws, pair_capacity: int, flags: int = 0, stream=None,
                   raise_on_capacity=True, slot_capacity: int = 0) -> int:
        arr = cams if isinstance(cams, ctypes.Array) else camera_array(cams)
        r = self.L.rogs_step_fused(self.h, ctypes.byref(ts), arr, len(arr), ctypes.byref(opts),
                                   ctypes.byref(targets), ctypes.byref(optim), ptr(ws),
                                   ws.numel() * ws.element_size(), int(pair_capacity),
                                   int(slot_capacity), flags, _stream(stream))
        if r == ECAPACITY and not raise_on_capacity:
            return r
        self._check(r, "rogs_step_fused")
        return r

    def autotune(self, surf: Surfels, cams, opts: Optional[RenderOpts] = None,
                 cache_json: Optional[str] = None, reps: int = 3, stream=None, step=None):
        """rogs_autotune: returns (opts with the chosen tile shape and staging
        depth, ms per run, the rogs_camera.tile code of every view).  step:
        None times the render passes; (TrainStateC, Targets, Optim) times
        fused training steps on copies of that state."""
        o = RenderOpts.from_buffer_copy(opts if opts is not None else default_opts())
        arr = camera_array(cams)
        ms = ctypes.c_float(0.0)
        tiles = (ctypes.c_int32 * len(arr))()
        path = cache_json.encode() if cache_json else None
        ts = None
        if step is not None:
            ts = TuneStep(ctypes.pointer(step[0]), ctypes.pointer(step[1]),
                          ctypes.pointer(step[2]))
        self._check(self.L.rogs_autotune(self.h, ctypes.byref(surf), arr, len(arr), ctypes.byref(o),
                                         tiles, ctypes.byref(ts) if ts is not None else None,
                                         path, int(reps), ctypes.byref(ms), _stream(stream)),
                    "rogs_autotune")
        return o, float(ms.value), [int(t) for t in tiles]

    def elev_loss(self, n, z, nbr, lambda_smooth, zbar, lambda_z, dz, loss_out, scratch,
                  stream=None):
        """rogs_elev_loss: adds Eq. 10 / 11 terms into dz and loss_out."""
        self._check(self.L.rogs_elev_loss(self.h, int(n), ptr(z), ptr(nbr), float(lambda_smooth),
                                          ptr(zbar), float(lambda_z), ptr(dz), ptr(loss_out),
                                          ptr(scratch), scratch.numel() * scratch.element_size(),
                                          _stream(stream)), "rogs_elev_loss")

    def elev_loss_static(self, n, z, nbr, lambda_smooth, zbar, lambda_z, dz, loss_out,
                         stream=None, check=True):
        """rogs_elev_loss_static: rogs_elev_loss with the library's fixed
        partial-sum array (allocates nothing).  Returns the status when check
        is False."""
        r = self.L.rogs_elev_loss_static(self.h, int(n), ptr(z), ptr(nbr), float(lambda_smooth),
                                         ptr(zbar), float(lambda_z), ptr(dz), ptr(loss_out),
                                         _stream(stream))
        if check:
            self._check(r, "rogs_elev_loss_static")
        return r

    def lidar_targets(self, x, y, px, py, pz, zbar, idx=None, stream=None, scratch=None):
        """rogs_lidar_targets: zbar (and idx) of the nearest point in xy.
        scratch: a uint8 device tensor of rogs_lidar_scratch_bytes bytes
        (allocated from PyTorch when None)."""
        import torch
        need = int(self.L.rogs_lidar_scratch_bytes(x.numel(), px.numel()))
        if scratch is None:
            scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
        self._check(self.L.rogs_lidar_targets(self.h, x.numel(), ptr(x), ptr(y), px.numel(), ptr(px),
                                              ptr(py), ptr(pz), ptr(zbar), ptr(idx),
                                              ptr(scratch), scratch.numel(), _stream(stream)),
                    "rogs_lidar_targets")

    def meshgrid_layout(self, poses, x0, y0, spacing, W, H, radius_px, stream=None):
        """rogs_meshgrid_layout on device poses (uint8 view of rogs_pose
        records or a float32 [P, 12] tensor): returns a dict of device
        tensors idx [H, W], x, y, z, q [4, n], nbr [4, n]."""
        import torch
        n_poses = poses.numel() * poses.element_size() // ctypes.sizeof(Pose)
        dev = poses.device
        scratch = torch.empty(self.L.rogs_meshgrid_scratch_bytes(W, H, n_poses), dtype=torch.uint8,
                              device=dev)
        n = ctypes.c_int64(0)
        args = (float(x0), float(y0), float(spacing), int(W), int(H), int(radius_px))
        self._check(self.L.rogs_meshgrid_layout(self.h, ptr(poses), n_poses, *args, None, 0, None, None,
                                                None, None, None, ctypes.byref(n), ptr(scratch),
                                                scratch.numel(), _stream(stream)),
                    "rogs_meshgrid_layout")
        N = int(n.value)
        idx = torch.empty((H, W), dtype=torch.int32, device=dev)
        x = torch.empty(N, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        q = torch.empty((4, N), dtype=torch.float32, device=dev)
        nbr = torch.empty((4, N), dtype=torch.int32, device=dev)
        self._check(self.L.rogs_meshgrid_layout(self.h, ptr(poses), n_poses, *args, ptr(idx), N,
                                                ptr(x), ptr(y), ptr(z), ptr(q), ptr(nbr),
                                                ctypes.byref(n), ptr(scratch), scratch.numel(),
                                                _stream(stream)), "rogs_meshgrid_layout")
        return dict(idx=idx, x=x, y=y, z=z, q=q, nbr=nbr, n=N)

    def bev_export(self, surf: Surfels, opts: Optional[RenderOpts], x0, y0, W, H, m_per_px,
                   chunk_px, height, channels, out, pair_capacity=1 << 22, stream=None):
        """rogs_bev_export into `out` (planes x H x W); grows the pair capacity
        and retries if a chunk overflows.  Returns the largest chunk pair count."""
        import torch
        o = opts if opts is not None else default_opts()
        cap = int(pair_capacity)
        while True:
            size = ctypes.c_size_t(0)
            self._check(self.L.rogs_bev_workspace_size(ctypes.byref(surf), int(chunk_px),
                                                       ctypes.byref(o), cap, ctypes.byref(size)),
                        "rogs_bev_workspace_size")
            ws = torch.empty(size.value, dtype=torch.uint8, device=out.device)
            worst = ctypes.c_int64(0)
            r = self.L.rogs_bev_export(self.h, ctypes.byref(surf), ctypes.byref(o), float(x0),
                                       float(y0), int(W), int(H), float(m_per_px), int(chunk_px),
                                       float(height), int(channels), ptr(out), ptr(ws), size.value,
                                       cap, ctypes.byref(worst), _stream(stream))
            if r == ECAPACITY:
                cap = int(worst.value * 1.25) + 4096
                continue
            self._check(r, "rogs_bev_export")
            return int(worst.value)

    def debug_work(self, ws, stream=None):
        """(evaluated, contributing) list entries over all pixels of the batch."""
        e, k = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(self.L.rogs_debug_work(self.h, ptr(ws), ctypes.byref(e), ctypes.byref(k),
                                           _stream(stream)), "rogs_debug_work")
        return int(e.value), int(k.value)

    def fused_status(self) -> dict:
        st = np.zeros(8, np.int64)
        loss = ctypes.c_float(0.0)
        self._check(self.L.rogs_fused_status(self.h, st.ctypes.data, ctypes.byref(loss)),
                    "rogs_fused_status")
        return dict(pairs=int(st[0]), overflow=int(st[1]), visible=int(st[2]), step=int(st[3]),
                    skipped=int(st[4]), pixels=int(st[5]), tiles=int(st[6]), slots=int(st[7]),
                    loss=float(loss.value))

    def debug_pairs(self, ws, cap: int, n_tiles: int, stream=None):
        keys = np.zeros(max(cap, 1), np.uint64)
        ids = np.zeros(max(cap, 1), np.int32)
        views = np.zeros(max(cap, 1), np.int32)
        ranges = np.zeros((max(n_tiles, 1), 2), np.uint32)
        self._check(self.L.rogs_debug_pairs(self.h, ptr(ws), keys.ctypes.data, ids.ctypes.data,
                                            views.ctypes.data, int(cap), ranges.ctypes.data,
                                            int(n_tiles), _stream(stream)), "rogs_debug_pairs")
        return keys, ids, views, ranges

    def debug_records(self, ws, n_views: int, n: int, stream=None):
        rec = np.zeros((n_views, n, 8), np.float32)
        rect = np.zeros((n_views, n, 4), np.int32)
        cnt = np.zeros((n_views, n), np.uint32)
        self._check(self.L.rogs_debug_records(self.h, ptr(ws), rec.ctypes.data, rect.ctypes.data,
                                              cnt.ctypes.data, _stream(stream)), "rogs_debug_records")
        return rec, rect, cnt


class Server:
    """Continuous-batching render server (rogs_server_*) over a resident map.

    ``keep`` holds the tensors behind the map's pointers and the arena so they
    outlive the server."""

    def __init__(self, surf: Surfels, opts: Optional[RenderOpts], arena, max_views: int = 16,
                 lanes: int = 2, device: int = 0, keep=()):
        self.L = load_library()
        self.h = ctypes.c_void_p()
        self._keep = (surf, arena, tuple(keep))
        self.C = int(surf.n_sem)
        o = opts if opts is not None else default_opts()
        r = self.L.rogs_server_create(ctypes.byref(self.h), ctypes.byref(surf), ctypes.byref(o),
                                      ptr(arena), arena.numel() * arena.element_size(),
                                      int(max_views), int(lanes), int(device))
        if r != OK:
            raise RogsError(r, "rogs_server_create")

    def submit(self, cam, channels: int, out, elev_ref: float = 0.0,
               raise_on_reject: bool = True) -> int:
        req = Request(cam if isinstance(cam, Camera) else make_camera(cam), int(channels),
                      float(elev_ref), ptr(out))
        t = ctypes.c_uint64(0)
        r = self.L.rogs_serve_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if r != OK:
            if not raise_on_reject and r == EREJECT:
                return 0
            raise RogsError(r, "rogs_serve_submit")
        return int(t.value)

    def poll(self, ticket: int) -> Optional[dict]:
        """None while pending; the result dict once done (the ticket is released)."""
        res = Result()
        r = self.L.rogs_serve_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(res))
        if r == NOT_READY:
            return None
        if r != OK:
            raise RogsError(r, "rogs_serve_poll")
        return dict(status=res.status, batch_views=res.batch_views, t_arrive_ns=res.t_arrive_ns,
                    t_start_ns=res.t_start_ns, t_done_ns=res.t_done_ns)

    def wait(self, ticket: int, sleep_s: float = 0.0002) -> dict:
        import time
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            time.sleep(sleep_s)

    def stats(self) -> dict:
        st = np.zeros(7, np.int64)
        self.L.rogs_server_stats(self.h, st.ctypes.data)
        return dict(batches=int(st[0]), views=int(st[1]), splits=int(st[2]),
                    max_batch=int(st[3]), capacity_failures=int(st[4]), queued=int(st[5]),
                    max_in_flight=int(st[6]))

    def close(self):
        if self.h:
            self.L.rogs_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
