"""Device-resident training state and the per-step call sequences.

PyTorch provides device memory and the stream; every step of the path runs in
librogs through :mod:`binding`.  Two sequences are provided:

* :meth:`TrainState.step_plain` - one launch sequence per view (project,
  bin/sort with a host read-back of the pair count, forward, loss, backward),
  then one Adam step: the plain per-view path.
* :meth:`TrainState.step_batched` - all views of the step in one batch, the
  pair count kept on the device.
* :meth:`TrainState.step_fused` - the batched step with the loss fused into
  the forward and Adam into the projection adjoint, captured once as a
  hipGraph and replayed.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B

# Sec. 4.2 hyper-parameters
LAMBDA_C, LAMBDA_S = 1.0, 0.06
LAMBDA_SMOOTH, LAMBDA_Z = 0.003, 0.02   # Eq. 12 (lambda_smooth = 1 when LiDAR supervises z)
LR_ALPHA = LR_SCALE = LR_ROT = 1e-4
LR_RGB, LR_SEM, LR_EXPOSURE = 0.008, 0.1, 0.001
LR_Z_START, LR_Z_END = 1.6e-4, 1.6e-6      # times the scene size


def paper_optim(extent: float, total_steps: int) -> B.Optim:
    """Optimizer settings of Sec. 4.2: the per-group rates, and the height
    rate proportional to the scene size, from 1.6e-4 to 1.6e-6 of it over
    ``total_steps`` steps (the library evaluates the schedule per step)."""
    z0 = float(np.float32(extent * LR_Z_START))
    z1 = float(np.float32(extent * LR_Z_END))
    lr = B.LR(z0, LR_ROT, LR_SCALE, LR_ALPHA, LR_RGB, LR_SEM, LR_EXPOSURE)
    return B.Optim(lr, z0, z1, int(total_steps), 0.9, 0.999, 1e-8)


def n_out(C: int) -> int:
    return 5 + C


class TrainState:
    """Surfel parameters, Adam moments, targets and output buffers on the GPU."""

    def __init__(self, scene, device="cuda", opts=None, pair_capacity: Optional[int] = None,
                 autotune_cache: Optional[str] = None, autotune_for: str = "step"):
        """opts: RenderOpts, None (defaults) or "auto" (rogs_autotune picks the
        tile shape, the staging depth and a tile shape per resolution class for
        these surfels and views, optionally through a JSON cache file; the
        per-view shapes go into the cameras' tile codes).  autotune_for:
        "step" times the fused training step (on copies of this state; scenes
        without targets fall back to "render"), "render" the render passes."""
        self.scene = scene
        self.dev = torch.device(device)
        N, C = scene.n, scene.n_sem
        self.N, self.C, self.K = N, C, 11 + C
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=self.dev)
        P = torch.empty((self.K, N), dtype=torch.float32, device=self.dev)
        P[0] = f(scene.z)
        P[1:5] = f(scene.q)
        P[5:7] = f(scene.log_s)
        P[7] = f(scene.logit_a)
        P[8:11] = f(scene.rgb)
        P[11:] = f(scene.sem)
        self.params = P
        self.s_act = f(scene.s).clone()
        self.alpha_act = f(scene.alpha).clone()
        self.x = f(scene.x)
        self.y = f(scene.y)
        self.m = torch.zeros_like(P)
        self.v = torch.zeros_like(P)
        self.grads = torch.zeros_like(P)
        self.cams = list(scene.cams)
        V = len(self.cams)
        self.V = V
        self.npix = [c.w * c.h for c in self.cams]
        self.pix_off = np.concatenate([[0], np.cumsum(self.npix)]).astype(np.int64)
        self.total_pix = int(self.pix_off[-1])
        self.exposure = torch.zeros((V, 2), dtype=torch.float32, device=self.dev)
        self.d_exp = torch.zeros_like(self.exposure)
        self.m_exp = torch.zeros_like(self.exposure)
        self.v_exp = torch.zeros_like(self.exposure)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        NO = n_out(C)
        self.out = torch.zeros(NO * self.total_pix, dtype=torch.float32, device=self.dev)
        self.G = torch.zeros_like(self.out)
        if scene.targets:
            self.tgt_rgb = torch.cat([f(t.rgb).reshape(-1) for t in scene.targets])
            self.tgt_label = torch.cat([torch.as_tensor(t.label.reshape(-1), device=self.dev)
                                        for t in scene.targets])
            self.tgt_mask = torch.cat([torch.as_tensor(t.mask.reshape(-1), device=self.dev)
                                       for t in scene.targets])
        else:
            self.tgt_rgb = self.tgt_label = self.tgt_mask = None
        self.rg = B.Rogs()
        auto = isinstance(opts, str)
        if auto and opts != "auto":
            raise ValueError("opts must be RenderOpts, None or 'auto'")
        if autotune_for not in ("step", "render"):
            raise ValueError("autotune_for must be 'step' or 'render'")
        self.opts = B.make_opts() if auto or opts is None else opts
        self.cap_view = pair_capacity or 1 << 20
        self.cap_batch = pair_capacity or 1 << 22
        self.cap_fused = self.cap_batch
        self.scap_fused = 0          # visible-slot capacity; 0 = the pair capacity
        self._ws_view = None
        self._ws_batch = None
        self.step_count = 0
        self.nbr = self.zbar = None
        self.lambda_smooth = self.lambda_z = 0.0
        if auto:
            step = None
            if autotune_for == "step" and self.tgt_rgb is not None:
                step = (self.train_state(), self.targets(0, self.V),
                        paper_optim(self.scene.extent, 1000))
            self.opts, self.autotune_ms, tiles = self.rg.autotune(
                self.surfels(), self.cams, self.opts, cache_json=autotune_cache, step=step)
            self.cams = [dataclasses.replace(c, tile=t) for c, t in zip(self.cams, tiles)]

    # -------------------------------------------------------------- views
    def surfels(self) -> B.Surfels:
        P = self.params
        return B.Surfels(self.N, self.C, self.x.data_ptr(), self.y.data_ptr(), P[0].data_ptr(),
                         P[1].data_ptr(), self.s_act.data_ptr(), self.alpha_act.data_ptr(),
                         P[8].data_ptr(), P[11].data_ptr())

    def out_view(self, v: int, buf=None) -> torch.Tensor:
        buf = self.out if buf is None else buf
        NO = n_out(self.C)
        return buf[NO * int(self.pix_off[v]): NO * int(self.pix_off[v + 1])]

    def image(self, v: int, buf=None) -> torch.Tensor:
        """[5 + C, H, W] view of the rendered (or gradient) image of view v."""
        c = self.cams[v]
        return self.out_view(v, buf).view(n_out(self.C), c.h, c.w)

    def targets(self, v0: int, v1: int) -> B.Targets:
        o = int(self.pix_off[v0])
        return B.Targets(self.tgt_rgb.data_ptr() + 4 * 3 * o, self.tgt_label.data_ptr() + o,
                         self.tgt_mask.data_ptr() + o, self.exposure.data_ptr() + 8 * v0,
                         LAMBDA_C, LAMBDA_S, 1.0 / self.V, B.ptr(self.nbr), B.ptr(self.zbar),
                         self.lambda_smooth, self.lambda_z)

    # ------------------------------------------------------ grid-side terms
    def set_grid_terms(self, nbr=None, zbar=None, lambda_smooth: float = LAMBDA_SMOOTH,
                       lambda_z: float = LAMBDA_Z):
        """Enables the elevation smoothness (Eq. 10, neighbour table nbr[4][N])
        and/or the LiDAR elevation loss (Eq. 11, targets zbar[N]) in every
        training step (plain, batched and fused)."""
        dev = self.dev
        self.nbr = None if nbr is None else torch.as_tensor(np.ascontiguousarray(nbr, np.int32),
                                                            device=dev)
        self.zbar = None if zbar is None else torch.as_tensor(
            np.ascontiguousarray(zbar, np.float32), device=dev) if not torch.is_tensor(zbar) \
            else zbar.to(dev, torch.float32).contiguous()
        self.lambda_smooth = float(lambda_smooth) if nbr is not None else 0.0
        self.lambda_z = float(lambda_z) if zbar is not None else 0.0
        self._reg_scratch = torch.empty(max(4, B.elev_scratch_bytes(self.N)), dtype=torch.uint8,
                                        device=dev)

    def lidar_targets(self, points) -> torch.Tensor:
        """zbar[N]: height of the LiDAR point nearest to each surfel in the
        xy-plane (rogs_lidar_targets); points: float32 [3, M]."""
        pts = torch.as_tensor(np.ascontiguousarray(points, np.float32), device=self.dev)
        zbar = torch.empty(self.N, dtype=torch.float32, device=self.dev)
        self.rg.lidar_targets(self.x, self.y, pts[0], pts[1], pts[2], zbar)
        return zbar

    def _grid_terms(self):
        if self.nbr is None and self.zbar is None:
            return
        self.rg.elev_loss(self.N, self.params[0], self.nbr, self.lambda_smooth, self.zbar,
                          self.lambda_z, self.grads[0], self.loss, self._reg_scratch)

    # ---------------------------------------------------------- workspace
    def _workspace(self, cams, cap, which, scap=0):
        size = B.workspace_size(self.surfels(), cams, self.opts, cap, scap)
        cur = getattr(self, which)
        if cur is None or cur.numel() < size:
            cur = torch.empty(size, dtype=torch.uint8, device=self.dev)
            setattr(self, which, cur)
        return cur

    def project_and_sort(self, cams, cap_attr: str, ws_attr: str, sync: bool = True):
        """rogs_project + rogs_bin_sort, growing the pair capacity if needed."""
        while True:
            cap = getattr(self, cap_attr)
            ws = self._workspace(cams, cap, ws_attr)
            self.rg.project(self.surfels(), cams, self.opts, ws, cap)
            if not sync:
                self.rg.bin_sort(ws, 0)
                return ws, -1
            n = self.rg.bin_sort(ws, B.SYNC_COUNT, raise_on_capacity=False)
            if n >= 0:
                return ws, n
            st = self.rg.batch_stats(ws)
            setattr(self, cap_attr, int(max(st["pairs"], st["visible"]) * 1.25) + 4096)

    # -------------------------------------------------------------- steps
    def forward_view(self, v: int):
        ws, n = self.project_and_sort([self.cams[v]], "cap_view", "_ws_view")
        self.rg.render_fwd(self.surfels(), ws, self.out_view(v))
        return ws, n

    def step_plain(self, optim: Optional[B.Optim] = None, total_steps: int = 1,
                   adam: bool = True):
        """One training step, one launch sequence per view (the plain path)."""
        self.step_count += 1
        optim = optim or paper_optim(self.scene.extent, total_steps)
        self.loss.zero_()
        self.d_exp.zero_()
        surf = self.surfels()
        for v in range(self.V):
            ws, _ = self.forward_view(v)
            ov, gv = self.out_view(v), self.out_view(v, self.G)
            self.rg.loss(ws, ov, self.targets(v, v + 1), gv, self.loss, self.d_exp[v])
            self.rg.render_bwd(surf, ws, ov, gv, self.grads, B.ACCUMULATE if v else 0)
        self._grid_terms()
        if adam:
            self.adam(optim)

    def step_batched(self, optim: Optional[B.Optim] = None, total_steps: int = 1,
                     adam: bool = True, sync: bool = True):
        """One training step with every view in one batch."""
        self.step_count += 1
        optim = optim or paper_optim(self.scene.extent, total_steps)
        self.loss.zero_()
        self.d_exp.zero_()
        surf = self.surfels()
        ws, _ = self.project_and_sort(self.cams, "cap_batch", "_ws_batch", sync=sync)
        self.rg.render_fwd(surf, ws, self.out)
        self.rg.loss(ws, self.out, self.targets(0, self.V), self.G, self.loss, self.d_exp)
        self.rg.render_bwd(surf, ws, self.out, self.G, self.grads, 0)
        self._grid_terms()
        if adam:
            self.adam(optim)

    def adam(self, optim: B.Optim):
        self.rg.adam_step(self.N, self.C, self.params, self.grads, self.m, self.v, self.s_act,
                          self.alpha_act, optim, self.step_count, exposure=self.exposure,
                          d_exposure=self.d_exp, m_exp=self.m_exp, v_exp=self.v_exp,
                          n_views=self.V)

    # ------------------------------------------------------------ fused
    def train_state(self, grads_out: bool = False) -> B.TrainStateC:
        if not hasattr(self, "step_state"):
            self.step_state = torch.zeros(16, dtype=torch.int32, device=self.dev)
        P = self.params
        return B.TrainStateC(self.N, self.C, self.x.data_ptr(), self.y.data_ptr(), P.data_ptr(),
                             self.m.data_ptr(), self.v.data_ptr(), self.s_act.data_ptr(),
                             self.alpha_act.data_ptr(), self.exposure.data_ptr(),
                             self.m_exp.data_ptr(), self.v_exp.data_ptr(), self.d_exp.data_ptr(),
                             self.grads.data_ptr() if grads_out else None,
                             self.step_state.data_ptr())

    def step_fused(self, total_steps: int = 1, eager: bool = False, grads_out: bool = False,
                   check: bool = True):
        """One training step as one captured graph (or the same kernels eagerly).

        With check=True the call waits for the step and, if it overflowed the
        pair capacity (the device then skips the update), grows the capacity
        and runs the step again.  With check=False the call returns right
        after the launch (two steps stay in flight); an overflow is then
        reported by the call that waits for that step, which grows the
        capacity before launching its own step."""
        ts = self.train_state(grads_out)
        optim = paper_optim(self.scene.extent, total_steps)
        flags = B.FUSED_EAGER if eager else 0
        for _ in range(8):
            size = B.fused_workspace_size(ts, self.cams, self.opts, self.cap_fused, self.scap_fused)
            if getattr(self, "_ws_fused", None) is None or self._ws_fused.numel() < size:
                self._ws_fused = torch.empty(size, dtype=torch.uint8, device=self.dev)
            r = self.rg.step_fused(ts, self.cams, self.opts, self.targets(0, self.V), optim,
                                   self._ws_fused, self.cap_fused, flags, raise_on_capacity=False,
                                   slot_capacity=self.scap_fused)
            if r == B.ECAPACITY:
                self._grow_fused(self.rg.fused_status())
                continue
            if not check:
                return
            st = self.rg.fused_status()
            if not st["overflow"]:
                return
            self._grow_fused(st)
        raise RuntimeError("pair capacity did not converge")

    def _grow_fused(self, st, slack: float = 1.25):
        self.cap_fused = max(self.cap_fused, int(st["pairs"] * slack) + 4096)
        self.scap_fused = max(self.scap_fused, int(st["visible"] * slack) + 4096)

    def fit_fused_capacity(self, slack: float = 1.1):
        """Shrinks the fused step's capacities to the last step's counts plus a
        margin (kernels waiting for device-side counts are sized by them)."""
        st = self.rg.fused_status()
        self.cap_fused = int(st["pairs"] * slack) + 4096
        self.scap_fused = int(st["visible"] * slack) + 4096

    def fused_status(self) -> dict:
        """Waits for the last fused step and returns its statistics."""
        return self.rg.fused_status()

    # ------------------------------------------------------- checkpoints
    _CKPT = ("params", "m", "v", "s_act", "alpha_act", "exposure", "m_exp", "v_exp")

    def save_checkpoint(self, path: str) -> None:
        """Writes the optimisation state to an .npz file: raw parameters,
        Adam moments, the activated copies, exposure and its moments, the
        host step count and the fused step's device state (step count,
        skipped steps, last loss).  Waits for the device."""
        torch.cuda.synchronize(self.dev)
        arrs = {k: getattr(self, k).detach().cpu().numpy() for k in self._CKPT}
        arrs["step_count"] = np.array([self.step_count], np.int64)
        if hasattr(self, "step_state"):
            arrs["step_state"] = self.step_state.cpu().numpy()
        arrs["shape"] = np.array([self.N, self.C, self.V], np.int64)
        np.savez(path, **arrs)

    def load_checkpoint(self, path: str) -> None:
        """Restores a state written by save_checkpoint for the same surfel
        count, classes and views (no pickled objects are read)."""
        with np.load(path, allow_pickle=False) as f:
            if tuple(int(t) for t in f["shape"]) != (self.N, self.C, self.V):
                raise ValueError("checkpoint is for another surfel count, class count or views")
            for k in self._CKPT:
                getattr(self, k).copy_(torch.as_tensor(f[k], device=self.dev))
            self.step_count = int(f["step_count"][0])
            if "step_state" in f.files:
                if not hasattr(self, "step_state"):
                    self.step_state = torch.zeros(16, dtype=torch.int32, device=self.dev)
                self.step_state.copy_(torch.as_tensor(f["step_state"], device=self.dev))
        torch.cuda.synchronize(self.dev)

    def render_all_plain(self):
        for v in range(self.V):
            self.forward_view(v)
