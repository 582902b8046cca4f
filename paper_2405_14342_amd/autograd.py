"""torch.autograd wrapper of the splatting renderer.

:class:`RenderFn` renders every given view of the surfels in one batch
(``rogs_project`` + ``rogs_bin_sort`` + ``rogs_render_fwd``) and its backward
is ``rogs_render_bwd`` with the incoming dL/d(image): the adjoint of the
compositing of Eq. 6 chained through the projection of Eq. 2 and 5.  Inputs
are the activated render-domain surfel values (height z, unnormalised
quaternion q, scales s, opacity alpha, colour, semantic logits) as CUDA
float32 tensors; x and y are the fixed grid coordinates (no gradient).

The output is one flat float32 buffer holding, view after view, the planar
channels [R, G, B, sem_0 .. sem_{C-1}, D, A] of H x W pixels (use
:func:`split_views`).  Exposure compensation (Eq. 7) is not part of this
function: it belongs to the loss (``rogs_loss``), which applies it to the
composited colour.

Every call owns its own library context and workspace, so several renders may
be alive before their backward passes run.  There is no CPU path: CPU tensors
raise.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import binding as B


def _f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor (the renderer has no CPU path)")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.detach().contiguous()


class RenderFn(torch.autograd.Function):
    """images = RenderFn.apply(z, q, s, alpha, rgb, sem, x, y, cams, opts)

    Shapes: z [N], q [4, N], s [2, N], alpha [N], rgb [3, N], sem [C, N],
    x [N], y [N]; cams: a list of :class:`synth.Camera`-like objects or
    :class:`binding.Camera`; opts: :class:`binding.RenderOpts` or None."""

    @staticmethod
    def forward(ctx, z, q, s, alpha, rgb, sem, x, y, cams, opts=None, pair_capacity=1 << 20):
        z, q, s, alpha = _f32(z, "z"), _f32(q, "q"), _f32(s, "s"), _f32(alpha, "alpha")
        rgb, sem, x, y = _f32(rgb, "rgb"), _f32(sem, "sem"), _f32(x, "x"), _f32(y, "y")
        N = z.numel()
        C = sem.shape[0]
        if q.shape != (4, N) or s.shape != (2, N) or rgb.shape != (3, N) or sem.shape != (C, N) \
                or alpha.numel() != N or x.numel() != N or y.numel() != N:
            raise ValueError("surfel arrays must be z[N], q[4,N], s[2,N], alpha[N], rgb[3,N], "
                             "sem[C,N], x[N], y[N]")
        opts = opts or B.make_opts()
        cams = list(cams)
        surf = B.Surfels(N, C, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                         s.data_ptr(), alpha.data_ptr(), rgb.data_ptr(), sem.data_ptr())
        rg = B.Rogs()
        cap = int(pair_capacity)
        while True:
            ws = torch.empty(B.workspace_size(surf, cams, opts, cap), dtype=torch.uint8,
                             device=z.device)
            rg.project(surf, cams, opts, ws, cap)
            n = rg.bin_sort(ws, B.SYNC_COUNT, raise_on_capacity=False)
            if n >= 0:
                break
            st = rg.batch_stats(ws)
            cap = int(max(st["pairs"], st["visible"]) * 1.25) + 4096
        total_pix = sum(int(c.w) * int(c.h) for c in cams)
        out = torch.empty((5 + C) * total_pix, dtype=torch.float32, device=z.device)
        rg.render_fwd(surf, ws, out)
        ctx.save_for_backward(z, q, s, alpha, rgb, sem, x, y, out)
        ctx.rg, ctx.ws, ctx.NC = rg, ws, (N, C)
        return out

    @staticmethod
    def backward(ctx, g_out):
        z, q, s, alpha, rgb, sem, x, y, out = ctx.saved_tensors
        N, C = ctx.NC
        surf = B.Surfels(N, C, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                         s.data_ptr(), alpha.data_ptr(), rgb.data_ptr(), sem.data_ptr())
        g = g_out.detach().to(torch.float32).contiguous()
        grads = torch.empty((11 + C, N), dtype=torch.float32, device=z.device)
        ctx.rg.render_bwd(surf, ctx.ws, out, g, grads, 0)
        dz, dq, ds, da = grads[0], grads[1:5], grads[5:7], grads[7]
        drgb, dsem = grads[8:11], grads[11:]
        need = ctx.needs_input_grad
        pick = lambda i, t: t if need[i] else None
        return (pick(0, dz), pick(1, dq), pick(2, ds), pick(3, da), pick(4, drgb),
                pick(5, dsem), None, None, None, None, None)


def render(z, q, s, alpha, rgb, sem, x, y, cams, opts=None) -> torch.Tensor:
    """Differentiable batched render; see :class:`RenderFn`."""
    return RenderFn.apply(z, q, s, alpha, rgb, sem, x, y, cams, opts)


def split_views(out: torch.Tensor, cams: Sequence, C: int) -> List[torch.Tensor]:
    """Views [5 + C, H, W] of the flat output buffer."""
    views, o = [], 0
    for c in cams:
        n = (5 + C) * int(c.w) * int(c.h)
        views.append(out[o:o + n].view(5 + C, int(c.h), int(c.w)))
        o += n
    return views
