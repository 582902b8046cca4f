"""Comparison helpers shared by the GPU parity tests (not a test module).

Gradient bar, per parameter tensor: max |delta| <= tol * max |g_ref|, and
|delta| <= tol * |g_ref| elementwise where |g_ref| >= 1e-2 * max |g_ref|."""
import numpy as np

import oracle

ROWS = {"z": slice(0, 1), "q": slice(1, 5), "s": slice(5, 7), "alpha": slice(7, 8),
        "rgb": slice(8, 11), "sem": slice(11, None)}


def grads_compare(g_gpu, ref_flat, n, C, tol=1e-4, cols=None):
    """g_gpu: packed [11 + C][n] gradients; ref_flat: the oracle's flat FP64
    block.  cols (optional): surfel indices to compare."""
    ref = oracle.split_grads(ref_flat, n, C)
    for name, sl in ROWS.items():
        a = g_gpu[sl].reshape(ref[name].shape) if ref[name].ndim > 1 else g_gpu[sl].reshape(-1)
        r = ref[name]
        if cols is not None:
            a, r = a[..., cols], r[..., cols]
        mx = np.abs(r).max()
        if mx == 0.0:            # e.g. dL/dz under a top-down orthographic camera
            assert np.abs(a).max() == 0.0, name
            continue
        d = np.abs(a - r)
        assert d.max() <= tol * mx, (name, d.max() / mx)
        big = np.abs(r) >= 1e-2 * mx
        rel = d[big] / np.abs(r[big])
        assert rel.max() <= tol, (name, rel.max(), np.argmax(rel))


def oracle_work_counts(prm, cams, o):
    """Per batch, from the oracle's tile lists and forward: the list entries
    every pixel visits up to its termination (its n_last) and those whose
    binary32 3-sigma test passes; compared with rogs_debug_work."""
    e_ref = k_ref = 0
    for cam in cams:
        _, rec, _ = oracle.contract(prm, cam, o)
        _, ids, ranges = oracle.tile_lists(prm, cam, o)
        _, _, nl = oracle.render_fwd(prm, cam, o)
        tx = (cam.w + o.tile_w - 1) // o.tile_w
        for py in range(cam.h):
            for px in range(cam.w):
                t = (py // o.tile_h) * tx + px // o.tile_w
                a, _ = ranges[t]
                n = int(nl[py * cam.w + px])
                lst = ids[a:a + n]
                e_ref += len(lst)
                q = oracle.q32(rec[lst], [px], [py])[:, 0] if len(lst) else np.zeros(0)
                k_ref += int((q <= np.float32(o.q_cut)).sum())
    return e_ref, k_ref
