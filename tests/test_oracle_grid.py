"""Pins of the oracle's grid-side terms (CPU only): elevation smoothness
(Eq. 10), LiDAR elevation loss and its nearest-neighbour lookup (Eq. 11), the
meshgrid layout with its road mask and neighbour index (Sec. 3.1; supp.
Sec. 3.3) and the pose-based initialisation (Eq. 4; supp. Sec. 1)."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle
from paper_2405_14342_amd import synth


def _layout(n_along=60, step=0.5, radius_px=12, seed=3):
    traj = synth.Trajectory(n_along * synth.SPACING, seed)
    poses = synth.vehicle_poses(traj, step)
    h = np.float32(0.1)
    xy = poses[:, :2].astype(np.float64)
    x0 = float(np.floor(xy[:, 0].min()) - 2.0)
    y0 = float(np.floor(xy[:, 1].min()) - 2.0)
    W = int(math.ceil((xy[:, 0].max() + 2.0 - x0) / h)) + 1
    H = int(math.ceil((xy[:, 1].max() + 2.0 - y0) / h)) + 1
    return poses, oracle.meshgrid_layout(poses, x0, y0, h, W, H, radius_px), (x0, y0, h, W, H)


def test_road_mask_is_disk_dilation_of_pose_pixels():
    poses, L, (x0, y0, h, W, H) = _layout()
    img = np.zeros((H, W), bool)
    pix = L["pose_pixels"]
    img[pix[:, 1], pix[:, 0]] = True
    r = 12
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    disk = xx * xx + yy * yy <= r * r
    ref = ndimage.binary_dilation(img, structure=disk)
    np.testing.assert_array_equal(L["mask"].astype(bool), ref)
    # cell of a position = nearest pixel centre
    np.testing.assert_array_equal(pix[:, 0], np.floor((poses[:, 0].astype(np.float64) - x0) / h + 0.5))


def test_surfel_index_is_running_count_and_grid_positions():
    _, L, (x0, y0, h, W, H) = _layout()
    mask, idx = L["mask"].astype(bool), L["idx"]
    n = L["x"].size
    assert n == mask.sum()
    np.testing.assert_array_equal(idx[mask], np.arange(n))
    assert np.all(idx[~mask] == -1)
    rows, cols = np.nonzero(mask)
    np.testing.assert_array_equal(L["x"], (x0 + cols * np.float64(h)).astype(np.float32))
    np.testing.assert_array_equal(L["y"], (y0 + rows * np.float64(h)).astype(np.float32))


def test_neighbour_index_equals_brute_force_nearest():
    """The pixel-index lookup gives, for every surfel, the surfel one grid step
    away in each direction (found here by brute force over all surfels), or
    the surfel itself at the road's border."""
    _, L, (x0, y0, h, W, H) = _layout(n_along=30)
    x, y, nbr = L["x"].astype(np.float64), L["y"].astype(np.float64), L["nbr"]
    n = x.size
    step = float(np.float64(np.float32(0.1)))
    for d, (dx, dy) in enumerate([(0, -1), (0, 1), (-1, 0), (1, 0)]):
        tx, ty = x + dx * step, y + dy * step
        ref = np.arange(n)
        for i in range(n):
            dist = np.hypot(x - tx[i], y - ty[i])
            j = int(np.argmin(dist))
            if dist[j] < 0.25 * step:
                ref[i] = j
        np.testing.assert_array_equal(nbr[d], ref, err_msg=str(d))
    # the table is symmetric: up/down and left/right are mutual
    i = np.arange(n)
    assert np.all((nbr[1][nbr[0]] == i) | (nbr[0] == i))
    assert np.all((nbr[3][nbr[2]] == i) | (nbr[2] == i))


def test_pose_init_closed_form_on_a_tilted_plane():
    """Poses on the plane z = a x + b y + c with normal n3: Eq. 4 puts every
    surfel on that plane; the rotation is the nearest pose's."""
    a, b, c = 0.03, -0.02, 1.5
    nrm = np.array([-a, -b, 1.0]) / math.sqrt(a * a + b * b + 1.0)
    f = np.array([1.0, 0.0, a]) / math.sqrt(1 + a * a)
    left = np.cross(nrm, f)
    R = np.stack([f, left, nrm], axis=-1)
    P = 40
    xs = np.linspace(0.0, 10.0, P)
    poses = np.zeros((P, 12), np.float32)
    poses[:, 0] = xs
    poses[:, 1] = 0.3 * np.sin(xs)
    poses[:, 2] = a * poses[:, 0].astype(np.float64) + b * poses[:, 1].astype(np.float64) + c
    poses[:, 3:] = R.reshape(-1)
    L = oracle.meshgrid_layout(poses, -2.0, -3.0, np.float32(0.1), 140, 60, 15)
    Rf = poses[0, 3:].astype(np.float64).reshape(3, 3)
    n3 = Rf[:, 2]
    # the surfel's height solves n3 . (p - p_v) = 0 for its nearest pose p_v
    idx = oracle.lidar_nn(L["x"], L["y"], poses[:, 0], poses[:, 1])
    pv = poses[idx, :3].astype(np.float64)
    p = np.stack([L["x"], L["y"], L["z"]], axis=-1).astype(np.float64)
    resid = ((p - pv) @ n3)
    assert np.abs(resid).max() < 1e-6
    # rotation = the pose's (unit quaternion, w >= 0)
    q = L["q"]
    assert np.all(q[0] >= 0.0)
    Rq = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=-1)).as_matrix()
    assert np.abs(Rq - Rf[None]).max() < 1e-6


def test_smoothness_closed_form_and_gradient():
    _, L, (x0, y0, h, W, H) = _layout(n_along=30)
    nbr, x, y = L["nbr"], L["x"].astype(np.float64), L["y"].astype(np.float64)
    n = x.size
    # z = a * column: vertical neighbours add nothing, every horizontal edge
    # counts twice (once from each end), each with (a * 1)^2, over K = 4
    a = 0.75
    col = np.nonzero(L["mask"])[1].astype(np.float64)
    val, _ = oracle.smooth_loss(a * col, nbr, lam=1.0)
    i = np.arange(n)
    edges = (nbr[2] != i).sum() + (nbr[3] != i).sum()
    assert val == edges * a * a / 4.0
    # gradient against central differences
    rng = np.random.default_rng(4)
    z = rng.normal(0.0, 0.1, n)
    lam = 0.003
    _, dz = oracle.smooth_loss(z, nbr, lam)
    for k in rng.choice(n, 12, replace=False):
        e = np.zeros(n)
        e[k] = 1e-6
        fd = (oracle.smooth_loss(z + e, nbr, lam)[0] - oracle.smooth_loss(z - e, nbr, lam)[0]) / 2e-6
        assert fd == pytest.approx(dz[k], rel=1e-6, abs=1e-12)


def test_lidar_nearest_neighbour_and_loss():
    rng = np.random.default_rng(5)
    px, py = rng.uniform(0, 20, 3000).astype(np.float32), rng.uniform(0, 5, 3000).astype(np.float32)
    x, y = rng.uniform(0, 20, 800).astype(np.float32), rng.uniform(0, 5, 800).astype(np.float32)
    idx = oracle.lidar_nn(x, y, px, py)
    d, ref = cKDTree(np.stack([px, py], -1).astype(np.float64)).query(
        np.stack([x, y], -1).astype(np.float64), k=2)
    unique = d[:, 1] - d[:, 0] > 1e-9
    np.testing.assert_array_equal(idx[unique], ref[unique, 0])
    # Eq. 11, closed form: targets a constant c above the surfels give
    # lambda N c^2, and every height is pulled up by 2 lambda c
    z = rng.normal(0, 0.2, 800)
    c = 0.37
    val, dz = oracle.lidar_loss(z, z + c, 0.02)
    assert val == pytest.approx(0.02 * 800 * c * c, rel=1e-12)
    np.testing.assert_allclose(dz, np.full(800, -2.0 * 0.02 * c), rtol=1e-12)
    assert oracle.lidar_loss(z, z, 0.02)[0] == 0.0
    # gradient against central differences at random targets (the loss is
    # quadratic in each height, so a large step is exact up to rounding)
    zbar = rng.normal(0, 0.2, 800)
    _, dz = oracle.lidar_loss(z, zbar, 0.02)
    for k in rng.choice(800, 12, replace=False):
        e = np.zeros(800)
        e[k] = 1e-2
        fd = (oracle.lidar_loss(z + e, zbar, 0.02)[0] - oracle.lidar_loss(z - e, zbar, 0.02)[0]) / 2e-2
        assert fd == pytest.approx(dz[k], rel=1e-9, abs=1e-13)
