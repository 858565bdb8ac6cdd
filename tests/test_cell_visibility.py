"""Cell culling (rgs_cell_visibility) against brute force, on the CPU.

A KD cell may be dropped for a view only if none of its Gaussians can reach
the image.  The oracle's projection (the same fp32 decisions the GPU takes,
bit for bit) says which Gaussians have a non-empty rectangle on each view;
every such Gaussian's cell must be marked visible.  Views include oblique
and low ones, where footprints reach far beyond the perspective image of the
3-sigma sphere through the EWA linearisation, and very large Gaussians.
Sec. 3.4 (the manager hands a request only to the sub-models it concerns).
"""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2406_11836_amd import scenes


@pytest.fixture(scope="module")
def lib():
    from paper_2406_11836_amd import _lib as L
    return L.load()


def cell_bounds_np(p, kd):
    """[8][K] bounds by brute force: centre min / max per cell, largest scale."""
    K = 1 << kd["L"]
    m = np.asarray(p["means"], np.float32)
    cc = kd["center_cell"]
    smax = np.exp(np.asarray(p["log_scales"], np.float32).astype(np.float64)).astype(np.float32).max(0)
    cb = np.zeros((8, K), np.float32)
    for k in range(K):
        sel = cc == k
        if not sel.any():
            cb[0:3, k], cb[3:6, k], cb[6, k] = np.inf, -np.inf, 0.0
            continue
        cb[0:3, k] = m[:, sel].min(1)
        cb[3:6, k] = m[:, sel].max(1)
        cb[6, k] = smax[sel].max()
    return cb


def visibility(lib, cams, L, cb):
    from paper_2406_11836_amd import _lib as Lb
    arr = Lb.camera_array(cams)
    out = np.zeros(len(cams), np.uint64)
    cb = np.ascontiguousarray(cb, np.float32)
    assert lib.rgs_cell_visibility(arr, len(cams), L, cb.ctypes.data_as(C.c_void_p),
                                   out.ctypes.data_as(C.c_void_p)) == 0
    return out


def _cams(rng):
    cams = []
    for k in range(36):
        W, H = [(320, 180), (640, 360), (200, 300)][k % 3]
        alt = rng.uniform(15, 300)
        pitch = rng.uniform(-90, -5) if k % 4 else rng.uniform(-15, -2)   # some near-horizontal
        cams.append(scenes.aerial_camera(rng, W, H, 250.0, alt, pitch))
    # off-centre principal points, wide and narrow fields of view
    for k in range(6):
        eye = np.array([rng.uniform(-150, 150), rng.uniform(-150, 150), rng.uniform(20, 120)])
        tgt = np.array([rng.uniform(-150, 150), rng.uniform(-150, 150), 0.0])
        cams.append(scenes.make_camera(scenes.look_at(eye, tgt), eye, 256, 192, hfov_deg=[20, 60, 100][k % 3],
                                       z_near=0.5, cx=40.0 + 30 * k, cy=150.0 - 20 * k))
    return cams


def test_culled_cells_hold_no_visible_gaussian(orc, lib):
    p = scenes.scene_city(24000, seed=80, D=0, half=300.0, n_boxes=40)
    # a few very large Gaussians (tens of metres), the hardest case for a bound
    big = np.random.default_rng(81).choice(p["means"].shape[1], 60, replace=False)
    p["log_scales"][:, big] = np.log(np.random.default_rng(82).uniform(5.0, 40.0, size=(3, 60))).astype(np.float32)
    L = 6
    kd = orc.kd_partition(p["means"], p["log_scales"], L)
    cb = cell_bounds_np(p, kd)
    cams = _cams(np.random.default_rng(83))
    vis = visibility(lib, cams, L, cb)
    n_culled = 0
    n_checked = 0
    for v, cam in enumerate(cams):
        pr = orc.project(p, cam, kd, 0)
        reach = pr["count"] > 0
        cells = np.unique(kd["center_cell"][reach])
        mask = int(vis[v])
        for k in cells:
            assert (mask >> int(k)) & 1, ("view %d drops cell %d holding %d visible Gaussians"
                                          % (v, k, int((kd["center_cell"][reach] == k).sum())))
        n_checked += int(reach.sum())
        n_culled += 64 - bin(mask).count("1")
    assert n_checked > 10000
    # the test is not vacuous: a good part of the cells is culled
    assert n_culled > 0.3 * 64 * len(cams), n_culled


def test_bound_is_not_loose_beyond_need(orc, lib):
    """A cell whose Gaussians sit just outside the frustum is culled, and kept once
    one of them grows enough for its footprint to reach the image."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 128, 96, z_near=0.1)
    f = float(cam["fx"])
    # a tight clump at depth 10, 40 px beyond the right edge of the image
    x = (128 - 64 + 40) / f * 10.0
    means = np.array([[x, x + 0.01], [0.0, 0.01], [10.0, 10.01]], np.float32)
    for s, expect in ((0.01, 0), (2.0, 1)):
        ls = np.full((3, 2), math.log(s), np.float32)
        p = dict(means=means, log_scales=ls)
        kd = dict(L=0, center_cell=np.zeros(2, np.int32))
        cb = cell_bounds_np(p, kd)
        assert int(visibility(lib, [cam], 0, cb)[0]) == expect


def test_empty_and_nonfinite_cells(lib):
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 64, 64)
    cb = np.zeros((8, 4), np.float32)
    cb[0:3], cb[3:6] = np.inf, -np.inf          # every cell empty ...
    cb[0:3, 1], cb[3:6, 1], cb[6, 1] = [0, 0, 5], [0, 0, 5], 0.1      # ... but cell 1 in view
    cb[0:3, 2], cb[3:6, 2], cb[6, 2] = [0, 0, -5], [0, 0, -4], 0.1    # cell 2 behind the camera
    cb[0:3, 3], cb[3:6, 3], cb[6, 3] = [np.nan, 0, 5], [0, 0, 5], 0.1  # cell 3 not finite: kept
    assert int(visibility(lib, [cam], 2, cb)[0]) == 0b1010


def test_random_gaussians_at_the_frustum_edge(orc, lib):
    """Thousands of single-Gaussian cells placed around the four sides of the
    frustum, large and anisotropic, at every depth: whenever the oracle finds a
    non-empty rectangle, the cell is kept.  Many of these footprints reach the
    image although a sphere of radius 3 s around the centre lies entirely
    outside the frustum (the EWA Jacobian is taken at the clamped centre and
    the low-pass adds 0.3 px^2), so the test fails for a bound that ignores
    them."""
    rng = np.random.default_rng(84)
    L = 6
    K = 64
    sphere_outside_but_visible = 0
    n_visible = 0
    for trial in range(60):
        W, H = [(160, 120), (96, 200), (256, 64)][trial % 3]
        eye = rng.normal(size=3) * 5
        tgt = eye + rng.normal(size=3)
        cam = scenes.make_camera(scenes.look_at(eye, tgt), eye, W, H, hfov_deg=rng.uniform(20, 110), z_near=0.05,
                                 cx=rng.uniform(0.2, 0.8) * W, cy=rng.uniform(0.2, 0.8) * H)
        R = np.asarray(cam["R"], np.float64)
        fx, cx, cy = float(cam["fx"]), float(cam["cx"]), float(cam["cy"])
        z = np.exp(rng.uniform(np.log(0.3), np.log(60.0), K))
        side = rng.integers(0, 4, K)
        # image-plane position just beyond one side of the image, up to 40% of its size
        u = rng.uniform(0, W, K)
        v = rng.uniform(0, H, K)
        off = rng.uniform(0.0, 0.4, K)
        u = np.where(side == 0, -off * W, np.where(side == 1, W * (1 + off), u))
        v = np.where(side == 2, -off * H, np.where(side == 3, H * (1 + off), v))
        pc = np.stack([(u - cx) / fx * z, (v - cy) / fx * z, z], 0)
        means = (R.T @ pc + np.asarray(cam["o"], np.float64)[:, None]).astype(np.float32)
        s = z * np.exp(rng.uniform(np.log(0.002), np.log(0.3), K))
        ls = np.log(np.stack([s, s * rng.uniform(0.05, 1, K), s * rng.uniform(0.05, 1, K)])).astype(np.float32)
        q = rng.normal(size=(4, K)).astype(np.float32)
        p = dict(means=means, log_scales=ls, quats=q, opacity=np.full(K, 6.0, np.float32),
                 sh=np.zeros((3, K), np.float32), sh_degree=0)
        kd = dict(L=L, K=K, split=np.zeros(K - 1, np.float32), center_cell=np.arange(K, dtype=np.int32))
        pr = orc.project(p, cam, dict(L=0, K=1, split=np.zeros(0, np.float32)), 0)
        mask = int(visibility(lib, [cam], L, cell_bounds_np(p, kd))[0])
        for i in np.nonzero(pr["count"] > 0)[0]:
            assert (mask >> int(i)) & 1, (trial, i)
            n_visible += 1
            # would a 3-sigma sphere (largest scale) clear every side plane of the frustum?
            t = pc[:, i]
            smax = float(np.exp(ls[:, i].astype(np.float64)).max())
            planes = [(np.array([1.0, 0, cx / fx])), (np.array([-1.0, 0, (W - cx) / fx])),
                      (np.array([0, 1.0, cy / fx])), (np.array([0, -1.0, (H - cy) / fx]))]
            if any(pl @ t / np.linalg.norm(pl) < -3 * smax for pl in planes):
                sphere_outside_but_visible += 1
    assert n_visible > 500, n_visible
    assert sphere_outside_but_visible > 10, sphere_outside_but_visible
