"""Seeded synthetic scenes, cameras and targets.

This module holds input generation only (no rasterizer arithmetic), so that
the HIP path and the CPU oracle can both be fed the same arrays.  All draws
use numpy's PCG64 ``default_rng(seed)`` with seed = 10 * config + stream
(stream 0 scene, 1 cameras, 2 targets, 3 request trace, 4 finite-difference
weights), in the fixed order means, log-scales, quaternions, opacity, SH.

Parameter layout (structure of arrays, float32):
  means [3, N], log_scales [3, N], quats [4, N] (w, x, y, z),
  opacity [N] (logit), sh [3 (D+1)^2, N] with row 3 j + channel,
  j = l^2 + l + m the real-SH index.

The scenes stand in for the paper's datasets (MipNeRF-360, MatrixCity,
ScanNet++; Sec. 4) by shape only: Gaussian count, resolution, and spatial
structure (clusters plus a ground plane, or an aerial city of boxes).
"""
from __future__ import annotations

import math

import numpy as np

Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi)): degree-0 real SH


def _rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(10 * config + stream)


def _sh_from_rgb(rng, rgb: np.ndarray, D: int) -> np.ndarray:
    n = rgb.shape[1]
    nc = (D + 1) ** 2
    sh = np.zeros((3 * nc, n), np.float32)
    sh[0:3] = ((rgb - 0.5) / Y00).astype(np.float32)
    if nc > 1:
        sh[3:] = rng.normal(0.0, 0.2, size=(3 * (nc - 1), n)).astype(np.float32)
    return sh


def _common(rng, means: np.ndarray, mu_s, D: int) -> dict:
    """Draw log-scales, rotations, opacity and SH for given means."""
    n = means.shape[1]
    mu_s = np.broadcast_to(np.asarray(mu_s, np.float64), (n,))
    log_scales = (mu_s[None, :] + rng.normal(0.0, 0.5, size=(3, n))).astype(np.float32)
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    sh = _sh_from_rgb(rng, rgb, D)
    return dict(means=np.ascontiguousarray(means, np.float32), log_scales=log_scales,
                quats=q.astype(np.float32), opacity=opacity, sh=sh, sh_degree=D)


def random_rotation(rng) -> np.ndarray:
    q = rng.normal(0.0, 1.0, size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# ---------------------------------------------------------------- cameras
def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """World->camera rotation for OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(r) < 1e-12:
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    return np.stack([r, d, f], 0)


def make_camera(R, eye, W: int, H: int, hfov_deg: float = 60.0, z_near: float = 0.2,
                bg=(0.0, 0.0, 0.0), cx=None, cy=None) -> dict:
    """Pinhole camera; fx = fy from the horizontal field of view."""
    R = np.asarray(R, np.float64)
    eye = np.asarray(eye, np.float64)
    fx = (W / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    R32 = R.astype(np.float32)
    o32 = eye.astype(np.float32)
    t32 = (-(R32.astype(np.float64) @ o32.astype(np.float64))).astype(np.float32)
    return dict(R=R32, t=t32, o=o32, fx=np.float32(fx), fy=np.float32(fx),
                cx=np.float32(W / 2.0 if cx is None else cx), cy=np.float32(H / 2.0 if cy is None else cy),
                W=int(W), H=int(H), z_near=np.float32(z_near), bg=np.asarray(bg, np.float32))


def orbit_camera(radius: float, azim: float, elev: float, W: int, H: int, **kw) -> dict:
    eye = radius * np.array([math.cos(elev) * math.cos(azim), math.cos(elev) * math.sin(azim), math.sin(elev)])
    return make_camera(look_at(eye, (0.0, 0.0, 0.0)), eye, W, H, **kw)


# ---------------------------------------------------------------- scenes
def scene_uniform(n: int, seed: int, D: int = 0, mu_s: float = -4.5, extent: float = 1.0) -> dict:
    """Means uniform in [-extent, extent]^3 (the small plain-method scene)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-extent, extent, size=(3, n))
    return _common(rng, means, mu_s, D)


def scene_clusters(n: int, seed: int, D: int = 3, mu_s: float = -4.5, n_clusters: int = 64,
                   ground_frac: float = 0.3) -> dict:
    """Mixture of anisotropic clusters plus samples on the ground plane z = 0."""
    rng = np.random.default_rng(seed)
    n_ground = int(round(n * ground_frac))
    n_cl = n - n_ground
    sizes = np.full(n_clusters, n_cl // n_clusters, np.int64)
    sizes[: n_cl - sizes.sum()] += 1
    centres = np.stack([rng.uniform(-1.5, 1.5, n_clusters), rng.uniform(-1.5, 1.5, n_clusters),
                        rng.uniform(0.1, 1.5, n_clusters)], 1)
    stds = np.exp(rng.uniform(math.log(0.05), math.log(0.4), size=(n_clusters, 3)))
    rots = [random_rotation(rng) for _ in range(n_clusters)]
    parts = []
    for c in range(n_clusters):
        z = rng.normal(0.0, 1.0, size=(int(sizes[c]), 3)) * stds[c]
        parts.append(z @ rots[c].T + centres[c])
    ground = np.stack([rng.uniform(-2, 2, n_ground), rng.uniform(-2, 2, n_ground), np.zeros(n_ground)], 1)
    means = np.concatenate(parts + [ground], 0).T
    return _common(rng, means, mu_s, D)


def scene_city(n: int, seed: int, D: int = 3, half: float = 1000.0, n_boxes: int = 4000) -> dict:
    """Aerial city: ground plane over [-half, half]^2 (50%) plus box facades
    and roofs (50%, spread by area); log-scale mean ln(0.5 h) with h the
    mean spacing sqrt(area / count) of each part."""
    rng = np.random.default_rng(seed)
    n_ground = n // 2
    n_box = n - n_ground
    bx = rng.uniform(-0.95 * half, 0.95 * half, size=(n_boxes, 2))
    side = rng.uniform(10, 60, size=(n_boxes, 2))
    height = rng.uniform(10, 150, size=n_boxes)
    yaw = rng.uniform(0, math.pi / 2, size=n_boxes)
    # faces: 4 walls + roof per box, area-weighted
    a_walls = 2 * (side[:, 0] + side[:, 1]) * height
    a_roof = side[:, 0] * side[:, 1]
    area = a_walls + a_roof
    cnt = np.floor(n_box * area / area.sum()).astype(np.int64)
    cnt[: n_box - cnt.sum()] += 1
    bid = np.repeat(np.arange(n_boxes), cnt)
    u = rng.uniform(0, 1, size=(n_box, 3))
    sx, sy, h = side[bid, 0], side[bid, 1], height[bid]
    per = 2 * (sx + sy)
    roof = u[:, 0] < (a_roof[bid] / area[bid])
    # position along the perimeter for walls, uniform on top for roofs
    t = u[:, 1] * per
    lx = np.where(t < sx, t - sx / 2, np.where(t < sx + sy, sx / 2, np.where(t < 2 * sx + sy, sx / 2 - (t - sx - sy), -sx / 2)))
    ly = np.where(t < sx, -sy / 2, np.where(t < sx + sy, -sy / 2 + (t - sx), np.where(t < 2 * sx + sy, sy / 2, sy / 2 - (t - 2 * sx - sy))))
    lz = u[:, 2] * h
    rx = (u[:, 1] - 0.5) * sx
    ry = (u[:, 2] - 0.5) * sy
    lx = np.where(roof, rx, lx)
    ly = np.where(roof, ry, ly)
    lz = np.where(roof, h, lz)
    c, s = np.cos(yaw[bid]), np.sin(yaw[bid])
    X = bx[bid, 0] + c * lx - s * ly
    Yy = bx[bid, 1] + s * lx + c * ly
    gpos = rng.uniform(-half, half, size=(n_ground, 2))
    means = np.concatenate([np.stack([gpos[:, 0], gpos[:, 1], np.zeros(n_ground)], 1),
                            np.stack([X, Yy, lz], 1)], 0).T
    h_ground = math.sqrt((2 * half) ** 2 / max(n_ground, 1))
    h_box = math.sqrt(area.sum() / max(n_box, 1))
    mu_s = np.concatenate([np.full(n_ground, math.log(0.5 * h_ground)), np.full(n_box, math.log(0.5 * h_box))])
    return _common(rng, means, mu_s, D)


def target_image(seed: int, W: int, H: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(3, H, W)).astype(np.float32)


# ---------------------------------------------------------------- configs
def config1(L: int = 2):
    """20k Gaussians in [-1,1]^3, SH 0; camera at distance 3, 60 deg, 256^2."""
    params = scene_uniform(20000, seed=10, D=0)
    eye = 3.0 * np.array([math.cos(math.radians(20)) * math.cos(math.radians(30)),
                          math.cos(math.radians(20)) * math.sin(math.radians(30)), math.sin(math.radians(20))])
    cam = make_camera(look_at(eye, (0, 0, 0)), eye, 256, 256, z_near=0.2)
    return params, cam, target_image(12, 256, 256), L


def config2(n: int = 1_000_000, W: int = 1600, H: int = 1060, L: int = 3):
    """1M clustered Gaussians + ground plane, SH 3; orbit radius 4, elevation 25 deg."""
    params = scene_clusters(n, seed=20, D=3)
    rng = _rng(2, 1)
    azim = rng.uniform(0, 2 * math.pi)
    cam = orbit_camera(4.0, azim, math.radians(25.0), W, H, z_near=0.2)
    return params, cam, target_image(22, W, H), L


def config4_cameras(n_views: int = 16):
    rng = _rng(4, 1)
    res = [(960, 540), (1600, 1060), (1920, 1080), (3840, 2160)]
    cams = []
    for _ in range(n_views):
        azim = rng.uniform(0, 2 * math.pi)
        elev = math.radians(rng.uniform(10, 45))
        W, H = res[int(rng.integers(0, 4))]
        cams.append(orbit_camera(4.0, azim, elev, W, H, z_near=0.2))
    return cams


def aerial_camera(rng, W: int, H: int, xy_range: float, alt, pitch_deg) -> dict:
    x, y = rng.uniform(-xy_range, xy_range, 2)
    yaw = rng.uniform(0, 2 * math.pi)
    pitch = math.radians(pitch_deg)
    eye = np.array([x, y, alt])
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    return make_camera(look_at(eye, eye + fwd), eye, W, H, z_near=0.5)


def with_kd_axis_aligned_camera(split_x: float, W: int, H: int, dist: float = 3.0, z_near: float = 0.2):
    """Camera whose centre lies on the plane x = split_x, looking along +y with
    the world z axis pointing up; the plane maps to the image column u = W/2."""
    eye = np.array([split_x, -dist, 0.0], np.float64)
    # rows: camera x (right) = world +x, camera y (down) = world -z,
    # camera z (forward) = world +y; a proper rotation (det +1)
    R = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    cam = make_camera(R, eye, W, H, z_near=z_near)
    cam["o"] = np.array([np.float32(split_x), np.float32(-dist), np.float32(0.0)], np.float32)
    cam["t"] = (-(cam["R"].astype(np.float64) @ cam["o"].astype(np.float64))).astype(np.float32)
    return cam


def scene_city_device(n: int, seed: int, D: int = 3, half: float = 1000.0, n_boxes: int = 4000, device="cuda"):
    """The aerial-city layout of scene_city, drawn on the GPU with torch's
    Philox generator (for scenes too large to draw on the host); returns
    float32 device tensors in the same layout.  Not bit-identical to
    scene_city (different generator)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f32 = torch.float32

    def U(shape, a, b):
        return torch.rand(shape, generator=g, device=device, dtype=f32) * (b - a) + a

    def N(shape, m, s):
        return torch.randn(shape, generator=g, device=device, dtype=f32) * s + m

    n_ground = n // 2
    n_box = n - n_ground
    bx = U((n_boxes, 2), -0.95 * half, 0.95 * half)
    side = U((n_boxes, 2), 10.0, 60.0)
    height = U((n_boxes,), 10.0, 150.0)
    yaw = U((n_boxes,), 0.0, math.pi / 2)
    a_walls = 2 * (side[:, 0] + side[:, 1]) * height
    a_roof = side[:, 0] * side[:, 1]
    area = (a_walls + a_roof).double()
    cnt = torch.floor(n_box * area / area.sum()).long()
    cnt[: n_box - int(cnt.sum())] += 1
    bid = torch.repeat_interleave(torch.arange(n_boxes, device=device), cnt)
    u = torch.rand((n_box, 3), generator=g, device=device, dtype=f32)
    sx, sy, h = side[bid, 0], side[bid, 1], height[bid]
    per = 2 * (sx + sy)
    roof = u[:, 0] < (a_roof[bid] / (a_walls + a_roof)[bid])
    t = u[:, 1] * per
    lx = torch.where(t < sx, t - sx / 2, torch.where(t < sx + sy, sx / 2,
                     torch.where(t < 2 * sx + sy, sx / 2 - (t - sx - sy), -sx / 2)))
    ly = torch.where(t < sx, -sy / 2, torch.where(t < sx + sy, -sy / 2 + (t - sx),
                     torch.where(t < 2 * sx + sy, sy / 2, sy / 2 - (t - 2 * sx - sy))))
    lz = u[:, 2] * h
    lx = torch.where(roof, (u[:, 1] - 0.5) * sx, lx)
    ly = torch.where(roof, (u[:, 2] - 0.5) * sy, ly)
    lz = torch.where(roof, h, lz)
    c, s_ = torch.cos(yaw[bid]), torch.sin(yaw[bid])
    X = bx[bid, 0] + c * lx - s_ * ly
    Y = bx[bid, 1] + s_ * lx + c * ly
    means = torch.empty((3, n), device=device, dtype=f32)
    means[0, :n_ground] = U((n_ground,), -half, half)
    means[1, :n_ground] = U((n_ground,), -half, half)
    means[2, :n_ground] = 0.0
    means[0, n_ground:], means[1, n_ground:], means[2, n_ground:] = X, Y, lz
    h_ground = math.sqrt((2 * half) ** 2 / max(n_ground, 1))
    h_box = math.sqrt(float(area.sum()) / max(n_box, 1))
    mu_s = torch.empty(n, device=device, dtype=f32)
    mu_s[:n_ground] = math.log(0.5 * h_ground)
    mu_s[n_ground:] = math.log(0.5 * h_box)
    log_scales = mu_s[None, :] + N((3, n), 0.0, 0.5)
    q = torch.randn((4, n), generator=g, device=device, dtype=f32)
    q = q / q.norm(dim=0, keepdim=True)
    opacity = N((n,), 0.0, 1.0)
    nc = (D + 1) ** 2
    sh = torch.empty((3 * nc, n), device=device, dtype=f32)
    sh[0:3] = (U((3, n), 0.0, 1.0) - 0.5) / Y00
    if nc > 1:
        sh[3:] = N((3 * (nc - 1), n), 0.0, 0.2)
    return dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=q.contiguous(),
                opacity=opacity.contiguous(), sh=sh.contiguous(), sh_degree=D)
