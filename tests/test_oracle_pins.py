"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: textbook
closed forms (SH, EWA of an isotropic Gaussian, one- and two-Gaussian
blends), invariances (quaternion sign/scale, world rotation), brute force
(rectangles, cell sets, ray-box entry order, order statistics), the paper's
equivalence of the merged partials with the single-worker render (Sec. 3.2,
Eq. 5 and the appendix proof), its validity experiment (Sec. 4.2, camera on a
dividing plane) and finite differences of the oracle's own forward.
"""
import math

import numpy as np
import pytest

from paper_2406_11836_amd import scenes


# ------------------------------------------------------------------ helpers
def manual_scene(means, log_scales, quats=None, opacity=None, rgb=None, D=0):
    means = np.asarray(means, np.float32).reshape(3, -1)
    n = means.shape[1]
    ls = np.asarray(log_scales, np.float32).reshape(3, n)
    q = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)) if quats is None else np.asarray(quats, np.float32)
    op = np.full(n, 2.0, np.float32) if opacity is None else np.asarray(opacity, np.float32)
    rgb = np.full((3, n), 0.7) if rgb is None else np.asarray(rgb, np.float64)
    nc = (D + 1) ** 2
    sh = np.zeros((3 * nc, n), np.float32)
    sh[0:3] = ((rgb - 0.5) / scenes.Y00).astype(np.float32)
    return dict(means=means, log_scales=ls, quats=q, opacity=op, sh=sh, sh_degree=D)


def axis_camera(W=64, H=64, f=None, z_near=0.1):
    """Camera at the origin looking along +z (R = I)."""
    cam = scenes.make_camera(np.eye(3), np.zeros(3), W, H, z_near=z_near)
    if f is not None:
        cam["fx"] = cam["fy"] = np.float32(f)
    return cam


def kd_trivial():
    return dict(L=0, K=1, split=np.zeros(0, np.float32))


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def f32(x):
    return float(np.float32(x))


def scale32(s):
    """The scale the oracle sees for a log-scale stored as float32."""
    return math.exp(f32(math.log(s)))


# ------------------------------------------------------------------ SH (Sec. 3.1: colour through SH)
def test_sh_orthonormal(orc):
    """Gram matrix of the 16 real SH by exact quadrature is the identity."""
    zs, wz = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phis = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros((16, 16))
    for z, w in zip(zs, wz):
        r = math.sqrt(1 - z * z)
        for ph in phis:
            Y, _ = orc.sh_basis(3, [r * math.cos(ph), r * math.sin(ph), z])
            G += np.outer(Y, Y) * w * (2 * np.pi / nphi)
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_band_sums(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y, _ = orc.sh_basis(3, d)
        for l in range(4):
            s = sum(Y[l * l + l + m] ** 2 for m in range(-l, l + 1))
            assert abs(s - (2 * l + 1) / (4 * np.pi)) < 1e-13


def test_sh_textbook_values(orc):
    """Standard real SH with the Condon-Shortley phase (tabulated forms)."""
    d = np.array([0.48, -0.6, 0.64])
    x, y, z = d
    Y, _ = orc.sh_basis(3, d)
    pi = math.pi
    ref = {
        0: 0.5 / math.sqrt(pi),
        1: -math.sqrt(3 / (4 * pi)) * y,
        2: math.sqrt(3 / (4 * pi)) * z,
        3: -math.sqrt(3 / (4 * pi)) * x,
        4: 0.5 * math.sqrt(15 / pi) * x * y,
        6: 0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),
        8: 0.25 * math.sqrt(15 / pi) * (x * x - y * y),
        12: 0.25 * math.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),
        15: -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),
    }
    for j, v in ref.items():
        assert abs(Y[j] - v) < 1e-14, j


def test_sh_gradient_fd(orc):
    d = np.array([0.3, -0.5, 0.7])
    _, dY = orc.sh_basis(3, d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3); e[a] = h
        Yp, _ = orc.sh_basis(3, d + e)
        Ym, _ = orc.sh_basis(3, d - e)
        assert np.abs((Yp - Ym) / (2 * h) - dY[:, a]).max() < 1e-8


def test_degree0_colour_is_rgb(orc):
    p = scenes.scene_uniform(200, seed=3, D=0)
    cam = scenes.orbit_camera(3.0, 0.3, 0.2, 64, 64)
    kd = orc.kd_partition(p["means"], p["log_scales"], 1)
    pr = orc.project(p, cam, kd, 1)
    rgb = p["sh"][0:3].astype(np.float64) * scenes.Y00 + 0.5
    v = pr["vis"] == 1
    assert v.sum() > 50
    assert np.abs(pr["val"][v, 7:10] - np.clip(rgb[:, v].T, 0, None)).max() < 1e-7


# ------------------------------------------------------------------ EWA (Sec. 3.1, Zwicker et al.)
@pytest.mark.parametrize("s,z", [(0.05, 2.0), (0.01, 5.0), (0.2, 1.0)])
def test_ewa_isotropic_on_axis(orc, s, z):
    cam = axis_camera(128, 96)
    f = float(cam["fx"])
    p = manual_scene([[0.0], [0.0], [z]], [[math.log(s)]] * 3)
    pr = orc.project(p, cam, kd_trivial(), 1)
    var = (f * s / z) ** 2 + 0.3
    v = pr["val"][0]
    assert pr["vis"][0] == 1
    assert abs(v[0] - 64.0) < 1e-9 and abs(v[1] - 48.0) < 1e-9
    assert abs(v[2] * var - 1) < 1e-6 and abs(v[4] * var - 1) < 1e-6 and abs(v[3]) < 1e-12
    d = pr["dec32"][0]
    assert abs(d[2] * var - 1) < 1e-5 and abs(d[4] * var - 1) < 1e-5
    assert abs(v[10] - min(9.0, 2 * math.log(255 * sigmoid(2.0)))) < 1e-12


def test_ewa_isotropic_off_axis(orc):
    cam = axis_camera(128, 128)
    f = float(cam["fx"])
    s = 0.07
    X, Y, Z = (float(np.float32(v)) for v in (0.3, -0.2, 1.5))
    s = float(np.exp(np.float64(np.float32(math.log(s)))))
    p = manual_scene([[X], [Y], [Z]], [[math.log(s)]] * 3)
    pr = orc.project(p, cam, kd_trivial(), 1)
    J = np.array([[f / Z, 0, -f * X / Z ** 2], [0, f / Z, -f * Y / Z ** 2]])
    S2 = s * s * J @ J.T + 0.3 * np.eye(2)
    Cn = np.linalg.inv(S2)
    v = pr["val"][0]
    assert np.allclose([v[2], v[3], v[4]], [Cn[0, 0], Cn[0, 1], Cn[1, 1]], rtol=1e-6, atol=1e-12)
    assert abs(v[0] - (f * X / Z + 64)) < 1e-9 and abs(v[1] - (f * Y / Z + 64)) < 1e-9


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _quat_to_R(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_ewa_world_rotation_invariance(orc):
    """Rotating the whole world (Gaussians and camera) leaves the 2D result unchanged;
    catches transposed camera rotations and quaternion conventions."""
    rng = np.random.default_rng(5)
    p = scenes.scene_uniform(64, seed=6, D=0, mu_s=-3.0, extent=0.5)
    cam = scenes.orbit_camera(2.5, 0.7, 0.4, 96, 80)
    qr = rng.normal(size=4); qr /= np.linalg.norm(qr)
    Q = _quat_to_R(qr)
    p2 = dict(p)
    p2["means"] = (Q @ p["means"].astype(np.float64)).astype(np.float64)
    p2["quats"] = np.stack([_quat_mul(qr, p["quats"][:, i].astype(np.float64)) for i in range(64)], 1)
    cam2 = dict(cam)
    cam2["R"] = cam["R"].astype(np.float64) @ Q.T
    cam2["o"] = Q @ cam["o"].astype(np.float64)
    cam2["t"] = -(cam2["R"] @ cam2["o"])
    cam["t"] = -(cam["R"].astype(np.float64) @ cam["o"].astype(np.float64))
    kd = kd_trivial()
    a = orc.project(p, cam, kd, 1)
    b = orc.project(p2, cam2, kd, 1)
    v = a["vis"] == 1
    assert v.sum() > 20 and np.array_equal(a["vis"], b["vis"])
    assert np.allclose(a["val"][v, :7], b["val"][v, :7], rtol=1e-9, atol=1e-9)


def test_quaternion_sign_and_scale_invariance(orc):
    p = scenes.scene_uniform(50, seed=8, D=0, mu_s=-3.0, extent=0.5)
    cam = scenes.orbit_camera(2.5, 0.1, 0.3, 64, 64)
    kd = kd_trivial()
    a = orc.project(p, cam, kd, 1)
    for c in (-1.0, 2.5, -0.3):
        p2 = dict(p)
        p2["quats"] = (p["quats"].astype(np.float64) * c)
        b = orc.project(p2, cam, kd, 1)
        assert np.allclose(a["val"][:, :7], b["val"][:, :7], rtol=1e-10, atol=1e-12)


def test_isotropic_ignores_rotation(orc):
    p = scenes.scene_uniform(30, seed=9, D=0, mu_s=-3.0, extent=0.5)
    p["log_scales"] = np.repeat(p["log_scales"][:1], 3, 0)
    cam = scenes.orbit_camera(2.5, 0.1, 0.3, 64, 64)
    a = orc.project(p, cam, kd_trivial(), 1)
    p2 = dict(p)
    p2["quats"] = np.random.default_rng(1).normal(size=(4, 30))
    b = orc.project(p2, cam, kd_trivial(), 1)
    assert np.allclose(a["val"][:, 2:5], b["val"][:, 2:5], rtol=1e-9)


def test_culling_rules(orc):
    """Behind z_near, zero quaternion, alpha < 1/255: culled with count 0."""
    cam = axis_camera(64, 64)
    means = [[0.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0], [1.0, 0.05, 1.0, 1.0]]
    q = np.array([[1, 1, 0, 1], [0, 0, 0, 0], [0, 0, 0, 0], [0, 0, 0, 0]], np.float32)
    op = np.array([2.0, 2.0, 2.0, math.log(1 / 254.0) - 0.05], np.float32)  # last: alpha just below 1/255
    p = manual_scene(means, [[-3.0] * 4] * 3, quats=q, opacity=op)
    for mode in (0, 1):
        pr = orc.project(p, cam, kd_trivial(), mode)
        assert list(pr["vis"]) == [1, 0, 0, 0]
        assert list(pr["count"][1:]) == [0, 0, 0]


# ------------------------------------------------------------------ blending (Eq. 2) closed forms
def test_single_gaussian_closed_form(orc):
    cam = axis_camera(48, 48)
    f = float(cam["fx"])
    s, z, a = 0.02, 1.0, 1.0
    p = manual_scene([[0.0], [0.0], [z]], [[math.log(s)]] * 3, opacity=[a], rgb=[[0.9], [0.4], [0.1]])
    pr = orc.project(p, cam, kd_trivial(), 1)
    s = scale32(s)
    var = (f * s / z) ** 2 + 0.3
    alpha = sigmoid(a)
    tau = min(9.0, 2 * math.log(255 * alpha))
    pix = orc.all_pixels(48, 48)
    r = orc.render(pr, cam, kd_trivial(), np.zeros(1, np.int32), pix)
    for q, (x, y) in enumerate(pix):
        r2 = (x + 0.5 - 24) ** 2 + (y + 0.5 - 24) ** 2
        d2 = r2 / var
        sig = min(0.99, alpha * math.exp(-0.5 * d2)) if d2 <= tau else 0.0
        c = 0.5 + f32((0.9 - 0.5) / scenes.Y00) * scenes.Y00
        assert abs(r["img"][q, 0] - c * sig) < 1e-12
        assert abs(r["T"][q] - (1 - sig)) < 1e-12


def test_two_gaussians_closed_form(orc):
    cam = axis_camera(32, 32)
    f = float(cam["fx"])
    s1, z1, s2, z2 = 0.03, 1.0, 0.05, 1.6
    p = manual_scene([[0.0, 0.0], [0.0, 0.0], [z2, z1]], [[math.log(s2), math.log(s1)]] * 3,
                     opacity=[0.5, 1.5], rgb=[[0.2, 0.9], [0.5, 0.1], [0.8, 0.3]])
    pr = orc.project(p, cam, kd_trivial(), 1)
    pix = orc.all_pixels(32, 32)
    r = orc.render(pr, cam, kd_trivial(), np.zeros(1, np.int32), pix)
    for q, (x, y) in enumerate(pix):
        r2 = (x + 0.5 - 16) ** 2 + (y + 0.5 - 16) ** 2
        sig = []
        for s, z, op in ((s1, z1, 1.5), (s2, z2, 0.5)):   # front (z1) first
            s, z = scale32(s), f32(z)
            var = (f * s / z) ** 2 + 0.3
            al = sigmoid(op)
            tau = min(9.0, 2 * math.log(255 * al))
            sig.append(min(0.99, al * math.exp(-0.5 * r2 / var)) if r2 / var <= tau else 0.0)
        def col(v):
            return np.array([0.5 + f32((c - 0.5) / scenes.Y00) * scenes.Y00 for c in v])
        c1 = col([0.9, 0.1, 0.3]); c2 = col([0.2, 0.5, 0.8])
        C = c1 * sig[0] + c2 * sig[1] * (1 - sig[0])
        assert np.abs(r["img"][q] - C).max() < 1e-12
        assert abs(r["T"][q] - (1 - sig[0]) * (1 - sig[1])) < 1e-12


# ------------------------------------------------------------------ rectangles, cell sets (brute force)
def _tiny_scene(n=48, seed=0, D=3, mu_s=-2.2, extent=0.4):
    return scenes.scene_uniform(n, seed=seed, D=D, mu_s=mu_s, extent=extent)


def test_rect_conservative_brute_force(orc):
    p = _tiny_scene(120, seed=1)
    cam = scenes.orbit_camera(2.0, 0.4, 0.3, 40, 36)
    pr = orc.project(p, cam, kd_trivial(), 0)
    xs = np.arange(40) + 0.5
    ys = np.arange(36) + 0.5
    X, Y = np.meshgrid(xs, ys)
    checked = 0
    for i in np.nonzero(pr["vis"])[0]:
        mx, my, ca, cb, cc, tau = [float(v) for v in pr["dec32"][i, :6]]
        d2 = ca * (X - mx) ** 2 + 2 * cb * (X - mx) * (Y - my) + cc * (Y - my) ** 2
        inside = d2 <= tau * (1 + 2e-6)
        xl, xh, yl, yh = pr["rect"][i]
        rx = (X - 0.5 >= xl) & (X - 0.5 <= xh) & (Y - 0.5 >= yl) & (Y - 0.5 <= yh)
        assert not np.any(inside & ~rx), i
        checked += int(inside.sum())
    assert checked > 500


def test_rect_conservative_elongated(orc):
    """Needle-like footprints (s00 s11 / det up to ~10^6): the rectangle holds
    every pixel centre whose d^2 = ca (dx + k dy)^2 + e dy^2 (fp64 on the fp32
    decision values) is at most tau (1 + 2^-21 (1 + rk)), rk = sqrt(1 + k^2
    ca / e) -- the most the fp32 per-pixel test can accept."""
    rng = np.random.default_rng(5)
    n = 20000
    p = scenes.scene_uniform(n, seed=11, D=0, mu_s=-3.0, extent=0.6)
    ls = p["log_scales"].copy()
    ls[0] += rng.uniform(0, 4.0, n).astype(np.float32)
    ls[1] -= rng.uniform(0, 4.0, n).astype(np.float32)
    ls[2] -= rng.uniform(0, 4.0, n).astype(np.float32)
    p["log_scales"] = ls
    W, H = 640, 480
    cam = scenes.orbit_camera(1.6, 0.4, 0.3, W, H, z_near=0.05)
    pr = orc.project(p, cam, kd_trivial(), 0)
    n_checked = 0
    kmax = 0.0
    for i in np.nonzero(pr["vis"])[0]:
        mx, my, ca, tau, k, e = [float(pr["dec32"][i, c]) for c in (0, 1, 2, 5, 8, 9)]
        xl, xh, yl, yh = [int(v) for v in pr["rect"][i]]
        rk = math.sqrt(1 + k * k * ca / e)
        kmax = max(kmax, rk * rk)
        if rk < 30:  # rounding margins below the rectangle's fixed padding
            continue
        x0, x1, y0, y1 = max(xl - 3, 0), min(xh + 3, W - 1), max(yl - 3, 0), min(yh + 3, H - 1)
        X, Y = np.meshgrid(np.arange(x0, x1 + 1) + 0.5, np.arange(y0, y1 + 1) + 0.5)
        dx, dy = X - mx, Y - my
        q = ca * (dx + k * dy) ** 2 + e * dy * dy
        inside = q <= tau * (1 + 2.0 ** -21 * (1 + rk))
        in_rect = (X - 0.5 >= xl) & (X - 0.5 <= xh) & (Y - 0.5 >= yl) & (Y - 0.5 <= yh)
        assert not np.any(inside & ~in_rect), i
        n_checked += int(inside.sum())
    assert kmax > 1e5 and n_checked > 10**4


@pytest.mark.parametrize("mode", [0, 1])
def test_rect_boundary_sample_included(orc, mode):
    """A sample exactly on the ellipse's extreme x (d^2 = tau) lies in the rectangle."""
    z = 2.0
    for s in (0.01, 0.03, 0.05):
        p = manual_scene([[0.0], [0.0], [z]], [[math.log(s)]] * 3)
        base = axis_camera(96, 64)
        f = float(base["fx"])
        s_ = scale32(s)
        var = (f * s_ / f32(z)) ** 2 + 0.3
        tau = min(9.0, 2 * math.log(255 * sigmoid(2.0)))
        e = math.sqrt(tau * var)
        xs = 70
        base["cx"] = np.float32(xs + 0.5 - e)   # the Gaussian sits at x = cx
        pr = orc.project(p, base, kd_trivial(), mode)
        assert pr["vis"][0] == 1
        assert pr["rect"][0, 1] >= xs


def _random_footprints(rng, n, W, H):
    """Decision-path footprints (fp32 conic, tau, rectangle as the projection
    pads it) from random screen covariances, aspect ratios up to 10^4."""
    lam1 = np.exp(rng.uniform(np.log(0.3), np.log(3000.0), n))
    lam2 = lam1 / np.exp(rng.uniform(0.0, np.log(1e4), n))
    lam2 = np.maximum(lam2, 0.3)
    th = rng.uniform(0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    s00 = (c * c * lam1 + s * s * lam2).astype(np.float32)
    s01 = (c * s * (lam1 - lam2)).astype(np.float32)
    s11 = (s * s * lam1 + c * c * lam2).astype(np.float32)
    s00_, s01_, s11_ = s00.astype(np.float64), s01.astype(np.float64), s11.astype(np.float64)
    det64 = s00_ * s11_ - s01_ * s01_
    det = det64.astype(np.float32)
    ca, cb, cc = (s11_ / det64).astype(np.float32), (-s01_ / det64).astype(np.float32), (s00_ / det64).astype(np.float32)
    kk, ee = (-s01_ / s11_).astype(np.float32), (1.0 / s11_).astype(np.float32)
    tau = rng.uniform(0.05, 9.0, n).astype(np.float32)
    mx = rng.uniform(-30, W + 30, n).astype(np.float32)
    my = rng.uniform(-30, H + 30, n).astype(np.float32)
    ex = np.sqrt(tau * s00) * np.float32(1.00001) + np.float32(1e-3)
    ey = np.sqrt(tau * s11) * np.float32(1.00001) + np.float32(1e-3)
    xl = np.maximum(np.ceil(mx - ex - 0.5), 0); xh = np.minimum(np.floor(mx + ex - 0.5), W - 1)
    yl = np.maximum(np.ceil(my - ey - 0.5), 0); yh = np.minimum(np.floor(my + ey - 0.5), H - 1)
    ok = (xl <= xh) & (yl <= yh) & (det > 0)
    dec = np.zeros((n, 10), np.float32)
    dec[:, 0], dec[:, 1], dec[:, 2], dec[:, 3], dec[:, 4], dec[:, 5] = mx, my, ca, cb, cc, tau
    dec[:, 6] = rng.uniform(1, 10, n)
    dec[:, 8], dec[:, 9] = kk, ee
    rect = np.stack([xl, xh, yl, yh], 1).astype(np.int32)
    return dec[ok], rect[ok]


def test_tile_spans_conservative_and_tight(orc):
    """Row spans of the instance lists: every pixel centre of the rectangle
    within the ellipse d^2 = ca (dx + k dy)^2 + e dy^2 <= tau, enlarged to
    tau (1 + 2^-20 (1 + rk)) (twice what fp32 rounding of the per-pixel test
    can accept), lies in a listed tile, and every listed tile comes within
    0.1 px of the ellipse."""
    rng = np.random.default_rng(7)
    W = H = 256
    dec, rect = _random_footprints(rng, 3000, W, H)
    n = len(dec)
    pr = dict(n=n, dec32=dec, rect=rect, vis=np.ones(n, np.uint8), cellmask=np.ones(n, np.uint64),
              count=np.full(n, 10**6, np.uint32))
    keys, gids = orc.bins(pr, np.zeros(1, np.int32), 0, W // 16)
    kept = {}
    for k, g in zip(keys.tolist(), gids.tolist()):
        kept.setdefault(g, set()).add(k)
    n_pix = n_tiles = n_rect_tiles = n_elong = 0
    for i in range(n):
        mx, my, ca, tau, k, e = [float(dec[i, c]) for c in (0, 1, 2, 5, 8, 9)]
        cb, cc = k * ca, e + k * k * ca
        rk = math.sqrt(1 + k * k * ca / e)
        xl, xh, yl, yh = [int(v) for v in rect[i]]
        X, Y = np.meshgrid(np.arange(xl, xh + 1) + 0.5, np.arange(yl, yh + 1) + 0.5)
        dx, dy = X - mx, Y - my
        q = ca * (dx + k * dy) ** 2 + e * dy * dy
        inside = q <= tau * (1 + 2.0 ** -20 * (1 + rk))
        tiles = set(((Y[inside].astype(int) >> 4) * (W // 16) + (X[inside].astype(int) >> 4)).tolist())
        got = kept.get(i, set())
        assert tiles <= got, i
        n_pix += int(inside.sum())
        n_rect_tiles += ((xh >> 4) - (xl >> 4) + 1) * ((yh >> 4) - (yl >> 4) + 1)
        n_tiles += len(got)
        n_elong += rk > 10
        for t in got:
            ty, tx = divmod(t, W // 16)
            assert (xl >> 4) <= tx <= (xh >> 4) and (yl >> 4) <= ty <= (yh >> 4)
            # minimum of q over the tile's pixel-centre box inside the rectangle, grown by 0.1 px
            bx0 = max(tx * 16, xl) + 0.4 - mx; bx1 = min(tx * 16 + 15, xh) + 0.6 - mx
            by0 = max(ty * 16, yl) + 0.4 - my; by1 = min(ty * 16 + 15, yh) + 0.6 - my
            if bx0 <= 0 <= bx1 and by0 <= 0 <= by1:
                continue
            qm = math.inf
            for ex in (bx0, bx1):
                ey = min(max(-cb * ex / cc, by0), by1)
                qm = min(qm, ca * ex * ex + 2 * cb * ex * ey + cc * ey * ey)
            for ey in (by0, by1):
                ex = min(max(-cb * ey / ca, bx0), bx1)
                qm = min(qm, ca * ex * ex + 2 * cb * ex * ey + cc * ey * ey)
            assert qm <= tau * (1 + 1e-3), (i, t)
    assert n_pix > 10**5 and n_elong > 10
    assert n_tiles < 0.9 * n_rect_tiles  # the spans drop tiles the rectangle holds


def test_instance_count_matches_lists(orc):
    """count (cells x span tiles) sums to the length of the instance lists."""
    p = _tiny_scene(300, seed=3, mu_s=-2.0)
    kd = orc.kd_partition(p["means"], p["log_scales"], 2)
    cam = scenes.orbit_camera(2.0, 0.7, 0.2, 96, 80)
    order, rank_of = orc.cell_order(2, kd["split"], cam["o"])
    pr = orc.project(p, cam, kd, 0)
    keys, gids = orc.bins(pr, rank_of, 2, (96 + 15) // 16)
    assert len(keys) == int(pr["count"].astype(np.int64).sum()) > 1000
    per = np.bincount(gids.astype(np.int64), minlength=pr["n"])
    assert np.array_equal(per, pr["count"].astype(np.int64))


@pytest.mark.parametrize("mode", [0, 1])
def test_cell_sets_conservative(orc, mode):
    """Keeping each Gaussian only in its emitted cells changes no partial."""
    p = _tiny_scene(200, seed=2, mu_s=-2.0)
    kd = orc.kd_partition(p["means"], p["log_scales"], 3)
    for k, cam in enumerate([scenes.orbit_camera(2.0, 0.4 + k, 0.3 * k - 0.2, 48, 40) for k in range(3)]):
        order, _ = orc.cell_order(3, kd["split"], cam["o"])
        pr = orc.project(p, cam, kd, mode)
        pix = orc.all_pixels(48, 40)
        a = orc.render(pr, cam, kd, order, pix)
        b = orc.render(pr, cam, kd, order, pix, restrict=True)
        assert np.array_equal(a["partC"], b["partC"]) and np.array_equal(a["partT"], b["partT"])
        assert (np.count_nonzero(pr["cellmask"] & (pr["cellmask"] - np.uint64(1)))) > 5  # multi-cell Gaussians exist


# ------------------------------------------------------------------ KD tree (Sec. 3.3)
def test_kd_order_statistics_and_balance(orc):
    rng = np.random.default_rng(4)
    n = 1001
    means = rng.normal(size=(3, n)).astype(np.float32)
    ls = np.full((3, n), -3.0, np.float32)
    kd = orc.kd_partition(means, ls, 3)
    # root: floor(n/2)-th smallest x
    assert kd["split"][0] == np.sort(means[0])[n // 2]
    left = means[0] < kd["split"][0]
    assert left.sum() == n // 2
    assert kd["split"][1] == np.sort(means[1, left])[left.sum() // 2]
    assert kd["split"][2] == np.sort(means[1, ~left])[(~left).sum() // 2]
    assert sorted(kd["counts"].tolist()) == sorted([125, 125, 125, 125, 125, 125, 125, 126])
    # every centre lies in its (half-open) leaf box
    cc = kd["center_cell"]
    for a in range(3):
        assert np.all(means[a] >= kd["box_lo"][a, cc]) and np.all(means[a] < kd["box_hi"][a, cc])
    assert np.array_equal(np.bincount(cc, minlength=8), kd["counts"])


def test_kd_config1_counts(orc):
    p, cam, _, L = scenes.config1()
    kd = orc.kd_partition(p["means"], p["log_scales"], L)
    assert kd["counts"].tolist() == [5000] * 4


def test_kd_ties_go_right(orc):
    """A ground plane under a Z split: equal coordinates all go to the right child."""
    n = 64
    means = np.zeros((3, n), np.float32)
    means[0] = np.arange(n)
    means[1] = np.arange(n)[::-1]
    means[2, : n // 4] = 1.0
    kd = orc.kd_partition(means, np.full((3, n), -3.0, np.float32), 3)
    # level 2 (axis Z) nodes: most members at z = 0, so the median is 0 and all z = 0 go right
    for nd in range(3, 7):
        assert kd["axis"][nd] == 2
    cc = kd["center_cell"]
    assert np.all(cc[means[2] == 0.0] % 2 == 1)


def test_paper_subsets_brute_force(orc):
    """N_k = { i : centre within the leaf box inflated by D_i = 3 max scale } (Sec. 3.3)."""
    p = scenes.scene_uniform(500, seed=11, D=0, mu_s=-2.5)
    kd = orc.kd_partition(p["means"], p["log_scales"], 3, 3.0)
    D = 3.0 * np.exp(p["log_scales"].astype(np.float64)).max(0)
    K = 8
    for i in range(500):
        for k in range(K):
            inside = True
            for a in range(3):
                u = float(p["means"][a, i])
                if kd["box_lo"][a, k] - u > D[i] * (1 + 1e-6) or u - kd["box_hi"][a, k] > D[i] * (1 + 1e-6):
                    inside = False
            bit = bool((kd["own_mask"][i, 0] >> k) & 1)
            if bit != inside:
                # only fp32-vs-fp64 ties at the margin may disagree
                margin = min(abs(kd["box_lo"][a, k] - float(p["means"][a, i]) - D[i]) for a in range(3))
                assert margin < 1e-5
    # every Gaussian owned by its centre cell
    own = kd["own_mask"][:, 0]
    assert np.all((own >> kd["center_cell"].astype(np.uint32)) & 1)


# ------------------------------------------------------------------ merge order o_l (Eq. 5)
def _ray_box_entry(o, d, lo, hi):
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if abs(d[a]) < 1e-300:
            if not (lo[a] <= o[a] <= hi[a]):
                return None
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
    return t0 if t0 < t1 else None


def test_cell_order_matches_ray_box_entry(orc):
    rng = np.random.default_rng(12)
    means = rng.normal(size=(3, 400)).astype(np.float32)
    kd = orc.kd_partition(means, np.full((3, 400), -3.0, np.float32), 4)
    lo, hi = kd["box_lo"].astype(np.float64), kd["box_hi"].astype(np.float64)
    for _ in range(20):
        o = rng.normal(size=3) * 1.5
        order, rank_of = orc.cell_order(4, kd["split"], o)
        for _ in range(30):
            d = rng.normal(size=3)
            ent = [(t, k) for k in range(16) if (t := _ray_box_entry(o, d, lo[:, k], hi[:, k])) is not None]
            by_t = [k for t, k in sorted(ent)]
            by_pi = sorted([k for _, k in ent], key=lambda k: rank_of[k])
            assert by_t == by_pi


# ------------------------------------------------------------------ equivalence (Eq. 5, appendix)
@pytest.mark.parametrize("L", [1, 2, 3])
def test_merged_equals_plain_exact64(orc, L):
    p = _tiny_scene(300, seed=20 + L, mu_s=-2.4, extent=0.6)
    kd = orc.kd_partition(p["means"], p["log_scales"], L)
    for v in range(2):
        cam = scenes.orbit_camera(2.2, 1.0 + 2 * v, 0.5 - 0.6 * v, 64, 48)
        order, _ = orc.cell_order(L, kd["split"], cam["o"])
        pr = orc.project(p, cam, kd, 1)
        r = orc.render(pr, cam, kd, order, orc.all_pixels(64, 48), 0.0)
        assert r["ncon"].max() > 10
        assert np.abs(r["img"] - r["plain"]).max() < 1e-12
        assert np.abs(r["T"] - r["plainT"]).max() < 1e-12


def test_merged_equals_plain_mirror32_config1(orc):
    p, cam, _, L = scenes.config1()
    kd = orc.kd_partition(p["means"], p["log_scales"], L)
    order, _ = orc.cell_order(L, kd["split"], cam["o"])
    pr = orc.project(p, cam, kd, 0)
    pix = orc.all_pixels(256, 256)[::7]
    r = orc.render(pr, cam, kd, order, pix, 0.0)
    assert np.abs(r["img"] - r["plain"]).max() < 1e-12


def test_mirror32_decisions_match_exact64(orc):
    """The fp32 decision path (factored quadratic form, fp64 covariance chain)
    against the exact64 one on anisotropic, rotated Gaussians: the per-pixel
    contributor sets may differ only where d^2 is within rounding of tau, so
    the images agree to within a few boundary contributions (sigma ~ 1/255)."""
    rng = np.random.default_rng(21)
    n = 400
    p = scenes.scene_uniform(n, seed=22, D=0, mu_s=-2.6, extent=0.5)
    ls = p["log_scales"].copy()
    ls[0] += rng.uniform(0, 2.5, n).astype(np.float32)
    ls[1] -= rng.uniform(0, 2.5, n).astype(np.float32)
    p["log_scales"] = ls
    q = rng.normal(size=(4, n)).astype(np.float32)
    p["quats"] = q
    cam = scenes.orbit_camera(2.0, 0.5, 0.35, 96, 80)
    kd = kd_trivial()
    order = np.zeros(1, np.int32)
    pix = orc.all_pixels(96, 80)
    a = orc.render(orc.project(p, cam, kd, 0), cam, kd, order, pix, 0.0)
    b = orc.render(orc.project(p, cam, kd, 1), cam, kd, order, pix, 0.0)
    d = np.abs(a["img"] - b["img"])
    assert np.count_nonzero(a["ncon"]) > 0.8 * len(pix)
    assert d.max() < 0.02 and np.mean(d > 1e-6) < 0.01


def test_k1_is_identity(orc):
    p = _tiny_scene(100, seed=30)
    cam = scenes.orbit_camera(2.0, 0.2, 0.3, 32, 32)
    pr = orc.project(p, cam, kd_trivial(), 1)
    r = orc.render(pr, cam, kd_trivial(), np.zeros(1, np.int32), orc.all_pixels(32, 32), 0.0)
    assert np.array_equal(r["partC"][:, 0], r["plain"]) or np.abs(r["partC"][:, 0] - r["plain"]).max() < 1e-15
    assert np.abs(r["partT"][:, 0] - r["plainT"]).max() < 1e-15


def test_merge_operator_associative(orc):
    """(C, T) o (C', T') = (C + T C', T T') is associative; pre-merging KD subtrees
    (contiguous in every cell order) gives the same image."""
    p = _tiny_scene(300, seed=31, mu_s=-2.4, extent=0.6)
    kd = orc.kd_partition(p["means"], p["log_scales"], 3)
    cam = scenes.orbit_camera(2.2, 0.8, 0.4, 40, 40)
    order, _ = orc.cell_order(3, kd["split"], cam["o"])
    pr = orc.project(p, cam, kd, 1)
    r = orc.render(pr, cam, kd, order, orc.all_pixels(40, 40), 0.0)

    def op(a, b):
        return (a[0] + a[1][:, None] * b[0], a[1] * b[1])

    parts = [(r["partC"][:, k], r["partT"][:, k]) for k in order]
    left = parts[0]
    for q in parts[1:]:
        left = op(left, q)
    pairs = [op(parts[2 * i], parts[2 * i + 1]) for i in range(4)]
    tree = op(op(pairs[0], pairs[1]), op(pairs[2], pairs[3]))
    assert np.abs(left[0] - tree[0]).max() < 1e-14 and np.abs(left[1] - tree[1]).max() < 1e-14
    assert np.abs(left[0] - r["img"]).max() < 1e-14


def test_validity_camera_on_split_plane(orc):
    """Sec. 4.2: with the optical axis on the dividing plane, each half of the
    image is rendered by one side only: the far cell's partial is exactly C = 0,
    T = 1, including for Gaussians that straddle the plane."""
    p = _tiny_scene(400, seed=40, mu_s=-2.3, extent=0.5)
    kd = orc.kd_partition(p["means"], p["log_scales"], 1)
    s = float(kd["split"][0])
    cam = scenes.with_kd_axis_aligned_camera(s, 64, 48, dist=2.0)
    order, _ = orc.cell_order(1, kd["split"], cam["o"])
    for mode in (0, 1):
        pr = orc.project(p, cam, kd, mode)
        straddle = (pr["cellmask"] == 3).sum()
        assert straddle > 5
        pix = orc.all_pixels(64, 48)
        r = orc.render(pr, cam, kd, order, pix, 0.0)
        left_px = pix[:, 0] < 32
        # x(p) = o + z D(p), D_x(p) = (u - cx)/fx: left half -> x < s -> cell 0
        assert np.all(r["partC"][left_px, 1] == 0.0) and np.all(r["partT"][left_px, 1] == 1.0)
        assert np.all(r["partC"][~left_px, 0] == 0.0) and np.all(r["partT"][~left_px, 0] == 1.0)
        assert r["partC"][left_px, 0].max() > 0.1 and r["partC"][~left_px, 1].max() > 0.1


def test_early_termination_include_then_stop(orc):
    """With eps_T, each cell includes the contributor that drops T_k below eps_T and
    stops there; the tail changes the image by at most eps_T per cell."""
    p = _tiny_scene(300, seed=41, mu_s=-2.0, extent=0.3)
    p["opacity"][:] = 4.0
    kd = orc.kd_partition(p["means"], p["log_scales"], 2)
    cam = scenes.orbit_camera(1.6, 0.3, 0.2, 32, 32)
    order, _ = orc.cell_order(2, kd["split"], cam["o"])
    pr = orc.project(p, cam, kd, 1)
    pix = orc.all_pixels(32, 32)
    a = orc.render(pr, cam, kd, order, pix, 0.0)
    b = orc.render(pr, cam, kd, order, pix, 1e-2)
    assert np.any(a["partT"] < 1e-2)
    stopped = b["partT"] < 1e-2
    assert np.all(b["partT"][stopped] >= a["partT"][stopped])
    assert np.abs(a["img"] - b["img"]).max() <= 4 * 1e-2 * 1.0 + 1e-12


# ------------------------------------------------------------------ finite differences (backward)
def _fd_check(f, x, g, idx, tol=2e-4):
    bad = []
    skipped = 0
    for i in idx:
        xi = float(x.flat[i])
        h = 1e-6 * max(1.0, abs(xi))
        vals = []
        for hh in (h, h / 4):
            x.flat[i] = xi + hh; fp = f()
            x.flat[i] = xi - hh; fm = f()
            vals.append((fp - fm) / (2 * hh))
        x.flat[i] = xi
        scale = 1e-3 + abs(vals[0])
        if abs(vals[0] - vals[1]) > 1e-3 * scale:
            skipped += 1   # a decision flipped inside the stencil: not differentiable there
            continue
        if abs(vals[0] - g.flat[i]) > tol * (abs(vals[0]) + 1e-2):
            bad.append((i, vals[0], g.flat[i]))
    return bad, skipped


def test_render_bwd_fd_2d(orc):
    """Gradient of the merged render w.r.t. the 2D quantities (mean, conic, alpha,
    colour) against central differences, exact64 decisions, no early stop."""
    p = _tiny_scene(24, seed=50, mu_s=-1.9, extent=0.25)
    kd = orc.kd_partition(p["means"], p["log_scales"], 2)
    cam = scenes.orbit_camera(1.6, 0.3, 0.35, 24, 24, bg=(0.3, 0.6, 0.9))
    order, _ = orc.cell_order(2, kd["split"], cam["o"])
    pr = orc.project(p, cam, kd, 1)
    pix = orc.all_pixels(24, 24)
    rng = np.random.default_rng(51)
    w = rng.normal(size=(len(pix), 3))
    wT = rng.normal(size=len(pix))
    g2d = orc.render_bwd(pr, cam, kd, order, pix, w, wT)
    val = pr["val"]

    def f():
        r = orc.render(pr, cam, kd, order, pix, 0.0)
        return float((w * r["img"]).sum() + (wT * r["T"]).sum())

    vis = np.nonzero(pr["vis"])[0]
    cols = [0, 1, 2, 3, 4, 5, 7, 8, 9]   # val columns for g2d rows 0..8
    G = np.zeros_like(val)
    for c_g, c_v in enumerate(cols):
        G[:, c_v] = g2d[:, c_g]
    idx = [i * 12 + c for i in vis for c in cols]
    bad, skipped = _fd_check(f, val, G, idx, tol=5e-4)
    assert skipped < len(idx) // 10
    assert not bad, bad[:5]


def test_full_backward_fd_params(orc):
    """Gradient of sum(w * merged image) w.r.t. every parameter (means, log-scales,
    quaternions, opacity, SH degree 3) against central differences of the exact64
    forward, with the KD tree held fixed."""
    p = _tiny_scene(16, seed=60, mu_s=-1.9, extent=0.25)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        p[k] = p[k].astype(np.float64)
    kd = orc.kd_partition(p["means"], p["log_scales"], 2)
    cam = scenes.orbit_camera(1.5, 0.9, 0.3, 24, 24, bg=(0.7, 0.2, 0.5))
    order, _ = orc.cell_order(2, kd["split"], cam["o"])
    pix = orc.all_pixels(24, 24)
    rng = np.random.default_rng(61)
    w = rng.normal(size=(len(pix), 3))
    pr = orc.project(p, cam, kd, 1)
    g2d = orc.render_bwd(pr, cam, kd, order, pix, w, None)
    g = orc.project_bwd(p, cam, pr, g2d)

    def f():
        pr2 = orc.project(p, cam, kd, 1)
        r = orc.render(pr2, cam, kd, order, pix, 0.0)
        return float((w * r["img"]).sum())

    vis = np.nonzero(pr["vis"])[0]
    assert len(vis) >= 10
    total_skipped = 0
    for k, rows in (("means", 3), ("log_scales", 3), ("quats", 4), ("opacity", 1), ("sh", 48)):
        x = p[k]
        n = 16
        idx = [r * n + i for r in range(rows) for i in vis] if x.ndim == 2 else list(vis)
        bad, skipped = _fd_check(f, x, g[k], idx, tol=5e-4)
        total_skipped += skipped
        assert not bad, (k, bad[:5])
    assert total_skipped < 40


# ------------------------------------------------------------------ loss
def test_l1_closed_form(orc):
    rng = np.random.default_rng(70)
    x = rng.uniform(size=(3, 9, 7)); y = rng.uniform(size=(3, 9, 7))
    l, d = orc.loss(x, y, 0.0)
    assert abs(l - np.abs(x - y).mean()) < 1e-14
    assert np.array_equal(d, np.sign(x - y) / x.size)


def test_ssim_identity(orc):
    rng = np.random.default_rng(71)
    x = rng.uniform(size=(3, 20, 17))
    l, d = orc.loss(x, x.copy(), 0.2)
    assert abs(l) < 1e-14 and np.abs(d).max() < 1e-12


def test_ssim_constant_images_closed_form(orc):
    """Constant images a, b with zero padding: each pixel's window mass w(p) gives
    mu = a w, E[x^2] = a^2 w, E[xy] = a b w in closed form."""
    H, W, a, b = 13, 16, 0.6, 0.25
    g = np.exp(-((np.arange(11) - 5) ** 2) / (2 * 1.5 ** 2)); g /= g.sum()
    def mass1(n):
        return np.array([sum(g[k + 5 - i] for k in range(n) if 0 <= k + 5 - i < 11) for i in range(n)])
    wmap = np.outer(mass1(H), mass1(W))
    C1, C2 = 1e-4, 9e-4
    mx, my = a * wmap, b * wmap
    sxx, syy, sxy = a * a * wmap - mx ** 2, b * b * wmap - my ** 2, a * b * wmap - mx * my
    S = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx ** 2 + my ** 2 + C1) * (sxx + syy + C2))
    x = np.full((3, H, W), a); y = np.full((3, H, W), b)
    l, _ = orc.loss(x, y, 0.2)
    assert abs(l - (abs(a - b) + 0.2 * (1 - S.mean()))) < 1e-13


def test_loss_gradient_fd(orc):
    rng = np.random.default_rng(72)
    x = rng.uniform(size=(3, 12, 14)); y = rng.uniform(size=(3, 12, 14))
    _, d = orc.loss(x, y, 0.2)
    h = 1e-6
    for i in rng.choice(x.size, 60, replace=False):
        xi = x.flat[i]
        x.flat[i] = xi + h; lp, _ = orc.loss(x, y, 0.2)
        x.flat[i] = xi - h; lm, _ = orc.loss(x, y, 0.2)
        x.flat[i] = xi
        assert abs((lp - lm) / (2 * h) - d.flat[i]) < 1e-7
