"""Edge cases and full-size sampled parity on the GPU.

Edge cases: no Gaussians; every Gaussian culled; one screen-filling Gaussian;
many centres exactly on KD split planes.  Full size: the benchmark's own
workload (1M Gaussians, 1600x1060, K = 8, SH 3) in the same launch
configuration, checked against the oracle on a seeded sample of pixels
(image, partial maps) and on a sample of Gaussians (gradients of a seeded
linear objective, with the oracle run over every pixel of their rectangles);
the loss at full resolution on seeded images.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import device_params, gpu_partials_dense, grad_close, log, proj_bin
from paper_2406_11836_amd import raster, scenes

pytestmark = pytest.mark.gpu
EPS_T = 5e-5


@pytest.fixture(scope="module")
def rast():
    return raster.Rasterizer()


def test_no_gaussians(rast):
    p = scenes.scene_uniform(0, seed=1, D=1)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 2)
    cam = scenes.orbit_camera(3.0, 0.2, 0.3, 70, 50, bg=(0.25, 0.5, 0.75))
    st = rast.forward(dp, kd, [cam], EPS_T)
    img = st.image.view(3, 50, 70).cpu().numpy()
    assert np.all(img[0] == np.float32(0.25)) and np.all(img[1] == 0.5) and np.all(img[2] == 0.75)
    assert torch.all(st.T_final == 1.0)
    g = rast.backward(st, dp, torch.ones_like(st.image))
    assert g["means"].numel() == 0


def test_everything_culled(rast):
    """Camera looking away from the scene: no instance, image = background, zero gradients."""
    p = scenes.scene_uniform(5000, seed=2, D=2)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 3)
    eye = np.array([5.0, 0.0, 0.0])
    cam = scenes.make_camera(scenes.look_at(eye, eye + np.array([1.0, 0.0, 0.0])), eye, 64, 48, bg=(0.1, 0.1, 0.1))
    st = rast.forward(dp, kd, [cam], EPS_T)
    assert st.bins_struct.n_instances == 0
    assert torch.all(st.T_final == 1.0)
    g = rast.backward(st, dp, torch.ones_like(st.image))
    for k in raster.PARAM_KEYS:
        assert torch.count_nonzero(g[k]) == 0, k


def test_screen_filling_gaussian(rast):
    """One Gaussian covering the whole image plus a few small ones, K = 4."""
    p = scenes.scene_uniform(64, seed=3, D=0, mu_s=-3.0, extent=0.3)
    p["means"][:, 0] = 0.0
    p["log_scales"][:, 0] = np.log(2.0)
    p["opacity"][0] = 3.0
    dp = device_params(p)
    kd = rast.kd_partition(dp, 2)
    cam = scenes.orbit_camera(2.0, 0.4, 0.2, 96, 80, z_near=0.1)
    st = rast.forward(dp, kd, [cam], EPS_T)
    okd = oracle.kd_partition(p["means"], p["log_scales"], 2)
    order, _ = oracle.cell_order(2, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    assert pr["count"][0] >= 30 * 4 / 4  # spans every tile
    r = oracle.render(pr, cam, okd, order, oracle.all_pixels(96, 80), EPS_T)
    img = st.image.cpu().numpy().reshape(3, -1).T
    assert np.abs(img - r["img"]).max() <= 2e-4


def test_single_tile_one_cell(rast):
    """A 16x16 image and L = 0: the (tile, cell) key has no bits, so no sort
    pass runs; the instances stay in emission order and the image matches."""
    p = scenes.scene_uniform(400, seed=11, D=1, mu_s=-2.5, extent=0.5)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 0)
    cam = scenes.orbit_camera(2.0, 0.3, 0.2, 16, 16)
    st = rast.forward(dp, kd, [cam], EPS_T)
    n_inst = st.bins_struct.n_instances
    assert n_inst == 400
    vals = st.bins["vals"][:n_inst].cpu().numpy().view(np.uint64)
    assert np.array_equal(vals & np.uint64(0xffffffff), np.arange(n_inst, dtype=np.uint64))
    okd = oracle.kd_partition(p["means"], p["log_scales"], 0)
    order, _ = oracle.cell_order(0, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    r = oracle.render(pr, cam, okd, order, oracle.all_pixels(16, 16), EPS_T)
    img = st.image.cpu().numpy().reshape(3, -1).T
    assert np.abs(img - r["img"]).max() <= 2e-4


@pytest.mark.parametrize("L", [0, 2])
def test_stacked_opaque_exact_mode(rast, L):
    """40 nearly opaque Gaussians (alpha 0.98) stacked on one line of sight and
    rendered with eps_T = 0: without a floor the transmittance would underflow
    fp32 after about 25 layers.  Both sides stop a pixel once T_k < 2^-100;
    image and the 2D gradients (which the backward recovers by dividing back
    from the stored T_k) match the oracle."""
    n = 40
    rng = np.random.default_rng(17)
    means = np.stack([rng.uniform(-0.03, 0.03, n), rng.uniform(-0.03, 0.03, n), 2.0 + 0.05 * np.arange(n)])
    p = scenes.scene_uniform(n, seed=18, D=1, mu_s=np.log(0.15), extent=0.1)
    p["means"] = means.astype(np.float32)
    # slightly anisotropic, so that the rotation gradient is not identically
    # zero (an isotropic covariance does not depend on the quaternion)
    p["log_scales"] = np.log(np.array([[0.15], [0.12], [0.10]]) * np.ones((3, n))).astype(np.float32)
    p["opacity"] = np.full(n, np.log(0.98 / 0.02), np.float32)
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 64, 64, z_near=0.1, bg=(0.2, 0.4, 0.6))
    dp = device_params(p)
    kd = rast.kd_partition(dp, L)
    st = rast.forward(dp, kd, [cam], 0.0)
    rng2 = np.random.default_rng(19)
    dimg = rng2.normal(size=(3, 64 * 64)).astype(np.float32)
    dTf = rng2.normal(size=64 * 64).astype(np.float32)
    g = rast.backward(st, dp, torch.from_numpy(dimg.ravel()).cuda(), torch.from_numpy(dTf).cuda())
    torch.cuda.synchronize()
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    order, _ = oracle.cell_order(L, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    pix = oracle.all_pixels(64, 64)
    r = oracle.render(pr, cam, okd, order, pix, 0.0)
    assert r["ncon"].max() == n
    assert r["T"].min() < 1e-30 and r["T"].min() > 0.0
    img = st.image.cpu().numpy().reshape(3, -1).T
    assert np.abs(img - r["img"]).max() <= 2e-4
    g2d = oracle.render_bwd(pr, cam, okd, order, pix, dimg.T.astype(np.float64), dTf.astype(np.float64), 0.0)
    dproj = g["_dproj"][: 9 * n].view(9, n).cpu().numpy().T
    for c in range(9):
        ok, info = grad_close(dproj[:, c], g2d[:, c], 1e-3, "stacked d_proj row %d" % c)
        log(str(info))
        assert ok, info
    og = oracle.project_bwd(p, cam, pr, g2d)
    for k in raster.PARAM_KEYS:
        ok, info = grad_close(g[k].cpu().numpy(), og[k], 1e-3, k)
        assert ok, info


def test_centres_on_split_planes(rast):
    """Many centres share coordinates, so split values coincide with centres and
    with each other; bit-exact tree and parity of the image."""
    rng = np.random.default_rng(4)
    n = 3000
    p = scenes.scene_uniform(n, seed=5, D=1, mu_s=-3.5, extent=0.5)
    grid = np.round(p["means"] * 4) / 4          # coordinates on a 0.25 grid
    p["means"] = grid.astype(np.float32)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 3)
    okd = oracle.kd_partition(p["means"], p["log_scales"], 3)
    assert np.array_equal(kd.split.cpu().numpy()[:7].view(np.uint32), okd["split"].view(np.uint32))
    assert np.array_equal(kd.center_cell.cpu().numpy(), okd["center_cell"])
    on_plane = np.isin(p["means"][0], okd["split"][:1]).sum()
    assert on_plane > 10
    cam = scenes.orbit_camera(2.2, 0.7, 0.35, 120, 90)
    st = rast.forward(dp, kd, [cam], EPS_T)
    order, _ = oracle.cell_order(3, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    r = oracle.render(pr, cam, okd, order, oracle.all_pixels(120, 90), EPS_T)
    assert np.abs(st.image.cpu().numpy().reshape(3, -1).T - r["img"]).max() <= 2e-4


@pytest.fixture(scope="module")
def needles(rast):
    """6000 strongly elongated Gaussians (s00 s11 / det up to ~10^6), SH 1."""
    rng = np.random.default_rng(5)
    n = 6000
    p = scenes.scene_uniform(n, seed=11, D=1, mu_s=-3.0, extent=0.6)
    ls = p["log_scales"].copy()
    ls[0] += rng.uniform(0, 4.0, n).astype(np.float32)
    ls[1] -= rng.uniform(0, 4.0, n).astype(np.float32)
    ls[2] -= rng.uniform(0, 4.0, n).astype(np.float32)
    p["log_scales"] = ls
    W, H, L = 320, 240, 2
    cam = scenes.orbit_camera(1.6, 0.4, 0.3, W, H, z_near=0.05)
    log("needles: GPU forward")
    dp = device_params(p)
    kd = rast.kd_partition(dp, L)
    st = rast.forward(dp, kd, [cam], EPS_T)
    torch.cuda.synchronize()
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    order, rank_of = oracle.cell_order(L, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    return p, cam, L, dp, kd, st, okd, order, rank_of, pr


def test_needle_footprints(needles):
    """Needles: rectangles, counts and instance lists bit-exact; the image
    against the oracle (which tests pixel-in-rectangle explicitly, the kernels
    do not) within 2e-4."""
    p, cam, L, dp, kd, st, okd, order, rank_of, pr = needles
    n = p["means"].shape[1]
    W, H = cam["W"], cam["H"]
    vis = pr["vis"] == 1
    d = pr["dec32"][vis].astype(np.float64)
    assert (1 + d[:, 8] ** 2 * d[:, 2] / d[:, 9]).max() > 1e4  # s00 s11 / det
    assert np.array_equal(st.proj["count"][:n].cpu().numpy().view(np.uint32), pr["count"])
    rect = proj_bin(st, n)[0]
    assert np.array_equal(rect[vis], pr["rect"][vis])
    okeys, ogids = oracle.bins(pr, rank_of, L, (W + 15) // 16)
    n_inst = st.bins_struct.n_instances
    keys = st.bins["keys"][:n_inst].cpu().numpy().view(np.uint32)
    src = (st.bins["vals"][:n_inst].cpu().numpy().view(np.uint64) >> np.uint64(32)).astype(np.int64)
    assert np.array_equal(keys, okeys) and np.array_equal(src % n, ogids.astype(np.int64))
    r = oracle.render(pr, cam, okd, order, oracle.all_pixels(W, H), EPS_T)
    err = np.abs(st.image.cpu().numpy().reshape(3, -1).T - r["img"]).max()
    log("needles: image max err %.2e" % err)
    assert err <= 2e-4


def test_needle_gradients(rast, needles):
    """Needles: 2D and parameter gradients of a seeded linear objective within
    1e-3 (relative) of the oracle's fp64 backward."""
    p, cam, L, dp, kd, st, okd, order, rank_of, pr = needles
    n = p["means"].shape[1]
    W, H = cam["W"], cam["H"]
    rng = np.random.default_rng(9)
    dimg = rng.normal(size=(3, H * W)).astype(np.float32) * 1e-3
    dTf = rng.normal(size=(H * W,)).astype(np.float32) * 1e-3
    g = rast.backward(st, dp, torch.from_numpy(dimg.ravel()).cuda(), torch.from_numpy(dTf).cuda())
    torch.cuda.synchronize()
    dproj = g["_dproj"][: 9 * n].view(9, n).cpu().numpy().T
    g2d = oracle.render_bwd(pr, cam, okd, order, oracle.all_pixels(W, H), dimg.T.astype(np.float64),
                            dTf.astype(np.float64), EPS_T)
    for c in range(9):
        ok, info = grad_close(dproj[:, c], g2d[:, c], 1e-3, "d2d[%d]" % c)
        assert ok, info
    og = oracle.project_bwd(p, cam, pr, g2d)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        ok, info = grad_close(g[k].cpu().numpy(), og[k], 1e-3, k)
        log(str(info))
        assert ok, info


def test_large_footprints_bins(rast):
    """Every pair has a rectangle larger than the 8 x 15 tiles the record's
    descriptor holds, so emission takes all spans from the block's row pool
    and a chunk of 256 pairs (far more than 2048 tile rows) is taken in
    several runs: instance lists bit-exact against the oracle."""
    n = 1500
    p = scenes.scene_uniform(n, seed=41, D=0, mu_s=-1.2, extent=0.5)
    W, H, L = 1280, 720, 1
    cam = scenes.orbit_camera(1.8, 0.3, 0.25, W, H, z_near=0.05)
    dp = device_params(p)
    kd = rast.kd_partition(dp, L)
    st = rast.forward(dp, kd, [cam], EPS_T)
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    order, rank_of = oracle.cell_order(L, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    vis = (pr["vis"] == 1) & (pr["count"] > 0)
    r = pr["rect"][vis]
    big = (((r[:, 3] >> 4) - (r[:, 2] >> 4)) >= 8) | (((r[:, 1] >> 4) - (r[:, 0] >> 4)) >= 15)
    rows = ((r[:, 3] >> 4) - (r[:, 2] >> 4) + 1)[big]
    log("large footprints: %d of %d visible pairs beyond the descriptor, %d tile rows" % (big.sum(), vis.sum(), rows.sum()))
    assert big.sum() > 0.8 * vis.sum() and rows.sum() > 4 * 2048
    assert np.array_equal(st.proj["count"][:n].cpu().numpy().view(np.uint32), pr["count"])
    okeys, ogids = oracle.bins(pr, rank_of, L, (W + 15) // 16)
    n_inst = st.bins_struct.n_instances
    keys = st.bins["keys"][:n_inst].cpu().numpy().view(np.uint32)
    src = (st.bins["vals"][:n_inst].cpu().numpy().view(np.uint64) >> np.uint64(32)).astype(np.int64)
    assert n_inst == len(okeys)
    assert np.array_equal(keys, okeys) and np.array_equal(src % n, ogids.astype(np.int64))


# ---------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def full(rast):
    log("config 2 at full size: 1M Gaussians, 1600x1060, K = 8")
    p, cam, tgt, L = scenes.config2()
    dp = device_params(p)
    kd = rast.kd_partition(dp, L)
    st = rast.forward(dp, kd, [cam], EPS_T)
    torch.cuda.synchronize()
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    order, rank_of = oracle.cell_order(L, okd["split"], cam["o"])
    log("oracle projection of 1M Gaussians")
    pr = oracle.project(p, cam, okd, 0)
    return p, cam, L, dp, kd, st, okd, order, pr


def test_full_size_sampled_pixels(full):
    p, cam, L, dp, kd, st, okd, order, pr = full
    n = p["means"].shape[1]
    assert np.array_equal(st.proj["count"][:n].cpu().numpy().view(np.uint32), pr["count"])
    W, H = cam["W"], cam["H"]
    rng = np.random.default_rng(123)
    pix = np.stack([rng.integers(0, W, 1500), rng.integers(0, H, 1500)], 1).astype(np.int32)
    # include the ragged last tile row (1060 = 66 * 16 + 4)
    pix[:50, 1] = H - 1 - rng.integers(0, 4, 50)
    log("oracle on %d sampled pixels of the full view" % len(pix))
    r = oracle.render(pr, cam, okd, order, pix, EPS_T)
    idx = pix[:, 1] * W + pix[:, 0]
    img = st.image.cpu().numpy().reshape(3, -1).T[idx]
    Tf = st.T_final.cpu().numpy()[idx]
    partC, partT, _ = gpu_partials_dense(st)
    err = max(np.abs(img - r["img"]).max(), np.abs(Tf - r["T"]).max(), np.abs(partC[idx] - r["partC"]).max(),
              np.abs(partT[idx] - r["partT"]).max())
    log("full size: max err over image, T, partials = %.2e (contributors per pixel up to %d)" % (err, r["ncon"].max()))
    assert err <= 2e-4


def test_full_size_sampled_gradients(full, rast):
    """Gradients of sum(w * image) for 24 Gaussians with small footprints (the
    2D quantities and the parameters); the oracle covers every pixel of their
    rectangles."""
    p, cam, L, dp, kd, st, okd, order, pr = full
    W, H = cam["W"], cam["H"]
    rng = np.random.default_rng(77)
    w = rng.normal(size=(3, H * W)).astype(np.float32) * 1e-3
    g = rast.backward(st, dp, torch.from_numpy(w.ravel()).cuda())
    dproj = g["_dproj"].view(9, -1).cpu().numpy()
    vis = np.nonzero(pr["vis"])[0]
    area = (pr["rect"][vis, 1] - pr["rect"][vis, 0] + 1) * (pr["rect"][vis, 3] - pr["rect"][vis, 2] + 1)
    small = vis[(area >= 9) & (area <= 400)]
    chosen = rng.choice(small, 24, replace=False)
    pix = []
    for i in chosen:
        x0, x1, y0, y1 = pr["rect"][i]
        yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        pix.append(np.stack([xx.ravel(), yy.ravel()], 1))
    pix = np.unique(np.concatenate(pix), axis=0).astype(np.int32)
    log("oracle backward over %d pixels covering %d Gaussians" % (len(pix), len(chosen)))
    idx = pix[:, 1] * W + pix[:, 0]
    g2d = oracle.render_bwd(pr, cam, okd, order, pix, w[:, idx].T.astype(np.float64), None, EPS_T)
    ref = g2d[chosen]
    got = dproj[:, chosen].T
    ok, info = grad_close(got, ref, 1e-3, "d_proj (24 Gaussians)")
    log(str(info))
    assert ok, info
    # their parameter gradients: the projection backward is per Gaussian, so
    # the oracle runs it on the chosen Gaussians alone
    sub = {k: (p[k][..., chosen] if k != "sh_degree" else p[k]) for k in p}
    og = oracle.project_bwd(sub, cam, dict(vis=pr["vis"][chosen]), ref)
    for k in raster.PARAM_KEYS:
        ok, info = grad_close(g[k].cpu().numpy()[..., chosen], og[k], 1e-3, "%s (24 Gaussians)" % k)
        log(str(info))
        assert ok, info


def test_full_resolution_loss(rast):
    rng = np.random.default_rng(6)
    x = rng.uniform(size=(3, 1060, 1600)).astype(np.float32)
    y = rng.uniform(size=(3, 1060, 1600)).astype(np.float32)
    lv, d = rast.loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), 0.2)
    ol, od = oracle.loss(x.astype(np.float64), y.astype(np.float64), 0.2)
    assert abs(lv.item() - ol) <= 1e-5 * abs(ol)
    ok, info = grad_close(d.cpu().numpy(), od, 1e-3, "dimage 1600x1060")
    assert ok, info


def test_sixteen_views_sixty_four_cells(rast):
    """The largest batch and partition the ABI takes (16 views, L = 6): every
    pixel of every (ragged) view against the oracle, and one view rendered
    alone bit-identical to the same view inside the batch."""
    p = scenes.scene_clusters(20000, seed=61, D=2)
    sizes = [(48 + 8 * k, 32 + 5 * (k % 4)) for k in range(16)]
    cams = [scenes.orbit_camera(4.0, 0.4 * k, np.radians(10 + 3 * k), W, H, z_near=0.2, bg=(0.1, 0.02 * k, 0.3))
            for k, (W, H) in enumerate(sizes)]
    dp = device_params(p)
    kd = rast.kd_partition(dp, 6)
    st = rast.forward(dp, kd, cams, EPS_T)
    okd = oracle.kd_partition(p["means"], p["log_scales"], 6)
    worst = 0.0
    for v, (cam, (img, Tf)) in enumerate(zip(cams, st.images())):
        order, _ = oracle.cell_order(6, okd["split"], cam["o"])
        pr = oracle.project(p, cam, okd, 0)
        r = oracle.render(pr, cam, okd, order, oracle.all_pixels(cam["W"], cam["H"]), EPS_T)
        worst = max(worst, float(np.abs(img.cpu().numpy().reshape(3, -1).T - r["img"]).max()),
                    float(np.abs(Tf.cpu().numpy().ravel() - r["T"]).max()))
    log("16 views, K = 64: max err %.2e" % worst)
    assert worst <= 2e-4
    alone = rast.forward(dp, kd, [cams[7]], EPS_T)
    assert torch.equal(alone.image, st.images()[7][0].reshape(-1))


def test_merged_render_matches_separate_merge(rast):
    """rgs_render_partial_merged writes the partials rgs_render_partial writes
    and the image / T_final that rgs_merge_partials folds from them, bit for
    bit: three ragged views (tiles without any instance among them), K = 8
    and K = 64."""
    p = scenes.scene_clusters(20000, seed=71, D=2)
    sizes = [(200, 136), (96, 80), (33, 17)]
    cams = [scenes.orbit_camera(4.0, 0.7 * k, np.radians(12 + 5 * k), W, H, z_near=0.2, bg=(0.2, 0.1 * k, 0.3))
            for k, (W, H) in enumerate(sizes)]
    dp = device_params(p)
    for L in (3, 6):
        kd = rast.kd_partition(dp, L)
        a = rast.forward(dp, kd, cams, EPS_T, merged=True)
        ia, ta = a.image.clone(), a.T_final.clone()
        n = int(a.bins["counters"][2].item())
        pa = {k: v[: n * (768 if k == "C" else 256)].clone() for k, v in a.parts.items()}
        b = rast.forward(dp, kd, cams, EPS_T, merged=False)
        assert int(b.bins["counters"][2].item()) == n
        assert torch.equal(ia, b.image) and torch.equal(ta, b.T_final)
        for k, v in pa.items():
            assert torch.equal(v, b.parts[k][: v.numel()])
        # some tile of these views has no slot (background only)
        assert bool((ta == 1.0).any())

def test_slot_table_beyond_fold(rast):
    """A dense (tile, rank) table of more than 1024 scan tiles (16 views of
    1088x1056 at L = 6: 71,808 tiles, 4.6M entries) takes the slot build's
    path with a separate scan of the tile sums; each view rendered alone (a
    small table, the folded path) must be bit-identical to it in the batch."""
    p = scenes.scene_clusters(20000, seed=67, D=2)
    cams = [scenes.orbit_camera(4.0, 0.4 * k, np.radians(10 + 3 * k), 1088, 1056, z_near=0.2, bg=(0.1, 0.02 * k, 0.3))
            for k in range(16)]
    dp = device_params(p)
    kd = rast.kd_partition(dp, 6)
    st = rast.forward(dp, kd, cams, EPS_T)
    tiles = 16 * 68 * 66
    assert (tiles << 6) > 1024 * 4096
    n_slots = int(st.bins["counters"][2].item())
    assert 0 < n_slots <= tiles << 6
    for v in (0, 5, 15):
        alone = rast.forward(dp, kd, [cams[v]], EPS_T)
        assert torch.equal(alone.image, st.images()[v][0].reshape(-1))
