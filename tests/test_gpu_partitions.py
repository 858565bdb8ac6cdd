"""GPU parity of the partition variants against the oracle.

- The fixed-size grid partition (Sec. 4.2, Table 2) next to the KD tree:
  splits, leaf boxes, leaf of every centre, counts, N_k and the cell bounds
  used for culling, bit for bit; the merged image of a grid partition is
  still the single-worker render.
- The paper's own subsets N_k as the render set (Sec. 3.3): instance lists
  bit for bit, partials and image within 2e-4 of the oracle's restricted
  render, and the contributions lost ("escapes") counted exactly, for the
  margin factors 3, 4 and 6.
- Exclusive cells without the indicator of Eq. 6 (the cell-based methods of
  Sec. 2): the leaky border of the validity experiment (Sec. 4.2) matches
  the oracle's restricted render, pixel for pixel.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import device_params, gpu_partials_dense, grad_close, log, proj_bin
from paper_2406_11836_amd import _lib as L
from paper_2406_11836_amd import raster, scenes

pytestmark = pytest.mark.gpu
EPS_T = 5e-5


@pytest.fixture(scope="module")
def rast():
    return raster.Rasterizer()


def _cell_bounds_np(p, cc, K):
    m = np.asarray(p["means"], np.float32)
    smax = np.exp(np.asarray(p["log_scales"], np.float32).astype(np.float64)).astype(np.float32).max(0)
    cb = np.zeros((8, K), np.float32)
    for k in range(K):
        sel = cc == k
        if not sel.any():
            cb[0:3, k], cb[3:6, k], cb[6, k] = np.inf, -np.inf, 0.0
        else:
            cb[0:3, k], cb[3:6, k], cb[6, k] = m[:, sel].min(1), m[:, sel].max(1), smax[sel].max()
    return cb


def _scene(name):
    if name == "clusters":
        p = scenes.scene_clusters(60000, seed=20, D=3)
        cam = scenes.orbit_camera(4.0, 2.1, np.radians(25.0), 410, 266, z_near=0.2, bg=(0.1, 0.2, 0.3))
        return p, cam, 3
    if name == "near":
        p = scenes.scene_uniform(8000, seed=31, D=1, mu_s=-3.2, extent=0.8)
        cam = scenes.orbit_camera(0.9, 0.4, 0.2, 200, 150, z_near=0.05)
        return p, cam, 4
    p, cam, _, L_ = scenes.config1()
    return p, cam, L_


@pytest.mark.parametrize("rule", [L.RGS_SPLIT_MEDIAN, L.RGS_SPLIT_MIDPOINT])
@pytest.mark.parametrize("name", ["clusters", "near"])
def test_partition_rules_bit_exact(name, rule, rast):
    p, cam, Ld = _scene(name)
    K = 1 << Ld
    dp = device_params(p)
    kd = rast.kd_partition(dp, Ld, rule=rule)
    okd = oracle.kd_partition(p["means"], p["log_scales"], Ld, 3.0, rule=rule)
    assert np.array_equal(kd.split.cpu().numpy()[: K - 1].view(np.uint32), okd["split"].view(np.uint32))
    assert np.array_equal(kd.box_lo.cpu().numpy().reshape(3, K), okd["box_lo"])
    assert np.array_equal(kd.box_hi.cpu().numpy().reshape(3, K), okd["box_hi"])
    assert np.array_equal(kd.center_cell.cpu().numpy(), okd["center_cell"])
    assert np.array_equal(kd.counts.cpu().numpy(), okd["counts"])
    own = kd.own_mask.cpu().numpy().view(np.uint32).reshape(okd["own_mask"].shape)
    assert np.array_equal(own, okd["own_mask"])
    cb = _cell_bounds_np(p, okd["center_cell"], K)
    assert np.array_equal(kd.cell_bounds_host.view(np.uint32), cb.view(np.uint32))
    log("%s rule %d: counts %s" % (name, rule, kd.counts.cpu().numpy().tolist()))
    if rule == L.RGS_SPLIT_MIDPOINT:
        # still a BSP partition: the merged render equals the single-cell one
        st = rast.forward(dp, kd, [cam], 0.0)
        st1 = rast.forward(dp, rast.kd_partition(dp, 0), [cam], 0.0)
        assert (st.image - st1.image).abs().max().item() <= 2e-5


def _project_bins_render(rast, dp, kd, cam, cells, eps_T):
    stats = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = rast.forward(dp, kd, [cam], eps_T, stats=stats, cells=cells)
    torch.cuda.synchronize()
    return st, stats.cpu().numpy()


@pytest.mark.parametrize("cells", [L.RGS_CELLS_PAPER_SUBSETS, L.RGS_CELLS_EXCLUSIVE])
def test_subset_modes_parity(cells, rast):
    p, cam, Ld = _scene("clusters")
    n = p["means"].shape[1]
    dp = device_params(p)
    kd = rast.kd_partition(dp, Ld, d_factor=1.0)   # a small margin: many escapes
    okd = oracle.kd_partition(p["means"], p["log_scales"], Ld, 1.0)
    order, rank_of = oracle.cell_order(Ld, okd["split"], cam["o"])
    st, _ = _project_bins_render(rast, dp, kd, cam, cells, EPS_T)
    pr = oracle.project(p, cam, okd, 0, cells=cells)
    cnt = st.proj["count"][:n].cpu().numpy().view(np.uint32)
    assert np.array_equal(cnt, pr["count"])
    vis = pr["count"] > 0
    assert np.array_equal(proj_bin(st, n)[1][vis], pr["cellmask"][vis])
    okeys, ogids = oracle.bins(pr, rank_of, Ld, (cam["W"] + 15) // 16)
    n_inst = st.bins_struct.n_instances
    assert n_inst == len(okeys)
    keys = st.bins["keys"][:n_inst].cpu().numpy().view(np.uint32)
    src = (st.bins["vals"][:n_inst].cpu().numpy().view(np.uint64) >> np.uint64(32)).astype(np.int64)
    assert np.array_equal(keys, okeys) and np.array_equal(src % n, ogids.astype(np.int64))
    W, H = cam["W"], cam["H"]
    pix = oracle.all_pixels(W, H)
    r = oracle.render(pr, cam, okd, order, pix, EPS_T)
    partC, partT, _ = gpu_partials_dense(st)
    img = st.image.cpu().numpy().reshape(3, -1).T
    err = max(np.abs(img - r["img"]).max(), np.abs(partC - r["partC"]).max(), np.abs(partT - r["partT"]).max())
    exact = oracle.render(oracle.project(p, cam, okd, 0), cam, okd, order, pix, EPS_T)
    dev = np.abs(r["img"] - exact["img"]).max()
    log("cells mode %d: GPU vs oracle %.2e; the mode departs from the exact render by %.3e" % (cells, err, dev))
    assert err <= 2e-4
    assert dev > 1e-3          # the restriction is visible on this scene
    # the backward of the restricted render, against the oracle's
    rng = np.random.default_rng(9)
    dimg = rng.normal(size=(3, H * W)).astype(np.float32) * 1e-3
    g = rast.backward(st, dp, torch.from_numpy(dimg.ravel()).cuda())
    dproj = g["_dproj"][: 9 * n].view(9, n).cpu().numpy().T
    g2d = oracle.render_bwd(pr, cam, okd, order, pix, dimg.T.astype(np.float64), None, EPS_T)
    for c in range(9):
        ok, info = grad_close(dproj[:, c], g2d[:, c], 1e-3, "mode %d row %d" % (cells, c))
        assert ok, info


def test_escapes_against_margin(rast):
    """Contributions lost by rendering from N_k (Sec. 3.3), for D_i = f max scale
    with f in {3, 4, 6}: the GPU's contributing-pair count falls short of the
    exact mode's by exactly the oracle's count of escapes (no early stop:
    eps_T = 0), and the loss shrinks as the margin grows."""
    p, cam, Ld = _scene("near")
    dp = device_params(p)
    pix = oracle.all_pixels(cam["W"], cam["H"])
    out = []
    for f in (3.0, 4.0, 6.0):
        kd = rast.kd_partition(dp, Ld, d_factor=f)
        okd = oracle.kd_partition(p["means"], p["log_scales"], Ld, f)
        order, _ = oracle.cell_order(Ld, okd["split"], cam["o"])
        _, s0 = _project_bins_render(rast, dp, kd, cam, L.RGS_CELLS_EXACT, 0.0)
        st1, s1 = _project_bins_render(rast, dp, kd, cam, L.RGS_CELLS_PAPER_SUBSETS, 0.0)
        r0 = oracle.render(oracle.project(p, cam, okd, 0), cam, okd, order, pix, 0.0)
        r1 = oracle.render(oracle.project(p, cam, okd, 0, cells=1), cam, okd, order, pix, 0.0)
        esc_oracle = int(r0["ncon"].sum() - r1["ncon"].sum())
        assert int(s0[1]) == int(r0["ncon"].sum()) and int(s1[1]) == int(r1["ncon"].sum())
        assert int(s0[1] - s1[1]) == esc_oracle
        img_err = float(np.abs(st1.image.cpu().numpy().reshape(3, -1).T - r0["img"]).max())
        out.append((f, esc_oracle, img_err))
    log("escapes and image error against the exact render, per margin factor: %s" % out)
    assert out[0][1] > 0 and out[0][1] >= out[1][1] >= out[2][1]


def test_exclusive_cells_leak_like_the_oracle(rast):
    """Validity experiment (Sec. 4.2) with cell-based exclusive subsets: the far
    cell's partial is no longer (0, 1) across the border, on the GPU as in the
    oracle, and the GPU's partials match the oracle's everywhere."""
    p = scenes.scene_uniform(20000, seed=40, D=0, mu_s=-3.5, extent=0.6)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 1)
    s = float(kd.split_host[0])
    cam = scenes.with_kd_axis_aligned_camera(s, 128, 96, dist=2.0)
    st = rast.forward(dp, kd, [cam], EPS_T, cells=L.RGS_CELLS_EXCLUSIVE)
    okd = oracle.kd_partition(p["means"], p["log_scales"], 1)
    order, _ = oracle.cell_order(1, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0, cells=2)
    r = oracle.render(pr, cam, okd, order, oracle.all_pixels(128, 96), EPS_T)
    partC, partT, _ = gpu_partials_dense(st)
    x = np.tile(np.arange(128), 96)
    left = x < 64
    leaks = int((partT[left, 1] < 1.0).sum() + (partT[~left, 0] < 1.0).sum())
    log("exclusive cells: %d pixels receive the far cell's colour" % leaks)
    assert leaks > 20
    assert np.abs(partC - r["partC"]).max() <= 2e-4 and np.abs(partT - r["partT"]).max() <= 2e-4
    assert np.abs(st.image.cpu().numpy().reshape(3, -1).T - r["img"]).max() <= 2e-4
