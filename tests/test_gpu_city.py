"""Parity at the size of one GPU's share of a billion-scale aerial scene.

16M Gaussians of the aerial-city layout (ground plane plus box facades, SH
degree 3), one 3840x2160 view at 150 m altitude pitched down 45 degrees, and
a K = 32 KD tree built on the whole scene, rendered in the launch
configuration the training step uses.  Checked against the oracle:
  - per-Gaussian counts of all 16M Gaussians, bit for bit;
  - image, final transmittance and every per-cell partial on a seeded
    sample of pixels;
  - the 2D and parameter gradients of a seeded linear objective for a
    sample of visible Gaussians (the oracle walks every pixel of their
    rectangles, so their gradients are complete).
The oracle's inputs are the host copies of the drawn scene; its KD tree is
built by the oracle itself.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import gpu_partials_dense, grad_close, log
from paper_2406_11836_amd import raster, scenes

pytestmark = pytest.mark.gpu
EPS_T = 5e-5
N_CITY = 16_000_000
L_CITY = 5


@pytest.fixture(scope="module")
def city():
    log("aerial city: %d Gaussians SH3, 3840x2160, K = %d" % (N_CITY, 1 << L_CITY))
    dp = scenes.scene_city_device(N_CITY, seed=30, D=3)
    rng = np.random.default_rng(31)
    cam = scenes.aerial_camera(rng, 3840, 2160, 800.0, 150.0, -45.0)
    rast = raster.Rasterizer()
    kd = rast.kd_partition(dp, L_CITY)
    st = rast.forward(dp, kd, [cam], EPS_T)
    torch.cuda.synchronize()
    p = {k: dp[k].cpu().numpy() for k in raster.PARAM_KEYS}
    p["sh_degree"] = 3
    log("oracle: KD tree and projection of %d Gaussians" % N_CITY)
    okd = oracle.kd_partition(p["means"], p["log_scales"], L_CITY)
    order, _ = oracle.cell_order(L_CITY, okd["split"], cam["o"])
    pr = oracle.project(p, cam, okd, 0)
    return rast, dp, kd, st, cam, p, okd, order, pr


def test_city_counts_and_splits_bit_exact(city):
    rast, dp, kd, st, cam, p, okd, order, pr = city
    K = 1 << L_CITY
    assert np.array_equal(kd.split.cpu().numpy()[: K - 1].view(np.uint32), okd["split"].view(np.uint32))
    assert np.array_equal(kd.counts.cpu().numpy(), okd["counts"])
    got = st.proj["count"][:N_CITY].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, pr["count"])
    log("visible %d, instances %d" % (int(pr["vis"].sum()), int(pr["count"].astype(np.int64).sum())))
    assert st.bins_struct.n_instances == int(pr["count"].astype(np.int64).sum())


def test_city_sampled_pixels(city):
    rast, dp, kd, st, cam, p, okd, order, pr = city
    W, H = cam["W"], cam["H"]
    rng = np.random.default_rng(321)
    pix = np.stack([rng.integers(0, W, 600), rng.integers(0, H, 600)], 1).astype(np.int32)
    # the image's last tile row and column
    pix[:40, 1] = H - 1 - rng.integers(0, 16, 40)
    pix[40:80, 0] = W - 1 - rng.integers(0, 16, 40)
    log("oracle on %d sampled pixels of the 3840x2160 view" % len(pix))
    r = oracle.render(pr, cam, okd, order, pix, EPS_T)
    idx = pix[:, 1] * W + pix[:, 0]
    img = st.image.cpu().numpy().reshape(3, -1).T[idx]
    Tf = st.T_final.cpu().numpy()[idx]
    partC, partT, _ = gpu_partials_dense(st)
    err = max(np.abs(img - r["img"]).max(), np.abs(Tf - r["T"]).max(), np.abs(partC[idx] - r["partC"]).max(),
              np.abs(partT[idx] - r["partT"]).max())
    log("city: max err over image, T, partials = %.2e (contributors per pixel up to %d, covered %d of %d)"
        % (err, r["ncon"].max(), int((r["ncon"] > 0).sum()), len(pix)))
    assert (r["ncon"] > 0).sum() > len(pix) // 2
    assert err <= 2e-4


def _sampled_gradients(rast, dp, st, cam, p, okd, order, pr, seed, n_pick, tag):
    """GPU gradients of sum(w * image) for n_pick visible Gaussians with small
    rectangles against the oracle's, which walks every pixel of their
    rectangles: the 2D quantities and the parameters."""
    W, H = cam["W"], cam["H"]
    rng = np.random.default_rng(seed)
    w = (rng.normal(size=(3, H * W)) * 1e-3).astype(np.float32)
    g = rast.backward(st, dp, torch.from_numpy(w.ravel()).cuda())
    torch.cuda.synchronize()
    n = pr["n"]
    dproj = g["_dproj"][: 9 * n].view(9, n).cpu().numpy()
    vis = np.nonzero(pr["vis"])[0]
    area = (pr["rect"][vis, 1] - pr["rect"][vis, 0] + 1) * (pr["rect"][vis, 3] - pr["rect"][vis, 2] + 1)
    small = vis[(area >= 9) & (area <= 400)]
    chosen = np.sort(rng.choice(small, n_pick, replace=False))
    pix = []
    for i in chosen:
        x0, x1, y0, y1 = pr["rect"][i]
        yy, xx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        pix.append(np.stack([xx.ravel(), yy.ravel()], 1))
    pix = np.unique(np.concatenate(pix), axis=0).astype(np.int32)
    log("%s: oracle backward over %d pixels covering %d Gaussians" % (tag, len(pix), len(chosen)))
    idx = pix[:, 1] * W + pix[:, 0]
    g2d = oracle.render_bwd(pr, cam, okd, order, pix, w[:, idx].T.astype(np.float64), None, EPS_T)
    ok, info = grad_close(dproj[:, chosen].T, g2d[chosen], 1e-3, "%s d_proj (%d Gaussians)" % (tag, len(chosen)))
    log(str(info))
    assert ok, info
    # parameter gradients of the chosen Gaussians (the projection backward is
    # per Gaussian, so the oracle runs it on the chosen ones alone)
    sub = {k: (p[k][..., chosen] if k != "sh_degree" else p[k]) for k in p}
    sub_pr = dict(vis=pr["vis"][chosen])
    og = oracle.project_bwd(sub, cam, sub_pr, g2d[chosen])
    for k in raster.PARAM_KEYS:
        got = g[k].cpu().numpy()[..., chosen]
        ok, info = grad_close(got, og[k], 1e-3, "%s %s (%d Gaussians)" % (tag, k, len(chosen)))
        log(str(info))
        assert ok, info


def test_city_sampled_gradients(city):
    rast, dp, kd, st, cam, p, okd, order, pr = city
    _sampled_gradients(rast, dp, st, cam, p, okd, order, pr, 77, 24, "city")
