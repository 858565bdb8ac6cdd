"""The training loop on the GPU (Sec. 3.4, Sec. 4): the fused Adam kernel
against the oracle's Adam, the reorder that follows a re-partition, and a
short run that fits a synthetic target."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import device_params, log
from paper_2406_11836_amd import raster, scenes, train

pytestmark = pytest.mark.gpu

KEYS = raster.PARAM_KEYS


def _rand_set(rng, n, D, scale=1.0):
    nc = (D + 1) ** 2
    return dict(means=rng.normal(size=(3, n)) * scale, log_scales=rng.normal(size=(3, n)) * scale,
                quats=rng.normal(size=(4, n)) * scale, opacity=rng.normal(size=n) * scale,
                sh=rng.normal(size=(3 * nc, n)) * scale, sh_degree=D)


def _dev(d):
    out = {k: torch.from_numpy(np.ascontiguousarray(d[k], np.float32)).cuda() for k in KEYS}
    out["sh_degree"] = d["sh_degree"]
    return out


@pytest.mark.parametrize("n", [1, 1001, 70000])
def test_adam_kernel_matches_oracle(n):
    """Four steps of rgs_adam_step (fp32) against the oracle's Adam (fp64) on
    seeded parameters and gradients, per-group rates, SH degree 3; ragged n
    exercises the element-wise tail."""
    from paper_2406_11836_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(100 + n)
    D = 3
    p = _rand_set(rng, n, D)
    p32 = {k: np.asarray(p[k], np.float32).astype(np.float64) for k in KEYS}
    m = {k: np.zeros_like(p32[k]) for k in KEYS}
    v = {k: np.zeros_like(p32[k]) for k in KEYS}
    dp = _dev(p32 | {"sh_degree": D})
    dm = {k: torch.zeros_like(dp[k]) for k in KEYS}
    dv = {k: torch.zeros_like(dp[k]) for k in KEYS}
    # the first moment's recursion on |g|: fp32 rounding of each step's two
    # products and one sum moves m by a few 2^-24 of this, whatever the signs
    mabs = {k: np.zeros_like(p32[k]) for k in KEYS}
    lr = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4)
    for step in range(1, 5):
        g = _rand_set(rng, n, D, scale=10.0 ** rng.uniform(-3, 1))
        g32 = {k: np.asarray(g[k], np.float32).astype(np.float64) for k in KEYS}
        for k in KEYS:
            mabs[k] = 0.9 * mabs[k] + 0.1 * np.abs(g32[k])
        train.adam_step(lib, dp, _dev(g32 | {"sh_degree": D}), dm, dv, step, lr, eps=1e-15)
        oracle.adam_step(p32, g32, m, v, dict(beta1=0.9, beta2=0.999, eps=1e-15, step=step,
                                               lr=dict(lr, means=1.6e-4)))
    torch.cuda.synchronize()
    for k in KEYS:
        got = dp[k].cpu().numpy().astype(np.float64)
        # the update is a few lr in size; fp32 storage of p rounds at 2^-24 |p|
        assert np.abs(got - p32[k]).max() <= 1e-6 * np.abs(p32[k]).max() + 1e-7, k
        # four steps of at most three roundings each (2^-24 = 6e-8), plus the
        # fp32 rounding of b1 and 1 - b1: well inside 2e-6 of the |g| recursion
        assert np.all(np.abs(dm[k].cpu().numpy() - m[k]) <= 2e-6 * mabs[k]), k
        # v sums positive terms, so its relative error stays a few 2^-24
        assert np.all(np.abs(dv[k].cpu().numpy() - v[k]) <= 2e-6 * v[k]), k


def test_permute_matches_indexing():
    from paper_2406_11836_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(7)
    src = _dev(_rand_set(rng, 5003, 2))
    perm = torch.from_numpy(rng.permutation(5003).astype(np.int32)).cuda()
    out = train.permute(lib, src, perm)
    pl = perm.long()
    for k in KEYS:
        ref = src[k][..., pl] if src[k].dim() == 2 else src[k][pl]
        assert torch.equal(out[k], ref), k


def test_repartition_carries_state():
    """After some steps, re-partitioning regroups parameters and both Adam
    moments with one permutation: row j of each is the old row perm[j]; the
    tree is rebuilt on the moved centres, still balanced; the image only
    changes among exactly equal depths."""
    p, cam, tgt, Ld = scenes.config1()
    tr = train.Trainer(device_params(p), Ld, max_steps=100, ssim_weight=0.0)
    target = torch.from_numpy(tgt).cuda()
    for _ in range(3):
        tr.step([cam], [target])
    old_p = {k: tr.params[k].clone() for k in KEYS}
    old_m = {k: tr.m[k].clone() for k in KEYS}
    old_v = {k: tr.v[k].clone() for k in KEYS}
    img0 = tr.rast.forward(tr.params, tr.kd, [cam], 5e-5).image.clone()
    perm = tr.repartition().long()
    for k in KEYS:
        for new, old in ((tr.params, old_p), (tr.m, old_m), (tr.v, old_v)):
            ref = old[k][..., perm] if old[k].dim() == 2 else old[k][perm]
            assert torch.equal(new[k], ref), k
    counts = tr.kd.counts.cpu().numpy()
    assert counts.max() - counts.min() <= 1
    cc = tr.kd.center_cell.cpu().numpy()
    assert np.all(np.diff(cc) >= 0)       # grouped by cell
    img1 = tr.rast.forward(tr.params, tr.kd, [cam], 5e-5).image
    assert float(((img1 - img0).abs() > 1e-6).float().mean()) <= 1e-3


def test_short_run_fits_a_target():
    """Fit a perturbed copy of a scene to renders of the original from four
    views (L1 + 0.2 (1 - SSIM), K = 4, re-partition every 10 steps): the loss
    falls by more than a third in 40 steps."""
    p, cam, _, Ld = scenes.config1()
    cams = [scenes.orbit_camera(3.0, a, 0.35, 192, 160) for a in (0.3, 1.8, 3.3, 4.8)]
    ref = device_params(p)
    rast = raster.Rasterizer()
    kd = rast.kd_partition(ref, Ld)
    targets = [img.clone() for img, _ in rast.forward(ref, kd, cams, 5e-5).images()]
    rng = np.random.default_rng(5)
    q = dict(p)
    q["sh"] = (p["sh"] + rng.normal(size=p["sh"].shape) * 0.6).astype(np.float32)
    q["opacity"] = (p["opacity"] + rng.normal(size=p["opacity"].shape)).astype(np.float32)
    tr = train.Trainer(device_params(q), Ld, max_steps=40, repartition_every=10, ssim_weight=0.2)
    losses = []
    for _ in range(40):
        losses.append(float(tr.step(cams, targets).item()))
    log("loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert losses[-1] < 0.66 * losses[0]
    assert all(np.isfinite(losses))
