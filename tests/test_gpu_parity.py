"""GPU parity of every step of the hot path against the CPU oracle.

Bit-exact: KD splits, boxes and leaf assignment; per-pair projection decision
quantities (screen mean, conic, tau, depth, alpha), rectangles, cell sets and
instance counts; the sorted instance lists.  Within tolerance: partial maps
and merged image (2e-4 max abs against fp64 values), loss and gradients
(1e-3 relative).  All inputs are seeded synthetic scenes.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import device_params, gpu_partials_dense, grad_close, log, oracle_scene, proj_bin
from paper_2406_11836_amd import scenes

pytestmark = pytest.mark.gpu

EPS_T = 5e-5


def case(name):
    if name == "c1":
        p, cam, tgt, L = scenes.config1()
        return p, cam, tgt, L
    if name == "mini2":
        p = scenes.scene_clusters(60000, seed=20, D=3)
        cam = scenes.orbit_camera(4.0, 2.1, np.radians(25.0), 410, 266, z_near=0.2, bg=(0.1, 0.2, 0.3))
        return p, cam, scenes.target_image(22, 410, 266), 3
    if name == "near":
        # camera inside the cloud: large footprints, many cells per Gaussian
        p = scenes.scene_uniform(8000, seed=31, D=1, mu_s=-3.2, extent=0.8)
        cam = scenes.orbit_camera(0.9, 0.4, 0.2, 200, 150, z_near=0.05)
        return p, cam, scenes.target_image(32, 200, 150), 4
    raise KeyError(name)


@pytest.fixture(scope="module")
def rast():
    from paper_2406_11836_amd import raster
    return raster.Rasterizer()


_cache = {}


def run_case(name, rast):
    if name in _cache:
        return _cache[name]
    from paper_2406_11836_amd import raster
    log("case %s: generating" % name)
    p, cam, tgt, L = case(name)
    dp = device_params(p)
    log("case %s: kd_partition (GPU)" % name)
    kd = rast.kd_partition(dp, L)
    log("case %s: forward (GPU)" % name)
    st = rast.forward(dp, kd, [cam], EPS_T)
    torch.cuda.synchronize()
    log("case %s: oracle" % name)
    okd, order, rank_of, pr = oracle_scene(p, cam, L)
    _cache[name] = (p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr)
    return _cache[name]


@pytest.mark.parametrize("name", ["c1", "mini2", "near"])
def test_kd_partition_bit_exact(name, rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    K = 1 << L
    assert np.array_equal(kd.split.cpu().numpy()[: K - 1].view(np.uint32), okd["split"].view(np.uint32))
    assert np.array_equal(kd.box_lo.cpu().numpy().reshape(3, K), okd["box_lo"])
    assert np.array_equal(kd.box_hi.cpu().numpy().reshape(3, K), okd["box_hi"])
    assert np.array_equal(kd.center_cell.cpu().numpy(), okd["center_cell"])
    assert np.array_equal(kd.counts.cpu().numpy(), okd["counts"])
    own = kd.own_mask.cpu().numpy().view(np.uint32).reshape(okd["own_mask"].shape)
    assert np.array_equal(own, okd["own_mask"])


def test_kd_partition_full_size_1m(rast):
    """The headline scene's 1M centres, K = 8: splits and leaf counts bit-exact."""
    p = scenes.scene_clusters(1_000_000, seed=20, D=0)
    dp = device_params(p)
    log("kd 1M (GPU)")
    kd = rast.kd_partition(dp, 3)
    okd = oracle.kd_partition(p["means"], p["log_scales"], 3)
    assert np.array_equal(kd.split.cpu().numpy()[:7].view(np.uint32), okd["split"].view(np.uint32))
    assert np.array_equal(kd.counts.cpu().numpy(), okd["counts"])
    assert np.array_equal(kd.center_cell.cpu().numpy(), okd["center_cell"])


@pytest.mark.parametrize("name", ["c1", "mini2", "near"])
def test_project_bit_exact(name, rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    n = p["means"].shape[1]
    rec = st.proj["rec"][: n * 16].view(n, 16).cpu().numpy()
    cnt = st.proj["count"][:n].cpu().numpy().view(np.uint32)
    assert np.array_equal(cnt, pr["count"]), "instance counts"
    vis = pr["vis"] == 1
    assert vis.sum() > 0.3 * n
    rect, mask, bcnt, bnt = proj_bin(st, n)
    assert np.array_equal(mask[vis], pr["cellmask"][vis])
    assert np.array_equal(rect[vis], pr["rect"][vis])
    # the binning record repeats the count, and its tiles per cell divide it by the cells
    assert np.array_equal(bcnt[vis], pr["count"][vis])
    ncell = np.array([bin(int(x)).count("1") for x in pr["cellmask"][vis]], np.uint32)
    assert np.array_equal(bnt[vis] * ncell, pr["count"][vis])
    # the render record carries the same rectangle (x_lo | x_hi << 16, y_lo | y_hi << 16)
    packed = rec[vis][:, 12:14].view(np.uint32)
    unpack = np.stack([packed[:, 0] & 0xffff, packed[:, 0] >> 16, packed[:, 1] & 0xffff, packed[:, 1] >> 16], 1)
    assert np.array_equal(unpack.astype(np.int16).astype(np.int32), pr["rect"][vis])
    # decision quantities: record (mx, my, ca, k | e, alpha, tau, z) against the
    # oracle's (mx, my, ca, cb, cc, tau, z, alpha, k, e)
    gpu_dec = rec[vis][:, :8]
    ora_dec = pr["dec32"][vis][:, [0, 1, 2, 8, 9, 7, 5, 6]]
    assert np.array_equal(gpu_dec.view(np.uint32), ora_dec.view(np.uint32))
    # the dense depth array (binning's sort key) is the record's z, bit for bit
    depth = st.proj["depth"][:n].cpu().numpy()
    assert np.array_equal(depth[vis].view(np.uint32), pr["dec32"][vis][:, 6].view(np.uint32))
    # colour (value path, fp32 vs fp64)
    assert np.abs(rec[vis][:, 8:11] - pr["val"][vis][:, 7:10]).max() < 2e-5
    flags = rec[:, 11].view(np.uint32)
    single = np.array([bin(int(m)).count("1") == 1 for m in pr["cellmask"]])
    assert np.array_equal((flags[vis] & 1) == 1, single[vis])


@pytest.mark.parametrize("name", ["c1", "mini2", "near"])
def test_bins_bit_exact(name, rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    n = p["means"].shape[1]
    tiles_x = (cam["W"] + 15) // 16
    okeys, ogids = oracle.bins(pr, rank_of, L, tiles_x)
    n_inst = st.bins_struct.n_instances
    assert n_inst == len(okeys)
    keys = st.bins["keys"][:n_inst].cpu().numpy().view(np.uint32)
    vals = st.bins["vals"][:n_inst].cpu().numpy().view(np.uint64)
    src = (vals >> np.uint64(32)).astype(np.int64)
    assert np.array_equal(keys, okeys)
    assert np.array_equal(src % n, ogids.astype(np.int64))
    # emission positions: a permutation, contiguous per pair in (depth, gid) order
    pos = (vals & np.uint64(0xffffffff)).astype(np.int64)
    assert np.array_equal(np.sort(pos), np.arange(n_inst))


@pytest.mark.parametrize("name", ["c1", "mini2", "near"])
def test_render_and_merge_parity(name, rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    W, H = cam["W"], cam["H"]
    pix = oracle.all_pixels(W, H)
    log("oracle render %s (%d px)" % (name, len(pix)))
    r = oracle.render(pr, cam, okd, order, pix, EPS_T)
    partC, partT, last = gpu_partials_dense(st)
    err_c = np.abs(partC - r["partC"]).max()
    err_t = np.abs(partT - r["partT"]).max()
    img = st.image.cpu().numpy().reshape(3, H * W).T
    Tf = st.T_final.cpu().numpy()
    err_i = np.abs(img - r["img"]).max()
    err_T = np.abs(Tf - r["T"]).max()
    log("%s: partial C %.2e T %.2e image %.2e T_final %.2e" % (name, err_c, err_t, err_i, err_T))
    assert err_c <= 2e-4 and err_t <= 2e-4
    assert err_i <= 2e-4 and err_T <= 2e-4
    assert r["ncon"].max() > 5


@pytest.mark.parametrize("name", ["c1", "mini2"])
def test_merged_equals_plain_on_gpu(name, rast):
    """Sec. 3.2: the merged K-cell image equals the single-cell (K = 1) render."""
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    kd1 = rast.kd_partition(dp, 0)
    st1 = rast.forward(dp, kd1, [cam], 0.0)
    stK = rast.forward(dp, kd, [cam], 0.0)
    d = (st1.image - stK.image).abs().max().item()
    log("%s: |merged K - plain| = %.3e" % (name, d))
    assert d <= 2e-5


def test_validity_camera_on_split_plane(rast):
    """Sec. 4.2: camera centre on the root plane, axis-aligned: each half of the
    image comes from one cell; the other cell's partial is exactly (0, 1)."""
    p = scenes.scene_uniform(20000, seed=40, D=0, mu_s=-3.5, extent=0.6)
    dp = device_params(p)
    kd = rast.kd_partition(dp, 1)
    s = float(kd.split_host[0])
    cam = scenes.with_kd_axis_aligned_camera(s, 128, 96, dist=2.0)
    st = rast.forward(dp, kd, [cam], EPS_T)
    partC, partT, _ = gpu_partials_dense(st)
    x = np.tile(np.arange(128), 96)
    left = x < 64
    assert np.all(partC[left, 1] == 0.0) and np.all(partT[left, 1] == 1.0)
    assert np.all(partC[~left, 0] == 0.0) and np.all(partT[~left, 0] == 1.0)
    assert partC[left, 0].max() > 0.05 and partC[~left, 1].max() > 0.05
    mask = proj_bin(st, 20000)[1][st.proj["count"][: 20000].cpu().numpy() != 0]
    assert (mask == 3).sum() > 10   # Gaussians straddling the plane are in both cells


@pytest.mark.parametrize("ssim_w", [0.0, 0.2])
def test_loss_parity(ssim_w, rast):
    rng = np.random.default_rng(5)
    for (H, W) in [(37, 53), (266, 410)]:
        x = rng.uniform(size=(3, H, W)).astype(np.float32)
        y = rng.uniform(size=(3, H, W)).astype(np.float32)
        lv, d = rast.loss(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), ssim_w)
        ol, od = oracle.loss(x.astype(np.float64), y.astype(np.float64), ssim_w)
        assert abs(lv.item() - ol) <= 1e-5 * max(1.0, abs(ol))
        ok, info = grad_close(d.cpu().numpy(), od, 1e-3, "dimage")
        assert ok, info


@pytest.mark.parametrize("name", ["c1", "mini2", "near"])
def test_backward_parity(name, rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case(name, rast)
    W, H = cam["W"], cam["H"]
    n = p["means"].shape[1]
    rng = np.random.default_rng(77)
    dimg = rng.normal(size=(3, H * W)).astype(np.float32) * 1e-3
    dTf = rng.normal(size=(H * W,)).astype(np.float32) * 1e-3
    log("GPU backward %s" % name)
    g = rast.backward(st, dp, torch.from_numpy(dimg.ravel()).cuda(), torch.from_numpy(dTf).cuda())
    torch.cuda.synchronize()
    dproj = g["_dproj"][: 9 * n].view(9, n).cpu().numpy().T
    log("oracle backward %s" % name)
    pix = oracle.all_pixels(W, H)
    g2d = oracle.render_bwd(pr, cam, okd, order, pix, dimg.T.astype(np.float64), dTf.astype(np.float64), EPS_T)
    names = ["d_mx", "d_my", "d_ca", "d_cb", "d_cc", "d_alpha", "d_r", "d_g", "d_b"]
    for c in range(9):
        ok, info = grad_close(dproj[:, c], g2d[:, c], 1e-3, names[c])
        log(str(info))
        assert ok, info
    og = oracle.project_bwd(p, cam, pr, g2d)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        ok, info = grad_close(g[k].cpu().numpy(), og[k], 1e-3, k)
        log(str(info))
        assert ok, info


def test_combined_backward_equals_split_calls(rast):
    """rgs_render_partial_bwd (one call) gives the same per-pair gradients, bit
    for bit, as rgs_render_partial_bwd_records followed by rgs_pair_reduce."""
    import ctypes as C
    from paper_2406_11836_amd import _lib as L
    p, cam, tgt, Ld, dp, kd, st, okd, order, rank_of, pr = run_case("mini2", rast)
    d = torch.from_numpy(np.random.default_rng(3).normal(size=st.image.numel()).astype(np.float32)).cuda()
    g = rast.backward(st, dp, d)
    torch.cuda.synchronize()
    lib = rast.lib
    pgs = L.PartialsGrad(g["_dparts"]["dC"].data_ptr(), g["_dparts"]["dT"].data_ptr())
    pt, ps, ks, bs = st.parts_struct(), st.proj_struct(), st.kd.struct(), st.bins_struct
    m = st.n
    dproj = torch.empty(9 * m, dtype=torch.float32, device="cuda")
    ws_bytes = lib.rgs_render_bwd_workspace(bs.capacity)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    L.check("rgs_render_partial_bwd", lib.rgs_render_partial_bwd(
        C.byref(pgs), C.byref(pt), C.byref(bs), C.byref(ps), st.n, st.cam_arr, 1, C.c_void_p(st.views.data_ptr()),
        C.byref(ks), C.c_void_p(dproj.data_ptr()), C.c_void_p(ws.data_ptr()), ws_bytes,
        C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    assert torch.equal(dproj, g["_dproj"][: 9 * m])


def test_async_binning_equals_sync():
    """Binning without the host wait gives the same image and gradients, bit for
    bit, once an earlier pass sized the buffers; a pass over capacity reports the
    required count and renders only the background."""
    from paper_2406_11836_amd import raster
    r = raster.Rasterizer()
    p, cam, tgt, Ld, dp, kd, st, okd, order, rank_of, pr = run_case("mini2", r)
    a = r.forward(dp, kd, [cam], EPS_T)                    # synchronous (sets the capacity)
    b = r.forward(dp, kd, [cam], EPS_T, no_sync=True)      # asynchronous
    assert b.bins_struct.n_instances == -1
    assert b.overflow() == 0
    assert torch.equal(a.image, b.image) and torch.equal(a.T_final, b.T_final)
    d = torch.from_numpy(np.random.default_rng(2).normal(size=a.image.numel()).astype(np.float32)).cuda()
    ga, gb = r.backward(a, dp, d), r.backward(b, dp, d)
    for k in raster.PARAM_KEYS:
        assert torch.equal(ga[k], gb[k]), k
    need = int(a.bins_struct.n_instances)
    r.capacity_hint = need // 3
    c = r.forward(dp, kd, [cam], EPS_T, no_sync=True)
    assert c.overflow() == need
    bg = torch.tensor(cam.get("bg", (0.0, 0.0, 0.0)), dtype=torch.float32,
                      device="cuda").repeat_interleave(cam["W"] * cam["H"])
    assert torch.equal(c.image, bg) and torch.all(c.T_final == 1.0)
    r.capacity_hint = 0
    e = r.forward(dp, kd, [cam], EPS_T)                    # grown again, synchronously
    assert torch.equal(e.image, a.image)


def test_deterministic_runs(rast):
    p, cam, tgt, L, dp, kd, st, okd, order, rank_of, pr = run_case("mini2", rast)
    a = rast.forward(dp, kd, [cam], EPS_T)
    b = rast.forward(dp, kd, [cam], EPS_T)
    assert torch.equal(a.image, b.image)
    d = torch.from_numpy(np.random.default_rng(1).normal(size=a.image.numel()).astype(np.float32)).cuda()
    ga = rast.backward(a, dp, d)
    gb = rast.backward(b, dp, d)
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        assert torch.equal(ga[k], gb[k]), k


# ---------------------------------------------------------------- batched views
def _batch_case():
    p = scenes.scene_clusters(40000, seed=44, D=3)
    cams = [scenes.orbit_camera(4.0, 0.3 + 1.7 * k, np.radians(15 + 12 * k), W, H, z_near=0.2, bg=(0.05 * k, 0.1, 0.2))
            for k, (W, H) in enumerate([(240, 136), (333, 201), (160, 90)])]
    return p, cams, 3


def test_batched_views_parity(rast):
    """Several views of different (ragged) sizes in one call: every view's image
    against the oracle, the summed gradient against the oracle's per-view sum,
    and each view bit-identical to the same view rendered alone."""
    p, cams, L = _batch_case()
    dp = device_params(p)
    kd = rast.kd_partition(dp, L)
    log("batched forward (3 views)")
    st = rast.forward(dp, kd, cams, EPS_T)
    okd = oracle.kd_partition(p["means"], p["log_scales"], L)
    rng = np.random.default_rng(9)
    d_img = rng.normal(size=st.image.numel()).astype(np.float32) * 1e-3
    g = rast.backward(st, dp, torch.from_numpy(d_img).cuda())
    torch.cuda.synchronize()
    og_sum = None
    po = 0
    for v, (cam, (img, Tf)) in enumerate(zip(cams, st.images())):
        W, H = cam["W"], cam["H"]
        order, rank_of = oracle.cell_order(L, okd["split"], cam["o"])
        pr = oracle.project(p, cam, okd, 0)
        pix = oracle.all_pixels(W, H)
        r = oracle.render(pr, cam, okd, order, pix, EPS_T)
        err = np.abs(img.cpu().numpy().reshape(3, -1).T - r["img"]).max()
        log("view %d (%dx%d): image err %.2e" % (v, W, H, err))
        assert err <= 2e-4
        alone = rast.forward(dp, kd, [cam], EPS_T)
        assert torch.equal(alone.image, img.reshape(-1)), "view %d differs alone vs batched" % v
        dv = d_img[3 * po: 3 * po + 3 * H * W].reshape(3, H * W).T.astype(np.float64)
        po += H * W
        g2d = oracle.render_bwd(pr, cam, okd, order, pix, dv, None, EPS_T)
        og = oracle.project_bwd(p, cam, pr, g2d)
        og_sum = og if og_sum is None else {k: og_sum[k] + og[k] for k in og}
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        ok, info = grad_close(g[k].cpu().numpy(), og_sum[k], 1e-3, k)
        log(str(info))
        assert ok, info
