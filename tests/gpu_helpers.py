"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import sys
import time

import numpy as np

import oracle
from paper_2406_11836_amd import scenes


def log(msg):
    print("[%s] %s" % (time.strftime("%H:%M:%S"), msg), flush=True)
    sys.stdout.flush()


def device_params(params):
    from paper_2406_11836_amd import raster
    return raster.to_device(params)


def oracle_scene(params, cam, L):
    """Oracle KD tree, cell order and mirror32 projection for one view."""
    kd = oracle.kd_partition(params["means"], params["log_scales"], L)
    order, rank_of = oracle.cell_order(L, kd["split"], cam["o"])
    pr = oracle.project(params, cam, kd, 0)
    return kd, order, rank_of, pr


def proj_bin(st, n):
    """The first n binning records of a projection: rectangle (int32 [n, 4]:
    x_lo, x_hi, y_lo, y_hi), cell mask (uint64 [n]), instance count and tiles
    per cell (uint32 [n] each).  Only rows with a non-zero count are defined."""
    b = st.proj["bin"][: 8 * n].view(n, 8).cpu().numpy().view(np.uint32)
    rect = np.ascontiguousarray(b[:, :2]).view(np.int16).astype(np.int32)
    mask = np.ascontiguousarray(b[:, 4:6]).view(np.uint64)[:, 0]
    return rect, mask, b[:, 6].copy(), b[:, 7].copy()


def gpu_partials_dense(st, view=0):
    """GPU per-slot partials scattered to [H*W, K] per-cell maps of one view
    (cells without a slot in a tile: C = 0, T = 1)."""
    cams = st.cams
    Ld = st.kd.L
    K = 1 << Ld
    cam = cams[view]
    W, H = int(cam["W"]), int(cam["H"])
    tx_n = (W + 15) // 16
    tile_off = sum(((int(c["W"]) + 15) // 16) * ((int(c["H"]) + 15) // 16) for c in cams[:view])
    ntiles = tx_n * ((H + 15) // 16)
    counters = st.bins["counters"].cpu().numpy()
    S = int(counters[2])
    keys = st.bins["slot_key"][:S].cpu().numpy().astype(np.int64)
    Cs = st.parts["C"][: S * 768].view(S, 3, 256).cpu().numpy()
    Ts = st.parts["T"][: S * 256].view(S, 256).cpu().numpy()
    Ls = st.parts["last"][: S * 256].view(S, 256).cpu().numpy()
    ranks = np.zeros((K,), np.int64)
    from paper_2406_11836_amd import raster  # noqa
    rk = st_ranks(st)[view]
    cell_of_rank = np.argsort(rk)
    partC = np.zeros((H * W, K, 3))
    partT = np.ones((H * W, K))
    last = np.zeros((H * W, K), np.int64)
    gt = keys >> Ld
    sel = (gt >= tile_off) & (gt < tile_off + ntiles)
    p = np.arange(256)
    px_in, py_in = p % 16, p // 16
    for s in np.nonzero(sel)[0]:
        lt = int(gt[s] - tile_off)
        tx, ty = lt % tx_n, lt // tx_n
        cell = int(cell_of_rank[int(keys[s] & (K - 1))])
        x = tx * 16 + px_in
        y = ty * 16 + py_in
        ok = (x < W) & (y < H)
        idx = y[ok] * W + x[ok]
        partC[idx, cell] = Cs[s][:, ok].T
        partT[idx, cell] = Ts[s][ok]
        last[idx, cell] = Ls[s][ok]
    return partC, partT, last


def st_ranks(st):
    from paper_2406_11836_amd import raster  # noqa
    r = raster.Rasterizer.__new__(raster.Rasterizer)
    r.lib = st_lib()
    return r.cell_ranks(st.kd, st.cams)


def st_lib():
    from paper_2406_11836_amd import _lib
    return _lib.load()


def grad_close(g, ref, rel=1e-3, name=""):
    """Per-tensor ||g - ref|| <= rel ||ref||; per element |d| <= rel |ref| + rel max|ref|."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.abs(g - ref)
    nr = np.linalg.norm(ref)
    mx = np.abs(ref).max() if ref.size else 0.0
    ok_norm = np.linalg.norm(g - ref) <= rel * nr + 1e-30
    bad = d > rel * np.abs(ref) + rel * mx
    return ok_norm and not bad.any(), dict(name=name, norm_ref=float(nr), norm_err=float(np.linalg.norm(g - ref)),
                                           n_bad=int(bad.sum()), max_err=float(d.max()) if d.size else 0.0,
                                           max_ref=float(mx))
