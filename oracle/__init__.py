"""Plain CPU oracle for the partitioned 3DGS rasterizer (RetinaGS, arXiv 2406.11836).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does.

Thin numpy/ctypes marshalling over ``oracle.c`` (see that file's header for
what each function computes and which passage of the paper it follows).
``build()`` compiles the C file with gcc (-O2 -ffp-contract=off -fopenmp).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def pack_camera(cam) -> np.ndarray:
    """Oracle camera layout: R(9) t(3) o(3) fx fy cx cy W H z_near bg(3)."""
    v = np.zeros(25, np.float64)
    v[0:9] = np.asarray(cam["R"], np.float64).reshape(9)
    v[9:12] = cam["t"]
    v[12:15] = cam["o"]
    v[15], v[16], v[17], v[18] = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    v[19], v[20], v[21] = cam["W"], cam["H"], cam["z_near"]
    v[22:25] = cam.get("bg", (0.0, 0.0, 0.0))
    return v


def sh_basis(D: int, d):
    d = _f64(d)
    Y = np.zeros(16, np.float64)
    dY = np.zeros(48, np.float64)
    lib().orc_sh_basis(C.c_int(D), _p(d), _p(Y), _p(dY))
    n = (D + 1) ** 2
    return Y[:n], dY[: 3 * n].reshape(n, 3)


def kd_partition(means, log_scales, L: int, d_factor: float = 3.0, rule: int = 0):
    """rule 0: equal-count bisection (the paper's KD tree); 1: fixed-size grid."""
    means = _f64(means)
    ls = _f64(log_scales)
    n = means.shape[1]
    K = 1 << L
    Wm = (K + 31) // 32
    split = np.zeros(max(K - 1, 1), np.float32)
    axis = np.zeros(max(K - 1, 1), np.uint8)
    lo = np.zeros((3, K), np.float32)
    hi = np.zeros((3, K), np.float32)
    cc = np.zeros(max(n, 1), np.int32)
    counts = np.zeros(K, np.int32)
    own = np.zeros((max(n, 1), Wm), np.uint32)
    f = lib().orc_kd_partition
    f.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_int] + [C.c_void_p] * 7
    rc = f(n, _p(means), _p(ls), L, d_factor, rule, _p(split), _p(axis), _p(lo), _p(hi), _p(cc),
           _p(counts), _p(own))
    if rc != 0:
        raise ValueError("orc_kd_partition failed")
    return dict(L=L, K=K, split=split[: K - 1], axis=axis[: K - 1], box_lo=lo, box_hi=hi,
                center_cell=cc[:n], counts=counts, own_mask=own[:n])


def cell_order(L: int, split, o):
    K = 1 << L
    order = np.zeros(K, np.int32)
    rank_of = np.zeros(K, np.int32)
    sp = np.ascontiguousarray(split, np.float32)
    if sp.size == 0:
        sp = np.zeros(1, np.float32)
    o = _f64(o)
    lib().orc_cell_order(C.c_int(L), _p(sp), _p(o), _p(order), _p(rank_of))
    return order, rank_of


def _split_arr(kd):
    sp = np.ascontiguousarray(kd["split"], np.float32)
    return sp if sp.size else np.zeros(1, np.float32)


def _cell_arrays(kd, n, cells):
    """center_cell and own_mask rows for the subset modes (cells 1 and 2)."""
    K = 1 << kd["L"]
    Wm = (K + 31) // 32
    if cells == 0:
        return np.zeros(1, np.int32), np.zeros(1, np.uint32)
    cc = np.ascontiguousarray(kd["center_cell"], np.int32).reshape(-1)
    own = np.ascontiguousarray(kd["own_mask"], np.uint32).reshape(-1)
    if cc.size < max(n, 1) or own.size < max(n, 1) * Wm:
        raise ValueError("kd lacks center_cell / own_mask for this scene")
    return cc, own


def project(params, cam, kd, mode: int = 0, cells: int = 0):
    """Per-Gaussian projection; mode 0 = mirror32 decisions, 1 = exact64.
    cells: 0 the exact per-view cell sets, 1 the paper's subsets N_k,
    2 exclusive subsets (the cell of the centre; cell-based methods)."""
    means, ls, q = _f64(params["means"]), _f64(params["log_scales"]), _f64(params["quats"])
    op, sh = _f64(params["opacity"]), _f64(params["sh"])
    D = int(params["sh_degree"])
    n = means.shape[1]
    nn = max(n, 1)
    dec = np.zeros((nn, 10), np.float32)
    val = np.zeros((nn, 12), np.float64)
    rect = np.zeros((nn, 4), np.int32)
    vis = np.zeros(nn, np.uint8)
    mask = np.zeros(nn, np.uint64)
    count = np.zeros(nn, np.uint32)
    camv = pack_camera(cam)
    sp = _split_arr(kd)
    cc, own = _cell_arrays(kd, n, cells)
    f = lib().orc_project
    f.argtypes = [C.c_int64, C.c_int] + [C.c_void_p] * 6 + [C.c_int, C.c_void_p, C.c_int, C.c_int] + \
        [C.c_void_p] * 8
    rc = f(n, D, _p(means), _p(ls), _p(q), _p(op), _p(sh), _p(camv), kd["L"], _p(sp),
           mode, cells, _p(cc), _p(own), _p(dec), _p(val), _p(rect), _p(vis), _p(mask), _p(count))
    if rc != 0:
        raise ValueError("orc_project failed")
    return dict(n=n, mode=mode, cells=cells, dec32=dec[:n], val=val[:n], rect=rect[:n], vis=vis[:n],
                cellmask=mask[:n], count=count[:n])


def bins(proj, rank_of, L: int, tiles_x: int):
    n = proj["n"]
    tot = int(proj["count"].astype(np.int64).sum())
    keys = np.zeros(max(tot, 1), np.uint32)
    gids = np.zeros(max(tot, 1), np.uint32)
    f = lib().orc_bins
    f.restype = C.c_int64
    f.argtypes = [C.c_int64] + [C.c_void_p] * 5 + [C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_void_p]
    ro = np.ascontiguousarray(rank_of, np.int32)
    dec, rect = np.ascontiguousarray(proj["dec32"]), np.ascontiguousarray(proj["rect"])
    vis, cm = np.ascontiguousarray(proj["vis"]), np.ascontiguousarray(proj["cellmask"])
    m = f(n, _p(dec), _p(rect), _p(vis), _p(cm), _p(ro), L, tiles_x, tot, _p(keys), _p(gids))
    if m < 0:
        raise RuntimeError("orc_bins capacity")
    return keys[:m], gids[:m]


def _cells_args(proj, kd, keep):
    cells = int(proj.get("cells", 0))
    cc, own = _cell_arrays(kd, proj["n"], cells)
    keep.extend([cc, own])
    return cells, _p(cc), _p(own)


def _render_args(proj, cam, kd, order, keep):
    """Argument prefix of the render calls; arrays are appended to ``keep`` so
    that they outlive the foreign call."""
    arrs = [np.ascontiguousarray(proj["dec32"]), np.ascontiguousarray(proj["val"]),
            np.ascontiguousarray(proj["rect"]), np.ascontiguousarray(proj["vis"]), pack_camera(cam),
            _split_arr(kd), np.ascontiguousarray(order, np.int32)]
    keep.extend(arrs)
    return (proj["n"], _p(arrs[0]), _p(arrs[1]), _p(arrs[2]), _p(arrs[3]), _p(arrs[4]), kd["L"],
            _p(arrs[5]), _p(arrs[6]))


def all_pixels(W: int, H: int) -> np.ndarray:
    yy, xx = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32), indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], 1).astype(np.int32)


def render(proj, cam, kd, order, pix, eps_T: float = 0.0, restrict: bool = False):
    """Merged (Eq. 5), plain (Eq. 2) and per-cell partial values at pixels.

    ``restrict`` keeps a Gaussian only in the cells of its emitted cell set
    (a diagnostic: with conservative cell sets nothing changes)."""
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    P = pix.shape[0]
    K = 1 << kd["L"]
    img = np.zeros((P, 3)); Tf = np.zeros(P); plain = np.zeros((P, 3)); Tp = np.zeros(P)
    pc = np.zeros((P, K, 3)); pt = np.zeros((P, K)); ncon = np.zeros(P, np.int32)
    f = lib().orc_render
    f.argtypes = [C.c_int64] + [C.c_void_p] * 5 + [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                                   C.c_int64] + [C.c_void_p] * 9 + [C.c_int, C.c_void_p, C.c_void_p]
    keep = []
    a = _render_args(proj, cam, kd, order, keep)
    mode = proj["mode"] | (2 if restrict else 0)
    cm = np.ascontiguousarray(proj["cellmask"])
    if f(*a, mode, eps_T, P, _p(pix), _p(img), _p(Tf), _p(plain), _p(Tp), _p(pc), _p(pt), _p(ncon), _p(cm),
         *_cells_args(proj, kd, keep)) != 0:
        raise ValueError("orc_render failed")
    return dict(img=img, T=Tf, plain=plain, plainT=Tp, partC=pc, partT=pt, ncon=ncon)


def render_bwd(proj, cam, kd, order, pix, dimg, dTf=None, eps_T: float = 0.0):
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    P = pix.shape[0]
    g2d = np.zeros((max(proj["n"], 1), 9))
    dimg = _f64(dimg).reshape(P, 3)
    f = lib().orc_render_bwd
    f.argtypes = [C.c_int64] + [C.c_void_p] * 5 + [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_double,
                                                   C.c_int64] + [C.c_void_p] * 4 + [C.c_int, C.c_void_p, C.c_void_p]
    keep = []
    a = _render_args(proj, cam, kd, order, keep)
    dT = _f64(dTf).reshape(P) if dTf is not None else None
    if f(*a, proj["mode"], eps_T, P, _p(pix), _p(dimg), _p(dT) if dT is not None else None, _p(g2d),
         *_cells_args(proj, kd, keep)) != 0:
        raise ValueError("orc_render_bwd failed")
    return g2d[: proj["n"]]


def project_bwd(params, cam, proj, g2d):
    means, ls, q = _f64(params["means"]), _f64(params["log_scales"]), _f64(params["quats"])
    op, sh = _f64(params["opacity"]), _f64(params["sh"])
    D = int(params["sh_degree"])
    n = means.shape[1]
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity=np.zeros(n), sh=np.zeros(sh.shape))
    f = lib().orc_project_bwd
    f.argtypes = [C.c_int64, C.c_int] + [C.c_void_p] * 13
    g = np.ascontiguousarray(g2d, np.float64)
    camv = pack_camera(cam)
    vis = np.ascontiguousarray(proj["vis"])
    f(n, D, _p(means), _p(ls), _p(q), _p(op), _p(sh), _p(camv), _p(vis), _p(g), _p(out["means"]), _p(out["log_scales"]),
      _p(out["quats"]), _p(out["opacity"]), _p(out["sh"]))
    return out


def loss(img, tgt, ssim_w: float = 0.0):
    img = _f64(img); tgt = _f64(tgt)
    Cc, H, W = img.shape
    d = np.zeros_like(img)
    lv = np.zeros(1)
    f = lib().orc_loss
    f.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
    f(Cc, H, W, _p(img), _p(tgt), ssim_w, _p(lv), _p(d))
    return float(lv[0]), d


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results are the same at any count)."""
    lib().orc_set_threads(C.c_int(int(n)))


# ------------------------------------------------------------------ training (Sec. 4, implementation details)
SH_GROUP_ROWS = 3   # SH rows of degree 0 (one per colour channel)


def expon_lr(step: int, lr_init: float, lr_final: float, max_steps: int) -> float:
    """Exponential decay from lr_init at step 0 to lr_final at max_steps (the
    paper's position schedule, 1.6e-4 -> 1.6e-6): log-linear in the step,
    held at lr_final afterwards."""
    t = min(max(step / max_steps, 0.0), 1.0)
    return float(np.exp(np.log(lr_init) * (1.0 - t) + np.log(lr_final) * t))


def adam_step(params, grads, m, v, hp: dict):
    """One Adam step (Kingma and Ba), fp64, in place on the numpy arrays of
    params, m and v; per-group learning rates hp["lr"][key], with the SH
    degree-0 rows at hp["lr"]["sh_dc"] and the others at hp["lr"]["sh_rest"].
    hp: beta1, beta2, eps, step (1-based)."""
    b1, b2, eps, t = hp["beta1"], hp["beta2"], hp["eps"], hp["step"]
    for k in ("means", "log_scales", "quats", "opacity", "sh"):
        g = np.asarray(grads[k], np.float64)
        m[k][...] = b1 * m[k] + (1.0 - b1) * g
        v[k][...] = b2 * v[k] + (1.0 - b2) * g * g
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        if k == "sh":
            lr = np.full(g.shape[0], hp["lr"]["sh_rest"])
            lr[:SH_GROUP_ROWS] = hp["lr"]["sh_dc"]
            lr = lr[:, None]
        else:
            lr = hp["lr"][k]
        params[k][...] = params[k] - lr * mh / (np.sqrt(vh) + eps)
