"""ctypes binding of librgs.so (declared in include/rgs.h).

Argument marshalling only: every step runs in the HIP library.  The library
is loaded from this package directory; if it has not been built, importing
raises ``RuntimeError`` (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgs.so")

RGS_OK, RGS_E_ARG, RGS_E_CAPACITY, RGS_E_HIP, RGS_E_UNSUPPORTED = 0, -1, -2, -3, -4
RGS_SPLIT_MEDIAN, RGS_SPLIT_MIDPOINT = 0, 1
RGS_CELLS_EXACT, RGS_CELLS_PAPER_SUBSETS, RGS_CELLS_EXCLUSIVE = 0, 1, 2
RGS_T_FLOOR = 2.0 ** -100
RGS_MAX_VIEWS = 16
RGS_MAX_L = 6
REC_FLOATS = 16

vp = C.c_void_p
i32, i64, f32, sz = C.c_int32, C.c_int64, C.c_float, C.c_size_t


class Gaussians(C.Structure):
    _fields_ = [("n", i64), ("sh_degree", i32), ("means", vp), ("log_scales", vp), ("quats", vp),
                ("opacity", vp), ("sh", vp)]


class GaussiansGrad(C.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity", vp), ("sh", vp)]


class Camera(C.Structure):
    _fields_ = [("R", f32 * 9), ("t", f32 * 3), ("campos", f32 * 3), ("fx", f32), ("fy", f32), ("cx", f32),
                ("cy", f32), ("width", i32), ("height", i32), ("z_near", f32), ("bg", f32 * 3)]


class KdTree(C.Structure):
    _fields_ = [("L", i32), ("split", vp), ("box_lo", vp), ("box_hi", vp), ("center_cell", vp), ("counts", vp),
                ("own_mask", vp), ("cell_bounds", vp)]


class Projected(C.Structure):
    _fields_ = [("rec", vp), ("bin", vp), ("count", vp), ("depth", vp)]


class Bins(C.Structure):
    _fields_ = [("capacity", i64), ("slot_capacity", i64), ("keys", vp), ("vals", vp), ("pair_src", vp),
                ("pair_off", vp), ("pair_rank", vp), ("slot_key", vp), ("slot_range", vp), ("tile_slot", vp),
                ("slot_order", vp), ("tile_order", vp), ("counters", vp), ("n_instances", i64)]


class AdamParams(C.Structure):
    _fields_ = [("lr_means", f32), ("lr_log_scales", f32), ("lr_quats", f32), ("lr_opacity", f32),
                ("lr_sh_dc", f32), ("lr_sh_rest", f32), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("step", i32)]


class Partials(C.Structure):
    _fields_ = [("C", vp), ("T", vp), ("last", vp)]


class PartialsGrad(C.Structure):
    _fields_ = [("dC", vp), ("dT", vp)]


P = C.POINTER
_SIGS = {
    "rgs_abi_version": (i32, []),
    "rgs_status_string": (C.c_char_p, [i32]),
    "rgs_last_hip_error": (i32, []),
    "rgs_views_bytes": (sz, []),
    "rgs_views_upload": (i32, [P(Camera), i32, i32, vp, vp, vp, vp]),
    "rgs_views_pack": (i32, [P(Camera), i32, i32, vp, vp, vp]),
    "rgs_total_tiles": (i64, [P(Camera), i32]),
    "rgs_kd_partition_workspace": (sz, [i64, i32]),
    "rgs_kd_partition": (i32, [P(Gaussians), i32, f32, i32, P(KdTree), vp, sz, vp]),
    "rgs_cell_order": (i32, [i32, vp, vp, vp, vp]),
    "rgs_cell_visibility": (i32, [P(Camera), i32, i32, vp, vp]),
    "rgs_group_by_cell_workspace": (sz, [i64]),
    "rgs_group_by_cell": (i32, [P(Gaussians), P(KdTree), i32, P(Gaussians), vp, vp, sz, vp]),
    "rgs_project_sh": (i32, [P(Gaussians), P(Camera), i32, vp, P(KdTree), i32, P(Projected), vp]),
    "rgs_bin_sort_workspace": (sz, [i64, i32, i64, i32, i64]),
    "rgs_bin_sort": (i32, [P(Projected), i64, P(Camera), i32, vp, i32, P(Bins), P(i64), vp, sz, vp]),
    "rgs_bin_sort_async": (i32, [P(Projected), i64, P(Camera), i32, vp, i32, P(Bins), vp, sz, vp]),
    "rgs_render_partial": (i32, [P(Projected), i64, P(Bins), P(Camera), i32, vp, P(KdTree), f32, P(Partials), vp, vp]),
    "rgs_render_partial_merged": (i32, [P(Projected), i64, P(Bins), P(Camera), i32, vp, P(KdTree), f32, P(Partials),
                                        vp, vp, vp, vp]),
    "rgs_merge_partials": (i32, [P(Partials), P(Bins), P(Camera), i32, vp, vp, vp, vp]),
    "rgs_loss_workspace": (sz, [i32, i32]),
    "rgs_loss_l1_ssim": (i32, [vp, vp, i32, i32, f32, vp, vp, vp, sz, vp]),
    "rgs_loss_l1_ssim_noalloc": (i32, [vp, vp, i32, i32, f32, vp, vp, vp]),
    "rgs_merge_partials_bwd": (i32, [vp, vp, P(Partials), P(Bins), P(Camera), i32, vp, P(PartialsGrad), vp]),
    "rgs_render_bwd_workspace": (sz, [i64]),
    "rgs_render_partial_bwd": (i32, [P(PartialsGrad), P(Partials), P(Bins), P(Projected), i64, P(Camera), i32, vp,
                                     P(KdTree), vp, vp, sz, vp]),
    "rgs_render_partial_bwd_records": (i32, [P(PartialsGrad), P(Partials), P(Bins), P(Projected), i64, P(Camera), i32, vp,
                                           P(KdTree), vp, sz, vp, vp]),
    "rgs_pair_reduce": (i32, [P(Bins), P(Projected), i64, i32, vp, vp, sz, vp]),
    "rgs_project_sh_bwd": (i32, [vp, P(Gaussians), P(Projected), P(Camera), i32, vp, P(GaussiansGrad), vp]),
    "rgs_adam_step": (i32, [P(GaussiansGrad), P(GaussiansGrad), P(GaussiansGrad), P(GaussiansGrad), i64, i32,
                            P(AdamParams), vp]),
    "rgs_permute_gaussians": (i32, [P(Gaussians), vp, P(GaussiansGrad), vp]),
}

EXPORTED = tuple(_SIGS)
_lib = None


class RGSError(RuntimeError):
    def __init__(self, fn: str, status: int):
        lib = _lib
        msg = lib.rgs_status_string(status).decode() if lib else str(status)
        hip = lib.rgs_last_hip_error() if (lib and status == RGS_E_HIP) else 0
        super().__init__("%s failed: %s (status %d%s)" % (fn, msg, status, ", hip error %d" % hip if hip else ""))
        self.status = status


def load(path: str = LIB_PATH):
    """Load librgs.so and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librgs.so is not built (%s); run __graft_entry__.build()" % path)
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(fn: str, status: int) -> int:
    if status != RGS_OK:
        raise RGSError(fn, status)
    return status


def camera_struct(cam) -> Camera:
    c = Camera()
    R = [float(v) for v in list(getattr(cam["R"], "ravel", lambda: cam["R"])())]
    for k in range(9):
        c.R[k] = R[k]
    for k in range(3):
        c.t[k] = float(cam["t"][k])
        c.campos[k] = float(cam["o"][k])
        c.bg[k] = float(cam.get("bg", (0.0, 0.0, 0.0))[k])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height, c.z_near = int(cam["W"]), int(cam["H"]), float(cam["z_near"])
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr
