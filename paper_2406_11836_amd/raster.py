"""One forward/backward pass of the partitioned rasterizer, driven through librgs.

``Rasterizer`` allocates device buffers with torch (memory and streams only)
and calls the C ABI in order:

  forward:  rgs_views_upload -> rgs_project_sh -> rgs_bin_sort
            -> rgs_render_partial_merged (or rgs_render_partial -> rgs_merge_partials)
  backward: rgs_merge_partials_bwd -> rgs_render_partial_bwd
            -> rgs_project_sh_bwd

``RetinaRasterize`` wraps the pair in a ``torch.autograd.Function``.  Every
arithmetic step runs in the HIP library; this module only marshals
arguments and owns buffers.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

PARAM_KEYS = ("means", "log_scales", "quats", "opacity", "sh")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mark(marks, name):
    """Record a timing event on the launch stream (measurement only)."""
    if marks is not None:
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        marks.append((name, e))


def to_device(params, device="cuda"):
    """numpy/torch parameter dict -> contiguous float32 device tensors."""
    out = {}
    for k in PARAM_KEYS:
        v = params[k]
        t = v if isinstance(v, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(v, np.float32))
        out[k] = t.to(device=device, dtype=torch.float32).contiguous()
    out["sh_degree"] = int(params["sh_degree"])
    return out


def gaussians_struct(params) -> L.Gaussians:
    g = L.Gaussians()
    g.n = int(params["means"].shape[1])
    g.sh_degree = int(params["sh_degree"])
    for k in PARAM_KEYS:
        setattr(g, k, params[k].data_ptr())
    return g


@dataclass
class KD:
    L: int
    split: torch.Tensor
    box_lo: torch.Tensor
    box_hi: torch.Tensor
    center_cell: torch.Tensor
    counts: torch.Tensor
    own_mask: torch.Tensor | None
    split_host: np.ndarray
    cell_bounds: torch.Tensor | None = None
    cell_bounds_host: np.ndarray | None = None

    def struct(self) -> L.KdTree:
        k = L.KdTree()
        k.L = self.L
        k.split, k.box_lo, k.box_hi = self.split.data_ptr(), self.box_lo.data_ptr(), self.box_hi.data_ptr()
        k.center_cell, k.counts = self.center_cell.data_ptr(), self.counts.data_ptr()
        k.own_mask = self.own_mask.data_ptr() if self.own_mask is not None else None
        k.cell_bounds = self.cell_bounds.data_ptr() if self.cell_bounds is not None else None
        return k


@dataclass
class FwdState:
    """Device buffers of one forward pass, kept for the backward."""
    n: int
    cams: list
    cam_arr: object
    kd: KD
    views: torch.Tensor
    proj: dict
    bins: dict
    bins_struct: L.Bins
    parts: dict
    image: torch.Tensor
    T_final: torch.Tensor
    eps_T: float
    total_tiles: int
    slot_capacity: int
    keep: list = field(default_factory=list)

    def proj_struct(self) -> L.Projected:
        s = L.Projected()
        s.rec, s.bin = self.proj["rec"].data_ptr(), self.proj["bin"].data_ptr()
        s.count = self.proj["count"].data_ptr()
        s.depth = self.proj["depth"].data_ptr()
        return s

    def overflow(self) -> int:
        """Instances required beyond the capacity by an asynchronous binning
        (0: the pass is valid).  Reads one device counter."""
        return int(self.bins["counters"][3].item())

    def parts_struct(self) -> L.Partials:
        s = L.Partials()
        s.C, s.T, s.last = self.parts["C"].data_ptr(), self.parts["T"].data_ptr(), self.parts["last"].data_ptr()
        return s

    def images(self):
        """Per-view (image [3,H,W], T_final [H,W]) views of the concatenated outputs."""
        out = []
        po = 0
        for c in self.cams:
            H, W = int(c["H"]), int(c["W"])
            out.append((self.image[3 * po: 3 * po + 3 * H * W].view(3, H, W), self.T_final[po: po + H * W].view(H, W)))
            po += H * W
        return out


class Rasterizer:
    """reuse=True keeps the forward pass's buffers between calls (grow-only, one
    set per Rasterizer): no allocation once warm, but a FwdState is only valid
    until the next forward call on the same Rasterizer.  For serving loops."""

    def __init__(self, device: str = "cuda", reuse: bool = False):
        self.lib = L.load()
        self.device = torch.device(device)
        self.capacity_hint = 0
        self.reuse = reuse
        self._pool = {}

    def _empty(self, n, dtype):
        return torch.empty(int(max(n, 1)), dtype=dtype, device=self.device)

    def _buf(self, key, n, dtype):
        if not self.reuse:
            return self._empty(n, dtype)
        esz = torch.empty(0, dtype=dtype).element_size()
        nbytes = int(max(n, 1)) * esz
        t = self._pool.get(key)
        if t is None or t.numel() < nbytes:
            self._pool.pop(key, None)
            t = torch.empty(int(nbytes * 1.25) + 256, dtype=torch.uint8, device=self.device)
            self._pool[key] = t
        return t[:nbytes].view(dtype)

    # ------------------------------------------------------------ KD tree
    def kd_partition(self, params, Ldepth: int, d_factor: float = 3.0, own_mask: bool = True,
                     rule: int = L.RGS_SPLIT_MEDIAN) -> KD:
        """rule: RGS_SPLIT_MEDIAN (the paper's KD tree) or RGS_SPLIT_MIDPOINT (fixed-size grid)."""
        n = int(params["means"].shape[1])
        K = 1 << Ldepth
        kd = KD(L=Ldepth, split=self._empty(max(K - 1, 1), torch.float32),
                box_lo=self._empty(3 * K, torch.float32), box_hi=self._empty(3 * K, torch.float32),
                center_cell=self._empty(n, torch.int32), counts=self._empty(K, torch.int32),
                own_mask=self._empty(n * ((K + 31) // 32), torch.int32) if own_mask else None,
                split_host=np.zeros(max(K - 1, 1), np.float32), cell_bounds=self._empty(8 * K, torch.float32))
        ws_bytes = self.lib.rgs_kd_partition_workspace(n, Ldepth)
        ws = self._empty(ws_bytes, torch.uint8)
        g = gaussians_struct(params)
        ks = kd.struct()
        L.check("rgs_kd_partition", self.lib.rgs_kd_partition(C.byref(g), Ldepth, d_factor, int(rule), C.byref(ks),
                                                               _p(ws), ws_bytes, _stream()))
        kd.split_host = kd.split.cpu().numpy().copy()
        kd.cell_bounds_host = kd.cell_bounds.cpu().numpy().reshape(8, K).copy()
        return kd

    def cell_visibility(self, kd: KD, cams) -> np.ndarray:
        """Per view, the mask of KD cells that may reach it (rgs_cell_visibility)."""
        cam_arr = L.camera_array(cams)
        out = np.zeros(len(cams), np.uint64)
        cb = np.ascontiguousarray(kd.cell_bounds_host, np.float32)
        L.check("rgs_cell_visibility", self.lib.rgs_cell_visibility(cam_arr, len(cams), kd.L,
                                                                     cb.ctypes.data_as(C.c_void_p),
                                                                     out.ctypes.data_as(C.c_void_p)))
        return out

    def group_by_cell(self, params, kd: KD):
        """Copy of the parameters grouped by KD cell (Morton order inside a
        cell) and its permutation perm (new index -> old gid, int32)."""
        n = int(params["means"].shape[1])
        out = {k: torch.empty_like(params[k]) for k in PARAM_KEYS}
        out["sh_degree"] = int(params["sh_degree"])
        perm = self._empty(n, torch.int32)
        ws_bytes = self.lib.rgs_group_by_cell_workspace(n)
        ws = self._empty(ws_bytes, torch.uint8)
        gi, go = gaussians_struct(params), gaussians_struct(out)
        ks = kd.struct()
        L.check("rgs_group_by_cell", self.lib.rgs_group_by_cell(C.byref(gi), C.byref(ks), kd.L, C.byref(go), _p(perm),
                                                                 _p(ws), ws_bytes, _stream()))
        return out, perm

    def cell_ranks(self, kd: KD, cams) -> np.ndarray:
        K = 1 << kd.L
        ranks = np.zeros((len(cams), K), np.int32)
        order = np.zeros(K, np.int32)
        for v, c in enumerate(cams):
            o = np.asarray(c["o"], np.float32)
            rk = np.zeros(K, np.int32)
            L.check("rgs_cell_order", self.lib.rgs_cell_order(kd.L, kd.split_host.ctypes.data_as(C.c_void_p),
                                                               o.ctypes.data_as(C.c_void_p),
                                                               order.ctypes.data_as(C.c_void_p),
                                                               rk.ctypes.data_as(C.c_void_p)))
            ranks[v] = rk
        return ranks

    # ------------------------------------------------------------ forward
    def forward(self, params, kd: KD, cams, eps_T: float = 5e-5, stats: torch.Tensor | None = None,
                marks: list | None = None, cell_visible=None, no_sync: bool = False, cull: bool = False,
                cells: int = L.RGS_CELLS_EXACT, merged: bool = True) -> FwdState:
        """stats: optional int64 device tensor [2] (evaluated, contributing pairs), incremented.
        merged: the partial render writes the merged image too (rgs_render_partial_merged);
        False runs rgs_render_partial, then rgs_merge_partials (bit-identical results).
        marks: optional list receiving (stage, event) pairs at stage ends.
        cell_visible: optional per-view uint64 masks of the KD cells that may reach each view;
        cull=True computes them with rgs_cell_visibility (changes no output).
        cells: RGS_CELLS_EXACT / _PAPER_SUBSETS / _EXCLUSIVE (which Gaussians each cell renders)."""
        lib = self.lib
        _mark(marks, "start")
        V = len(cams)
        if V < 1 or V > L.RGS_MAX_VIEWS:
            raise ValueError("1..%d views per call" % L.RGS_MAX_VIEWS)
        n = int(params["means"].shape[1])
        cam_arr = L.camera_array(cams)
        stream = _stream()
        ranks = self.cell_ranks(kd, cams)
        vb = lib.rgs_views_bytes()
        views = self._buf("views", vb, torch.uint8)
        if cell_visible is None and cull and kd.L > 0:
            cell_visible = self.cell_visibility(kd, cams)
        vis = None if cell_visible is None else np.ascontiguousarray(cell_visible, np.uint64)
        # packed on the host into pinned memory and copied on the stream without waiting
        # (torch's pinned allocator does not reuse the block before the copy is done)
        host = torch.empty(vb, dtype=torch.uint8, pin_memory=True)
        L.check("rgs_views_pack", lib.rgs_views_pack(cam_arr, V, kd.L, ranks.ctypes.data_as(C.c_void_p),
                                                     None if vis is None else vis.ctypes.data_as(C.c_void_p),
                                                     C.c_void_p(host.data_ptr())))
        views.copy_(host, non_blocking=True)
        _mark(marks, "views")
        g = gaussians_struct(params)
        ks = kd.struct()
        m = V * n
        proj = dict(rec=self._buf("rec", m * L.REC_FLOATS, torch.float32), bin=self._buf("bin", m * 8, torch.int32),
                    count=self._buf("count", m, torch.int32),
                    depth=self._buf("depth", m, torch.float32))
        ps = L.Projected(proj["rec"].data_ptr(), proj["bin"].data_ptr(), proj["count"].data_ptr(),
                         proj["depth"].data_ptr())
        L.check("rgs_project_sh", lib.rgs_project_sh(C.byref(g), cam_arr, V, _p(views), C.byref(ks), int(cells), C.byref(ps),
                                                     stream))
        _mark(marks, "project")
        T = int(lib.rgs_total_tiles(cam_arr, V))
        K = 1 << kd.L
        bins = dict(pair_src=self._buf("pair_src", m, torch.int32), pair_off=self._buf("pair_off", m + 1, torch.int32),
                    pair_rank=self._buf("pair_rank", m, torch.int32), tile_slot=self._buf("tile_slot", T + 1, torch.int32),
                    tile_order=self._buf("tile_order", T, torch.int32),
                    counters=self._buf("counters", 4, torch.int32))
        cap = max(self.capacity_hint, 1)
        # no host wait in binning when an earlier pass sized the buffers and the
        # slot bound stays small (the caller checks FwdState.overflow())
        use_async = no_sync and self.capacity_hint > 0 and min(cap, T * K) <= (1 << 18)
        while True:
            slot_cap = min(cap, T * K)
            bins["keys"] = self._buf("keys", cap, torch.int32)
            bins["vals"] = self._buf("vals", cap, torch.int64)
            bins["slot_key"] = self._buf("slot_key", slot_cap, torch.int32)
            bins["slot_range"] = self._buf("slot_range", 2 * slot_cap, torch.int32)
            bins["slot_order"] = self._buf("slot_order", slot_cap, torch.int32)
            bs = L.Bins()
            bs.capacity, bs.slot_capacity = cap, slot_cap
            for k in ("keys", "vals", "pair_src", "pair_off", "pair_rank", "slot_key", "slot_range", "tile_slot",
                      "slot_order", "tile_order", "counters"):
                setattr(bs, k, bins[k].data_ptr())
            ws_bytes = lib.rgs_bin_sort_workspace(n, V, T, kd.L, cap)
            ws = self._buf("bin_ws", ws_bytes, torch.uint8)
            need = C.c_int64(0)
            if use_async:
                L.check("rgs_bin_sort_async", lib.rgs_bin_sort_async(C.byref(ps), n, cam_arr, V, _p(views), kd.L,
                                                                     C.byref(bs), _p(ws), ws_bytes, stream))
                break
            st = lib.rgs_bin_sort(C.byref(ps), n, cam_arr, V, _p(views), kd.L, C.byref(bs), C.byref(need), _p(ws),
                                  ws_bytes, stream)
            if st == L.RGS_E_CAPACITY:
                cap = int(need.value * 1.15) + 1024
                self.capacity_hint = cap
                continue
            L.check("rgs_bin_sort", st)
            break
        _mark(marks, "bin_sort")
        n_inst = int(bs.n_instances)
        slot_cap = int(bs.slot_capacity)
        if slot_cap > (1 << 18) and not use_async:
            # large bound (many views / tiles): size the partial maps by the
            # actual slot count instead (one small device-to-host read)
            slot_cap = max(int(bins["counters"][2].item()), 1)
            bs.slot_capacity = slot_cap
        parts = dict(C=self._buf("C", slot_cap * 768, torch.float32), T=self._buf("T", slot_cap * 256, torch.float32),
                     last=self._buf("last", slot_cap * 256, torch.int32))
        pt = L.Partials(parts["C"].data_ptr(), parts["T"].data_ptr(), parts["last"].data_ptr())
        npix = sum(int(c["W"]) * int(c["H"]) for c in cams)
        image = self._buf("image", 3 * npix, torch.float32)
        T_final = self._buf("T_final", npix, torch.float32)
        if merged:
            L.check("rgs_render_partial_merged",
                    lib.rgs_render_partial_merged(C.byref(ps), n, C.byref(bs), cam_arr, V, _p(views), C.byref(ks),
                                                  float(eps_T), C.byref(pt), _p(image), _p(T_final), _p(stats), stream))
            _mark(marks, "render_fwd")
        else:
            L.check("rgs_render_partial", lib.rgs_render_partial(C.byref(ps), n, C.byref(bs), cam_arr, V, _p(views),
                                                                 C.byref(ks), float(eps_T), C.byref(pt), _p(stats),
                                                                 stream))
            _mark(marks, "render_fwd")
            L.check("rgs_merge_partials", lib.rgs_merge_partials(C.byref(pt), C.byref(bs), cam_arr, V, _p(views),
                                                                 _p(image), _p(T_final), stream))
            _mark(marks, "merge")
        return FwdState(n=n, cams=list(cams), cam_arr=cam_arr, kd=kd, views=views, proj=proj, bins=bins,
                        bins_struct=bs, parts=parts, image=image, T_final=T_final, eps_T=eps_T, total_tiles=T,
                        slot_capacity=slot_cap, keep=[ws, n_inst])

    # ------------------------------------------------------------ backward
    def backward(self, st: FwdState, params, d_image: torch.Tensor, d_T_final: torch.Tensor | None = None,
                 marks: list | None = None, stats: torch.Tensor | None = None):
        """stats: optional int64 device tensor [2] (pairs re-tested, contributing pairs of the
        partial-render backward), incremented."""
        lib = self.lib
        _mark(marks, "bwd_start")
        V = len(st.cams)
        stream = _stream()
        d_image = d_image.contiguous()
        if d_T_final is not None:
            d_T_final = d_T_final.contiguous()
        pg = dict(dC=self._empty(st.slot_capacity * 768, torch.float32), dT=self._empty(st.slot_capacity * 256, torch.float32))
        pgs = L.PartialsGrad(pg["dC"].data_ptr(), pg["dT"].data_ptr())
        pt = st.parts_struct()
        bs = st.bins_struct
        L.check("rgs_merge_partials_bwd", lib.rgs_merge_partials_bwd(_p(d_image), _p(d_T_final), C.byref(pt), C.byref(bs),
                                                                     st.cam_arr, V, _p(st.views), C.byref(pgs), stream))
        _mark(marks, "merge_bwd")
        ps = st.proj_struct()
        ks = st.kd.struct()
        m = V * st.n
        dproj = self._empty(9 * m, torch.float32)
        ws_bytes = lib.rgs_render_bwd_workspace(bs.capacity)
        ws = self._empty(ws_bytes, torch.uint8)
        L.check("rgs_render_partial_bwd_records",
                lib.rgs_render_partial_bwd_records(C.byref(pgs), C.byref(pt), C.byref(bs), C.byref(ps), st.n, st.cam_arr,
                                                   V, _p(st.views), C.byref(ks), _p(ws), ws_bytes, _p(stats), stream))
        _mark(marks, "render_bwd")
        L.check("rgs_pair_reduce", lib.rgs_pair_reduce(C.byref(bs), C.byref(ps), st.n, V, _p(dproj), _p(ws), ws_bytes,
                                                       stream))
        _mark(marks, "pair_reduce")
        grads = {k: torch.empty_like(params[k]) for k in PARAM_KEYS}
        gg = L.GaussiansGrad(*[grads[k].data_ptr() for k in PARAM_KEYS])
        g = gaussians_struct(params)
        L.check("rgs_project_sh_bwd", lib.rgs_project_sh_bwd(_p(dproj), C.byref(g), C.byref(ps), st.cam_arr, V,
                                                             _p(st.views), C.byref(gg), stream))
        _mark(marks, "project_bwd")
        grads["_dproj"] = dproj
        grads["_dparts"] = pg
        return grads

    # ------------------------------------------------------------ loss
    def loss(self, image: torch.Tensor, target: torch.Tensor, ssim_weight: float = 0.0):
        """L1 + w (1 - SSIM) of one [3,H,W] view: (loss scalar tensor, d loss / d image)."""
        _, H, W = image.shape
        lossv = torch.empty(1, dtype=torch.float32, device=self.device)
        d = torch.empty_like(image)
        ws_bytes = self.lib.rgs_loss_workspace(H, W)
        ws = self._empty(ws_bytes, torch.uint8)
        L.check("rgs_loss_l1_ssim", self.lib.rgs_loss_l1_ssim(_p(image.contiguous()), _p(target.contiguous()), H, W,
                                                              float(ssim_weight), _p(lossv), _p(d), _p(ws), ws_bytes,
                                                              _stream()))
        return lossv, d


class RetinaRasterize(torch.autograd.Function):
    """(means, log_scales, quats, opacity, sh) -> (image, T_final) for the
    views in ``cams``, merged over the KD cells of ``kd``."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity, sh, cams, kd, rast, sh_degree, eps_T):
        params = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                      opacity=opacity.contiguous(), sh=sh.contiguous(), sh_degree=sh_degree)
        st = rast.forward(params, kd, cams, eps_T)
        ctx.st, ctx.rast, ctx.params = st, rast, params
        return st.image, st.T_final

    @staticmethod
    def backward(ctx, d_image, d_T_final):
        g = ctx.rast.backward(ctx.st, ctx.params, d_image, d_T_final)
        return g["means"], g["log_scales"], g["quats"], g["opacity"], g["sh"], None, None, None, None, None


def rasterize(params, cams, kd: KD, rast: Rasterizer, eps_T: float = 5e-5):
    return RetinaRasterize.apply(params["means"], params["log_scales"], params["quats"], params["opacity"],
                                 params["sh"], cams, kd, rast, int(params["sh_degree"]), eps_T)
