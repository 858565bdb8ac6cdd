"""Training loop around the partitioned rasterizer (Sec. 3.4 and Sec. 4).

One step renders a batch of views through the KD cells (projection, binning,
partial render, merge), takes the loss of every view, sends its gradient
back through the merge to every cell and on to the parameters, and updates
them with the library's fused Adam (fp32 moments, one learning rate per
parameter group).  The position rate decays exponentially from 1.6e-4 to
1.6e-6 over the run (the paper's setting, 1/100 of 3DGS's positions rate at
the end) and the number of Gaussians stays fixed (the paper disables
densification).  Every ``repartition_every`` steps the KD tree is rebuilt on
the current centres and the parameters and both Adam moments are regrouped
by cell with one permutation (rgs_group_by_cell, rgs_permute_gaussians), as
the paper repartitions after a set number of epochs.

Every arithmetic step runs in librgs; this module owns buffers and the
schedule.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L
from . import raster

# 3DGS's per-group learning rates (positions decayed, the rest constant)
DEFAULT_LR = dict(means_init=1.6e-4, means_final=1.6e-6, log_scales=5e-3, quats=1e-3, opacity=5e-2,
                  sh_dc=2.5e-3, sh_rest=2.5e-3 / 20.0)


def expon_lr(step: int, lr_init: float, lr_final: float, max_steps: int) -> float:
    """Log-linear decay from lr_init (step 0) to lr_final (max_steps), then held."""
    t = min(max(step / max(max_steps, 1), 0.0), 1.0)
    return math.exp(math.log(lr_init) * (1.0 - t) + math.log(lr_final) * t)


def _grad_struct(d) -> L.GaussiansGrad:
    return L.GaussiansGrad(*[d[k].data_ptr() for k in raster.PARAM_KEYS])


def adam_step(lib, params, grads, m, v, step: int, lrs: dict, betas=(0.9, 0.999), eps: float = 1e-15):
    """rgs_adam_step on dicts of device tensors (params, m, v updated in place)."""
    hp = L.AdamParams(lrs["means"], lrs["log_scales"], lrs["quats"], lrs["opacity"], lrs["sh_dc"], lrs["sh_rest"],
                      betas[0], betas[1], eps, int(step))
    n = int(params["means"].shape[1])
    L.check("rgs_adam_step", lib.rgs_adam_step(C.byref(_grad_struct(params)), C.byref(_grad_struct(grads)),
                                               C.byref(_grad_struct(m)), C.byref(_grad_struct(v)), n,
                                               int(params["sh_degree"]), C.byref(hp), raster._stream()))


def permute(lib, src, perm: torch.Tensor):
    """New dict with row j = src row perm[j] in every parameter array."""
    out = {k: torch.empty_like(src[k]) for k in raster.PARAM_KEYS}
    out["sh_degree"] = int(src["sh_degree"])
    g = raster.gaussians_struct(src)
    L.check("rgs_permute_gaussians", lib.rgs_permute_gaussians(C.byref(g), C.c_void_p(perm.data_ptr()),
                                                               C.byref(_grad_struct(out)), raster._stream()))
    return out


class Trainer:
    def __init__(self, params, L_depth: int, *, max_steps: int, repartition_every: int = 0, d_factor: float = 3.0,
                 ssim_weight: float = 0.2, eps_T: float = 5e-5, lr: dict | None = None, device: str = "cuda"):
        self.rast = raster.Rasterizer(device)
        self.lib = self.rast.lib
        self.params = {k: params[k].contiguous() for k in raster.PARAM_KEYS}
        self.params["sh_degree"] = int(params["sh_degree"])
        self.m = {k: torch.zeros_like(self.params[k]) for k in raster.PARAM_KEYS}
        self.v = {k: torch.zeros_like(self.params[k]) for k in raster.PARAM_KEYS}
        self.m["sh_degree"] = self.v["sh_degree"] = self.params["sh_degree"]
        self.L = int(L_depth)
        self.max_steps = int(max_steps)
        self.repartition_every = int(repartition_every)
        self.d_factor = float(d_factor)
        self.ssim_weight = float(ssim_weight)
        self.eps_T = float(eps_T)
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.step_count = 0
        self.kd = self.rast.kd_partition(self.params, self.L, self.d_factor)

    def lrs(self, step: int) -> dict:
        return dict(means=expon_lr(step, self.lr["means_init"], self.lr["means_final"], self.max_steps),
                    log_scales=self.lr["log_scales"], quats=self.lr["quats"], opacity=self.lr["opacity"],
                    sh_dc=self.lr["sh_dc"], sh_rest=self.lr["sh_rest"])

    def repartition(self):
        """Rebuild the KD tree on the current centres and regroup parameters and
        Adam moments by cell with one permutation."""
        kd = self.rast.kd_partition(self.params, self.L, self.d_factor)
        grouped, perm = self.rast.group_by_cell(self.params, kd)
        self.m = permute(self.lib, self.m, perm)
        self.v = permute(self.lib, self.v, perm)
        self.params = grouped
        # the tree of the regrouped copy is the same; its leaf indices follow the new order
        self.kd = self.rast.kd_partition(self.params, self.L, self.d_factor)
        return perm

    def _grads(self, cams, targets, no_sync):
        st = self.rast.forward(self.params, self.kd, cams, self.eps_T, no_sync=no_sync)
        d = torch.empty_like(st.image)
        total = torch.zeros(1, dtype=torch.float32, device=st.image.device)
        po = 0
        for (img, _), tg in zip(st.images(), targets):
            lv, dv = self.rast.loss(img, tg, self.ssim_weight)
            nimg = img.numel()
            d[po: po + nimg] = dv.view(-1)
            total += lv
            po += nimg
        return st, self.rast.backward(st, self.params, d), total

    def step(self, cams, targets, no_sync: bool = True):
        """One step over the views in `cams` (targets: [3, H, W] device tensors).
        Returns the summed loss as a device scalar.  With no_sync, binning does
        not wait on the host (buffers sized by the previous step); one counter is
        read before the update, and a step that ran out of instance capacity is
        redone with the waiting binning."""
        if self.repartition_every and self.step_count > 0 and self.step_count % self.repartition_every == 0:
            self.repartition()
        st, g, total = self._grads(cams, targets, no_sync)
        if st.bins_struct.n_instances < 0 and st.overflow():
            st, g, total = self._grads(cams, targets, False)
        self.step_count += 1
        adam_step(self.lib, self.params, g, self.m, self.v, self.step_count, self.lrs(self.step_count - 1))
        return total
