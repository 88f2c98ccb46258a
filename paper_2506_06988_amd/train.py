"""Joint optimisation of Gaussians and texture map (Sec. 3.4; Alg. 1, stage 2).

One iteration renders one training view through the library, evaluates the
loss of Eq. 3 with the transmittance-aware term weighted by the Alg. 1
schedule, runs the backward into the Gaussian parameters and the texture, and
applies one Adam step to both. Every stage is a library entry point; this
module sequences them and owns the optimiser state and preallocated buffers.

Densification (clone / split / prune) is not performed here; the backward
accumulates the statistic it uses: per Gaussian, the sum over rendered views of
|dL/d mean2D| (pixel units) and the number of views in which it was visible.
A 3DGS-style threshold in NDC units converts as |g_ndc| = |g_px| * (W, H) / 2
per axis.

Learning rates and the position decay follow the 3DGS optimiser that the
paper trains with (Sec. 4: same schedule and hyperparameters); the texture
rate is not given by the paper and is a constructor argument.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Sequence

from . import hr


def lambda_t(i: int, lam: float = 0.1, warmup: int = 3000, densify_until: int = 15000) -> float:
    """L_t weight at iteration i (Alg. 1): on strictly between the end of the
    warm-up and the end of densification, off (L_c alone) elsewhere."""
    return lam if (i > warmup and i < densify_until) else 0.0


def exp_lr(step: int, lr_init: float, lr_final: float, max_steps: int) -> float:
    """Log-linear decay from lr_init at step 0 to lr_final at max_steps
    (clamped beyond), the 3DGS position-rate schedule."""
    t = min(max(step / max(1, max_steps), 0.0), 1.0)
    return math.exp((1.0 - t) * math.log(lr_init) + t * math.log(lr_final))


DEFAULT_LRS = dict(position_init=1.6e-4, position_final=1.6e-6, sh_dc=2.5e-3, sh_rest=2.5e-3 / 20,
                   opacity=0.05, scaling=5e-3, rotation=1e-3, texture=1e-3)


class Trainer:
    """Owns a Renderer over one view at a time, Adam moments and buffers.

    views: cameras of equal size; targets: one [3, H, W] float32 device tensor
    per view. `extent` scales the position rate (the 3DGS scene extent).
    """

    def __init__(self, gaussians: "hr.DevGaussians", mesh, views: Sequence, targets, extent=1.0,
                 max_iters=30000, lrs=None, lambda_c=0.2, lam=0.1, warmup=3000,
                 densify_until=15000, k=20.0, mask_mode="sigmoid", settings=None):
        import torch
        self.views = list(views)
        assert len(targets) == len(self.views) and self.views
        w, h = self.views[0].width, self.views[0].height
        assert all((c.width, c.height) == (w, h) for c in self.views), "views must share one size"
        self.r = hr.Renderer(gaussians, mesh, [self.views[0]], settings=settings)
        self.targets = [t.contiguous().reshape(-1) for t in targets]
        self.lrs = dict(DEFAULT_LRS, **(lrs or {}))
        self.extent, self.max_iters = float(extent), int(max_iters)
        self.lambda_c, self.lam, self.k = float(lambda_c), float(lam), float(k)
        self.warmup, self.densify_until = int(warmup), int(densify_until)
        self.mask_mode = hr.MASK_MODES[mask_mode]
        self.it = 0
        g = gaussians
        self.params = dict(means=g.means, log_scales=g.log_scales, quats=g.quats,
                           opacity_logits=g.opacity_logits, sh=g.sh)
        if mesh is not None:
            self.params["tex"] = mesh.tex
        for t in self.params.values():
            assert t.is_contiguous() and t.dtype == torch.float32
        self.grads = {k_: torch.zeros_like(v) for k_, v in self.params.items()}
        self.m = {k_: torch.zeros_like(v) for k_, v in self.params.items()}
        self.v = {k_: torch.zeros_like(v) for k_, v in self.params.items()}
        n = g.n
        self.grads["mean2d_norm"] = torch.zeros(n, dtype=torch.float32, device=g.means.device)
        self.grads["mean2d_count"] = torch.zeros(n, dtype=torch.int32, device=g.means.device)
        self.frame = self.r.new_frame()
        self._sizes = (C.c_int32 * 2)(w, h)
        nb = int(self.r.L.hr_full_loss_scratch_bytes(self._sizes, 1))
        self._scratch = torch.empty(nb, dtype=torch.uint8, device=g.means.device)
        P = w * h
        dev = g.means.device
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self._gi = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self._gt = torch.empty(P, dtype=torch.float32, device=dev)
        self._gm = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.K = (g.sh_degree + 1) ** 2

    def reset_densification_stats(self):
        self.grads["mean2d_norm"].zero_()
        self.grads["mean2d_count"].zero_()

    def adam_groups(self, it: int):
        lr = self.lrs
        pos = exp_lr(it, lr["position_init"] * self.extent, lr["position_final"] * self.extent,
                     self.max_iters)
        rates = dict(means=(pos,), log_scales=(lr["scaling"],), quats=(lr["rotation"],),
                     opacity_logits=(lr["opacity"],),
                     sh=(lr["sh_rest"], lr["sh_dc"], 3, 3 * self.K), tex=(lr["texture"],))
        return [(self.params[k_], self.grads[k_], self.m[k_], self.v[k_]) + rates[k_]
                for k_ in self.params]

    def step(self):
        """One iteration; returns the loss as a 1-element device tensor."""
        it = self.it
        self.it += 1
        vi = it % len(self.views)
        self.r.set_cameras([self.views[vi]])
        tex = self.params.get("tex")
        f = self.r.render_hybrid(frame=self.frame, tex=tex)
        lt = lambda_t(it, self.lam, self.warmup, self.densify_until)
        L = self.r.L
        hr.check(L.hr_full_loss(hr._ptr(f.image), hr._ptr(f.final_T), hr._ptr(f.mesh_rgb),
                                hr._ptr(f.tri_id), hr._ptr(self.targets[vi]), self._sizes, 1,
                                self.lambda_c, lt, self.k, self.mask_mode, 0, hr._ptr(self.loss),
                                hr._ptr(self._gi), hr._ptr(self._gt), hr._ptr(self._gm),
                                hr._ptr(self._scratch), hr._stream()))
        for k_ in self.params:
            self.grads[k_].zero_()
        self.r.render_hybrid_backward(self._gi, self._gt, self._gm, grads=self.grads, tex=tex)
        hr.adam_step(self.adam_groups(it), it + 1)
        return self.loss
