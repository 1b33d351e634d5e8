"""Batched multi-view training step: forward, loss and backward for V views in one batched
pass of the render path, optionally captured once into a HIP graph and replayed.

Each step: clod_project (all views), clod_bin_sort (one sort for all views: the view is part
of the key), clod_render_fwd, clod_loss (per-view L1 + point-count regulariser, Sec. 3.3
Eq. 3-5; the multi-view loss is the sum over views) and clod_render_bwd, whose per-Gaussian
gradients sum the views' contributions.

Graph replays read new poses and LoD scales from the device view table (write them with
``set_views`` between replays); resolutions are fixed at capture.  The duplicate buffer is
sized before capture; ``overflowed()`` reads the flag of the last step.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _clod as C
from .render import PLANES, Batch, Scene


class MultiViewTrainer:
    def __init__(self, scene: Scene, views, s_max: float, lambda_reg: float = 1.0, params=None,
                 dup_capacity: int | None = None, lambda_dssim: float = 0.0):
        self.scene = scene
        self.s_max = float(s_max)
        self.lambda_reg = float(lambda_reg)
        self.lambda_dssim = float(lambda_dssim)   # 0.2 gives the 3DGS L_render = 0.8 L1 + 0.2 D-SSIM
        self.batch = Batch(scene.n, views, params, dup_capacity=dup_capacity or 1)
        b = self.batch
        dev = "cuda"
        self.rgb = torch.empty(3 * b.pixels, device=dev, dtype=torch.float32)
        self.T = torch.empty(b.pixels, device=dev, dtype=torch.float32)
        self.last = torch.empty(b.pixels, dtype=torch.int32, device=dev)
        self.target = torch.zeros(3 * b.pixels, device=dev, dtype=torch.float32)
        self.loss = torch.empty(len(views), device=dev, dtype=torch.float32)
        self.dL = torch.empty_like(self.rgb)
        self.deta = torch.empty(len(views), device=dev, dtype=torch.float32)
        self.grads = {k: torch.zeros_like(v) for k, v in scene.t.items()}
        self.hdr = torch.empty(16, dtype=torch.uint8, pin_memory=True)
        # Per-pixel SSIM derivatives (36 B per pixel), only when the D-SSIM term is on.
        self.ssim_scratch = torch.empty(9 * b.pixels, device=dev, dtype=torch.float32) if self.lambda_dssim > 0 else None
        self.graph = None
        if dup_capacity is None:
            self.size_capacity()

    def size_capacity(self, views_list=None, margin: float = 1.25):
        """Runs the projection and sort eagerly for each set of views (default: the current
        ones) and sizes the duplicate buffer to the largest pair count times ``margin``."""
        b = self.batch
        sets = views_list or [b.views]
        dmax = 0
        for vs in sets:
            self.set_views(vs)
            b.project(self.scene)
            dmax = max(dmax, b.bin_sort())
        b._alloc_dup(int(dmax * margin) + 65536)
        self.set_views(sets[0])
        return dmax

    def set_views(self, views):
        """New poses and s_v (same resolutions) written into the device view table."""
        b = self.batch
        for v in views:
            if v.s_v > self.s_max:
                raise ValueError("s_v above s_max")
        b.update_views(views)

    def set_views_dev(self, table: torch.Tensor):
        """Copies a device view table (same resolutions, bytes of clod_view[V]) into place:
        a device-to-device copy, so replays can take inputs already resident in HBM."""
        self.batch.views_dev.copy_(table)

    def set_target(self, target_flat: torch.Tensor):
        self.target.copy_(target_flat)

    def _launch(self):
        b, sc = self.batch, self.scene
        bs = b.c_struct()
        s = sc.c_struct()
        C.clod_project(s, bs, b.counts)
        C.clod_bin_sort(bs, sync_count=False)
        C.clod_render_fwd(bs, self.rgb, self.T, self.last, None)
        if self.lambda_dssim > 0 and self.ssim_scratch is None:
            self.ssim_scratch = torch.empty(9 * b.pixels, device=self.rgb.device, dtype=torch.float32)
        C.clod_loss(bs, self.rgb, self.target, self.s_max, self.lambda_reg, self.loss, self.dL, self.deta,
                    lambda_dssim=self.lambda_dssim, ssim_scratch=self.ssim_scratch)
        C.clod_render_bwd(s, bs, self.T, self.last, self.dL, self.deta, False, C.make_grad(self.grads))
        ptr, _ = C.clod_inspect(bs, C.SEC_HEADER)
        off = ptr - b.ws.data_ptr()
        self.hdr.copy_(b.ws[off:off + 16], non_blocking=True)

    def step(self):
        """One fused step (eager, or the captured graph if ``capture`` was called)."""
        if self.graph is not None:
            self.graph.replay()
        else:
            self._launch()

    def capture(self):
        """Captures the step into a graph (warm-up launch first, as graph capture requires)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._launch()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._launch()
        torch.cuda.synchronize()
        self.graph = g

    def overflowed(self) -> bool:
        torch.cuda.current_stream().synchronize()
        return bool(self.hdr.view(torch.int64)[1].item())

    def n_dup(self) -> int:
        torch.cuda.current_stream().synchronize()
        return int(self.hdr.view(torch.int64)[0].item())

    def total_loss(self) -> float:
        return float(self.loss.sum().item())


# ---------------------------------------------------------------------------------------------
# Optimiser and schedule (Sec. 4.1)
# ---------------------------------------------------------------------------------------------

# 3DGS learning rates per parameter group; sigma_d uses 1e-2 (Sec. 4.1).  The position rate
# decays log-linearly over training (position_lr); SH degrees >= 1 use 1/20 of the DC rate.
DEFAULT_LRS = dict(mean=1.6e-4, log_scale=5e-3, quat=1e-3, opacity=2.5e-2, decay=1e-2, sh_dc=2.5e-3,
                   sh_rest=2.5e-3 / 20.0)


def position_lr(step: int, lr_init: float = 1.6e-4, lr_final: float = 1.6e-6, max_steps: int = 30000,
                extent: float = 1.0) -> float:
    t = min(max(step / max_steps, 0.0), 1.0)
    return float(np.exp(np.log(lr_init * extent) * (1 - t) + np.log(lr_final * extent) * t))


class FusedAdam:
    """Adam over every per-Gaussian parameter plane of a Scene in one launch (clod_adam_step):
    first and second moments in HBM beside the parameters, one read and one write per element."""

    def __init__(self, scene: Scene, betas=(0.9, 0.999), eps: float = 1e-15):
        self.scene = scene
        self.m = {k: torch.zeros_like(v) for k, v in scene.t.items()}
        self.v = {k: torch.zeros_like(v) for k, v in scene.t.items()}
        self.betas = betas
        self.eps = eps
        self.t = 0
        self._p = C.make_grad(scene.t)
        self._m = C.make_grad(self.m)
        self._v = C.make_grad(self.v)

    def step(self, grads: dict, lrs: dict, stream=None):
        self.t += 1
        hp = C.make_adam(lrs, self.t, self.betas[0], self.betas[1], self.eps)
        C.clod_adam_step(self.scene.n, self.scene.sh_degree, self._p, C.make_grad(grads), self._m, self._v, hp,
                         stream)


class LodSchedule:
    """Per-iteration training settings (Sec. 3.3 and Sec. 4.1): before `enable_at` the LoD
    mechanism is off (s_v = 1, no regulariser, sigma_d frozen); from then on every view draws
    its virtual distance scale from U(1, s_max) (log-uniform if law == "log") and the
    regulariser weight is lambda_reg.  The position learning rate decays over `total` steps."""

    def __init__(self, s_max: float, enable_at: int = 5000, total: int = 30000, lambda_reg: float = 1.0,
                 law: str = "uniform", lrs: dict | None = None, seed: int = 0):
        if law not in ("uniform", "log"):
            raise ValueError(law)
        self.s_max, self.enable_at, self.total, self.lambda_reg, self.law = s_max, enable_at, total, lambda_reg, law
        self.lrs = dict(DEFAULT_LRS if lrs is None else lrs)
        self.rng = np.random.default_rng(seed)

    def active(self, it: int) -> bool:
        return it >= self.enable_at

    def sample_sv(self, it: int, k: int) -> np.ndarray:
        if not self.active(it):
            return np.ones(k)
        if self.law == "uniform":
            return self.rng.uniform(1.0, self.s_max, size=k)
        return np.exp(self.rng.uniform(0.0, np.log(self.s_max), size=k))

    def lambda_at(self, it: int) -> float:
        return self.lambda_reg if self.active(it) else 0.0

    def lrs_at(self, it: int) -> dict:
        lr = dict(self.lrs)
        lr["mean"] = position_lr(it, lr_init=self.lrs["mean"], lr_final=self.lrs["mean"] / 100.0, max_steps=self.total)
        if not self.active(it):
            lr["decay"] = 0.0
        return lr
