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
                 dup_capacity: int | None = None):
        self.scene = scene
        self.s_max = float(s_max)
        self.lambda_reg = float(lambda_reg)
        self.batch = Batch(scene.n, views, params, dup_capacity=dup_capacity or 1)
        b = self.batch
        dev = "cuda"
        self.rgb = torch.empty(3 * b.pixels, device=dev)
        self.T = torch.empty(b.pixels, device=dev)
        self.last = torch.empty(b.pixels, dtype=torch.int32, device=dev)
        self.target = torch.zeros(3 * b.pixels, device=dev)
        self.loss = torch.empty(len(views), device=dev)
        self.dL = torch.empty_like(self.rgb)
        self.deta = torch.empty(len(views), device=dev)
        self.grads = {k: torch.zeros_like(v) for k, v in scene.t.items()}
        self.hdr = torch.empty(16, dtype=torch.uint8, pin_memory=True)
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
        C.clod_loss(bs, self.rgb, self.target, self.s_max, self.lambda_reg, self.loss, self.dL, self.deta)
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
