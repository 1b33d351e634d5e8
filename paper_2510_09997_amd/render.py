"""High-level use of libclod from PyTorch: device-resident scenes, view batches with their
workspaces, a differentiable render (torch.autograd.Function) and the fused training step.

PyTorch only allocates device memory and supplies the stream; every step of the render path
runs in libclod's HIP kernels.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _clod as C

PLANES = ("mean", "log_scale", "quat", "opacity", "decay", "sh")


class Scene:
    """A device-resident scene in the C layout (float32 planes, see include/clod.h)."""

    def __init__(self, planes: dict, device="cuda", packed_sh: bool = False, spatial_order: bool = False):
        self.n = int(planes["n"])
        self.sh_degree = int(planes["sh_degree"])
        self.t = {}
        for k in PLANES:
            v = planes[k]
            if isinstance(v, np.ndarray):
                v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32))
            self.t[k] = v.to(device=device, dtype=torch.float32).contiguous()
        # spatial_order: the Gaussians are stored along a Morton curve of their means
        # (clod_scene_reorder); self.perm[j] is the caller's index of stored Gaussian j.
        self.perm = None
        self.sh_packed = None
        if spatial_order and self.n > 0:
            if self.t["mean"].device.type != "cuda":
                raise ValueError("spatial_order needs the scene on the GPU (clod_scene_reorder takes device planes)")
            dst = {k: torch.empty_like(v) for k, v in self.t.items()}
            perm = torch.empty(self.n, dtype=torch.int32, device=device)
            ws = torch.empty(C.clod_scene_reorder_ws_bytes(self.n), dtype=torch.uint8, device=device)
            C.clod_scene_reorder(self.c_struct(), C.make_grad(dst), perm, ws)
            torch.cuda.synchronize()
            del ws
            self.t, self.perm = dst, perm
        # Static scenes (serving) may also keep the SH coefficients per Gaussian
        # ([n][K][3]), which the projection gathers far more cheaply for its sparse set.
        self.sh_packed = None
        if packed_sh:
            K = (self.sh_degree + 1) ** 2
            self.sh_packed = self.t["sh"].view(K, 3, self.n).permute(2, 0, 1).contiguous()

    def c_struct(self, planes: dict | None = None) -> C.clod_scene:
        d = dict(self.t if planes is None else planes)
        d["n"], d["sh_degree"] = self.n, self.sh_degree
        if planes is None and self.sh_packed is not None:
            d["sh_packed"] = self.sh_packed
        return C.make_scene(d)

    def zeros_like(self) -> dict:
        return {k: torch.zeros_like(v) for k, v in self.t.items()}

    def nbytes(self) -> int:
        extra = 0 if self.sh_packed is None else self.sh_packed.numel() * 4
        return sum(v.numel() * 4 for v in self.t.values()) + extra


def default_params(**kw) -> C.clod_params:
    return C.make_params(**kw)


class Batch:
    """A batch of views with its workspaces.  Pixel offsets of view v: ``self.pix_base[v]``."""

    def __init__(self, n: int, views, params: C.clod_params | None = None, dup_capacity: int | None = None,
                 device="cuda"):
        self.device = device
        self.views = list(views)
        self.params = params if params is not None else default_params()
        self.n = int(n)
        self.views_host = C.make_views(self.views)
        self.views_dev = C.views_to_device(self.views_host, device)
        V = len(self.views)
        self.sizes = [(v.height, v.width) for v in self.views]
        self.pix_base = np.concatenate([[0], np.cumsum([h * w for h, w in self.sizes])]).astype(np.int64)
        self.pixels = int(self.pix_base[-1])
        ws_bytes = C.clod_ws_bytes(self.n, self.views_host)
        if ws_bytes == 0:
            raise ValueError("invalid views")
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        if dup_capacity is None:
            dup_capacity = max(1 << 16, 4 * self.n * V)
        self._alloc_dup(dup_capacity)
        self.n_views = V
        self.counts = torch.zeros(V, 3, dtype=torch.int64, device=device)
        self.eta = torch.zeros(V, dtype=torch.float32, device=device)   # eta_actual per view (Eq. 4)

    def _alloc_dup(self, capacity: int):
        nbytes = C.clod_dup_bytes(int(capacity))
        self.dup = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.capacity = C.clod_dup_capacity(nbytes)

    def c_struct(self) -> C.clod_batch:
        b = C.clod_batch()
        b.n = self.n
        b.n_views = len(self.views)
        b.views_host = C.ctypes.cast(self.views_host, C.P)
        b.views_dev = self.views_dev.data_ptr()
        b.params = self.params
        b.ws = self.ws.data_ptr()
        b.ws_bytes = self.ws.numel()
        b.dup = self.dup.data_ptr()
        b.dup_bytes = self.dup.numel()
        return b

    def update_views(self, views):
        """New poses / s_v with the same resolutions (device copy updated in place)."""
        assert [(v.height, v.width) for v in views] == self.sizes
        self.views = list(views)
        self.views_host = C.make_views(self.views)
        self.views_dev.copy_(C.views_to_device(self.views_host, self.device))
        need = C.clod_ws_bytes(self.n, self.views_host)   # a budget view needs select histograms
        if need > self.ws.numel():
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)

    def split(self, flat: torch.Tensor, channels: int):
        out = []
        for v, (h, w) in enumerate(self.sizes):
            a = int(self.pix_base[v]) * channels
            out.append(flat[a:a + channels * h * w].view(channels, h, w) if channels > 1
                       else flat[a:a + h * w].view(h, w))
        return out

    # ---- stages --------------------------------------------------------------------------
    def project(self, scene: Scene):
        C.clod_project(scene.c_struct(), self.c_struct(), self.counts, eta=self.eta)

    def bin_sort(self, sync: bool = True, grow: float = 1.5) -> int | None:
        """Bins and sorts; with sync=True reads the pair count and grows the duplicate
        buffer (re-running the sort) when it was too small."""
        if not sync:
            C.clod_bin_sort(self.c_struct(), sync_count=False)
            return None
        while True:
            try:
                return C.clod_bin_sort(self.c_struct(), sync_count=True)
            except C.CapacityError:
                info = C.clod_read_info(self.c_struct())
                self._alloc_dup(int(info["n_dup"] * grow) + 1024)

    def render_fwd(self, pairs: torch.Tensor | None = None):
        rgb = torch.empty(3 * self.pixels, dtype=torch.float32, device=self.device)
        T = torch.empty(self.pixels, dtype=torch.float32, device=self.device)
        last = torch.empty(self.pixels, dtype=torch.int32, device=self.device)
        C.clod_render_fwd(self.c_struct(), rgb, T, last, pairs)
        return rgb, T, last

    def render_bwd(self, scene: Scene, T, last, dL_drgb, dL_deta=None, grads: dict | None = None,
                   accumulate: bool = False, pairs: torch.Tensor | None = None) -> dict:
        """pairs (int64 [3], zeroed by the caller) receives the adjoint loop's work counters."""
        if grads is None:
            grads = {k: torch.empty_like(v) for k, v in scene.t.items()}
        C.clod_render_bwd(scene.c_struct(), self.c_struct(), T, last, dL_drgb.contiguous(),
                          None if dL_deta is None else dL_deta.contiguous(), accumulate, C.make_grad(grads),
                          pairs=pairs)
        return grads

    def section(self, section: int, count: int | None = None) -> torch.Tensor:
        """A device tensor copy of an intermediate section (see clod_inspect)."""
        ptr, n = C.clod_inspect(self.c_struct(), section)
        if count is not None:
            n = min(n, int(count))
        elem = {C.SEC_KEYS: 4, C.SEC_VALUES: 4, C.SEC_RANGES: 8, C.SEC_REC: 64, C.SEC_ALPHA: 4,
                C.SEC_FLAGS: 1, C.SEC_DMAX: 8, C.SEC_GSCREEN: 36}[section]
        base = self.dup if section in (C.SEC_KEYS, C.SEC_VALUES) else self.ws
        off = ptr - base.data_ptr()
        assert 0 <= off and off + n * elem <= base.numel()
        raw = base[off:off + n * elem].clone()
        if section == C.SEC_GSCREEN:
            # Nine partials per (view, Gaussian), interleaved: returned as [VN, 9].
            return raw.view(torch.float32).view(n, 9)
        dt = {8: torch.int64, 4: torch.int32, 64: torch.float32, 1: torch.uint8}[elem]
        if section == C.SEC_ALPHA:
            dt = torch.float32
        t = raw.view(dt)
        if section == C.SEC_REC:
            t = t.view(n, 4, 4)
        if section == C.SEC_RANGES:
            t = raw.view(torch.int32).view(n, 2)
        return t

    def lod_count(self, scene: Scene) -> torch.Tensor:
        out = torch.empty(len(self.views), 3, dtype=torch.int64, device=self.device)
        C.clod_lod_count(scene.c_struct(), self.c_struct(), out)
        return out

    def loss(self, rgb, target, s_max: float, lambda_reg: float = 1.0, lambda_dssim: float = 0.0):
        loss = torch.empty(len(self.views), dtype=torch.float32, device=self.device)
        dL_drgb = torch.empty_like(rgb)
        dL_deta = torch.empty(len(self.views), dtype=torch.float32, device=self.device)
        scratch = torch.empty(9 * self.pixels, dtype=torch.float32, device=self.device) if lambda_dssim > 0 else None
        C.clod_loss(self.c_struct(), rgb, target, s_max, lambda_reg, loss, dL_drgb, dL_deta,
                    lambda_dssim=lambda_dssim, ssim_scratch=scratch)
        return loss, dL_drgb, dL_deta


def render(scene: Scene, views, params=None, batch: Batch | None = None):
    """Forward render of a list of views; returns (rgb list [3,H,W], T list, last list, batch)."""
    b = batch if batch is not None else Batch(scene.n, views, params)
    b.project(scene)
    b.bin_sort()
    rgb, T, last = b.render_fwd()
    return b.split(rgb, 3), b.split(T, 1), b.split(last, 1), b


class ClodRender(torch.autograd.Function):
    """Differentiable CLoD render of a batch of views.

    Inputs: the six parameter planes (leaf tensors in the C layout) and a ``Batch``.
    Outputs: rgb (flat, views concatenated as [3][H][W]) and eta [V] = n_mask / n, whose
    gradient is passed straight through to every alpha'' (the kept-primitive mass).
    """

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, decay, sh, batch: Batch, sh_degree: int):
        planes = dict(mean=mean.contiguous(), log_scale=log_scale.contiguous(), quat=quat.contiguous(),
                      opacity=opacity.contiguous(), decay=decay.contiguous(), sh=sh.contiguous(),
                      n=mean.shape[1], sh_degree=sh_degree)
        scene = C.make_scene(planes)
        C.clod_project(scene, batch.c_struct(), batch.counts, eta=batch.eta)
        batch.bin_sort()
        rgb, T, last = batch.render_fwd()
        eta = batch.eta.clone()
        ctx.batch = batch
        ctx.sh_degree = sh_degree
        ctx.save_for_backward(planes["mean"], planes["log_scale"], planes["quat"], planes["opacity"],
                              planes["decay"], planes["sh"], T, last)
        ctx.mark_non_differentiable(T, last)
        return rgb, eta, T, last

    @staticmethod
    def backward(ctx, g_rgb, g_eta, g_T, g_last):
        mean, log_scale, quat, opacity, decay, sh, T, last = ctx.saved_tensors
        planes = dict(mean=mean, log_scale=log_scale, quat=quat, opacity=opacity, decay=decay, sh=sh,
                      n=mean.shape[1], sh_degree=ctx.sh_degree)
        grads = {k: torch.empty_like(planes[k]) for k in PLANES}
        if g_rgb is None:
            g_rgb = torch.zeros(3 * ctx.batch.pixels, dtype=torch.float32, device=mean.device)
        C.clod_render_bwd(C.make_scene(planes), ctx.batch.c_struct(), T, last, g_rgb.contiguous(),
                          None if g_eta is None else g_eta.to(torch.float32).contiguous(), False,
                          C.make_grad(grads))
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity"], grads["decay"],
                grads["sh"], None, None)


def train_step(scene: Scene, batch: Batch, target_flat: torch.Tensor, s_max: float, lambda_reg: float = 1.0,
               grads: dict | None = None, sync_sort: bool = True):
    """One fused forward + loss + backward over the batch's views (Sec. 3.3, Eq. 5 with
    L_render = L1; multi-view loss = sum over views).  Returns (loss per view, grads)."""
    batch.project(scene)
    batch.bin_sort(sync=sync_sort)
    rgb, T, last = batch.render_fwd()
    loss, dL_drgb, dL_deta = batch.loss(rgb, target_flat, s_max, lambda_reg)
    grads = batch.render_bwd(scene, T, last, dL_drgb, dL_deta, grads=grads, accumulate=False)
    return loss, grads, rgb
