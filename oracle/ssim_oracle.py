"""Oracle for the D-SSIM part of the rendering loss.  TEST INFRASTRUCTURE ONLY: imported by
tests, the smoke check and the benchmark's CPU-baseline leg, never by the product path.

Sec. 3.3, Eq. (5): L_render is the 3DGS rendering loss, a weighted sum of L1 and D-SSIM:
    L_render = (1 - lambda_dssim) * L1 + lambda_dssim * (1 - SSIM),   lambda_dssim = 0.2,
with SSIM the structural similarity of Wang et al. (2004) computed per colour channel with an
11 x 11 Gaussian window (sigma 1.5, normalised to sum 1), C1 = 0.01^2, C2 = 0.03^2, the image
zero-padded by 5 pixels so the map has the image's size, and averaged over all pixels and
channels.  Per pixel, with the window-weighted means mu, variances sigma^2 and covariance:
    S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
    sigma_x^2 = E[x^2] - mu_x^2,  sigma_xy = E[xy] - mu_x mu_y.

Two independent float64 implementations: `ssim_map64` (numpy, explicit separable
correlation) and `dssim_torch64` (plain PyTorch conv2d, differentiated by autograd); tests pin
each against the other and against closed forms.
"""
from __future__ import annotations

import numpy as np
import torch

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WIN = 11
SIGMA = 1.5
LAMBDA_DSSIM = 0.2


def window1d() -> np.ndarray:
    k = np.arange(WIN) - WIN // 2
    g = np.exp(-(k * k) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def _filter(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Zero-padded 'same' correlation of a 2D image with the separable window g (x) g."""
    h, w = img.shape
    r = WIN // 2
    p = np.zeros((h + 2 * r, w + 2 * r))
    p[r:r + h, r:r + w] = img
    rows = sum(g[k] * p[:, k:k + w] for k in range(WIN))          # horizontal
    return sum(g[k] * rows[k:k + h, :] for k in range(WIN))        # vertical


def ssim_map64(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM map [C][H][W] of two images [C][H][W] (float64)."""
    g = window1d()
    out = np.empty(x.shape)
    for ch in range(x.shape[0]):
        a, b = x[ch].astype(np.float64), y[ch].astype(np.float64)
        mx, my = _filter(a, g), _filter(b, g)
        sxx = _filter(a * a, g) - mx * mx
        syy = _filter(b * b, g) - my * my
        sxy = _filter(a * b, g) - mx * my
        out[ch] = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return out


def ssim64(x: np.ndarray, y: np.ndarray) -> float:
    return float(ssim_map64(x, y).mean())


def dssim_torch64(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """1 - SSIM of two [C][H][W] float64 tensors with plain conv2d (differentiable)."""
    g = torch.from_numpy(window1d())
    w2 = (g[:, None] * g[None, :]).expand(x.shape[0], 1, WIN, WIN).contiguous()
    conv = lambda t: torch.nn.functional.conv2d(t[None], w2, padding=WIN // 2, groups=x.shape[0])[0]
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    s = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
    return 1.0 - s.mean()


def render_loss64(x: np.ndarray, y: np.ndarray, lambda_dssim: float = LAMBDA_DSSIM, abs_terms: bool = False):
    """L_render and its gradient with respect to x ([C][H][W]), float64.  With ``abs_terms``
    also the absolute adjoint of the gradient (per pixel, the sum of the magnitudes of its
    chain-rule terms; see abs_adjoint.py) as a third result."""
    def run(mode):
        xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
        yt = torch.tensor(np.asarray(y, np.float64))
        with mode:
            l1 = (xt - yt).abs().mean()
            loss = (1.0 - lambda_dssim) * l1 + lambda_dssim * dssim_torch64(xt, yt)
        loss.backward()
        return float(loss.detach()), xt.grad.numpy()

    import contextlib
    loss, g = run(contextlib.nullcontext())
    if not abs_terms:
        return loss, g
    from .abs_adjoint import AbsAdjointMode
    return loss, g, run(AbsAdjointMode())[1]
