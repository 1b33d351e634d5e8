"""Seeded synthetic inputs: scenes, cameras and request streams.

This module only draws inputs.  It holds none of the render method's arithmetic and is the
one piece shared by the HIP path and the CPU oracle (both read the float32 arrays it makes).

Every array is drawn with ``numpy.random.default_rng(seed)`` (PCG64): the large SH planes
directly in float32, everything else in float64 and cast to float32.  Scene draw order: means, log-scales, quaternions, opacity logits, SH
coefficients, decay parameters.  Cameras and requests use ``default_rng(seed + 1000)``.

Shapes follow the paper's scenes (Sec. 4.1 and the per-scene tables: 0.4M-8.6M Gaussians,
SH degree 3, one extra decay float per Gaussian, Sec. 3.2):

* ``mean``      float32 [3][n]   (plane-major)
* ``log_scale`` float32 [3][n]
* ``quat``      float32 [4][n]   (w, x, y, z), unit length
* ``opacity``   float32 [n]      logits
* ``decay``     float32 [n]      sigma_d
* ``sh``        float32 [(deg+1)^2][3][n]
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Standard deviation of the degree-0 SH coefficient that gives a degree-0 colour with
# standard deviation 0.2 around 0.5 (0.2 divided by the degree-0 basis value 0.28209...).
DC_STD = 0.7089815403622064
HIGHER_SH_STD = 0.05


def make_scene(n: int, sh_degree: int, layout: str = "uniform", seed: int = 0,
               n_clusters: int = 64, cluster_sigma: float = 0.3, box: float = 5.0,
               log_scale_mean: float = -4.0, log_scale_std: float = 0.5,
               decay_std: float = 0.5) -> dict:
    """A seeded scene.

    layout="uniform": means uniform in [-1, 1]^3.
    layout="mixture": ``n_clusters`` centres uniform in [-box, box]^3; each Gaussian picks a
    centre uniformly, adds N(0, cluster_sigma^2 I) and is clamped to the box.
    """
    if n < 0 or sh_degree not in (0, 1, 2, 3):
        raise ValueError("bad scene size or SH degree")
    rng = np.random.default_rng(seed)
    if layout == "uniform":
        mean = rng.uniform(-1.0, 1.0, size=(3, n))
    elif layout == "mixture":
        centres = rng.uniform(-box, box, size=(n_clusters, 3))
        pick = rng.integers(0, n_clusters, size=n)
        mean = centres[pick].T + rng.normal(0.0, cluster_sigma, size=(3, n))
        mean = np.clip(mean, -box, box)
    else:
        raise ValueError(layout)
    log_scale = rng.normal(log_scale_mean, log_scale_std, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.maximum(np.linalg.norm(q, axis=0, keepdims=True), 1e-30)
    opacity = rng.normal(0.0, 1.0, size=n)
    K = (sh_degree + 1) ** 2
    sh = np.empty((K, 3, n), dtype=np.float32)
    sh[0] = rng.standard_normal(size=(3, n), dtype=np.float32) * np.float32(DC_STD)
    if K > 1:
        sh[1:] = rng.standard_normal(size=(K - 1, 3, n), dtype=np.float32) * np.float32(HIGHER_SH_STD)
    decay = rng.normal(0.0, decay_std, size=n)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(n=n, sh_degree=sh_degree, mean=f(mean), log_scale=f(log_scale), quat=f(q),
                opacity=f(opacity), decay=f(decay), sh=f(sh))


@dataclasses.dataclass
class View:
    """A pinhole camera (OpenCV axes: x right, y down, z forward) plus its LoD scale.

    ``W`` is the row-major world-to-camera rotation, ``t`` the translation, ``c`` the camera
    centre; a pixel (i, j) covers [i, i+1) x [j, j+1).  ``s_v`` is the virtual distance scale;
    ``budget`` selects the LoD rule (0: alpha'' > tau s_v; K > 0: the K largest alpha'').
    """
    W: np.ndarray
    t: np.ndarray
    c: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    s_v: float = 1.0
    budget: int = 0   # 0: threshold mask; K > 0: keep the K largest alpha''
    frame_width: int = 0    # > 0: this view renders a viewport of a larger frame
    frame_height: int = 0
    vx: int = 0             # viewport origin in the frame (multiples of 16)
    vy: int = 0


def look_at(pos, target=(0.0, 0.0, 0.0), width=256, height=256, fov_deg=60.0, s_v=1.0) -> View:
    """Camera at ``pos`` looking at ``target``; world up +y (+z when nearly parallel);
    horizontal field of view ``fov_deg``; principal point at the image centre."""
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    W = np.stack([x, y, f])
    t = -W @ pos
    focal = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return View(W=W.astype(np.float32), t=t.astype(np.float32), c=pos.astype(np.float32),
                fx=float(np.float32(focal)), fy=float(np.float32(focal)),
                cx=float(width) / 2.0, cy=float(height) / 2.0,
                width=int(width), height=int(height), s_v=float(np.float32(s_v)))


def viewport(view: View, x: int, y: int, width: int, height: int, s_v: float | None = None,
             budget: int | None = None) -> View:
    """The window [x, x + width) x [y, y + height) of `view`'s image as a view of its own (x, y
    multiples of 16), optionally with its own virtual distance scale and budget: the frustum,
    its maximum distance and the pixel coordinates stay those of the whole frame."""
    fw = view.frame_width or view.width
    fh = view.frame_height or view.height
    return dataclasses.replace(view, width=int(width), height=int(height), frame_width=fw, frame_height=fh,
                               vx=view.vx + int(x), vy=view.vy + int(y),
                               s_v=view.s_v if s_v is None else float(np.float32(s_v)),
                               budget=view.budget if budget is None else int(budget))


def strips(view: View, s_values) -> list[View]:
    """Vertical strips of equal tile-aligned width covering `view`, strip r at s_values[r]
    (spatially varying virtual distance scale)."""
    k = len(s_values)
    tiles = (view.width + 15) // 16
    edges = [16 * ((tiles * r) // k) for r in range(k)] + [view.width]
    return [viewport(view, edges[r], 0, edges[r + 1] - edges[r], view.height, s_v=s_values[r]) for r in range(k)]


def unit_vectors(rng, k: int) -> np.ndarray:
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def log_uniform(rng, lo: float, hi: float, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))


def random_views(seed: int, k: int, radius=(4.0, 6.0), resolutions=((1297, 840),),
                 sv_range=(1.0, 8.0), fov_deg=60.0) -> list[View]:
    """k views on a sphere (direction uniform on S^2, radius uniform in ``radius``) looking
    at the origin; resolution uniform over ``resolutions``; s_v log-uniform in sv_range."""
    rng = np.random.default_rng(seed + 1000)
    dirs = unit_vectors(rng, k)
    radii = rng.uniform(radius[0], radius[1], size=k)
    res_idx = rng.integers(0, len(resolutions), size=k)
    svs = log_uniform(rng, sv_range[0], sv_range[1], size=k)
    out = []
    for j in range(k):
        w, h = resolutions[int(res_idx[j])]
        out.append(look_at(dirs[j] * radii[j], width=w, height=h, fov_deg=fov_deg, s_v=float(svs[j])))
    return out


def sweep_distances(k: int = 64, lo: float = 2.0, hi: float = 200.0) -> np.ndarray:
    """k distances log-spaced in [lo, hi] along one ray."""
    return lo * (hi / lo) ** (np.arange(k) / (k - 1))


def random_target(seed: int, height: int, width: int) -> np.ndarray:
    """Target image, uniform in [0, 1), float32 [3][H][W]."""
    rng = np.random.default_rng(seed + 2000)
    return rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    view: View


def poisson_requests(seed: int, count: int, rate_hz: float = 200.0, radius=(3.0, 30.0),
                     sv_range=(1.0, 16.0),
                     resolutions=((1280, 720), (1920, 1080), (3840, 2160))) -> list[Request]:
    """A Poisson request stream: exponential gaps at ``rate_hz``, pose direction uniform on
    S^2 with radius uniform in ``radius``, s_v log-uniform, resolution uniform."""
    rng = np.random.default_rng(seed + 1000)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    dirs = unit_vectors(rng, count)
    radii = rng.uniform(radius[0], radius[1], size=count)
    svs = log_uniform(rng, sv_range[0], sv_range[1], size=count)
    res_idx = rng.integers(0, len(resolutions), size=count)
    out = []
    for j in range(count):
        w, h = resolutions[int(res_idx[j])]
        out.append(Request(rid=j, arrival_s=float(t[j]),
                           view=look_at(dirs[j] * radii[j], width=w, height=h, s_v=float(svs[j]))))
    return out
