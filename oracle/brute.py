"""No-tile brute-force renderer in numpy float64, for tiny scenes.  TEST INFRASTRUCTURE ONLY.

It computes Eq. (1) of Sec. 3.1 for every pixel directly from its definition: the set of
rendered Gaussians that support the pixel (the 3-sigma screen rectangle of the Gaussian,
rounded out to 16x16 tiles, contains the pixel's tile), ordered by (depth, index), blended
front to back with the skip (alpha' < 1/255), clamp (0.99) and termination (T < 1e-4) rules.
Attenuated opacity and mask follow Sec. 3.2, Eq. (2).  Everything is double precision and
written independently of clod_oracle.c; it also reports how close each decision came to
its threshold so that tests can use seeds where float32 and float64 cannot disagree.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as _o


def _sh64(d: np.ndarray, deg: int) -> np.ndarray:
    X, Y, Z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    cols = [np.full_like(X, 1.0 / (2.0 * math.sqrt(pi)))]
    if deg >= 1:
        k = math.sqrt(3.0 / (4.0 * pi))
        cols += [k * Y, k * Z, k * X]
    if deg >= 2:
        a, b, c = 0.5 * math.sqrt(15 / pi), 0.25 * math.sqrt(5 / pi), 0.25 * math.sqrt(15 / pi)
        cols += [a * X * Y, a * Y * Z, b * (2 * Z * Z - X * X - Y * Y), a * X * Z, c * (X * X - Y * Y)]
    if deg >= 3:
        a = 0.25 * math.sqrt(35 / (2 * pi)); b = 0.5 * math.sqrt(105 / pi)
        c = 0.25 * math.sqrt(21 / (2 * pi)); e = 0.25 * math.sqrt(7 / pi); f = 0.25 * math.sqrt(105 / pi)
        t4 = 4 * Z * Z - X * X - Y * Y
        cols += [a * Y * (3 * X * X - Y * Y), b * X * Y * Z, c * Y * t4, e * Z * (2 * Z * Z - 3 * X * X - 3 * Y * Y),
                 c * X * t4, f * Z * (X * X - Y * Y), a * X * (X * X - 3 * Y * Y)]
    return np.stack(cols, axis=1)


def render(scene: dict, view, params: dict | None = None) -> dict:
    p = {**_o.DEFAULT_PARAMS, **(params or {})}
    n, deg = scene["n"], scene["sh_degree"]
    W = np.asarray(view.W, np.float64)
    t = np.asarray(view.t, np.float64)
    c = np.asarray(view.c, np.float64)
    mu = scene["mean"].astype(np.float64)                 # [3, n]
    pc = W @ mu + t[:, None]
    x, y, z = pc
    assert not getattr(view, "frame_width", 0), "the brute force renders whole frames only"
    w_img, h_img = view.width, view.height
    tanx = p["guard"] * (0.5 * w_img) / view.fx
    tany = p["guard"] * (0.5 * h_img) / view.fy
    F = (z > p["near"]) & (np.abs(x) <= tanx * z) & (np.abs(y) <= tany * z)
    margins = []
    e = mu - c[:, None]
    d = np.sqrt((e * e).sum(0))
    dmax = d[F].max() if F.any() else 1.0
    dn = d / dmax
    r = np.maximum(scene["decay"].astype(np.float64), 0.0)
    q = (dn * view.s_v) ** 2 / (2 * r * r + p["eps"])
    alpha = 1.0 / (1.0 + np.exp(-scene["opacity"].astype(np.float64)))
    a2 = alpha * np.exp(-q)
    thr = p["tau"] * view.s_v
    M = a2 > thr
    margins.append(np.abs(a2 - thr) / max(thr, 1e-30))
    margins.append(np.abs(z - p["near"]) / p["near"])
    margins.append(np.abs(np.abs(x) - tanx * z) / np.maximum(np.abs(z), 1e-9))
    margins.append(np.abs(np.abs(y) - tany * z) / np.maximum(np.abs(z), 1e-9))

    s = np.exp(scene["log_scale"].astype(np.float64))
    qv = scene["quat"].astype(np.float64)
    qv = qv / np.linalg.norm(qv, axis=0, keepdims=True)
    rendered = np.zeros(n, bool)
    rect = np.zeros((n, 4), np.int64)
    u = np.zeros(n); v = np.zeros(n); A = np.zeros(n); B = np.zeros(n); C = np.zeros(n)
    col = np.zeros((n, 3))
    TW, TH = (w_img + 15) // 16, (h_img + 15) // 16
    for i in np.nonzero(F & M)[0]:
        qw, qx, qy, qz = qv[:, i]
        R = np.array([[1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
                      [2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)],
                      [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)]])
        Sig = R @ np.diag(s[:, i] ** 2) @ R.T
        J = np.array([[view.fx / z[i], 0, -view.fx * x[i] / z[i] ** 2],
                      [0, view.fy / z[i], -view.fy * y[i] / z[i] ** 2]])
        cov = J @ W @ Sig @ W.T @ J.T + p["dilation"] * np.eye(2)
        det = np.linalg.det(cov)
        if det <= 0:
            continue
        inv = np.linalg.inv(cov)
        lam = 0.5 * (cov[0, 0] + cov[1, 1]) + math.sqrt(max(0.0, (0.5 * (cov[0, 0] + cov[1, 1])) ** 2 - det))
        r3 = 3.0 * math.sqrt(lam)
        rad = math.ceil(r3)
        margins.append(np.array([abs(r3 - round(r3))]))
        ui = view.fx * x[i] / z[i] + view.cx
        vi = view.fy * y[i] / z[i] + view.cy
        for val in ((ui - rad) / 16, (ui + rad) / 16, (vi - rad) / 16, (vi + rad) / 16):
            margins.append(np.array([abs(val - round(val))]))
        x0 = min(max(math.floor((ui - rad) / 16), 0), TW); x1 = min(max(math.floor((ui + rad) / 16) + 1, 0), TW)
        y0 = min(max(math.floor((vi - rad) / 16), 0), TH); y1 = min(max(math.floor((vi + rad) / 16) + 1, 0), TH)
        if x0 >= x1 or y0 >= y1:
            continue
        dirv = e[:, i] / d[i]
        Yb = _sh64(dirv[None, :], deg)[0]
        shc = scene["sh"][:, :, i].astype(np.float64)    # [K, 3]
        col[i] = np.maximum(Yb @ shc + 0.5, 0.0)
        rendered[i] = True
        rect[i] = (x0, x1, y0, y1)
        u[i], v[i] = ui, vi
        A[i], B[i], C[i] = inv[0, 0], inv[0, 1], inv[1, 1]

    rgb = np.zeros((3, h_img, w_img))
    T_img = np.ones((h_img, w_img))
    last = np.zeros((h_img, w_img), np.int64)
    tile_lists = {}
    bg = np.asarray(p["bg"], np.float64)
    ridx = np.nonzero(rendered)[0]
    for py in range(h_img):
        for px in range(w_img):
            tx, ty = px // 16, py // 16
            key = (tx, ty)
            if key not in tile_lists:
                sup = ridx[(rect[ridx, 0] <= tx) & (tx < rect[ridx, 1]) & (rect[ridx, 2] <= ty) & (ty < rect[ridx, 3])]
                order = np.lexsort((sup, z[sup]))
                tile_lists[key] = sup[order]
            lst = tile_lists[key]
            T = 1.0
            acc = np.zeros(3)
            lastk = 0
            for k, g in enumerate(lst):
                dx, dy = u[g] - (px + 0.5), v[g] - (py + 0.5)
                power = -0.5 * (A[g] * dx * dx + C[g] * dy * dy) - B[g] * dx * dy
                if power > 0:
                    continue
                a = min(_o.ALPHA_CLAMP, a2[g] * math.exp(power))
                margins.append(np.array([abs(a - _o.SKIP_ALPHA) / _o.SKIP_ALPHA]))
                if a < _o.SKIP_ALPHA:
                    continue
                Tn = T * (1 - a)
                margins.append(np.array([abs(Tn - _o.T_MIN) / _o.T_MIN]))
                if Tn < _o.T_MIN:
                    break
                acc += col[g] * a * T
                T = Tn
                lastk = k + 1
            rgb[:, py, px] = acc + T * bg
            T_img[py, px] = T
            last[py, px] = lastk
    m = np.concatenate([np.ravel(a) for a in margins]) if margins else np.array([1.0])
    return dict(rgb=rgb, T=T_img, last=last, tile_lists=tile_lists, rendered=rendered,
                F=F, M=M, a2=a2, dmax=dmax, min_margin=float(m.min()))
