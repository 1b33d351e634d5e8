"""CPU oracle for the CLoD-GS render path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this module.  It shares no code with the HIP library and never imports it.

Two halves:

* ``liboracle.so`` (clod_oracle.c): the binary32 contract path.  It takes every decision
  that produces an integer (frustum flag, LoD mask, tile rectangle, depth order, per-pixel
  skip/termination, last-contributor index) exactly as the arithmetic contract specifies,
  and also produces binary32 colour.
* The FP64 path below (plain PyTorch CPU ops in float64): the same formulas in double
  precision, replaying the binary32 decisions, so that colour is compared against a more
  accurate value and gradients come from autograd of a plainly written forward.

Paper passages followed (CLoD-GS, arXiv 2510.09997):
  Sec. 3.1 Eq. (1) front-to-back blending; Sec. 3.2 distance normalisation, Eq. (2)
  attenuated opacity and the mask M_i = alpha''_i > tau s_v; Sec. 3.3 Eq. (3)-(5) target
  ratio, point-count regulariser and weighted total loss; Sec. 4.1 hyperparameters.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "clod_oracle.c")

# Readings of constants the paper leaves open (documented with the arithmetic contract).
DEFAULT_PARAMS = dict(tau=1.0 / 255.0, eps=1e-6, near=0.2, guard=1.3, dilation=0.3,
                      bg=(0.0, 0.0, 0.0))
SKIP_ALPHA = 1.0 / 255.0
T_MIN = 1e-4
# The clamp value is the binary32 number 0.99f of the contract; the FP64 replay uses it too.
ALPHA_CLAMP = float(np.float32(0.99))


def build(force: bool = False) -> str:
    """Compile the binary32 oracle with contraction off (gcc, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_init.restype = None
        L.oracle_exp.argtypes = [P, P, i64]
        L.oracle_exp_scan.argtypes = [ctypes.c_float, ctypes.c_float, P]
        L.oracle_sh_basis.argtypes = [P, i64, ctypes.c_int, P]
        L.oracle_view_pass.argtypes = [i64, ctypes.c_int] + [P] * 9 + [P] * 7
        L.oracle_tile_lists.argtypes = [i64, P, P, P, ctypes.c_int, ctypes.c_int, P, P, i64]
        L.oracle_tile_lists.restype = i64
        L.oracle_blend.argtypes = [ctypes.c_int] * 4 + [P, P, P, P, P, P, P, P]
        L.oracle_blend.restype = i64
        L.oracle_tile_status.argtypes = [ctypes.c_int] * 4 + [i64, P, P, P, i64, P]
        L.oracle_blend_one.argtypes = [ctypes.c_int, ctypes.c_int, P, P, i64, P, P, P]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_init()
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def viewport_of(view):
    """(frame width, frame height, x, y) of a view's viewport; a plain view is its own frame."""
    fw, fh = int(getattr(view, "frame_width", 0)), int(getattr(view, "frame_height", 0))
    if fw == 0 and fh == 0:
        return view.width, view.height, 0, 0
    return fw, fh, int(view.vx), int(view.vy)


def pack_view(view) -> np.ndarray:
    v = np.zeros(28, dtype=np.float32)
    v[0:9] = np.asarray(view.W, dtype=np.float32).reshape(9)
    v[9:12] = view.t
    v[12:15] = view.c
    v[15:19] = (view.fx, view.fy, view.cx, view.cy)
    v[19] = view.width
    v[20] = view.height
    v[21] = view.s_v
    v[22:26] = viewport_of(view)
    return v


def pack_params(p: dict | None = None) -> np.ndarray:
    p = {**DEFAULT_PARAMS, **(p or {})}
    return np.array([p["tau"], p["eps"], p["near"], p["guard"], p["dilation"], *p["bg"]],
                    dtype=np.float32)


# ---------------------------------------------------------------------------------------
# binary32 contract path
# ---------------------------------------------------------------------------------------

def cexp(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().oracle_exp(_p(x), _p(y), x.size)
    return y


def exp_scan(lo: float, hi: float):
    out = np.zeros(4, dtype=np.float64)
    lib().oracle_exp_scan(ctypes.c_float(lo), ctypes.c_float(hi), _p(out))
    return dict(nonmonotone=int(out[0]), max_ulp=float(out[1]), visited=int(out[2]),
                max_rel_drop=float(out[3]))


def sh_basis32(dirs: np.ndarray, deg: int) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, dtype=np.float32)
    out = np.empty((dirs.shape[0], (deg + 1) ** 2), dtype=np.float32)
    lib().oracle_sh_basis(_p(dirs), dirs.shape[0], deg, _p(out))
    return out


def budget_mask(alpha2: np.ndarray, budget: int) -> np.ndarray:
    """Primitive-budget LoD selection (the Sec. 4 comparisons keep the Gaussians with the
    highest attenuated opacity): the `budget` largest alpha'', lower index first among equal
    values (the tie reading).  A plain sort of (-alpha'', index)."""
    n = alpha2.shape[0]
    m = np.zeros(n, dtype=np.uint8)
    order = np.lexsort((np.arange(n), -alpha2.astype(np.float64)))
    m[order[:min(int(budget), n)]] = 1
    return m


def view_pass(scene: dict, view, params: dict | None = None) -> dict:
    """Per-Gaussian binary32 pass for one view (Sec. 3.2 and the EWA projection).  A view with
    budget K > 0 keeps the K largest alpha'' (a first pass computes alpha'' for all Gaussians)."""
    budget = int(getattr(view, "budget", 0))
    mask = None
    if budget > 0:
        mask = budget_mask(_view_pass(scene, view, params, None)["rec"][:, 6], budget)
    return _view_pass(scene, view, params, mask)


def _view_pass(scene: dict, view, params: dict | None, mask) -> dict:
    n, deg = scene["n"], scene["sh_degree"]
    flags = np.zeros(n, dtype=np.uint8)
    rec = np.zeros((n, 10), dtype=np.float32)
    rect = np.zeros((n, 4), dtype=np.int32)
    aux = np.zeros((n, 6), dtype=np.float32)
    dmax = np.zeros(1, dtype=np.float32)
    arg = np.zeros(1, dtype=np.int64)
    counts = np.zeros(3, dtype=np.int64)
    v24, p8 = pack_view(view), pack_params(params)
    mask_c = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)   # alive across the call
    lib().oracle_view_pass(n, deg, _p(scene["mean"]), _p(scene["log_scale"]), _p(scene["quat"]),
                           _p(scene["opacity"]), _p(scene["decay"]), _p(scene["sh"]), _p(v24), _p(p8),
                           None if mask_c is None else _p(mask_c),
                           _p(flags), _p(rec), _p(rect), _p(aux), _p(dmax), _p(arg), _p(counts))
    _, _, vx, vy = viewport_of(view)
    return dict(flags=flags, rec=rec, rect=rect, aux=aux, dmax=float(dmax[0]), argmax=int(arg[0]),
                counts=counts, width=view.width, height=view.height, vx=vx, vy=vy)


def tile_lists(vp: dict):
    """Per tile, the rendered Gaussians whose rectangle contains it, in (depth, index) order."""
    w, h = vp["width"], vp["height"]
    T = ((w + 15) // 16) * ((h + 15) // 16)
    off = np.zeros(T + 1, dtype=np.int64)
    n = vp["flags"].shape[0]
    D = lib().oracle_tile_lists(n, _p(vp["flags"]), _p(vp["rec"]), _p(vp["rect"]), w, h, _p(off), None, 0)
    ent = np.zeros(max(D, 1), dtype=np.int32)
    lib().oracle_tile_lists(n, _p(vp["flags"]), _p(vp["rec"]), _p(vp["rect"]), w, h, _p(off), _p(ent), D)
    return off, ent[:D]


def blend(vp: dict, off: np.ndarray, ent: np.ndarray, params: dict | None = None):
    """Eq. (1) per pixel over its tile list.  Returns rgb [3][H][W], T [H][W], last [H][W],
    and the pair counts {evaluated, exponential needed, blended}."""
    w, h = vp["width"], vp["height"]
    bg = pack_params(params)[5:8].copy()
    rgb = np.zeros((3, h, w), dtype=np.float32)
    T = np.zeros((h, w), dtype=np.float32)
    last = np.zeros((h, w), dtype=np.int32)
    ent_c = np.ascontiguousarray(ent if ent.size else np.zeros(1, np.int32))
    classes = np.zeros(3, np.int64)
    lib().oracle_blend(w, h, vp["vx"], vp["vy"], _p(vp["rec"]), _p(off), _p(ent_c), _p(bg), _p(rgb), _p(T), _p(last),
                       _p(classes))
    return rgb, T, last, classes


def render32(scene: dict, view, params: dict | None = None) -> dict:
    vp = view_pass(scene, view, params)
    off, ent = tile_lists(vp)
    rgb, T, last, classes = blend(vp, off, ent, params)
    vp.update(tile_off=off, entries=ent, rgb=rgb, T=T, last=last, pairs=int(classes[0]), pair_classes=classes)
    return vp


def sorted_keys(vp: dict, tile_base: int = 0) -> np.ndarray:
    """The (tile, depth) keys in sorted order: (tile_base + tile) << 32 | bits(depth)."""
    off, ent = vp["tile_off"], vp["entries"]
    tiles = np.repeat(np.arange(off.size - 1, dtype=np.uint64), np.diff(off).astype(np.int64))
    depth_bits = vp["rec"][ent.astype(np.int64), 2].view(np.uint32).astype(np.uint64)
    return ((tiles + np.uint64(tile_base)) << np.uint64(32)) | depth_bits


def tile_status(vp: dict, tile: int, lmax: int) -> np.ndarray:
    st = np.zeros((256, max(lmax, 1)), dtype=np.uint8)
    ent_c = np.ascontiguousarray(vp["entries"] if vp["entries"].size else np.zeros(1, np.int32))
    lib().oracle_tile_status(vp["width"], vp["height"], vp["vx"], vp["vy"], tile, _p(vp["rec"]), _p(vp["tile_off"]),
                             _p(ent_c), max(lmax, 1), _p(st))
    return st[:, :lmax]


def blend_pixel(vp: dict, px: int, py: int):
    """One pixel's (rgb without background, T, last) from its tile list."""
    w = vp["width"]
    t = (py // 16) * ((w + 15) // 16) + px // 16
    a, b = int(vp["tile_off"][t]), int(vp["tile_off"][t + 1])
    lst = np.ascontiguousarray(vp["entries"][a:b]) if b > a else np.zeros(1, np.int32)
    rgb = np.zeros(3, np.float32)
    T = np.zeros(1, np.float32)
    last = np.zeros(1, np.int32)
    lib().oracle_blend_one(px + vp["vx"], py + vp["vy"], _p(vp["rec"]), _p(lst), b - a, _p(rgb), _p(T), _p(last))
    return rgb, float(T[0]), int(last[0])


# ---------------------------------------------------------------------------------------
# Loss scalars, Sec. 3.3
# ---------------------------------------------------------------------------------------

def eta_target(s_v):
    """Eq. (3)."""
    return 1.0 / s_v ** 1.5


def l_reg(s_v, eta_actual):
    """Eq. (4): (s_v - 1)^2 * ReLU(eta_actual - eta_target)^2."""
    return (s_v - 1.0) ** 2 * max(eta_actual - eta_target(s_v), 0.0) ** 2


def w_s(s_v, s_max):
    """Weight of Eq. (5): (1 - 0.5 s_v / max(s_v))^2, max(s_v) read as the training range's
    upper bound."""
    return (1.0 - 0.5 * s_v / s_max) ** 2


def total_loss(l_render, s_v, eta_actual, s_max, lam=1.0):
    """Eq. (5): w_s (L_render + lambda_reg L_reg); lambda_reg = 1.0 per Sec. 4.1."""
    return w_s(s_v, s_max) * (l_render + lam * l_reg(s_v, eta_actual))


# ---------------------------------------------------------------------------------------
# FP64 path (plain PyTorch CPU ops), replaying the binary32 decisions
# ---------------------------------------------------------------------------------------

def sh_basis64(dirs: torch.Tensor, deg: int) -> torch.Tensor:
    """Real spherical harmonics, l <= deg, on unit directions [..., 3] -> [..., (deg+1)^2]."""
    X, Y, Z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    pi = math.pi
    out = [torch.full_like(X, 0.5 * math.sqrt(1.0 / pi))]
    if deg >= 1:
        k1 = math.sqrt(3.0 / (4.0 * pi))
        out += [k1 * Y, k1 * Z, k1 * X]
    if deg >= 2:
        k2a, k2b, k2c = 0.5 * math.sqrt(15 / pi), 0.25 * math.sqrt(5 / pi), 0.25 * math.sqrt(15 / pi)
        out += [k2a * X * Y, k2a * Y * Z, k2b * (2 * Z * Z - X * X - Y * Y), k2a * X * Z,
                k2c * (X * X - Y * Y)]
    if deg >= 3:
        k3a = 0.25 * math.sqrt(35 / (2 * pi))
        k3b = 0.5 * math.sqrt(105 / pi)
        k3c = 0.25 * math.sqrt(21 / (2 * pi))
        k3d = 0.25 * math.sqrt(7 / pi)
        k3e = 0.25 * math.sqrt(105 / pi)
        t4 = 4 * Z * Z - X * X - Y * Y
        out += [k3a * Y * (3 * X * X - Y * Y), k3b * X * Y * Z, k3c * Y * t4,
                k3d * Z * (2 * Z * Z - 3 * X * X - 3 * Y * Y), k3c * X * t4,
                k3e * Z * (X * X - Y * Y), k3a * X * (X * X - 3 * Y * Y)]
    return torch.stack(out, dim=-1)


def scene_to_torch64(scene: dict, requires_grad: bool = True) -> dict:
    out = {}
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        t = torch.from_numpy(scene[k].astype(np.float64))
        out[k] = t.requires_grad_(requires_grad)
    out["n"] = scene["n"]
    out["sh_degree"] = scene["sh_degree"]
    return out


def quat_to_rot64(q: torch.Tensor) -> torch.Tensor:
    """q [4, m] (w, x, y, z), normalised here -> R [m, 3, 3]."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q[0], q[1], q[2], q[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def fp64_view_forward(sc: dict, view, vp: dict, params: dict | None = None,
                      tiles: list[int] | None = None):
    """FP64 forward for one view, replaying the binary32 decisions held in ``vp`` (the
    output of ``render32``).

    Returns (rgb [3][H][W], T [H][W], eta_ste, alpha2 [n]) as float64 tensors connected to
    the leaves in ``sc``.  eta_ste has the value n_M / N and, for the point-count
    regulariser, the gradient 1/N with respect to every alpha''_i (kept-primitive mass).
    ``tiles`` restricts the blend to a subset of tiles (other pixels stay zero).
    """
    p = {**DEFAULT_PARAMS, **(params or {})}
    n, deg = sc["n"], sc["sh_degree"]
    W = torch.from_numpy(np.asarray(view.W, dtype=np.float64))
    t = torch.from_numpy(np.asarray(view.t, dtype=np.float64))
    c = torch.from_numpy(np.asarray(view.c, dtype=np.float64))
    mean = sc["mean"]                                    # [3, n]
    pc = W @ mean + t[:, None]                           # camera-space means
    e = mean - c[:, None]
    d = torch.sqrt((e * e).sum(0))
    k = vp["argmax"]
    dmax = d[k] if k >= 0 else torch.tensor(1.0, dtype=torch.float64)
    dn = d / dmax
    r = torch.relu(sc["decay"])
    q = (dn * view.s_v) ** 2 / (2.0 * r * r + p["eps"])
    alpha = torch.sigmoid(sc["opacity"])
    alpha2 = alpha * torch.exp(-q)                       # Eq. (2)
    # Where the binary32 alpha'' is exactly 0 (the contract exponential returns 0 below -86, or
    # the product underflows), the replay takes that value too: no gradient flows through it.
    alpha2 = torch.where(torch.from_numpy(vp["rec"][:, 6] == 0), torch.zeros_like(alpha2), alpha2)
    mask_m = torch.from_numpy((vp["flags"] & 2) != 0)
    n_m = int(mask_m.sum())
    mass = alpha2.sum()
    eta = n_m / n + (mass - mass.detach()) / n           # Eq. (4) eta_actual, STE gradient

    H, Wd = view.height, view.width
    rgb = torch.zeros(3, H, Wd, dtype=torch.float64)
    Tim = torch.ones(H, Wd, dtype=torch.float64)
    flags = vp["flags"]
    ridx_np = np.nonzero(flags & 4)[0]
    if ridx_np.size == 0:
        bgv = torch.tensor(p["bg"], dtype=torch.float64)
        return rgb + bgv[:, None, None], Tim, eta, alpha2
    ridx = torch.from_numpy(ridx_np)

    # EWA projection of the rendered Gaussians.
    x, y, z = pc[0, ridx], pc[1, ridx], pc[2, ridx]
    s = torch.exp(sc["log_scale"][:, ridx])              # [3, m]
    R = quat_to_rot64(sc["quat"][:, ridx])               # [m, 3, 3]
    Mm = R * s.T[:, None, :]
    Sig = Mm @ Mm.transpose(1, 2)
    fx, fy = float(view.fx), float(view.fy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * x / (z * z)], -1),
                     torch.stack([zero, fy / z, -fy * y / (z * z)], -1)], -2)   # [m, 2, 3]
    Tm = J @ W
    cov = Tm @ Sig @ Tm.transpose(1, 2)
    ca = cov[:, 0, 0] + p["dilation"]
    cb = cov[:, 0, 1]
    cc = cov[:, 1, 1] + p["dilation"]
    det = ca * cc - cb * cb
    A, B, C = cc / det, -cb / det, ca / det
    u = fx * x / z + float(view.cx)
    v = fy * y / z + float(view.cy)
    dirs = (e[:, ridx] / d[ridx]).T
    Y = sh_basis64(dirs, deg)                            # [m, K]
    shr = sc["sh"][:, :, ridx]                           # [K, 3, m]
    col = torch.einsum("mk,kcm->mc", Y, shr) + 0.5
    clampm = torch.from_numpy(np.stack([(flags[ridx_np] >> (3 + ch)) & 1 for ch in range(3)], -1) != 0)
    col = torch.where(clampm, torch.zeros_like(col), col)
    a2r = alpha2[ridx]

    # Map Gaussian index -> position in the rendered subset.
    pos_of = np.full(n, -1, dtype=np.int64)
    pos_of[ridx_np] = np.arange(ridx_np.size)

    TW = (Wd + 15) // 16
    TH = (H + 15) // 16
    off, ent, last = vp["tile_off"], vp["entries"], vp["last"]
    bg = torch.tensor(p["bg"], dtype=torch.float64)
    rows_rgb, rows_T, idx_pix = [], [], []
    tile_iter = range(TW * TH) if tiles is None else tiles
    for tile in tile_iter:
        tx, ty = tile % TW, tile // TW
        px0, py0 = tx * 16, ty * 16
        ly, lx = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
        pxs, pys = (px0 + lx).reshape(-1), (py0 + ly).reshape(-1)
        valid = (pxs < Wd) & (pys < H)
        lmax = int(last[pys[valid], pxs[valid]].max()) if valid.any() else 0
        pix_flat = pys[valid] * Wd + pxs[valid]
        if lmax == 0:
            rows_rgb.append(torch.zeros(int(valid.sum()), 3, dtype=torch.float64))
            rows_T.append(torch.ones(int(valid.sum()), dtype=torch.float64))
            idx_pix.append(pix_flat)
            continue
        st = tile_status(vp, tile, lmax)[valid]          # [P, L] 0/1/2
        gidx = ent[off[tile]: off[tile] + lmax].astype(np.int64)
        gpos = torch.from_numpy(pos_of[gidx])            # [L]
        pcx = torch.from_numpy(pxs[valid].astype(np.float64) + vp.get("vx", 0) + 0.5)[:, None]
        pcy = torch.from_numpy(pys[valid].astype(np.float64) + vp.get("vy", 0) + 0.5)[:, None]
        dx = u[gpos][None, :] - pcx
        dy = v[gpos][None, :] - pcy
        power = -0.5 * (A[gpos][None, :] * dx * dx + C[gpos][None, :] * dy * dy) - B[gpos][None, :] * dx * dy
        st_t = torch.from_numpy(st)
        a = a2r[gpos][None, :] * torch.exp(power)
        a = torch.where(st_t == 2, torch.full_like(a, ALPHA_CLAMP), a)
        on = st_t > 0
        one_m = torch.where(on, 1.0 - a, torch.ones_like(a))
        Tincl = torch.cumprod(one_m, dim=1)
        Texcl = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], dim=1)
        wgt = torch.where(on, a * Texcl, torch.zeros_like(a))
        cpix = wgt @ col[gpos]                           # [P, 3]
        Tfin = Tincl[:, -1]
        rows_rgb.append(cpix + Tfin[:, None] * bg[None, :])
        rows_T.append(Tfin)
        idx_pix.append(pix_flat)
    rgb_flat = torch.zeros(H * Wd, 3, dtype=torch.float64)
    T_flat = torch.ones(H * Wd, dtype=torch.float64)
    if idx_pix:
        allpix = torch.from_numpy(np.concatenate(idx_pix))
        rgb_flat = rgb_flat.index_copy(0, allpix, torch.cat(rows_rgb))
        T_flat = T_flat.index_copy(0, allpix, torch.cat(rows_T))
    rgb = rgb_flat.T.reshape(3, H, Wd)
    Tim = T_flat.reshape(H, Wd)
    return rgb, Tim, eta, alpha2


def fp64_grads(scene: dict, view, vp: dict, dL_drgb: np.ndarray, dL_deta: float,
               params: dict | None = None, tiles: list[int] | None = None, abs_terms: bool = False) -> dict:
    """Gradients of  sum(dL_drgb * rgb) + dL_deta * eta  with respect to every parameter
    plane, by autograd of the FP64 forward.  Returns float64 numpy arrays in the scene's
    layout, plus the FP64 rgb and T.  With ``abs_terms`` also ``out["abs"][plane]``: the
    absolute adjoint of each element (the sum over chain-rule paths of the products of absolute
    partials, with |dL_drgb| and |dL_deta|; see abs_adjoint.py), the scale of its terms."""
    sc = scene_to_torch64(scene)
    rgb, T, eta, _ = fp64_view_forward(sc, view, vp, params, tiles)
    g = torch.from_numpy(np.asarray(dL_drgb, dtype=np.float64))
    L = (rgb * g).sum() + dL_deta * eta
    L.backward()
    out = {k: (sc[k].grad.detach().numpy().copy() if sc[k].grad is not None else np.zeros(sc[k].shape))
           for k in PLANES}
    out["rgb"] = rgb.detach().numpy()
    out["T"] = T.detach().numpy()
    if abs_terms:
        out["abs"] = fp64_abs_adjoint(scene, view, vp, dL_drgb, dL_deta, params, tiles)
    return out


PLANES = ("mean", "log_scale", "quat", "opacity", "decay", "sh")


def fp64_abs_adjoint(scene: dict, view, vp: dict, dL_drgb: np.ndarray, dL_deta: float,
                     params: dict | None = None, tiles: list[int] | None = None) -> dict:
    """Per element of every parameter plane, the sum of the magnitudes of the chain-rule terms
    of its gradient (the same forward as fp64_grads, differentiated with absolute partials)."""
    from .abs_adjoint import AbsAdjointMode
    sc = scene_to_torch64(scene)
    g = torch.from_numpy(np.abs(np.asarray(dL_drgb, dtype=np.float64)))
    with AbsAdjointMode():
        rgb, _, eta, _ = fp64_view_forward(sc, view, vp, params, tiles)
        L = (rgb * g).sum() + abs(float(dL_deta)) * eta
    L.backward()
    return {k: (sc[k].grad.detach().numpy().copy() if sc[k].grad is not None else np.zeros(sc[k].shape))
            for k in PLANES}


# Smallest normal binary32 number: differences below it are below the format's normal range.
FLT_MIN = float(np.finfo(np.float32).tiny)


def grad_elem_terms(g: np.ndarray, r: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Per element, (|g_i - r_i| - FLT_MIN)+ / S_i: the error measured against the magnitude of
    the element's terms (S_i, the absolute adjoint: S_i >= |r_i|, equal where the terms do not
    cancel, so this is the plain relative error there), less the binary32 underflow threshold
    (a binary32 evaluation cannot resolve differences below the smallest normal number).  An
    element with S_i = 0 has no terms: its error must stay below FLT_MIN (else inf)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    S = np.asarray(S, dtype=np.float64).ravel()
    d = np.maximum(np.abs(g - r) - FLT_MIN, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(S > 0.0, d / np.where(S > 0.0, S, 1.0), np.where(d > 0.0, np.inf, 0.0))
    return e


def grad_elem_error(g: np.ndarray, r: np.ndarray, S: np.ndarray) -> float:
    """max over elements of grad_elem_terms (0 for an empty plane)."""
    e = grad_elem_terms(g, r, S)
    return float(e.max()) if e.size else 0.0


def grad_rel_error(g: np.ndarray, r: np.ndarray) -> float:
    """Relative error of a gradient tensor in the max norm: max_i |g_i - r_i| / max_j |r_j|.
    Reported beside grad_elem_error; used alone only to compare two GPU runs of the same
    arithmetic (graph replay against the eager step)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    if r.size == 0:
        return 0.0
    scale = np.abs(r).max()
    if scale == 0.0:
        return float(np.abs(g).max())
    return float(np.abs(g - r).max() / scale)


def grad_floor_error(g: np.ndarray, r: np.ndarray, floor: float = 1e-3) -> float:
    """Element-wise relative error with a floor: max_i |g_i - r_i| / max(|r_i|, floor max_j |r_j|)
    (reported, not a gate: it ignores how strongly an element's terms cancel)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    if r.size == 0:
        return 0.0
    den = np.maximum(np.abs(r), floor * np.abs(r).max())
    if den.max() == 0.0:
        return float(np.abs(g).max())
    return float((np.abs(g - r) / np.where(den > 0, den, 1.0)).max())


def grad_l2_error(g: np.ndarray, r: np.ndarray) -> float:
    """||g - r||_2 / ||r||_2."""
    g = np.asarray(g, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    nr = np.linalg.norm(r)
    return float(np.linalg.norm(g - r) / nr) if nr > 0 else float(np.linalg.norm(g))


def num_threads() -> int:
    return int(lib().oracle_num_threads())
