"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, special cases, invariants, an independent no-tile brute force, Monte-Carlo
statistics and finite differences.  No GPU needed."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import brute, oracle as O
from paper_2510_09997_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_gaussian_scene(mean, log_scale=(-4.0, -4.0, -4.0), opacity=0.0, decay=1.0, deg=0,
                       dc=(0.0, 0.0, 0.0), quat=(1.0, 0.0, 0.0, 0.0)):
    n = len(mean)
    K = (deg + 1) ** 2
    sc = dict(n=n, sh_degree=deg,
              mean=np.ascontiguousarray(np.asarray(mean, np.float32).T),
              log_scale=np.ascontiguousarray(np.tile(np.asarray(log_scale, np.float32)[:, None], (1, n))),
              quat=np.ascontiguousarray(np.tile(np.asarray(quat, np.float32)[:, None], (1, n))),
              opacity=np.full(n, opacity, np.float32),
              decay=np.full(n, decay, np.float32),
              sh=np.zeros((K, 3, n), np.float32))
    sc["sh"][0] = np.asarray(dc, np.float32)[:, None]
    return sc


# ------------------------------------------------------------------ contract exponential

@pytest.mark.slow
def test_contract_exp_exhaustive_accuracy_and_glitch_bound():
    """Every binary32 input in [-86, 88]: error <= 1 ulp against exp, and any decrease
    between neighbouring inputs stays below 2^-23 relative (the LoD-count monotonicity
    argument needs exactly this bound)."""
    for lo, hi in ((-86.0, 0.0), (0.0, 88.0)):
        r = O.exp_scan(lo, hi)
        assert r["max_ulp"] <= 1.0, r
        assert r["max_rel_drop"] < 2.0 ** -23, r


def test_contract_exp_special_values():
    x = np.array([0.0, -0.0, -87.0, -1e30, 89.0, 1.0, -1.0], np.float32)
    y = O.cexp(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert y[2] == 0.0 and y[3] == 0.0
    assert np.isinf(y[4])
    assert abs(y[5] / math.e - 1) < 1.2e-7 and abs(y[6] * math.e - 1) < 1.2e-7


# ------------------------------------------------------------------ spherical harmonics

def _sphere_quadrature(nt=40, nphi=80):
    xs, ws = np.polynomial.legendre.leggauss(nt)        # cos(theta) nodes, exact to deg 79
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xs, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (np.repeat(ws, nphi) * (2 * math.pi / nphi))
    return d, w


def test_sh_basis_orthonormal_fp64():
    """The 16 real SH basis functions are orthonormal on S^2 (Gauss-Legendre x trapezoid
    quadrature, exact for these polynomial degrees)."""
    d, w = _sphere_quadrature()
    Y = O.sh_basis64(torch.from_numpy(d), 3).numpy()
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12
    assert abs(Y[0, 0] - 1 / (2 * math.sqrt(math.pi))) < 1e-15


def test_sh_basis_binary32_matches_fp64_and_is_orthonormal():
    d, w = _sphere_quadrature()
    Y32 = O.sh_basis32(d.astype(np.float32), 3).astype(np.float64)
    Y64 = O.sh_basis64(torch.from_numpy(d.astype(np.float32).astype(np.float64)), 3).numpy()
    assert np.abs(Y32 - Y64).max() < 2e-6
    G = (Y32 * w[:, None]).T @ Y32
    assert np.abs(G - np.eye(16)).max() < 1e-5


def test_sh_direction_points_from_camera_to_gaussian():
    """Reading of the view direction: (mu - c)/|mu - c|.  A Gaussian straight ahead of a
    camera on the -z axis sees direction +z, so a positive Y_1^0 coefficient brightens it."""
    sc = one_gaussian_scene([(0.0, 0.0, 0.0)], deg=1, decay=1e15)
    sc["sh"][2, :, 0] = 0.5                              # Y_1^0 (z) coefficient
    v = synth.look_at((0, 0, -3), width=64, height=64)
    vp = O.view_pass(sc, v)
    k1 = math.sqrt(3 / (4 * math.pi))
    assert vp["flags"][0] & 4
    np.testing.assert_allclose(vp["rec"][0, 7:10], 0.5 + 0.5 * k1, rtol=1e-6)


# ------------------------------------------------------------------ Eq. (2) and the mask

def test_single_gaussian_normalised_distance_is_one_and_eq2_value():
    """One Gaussian in view: it is the frustum maximum, so d' = 1 exactly and Eq. (2)
    reduces to alpha * exp(-s_v^2 / (2 sigma^2 + eps))."""
    eps = 1e-6
    for s_v in (1.0, 1.7, 2.5):
        sc = one_gaussian_scene([(0.1, -0.2, 0.3)], opacity=0.0, decay=1.0)
        v = synth.look_at((0, 0, -3), width=64, height=64, s_v=s_v)
        vp = O.view_pass(sc, v)
        a2 = vp["rec"][0, 6]
        ref = 0.5 * math.exp(-(s_v ** 2) / (2.0 + eps))
        assert abs(a2 - ref) <= 3e-7 * ref
    # Worked value at s_v = 1.
    assert abs(0.5 * math.exp(-1 / (2 + eps)) - 0.3032654) < 1e-7


def test_mask_threshold_crossing_at_closed_form_root():
    """M = alpha'' > tau s_v flips exactly where alpha exp(-s^2/(2 sigma^2+eps)) = tau s."""
    eps, tau = 1e-6, 1.0 / 255.0
    f = lambda s: 0.5 * math.exp(-s * s / (2 + eps)) - tau * s
    lo, hi = 1.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) > 0 else (lo, mid)
    s_star = 0.5 * (lo + hi)
    assert abs(s_star - 2.767706) < 1e-5
    sc = one_gaussian_scene([(0.0, 0.0, 0.0)], opacity=0.0, decay=1.0)
    for s_v, kept in ((s_star * (1 - 1e-4), True), (s_star * (1 + 1e-4), False)):
        vp = O.view_pass(sc, synth.look_at((0, 0, -3), width=64, height=64, s_v=s_v))
        assert bool(vp["flags"][0] & 2) == kept
        assert vp["counts"][1] == int(kept)


def test_frustum_max_ignores_gaussians_outside_view_and_ties_take_lowest_index():
    base = [(0.0, 0.0, 0.0), (0.3, 0.0, 0.0)]
    v = synth.look_at((0, 0, -3), width=64, height=64)
    a = O.view_pass(one_gaussian_scene(base), v)
    b = O.view_pass(one_gaussian_scene(base + [(0.0, 0.0, -50.0)]), v)   # behind the camera
    assert a["dmax"] == b["dmax"] and a["argmax"] == b["argmax"] == 1
    np.testing.assert_array_equal(a["rec"][:, 6], b["rec"][:2, 6])
    assert b["counts"][0] == 2
    # Two Gaussians at the same distance: the lower index is the argmax.
    c = O.view_pass(one_gaussian_scene([(0.0, 0.0, 0.0), (0.3, 0.0, 0.0), (-0.3, 0.0, 0.0)]), v)
    assert c["argmax"] == 1


def test_empty_frustum_uses_unit_normaliser():
    sc = one_gaussian_scene([(0.0, 0.0, -50.0)])
    vp = O.view_pass(sc, synth.look_at((0, 0, -3), width=64, height=64))
    assert vp["dmax"] == 1.0 and vp["argmax"] == -1 and vp["counts"][0] == 0 and vp["counts"][2] == 0


def test_lod_counts_non_increasing_in_virtual_distance_scale():
    """alpha'' is non-increasing in s_v and the threshold tau s_v increasing, while d' and
    the frustum do not depend on s_v: n_M and n_rendered never rise along an s_v sweep
    whose steps exceed 2^-19 relative (the contract exp's glitches are below 2^-23)."""
    sc = synth.make_scene(20000, 0, "mixture", seed=5)
    prev = None
    for s_v in synth.sweep_distances(64, 2.0, 200.0) / 2.0:
        vp = O.view_pass(sc, synth.look_at((0, 0, -8), width=320, height=240, s_v=float(s_v)))
        c = vp["counts"]
        if prev is not None:
            assert c[0] == prev[0] and c[1] <= prev[1] and c[2] <= prev[2]
        prev = c
    assert prev[1] < 20000


def test_scaling_scene_and_camera_by_two_is_bit_identical_for_decisions():
    """Multiplying all means and the camera position by 2 scales every intermediate of the
    normalised distance exactly, so d', F, M and the counts are bit-identical."""
    sc = synth.make_scene(5000, 0, "uniform", seed=7)
    v1 = synth.look_at((0.0, 0.0, -3.0), width=128, height=128, s_v=2.0)
    sc2 = dict(sc)
    sc2["mean"] = sc["mean"] * np.float32(2.0)
    v2 = synth.look_at((0.0, 0.0, -6.0), width=128, height=128, s_v=2.0)
    assert np.array_equal(v2.t, v1.t * np.float32(2)) and np.array_equal(v2.W, v1.W)
    a, b = O.view_pass(sc, v1), O.view_pass(sc2, v2)
    assert np.array_equal(a["flags"] & 3, b["flags"] & 3)
    assert np.array_equal(a["rec"][:, 6], b["rec"][:, 6])
    assert a["dmax"] * 2 == b["dmax"] and np.array_equal(a["counts"][:2], b["counts"][:2])


def test_huge_decay_reduces_to_plain_3dgs():
    """sigma_d -> infinity makes the exponent of Eq. (2) vanish: alpha'' = alpha exactly, and
    with tau = 0 every in-frustum Gaussian is rendered, i.e. the plain 3DGS forward.  The
    brute force with the LoD switched off in the same way must agree."""
    sc = synth.make_scene(64, 0, "uniform", seed=11, log_scale_mean=-2.5)
    sc["decay"][:] = 1e15
    v = synth.look_at((0, 0, -3), width=48, height=48, s_v=3.0)
    p = dict(tau=0.0)
    r = O.render32(sc, v, p)
    alpha = 1.0 / (1.0 + np.exp(-sc["opacity"].astype(np.float64)))
    np.testing.assert_allclose(r["rec"][:, 6], alpha, rtol=3e-7)
    assert r["counts"][1] == 64
    b = brute.render(sc, v, p)
    assert b["min_margin"] > 1e-5
    assert np.abs(b["rgb"] - r["rgb"]).max() < 1e-5
    assert np.array_equal(b["last"], r["last"])


# ------------------------------------------------------------------ projection (EWA)

def test_ewa_worked_on_axis_value():
    """Isotropic Gaussian on the optical axis: Sigma' = (f s / z)^2 I + 0.3 I, radius
    ceil(3 sqrt(lambda)), rectangle [7, 9)^2 in a 256x256 image."""
    s = math.exp(-4.0)
    sc = one_gaussian_scene([(0.0, 0.0, 0.0)], decay=1e15, dc=(1.0, 1.0, 1.0))
    v = synth.look_at((0, 0, -3), width=256, height=256)
    vp = O.view_pass(sc, v)
    f = 128.0 / math.tan(math.radians(30))
    assert abs(v.fx - f) < 1e-4 and abs(f - 221.70250) < 1e-4
    sig2 = (f * s / 3.0) ** 2 + 0.3
    assert abs(sig2 - 2.1320732) < 1e-6
    a, b, c, rad = vp["aux"][0, 2:6]
    assert abs(a - sig2) < 2e-6 * sig2 and abs(c - sig2) < 2e-6 * sig2 and abs(b) < 1e-6
    assert rad == 5.0
    assert list(vp["rect"][0]) == [7, 9, 7, 9]
    power = -0.5 * (0.25 + 0.25) / sig2
    assert abs(power + 0.1172568) < 1e-6 and abs(math.exp(power) - 0.8893568) < 1e-6


def test_ewa_covariance_matches_monte_carlo_projection():
    """The projected covariance equals the covariance of exactly projected samples of the
    3D Gaussian (first order); checks J, W and Sigma composition, signs and transposes."""
    rng = np.random.default_rng(0)
    sc = one_gaussian_scene([(0.3, -0.2, 0.4)], log_scale=(-2.0, -3.0, -2.5), decay=1e15,
                            quat=(0.8, 0.3, -0.4, 0.2))
    v = synth.look_at((1.0, 0.5, -3.0), width=256, height=256)
    vp = O.view_pass(sc, v)
    a, b, c = vp["aux"][0, 2:5]
    q = sc["quat"][:, 0].astype(np.float64)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    S = np.diag(np.exp(sc["log_scale"][:, 0].astype(np.float64)) ** 2)
    Sig = R @ S @ R.T
    pts = rng.multivariate_normal(sc["mean"][:, 0].astype(np.float64), Sig, size=400000)
    pc = pts @ v.W.T.astype(np.float64) + v.t.astype(np.float64)
    uv = np.stack([v.fx * pc[:, 0] / pc[:, 2], v.fy * pc[:, 1] / pc[:, 2]], 1)
    C = np.cov(uv.T)
    ref = np.array([[a - 0.3, b], [b, c - 0.3]])
    assert np.abs(C - ref).max() < 0.02 * np.abs(ref).max()
    # Rotation independence check: it is not the identity.
    assert abs(b) > 0.05 * max(a, c)


def test_projection_jacobian_matches_finite_differences():
    """The perspective Jacobian used by the oracle's FP64 path equals central differences
    of the pinhole map (x, y, z) -> (fx x/z + cx, fy y/z + cy)."""
    fx, fy = 300.0, 280.0
    X = np.array([0.3, -0.2, 2.5])
    pi = lambda P: np.array([fx * P[0] / P[2], fy * P[1] / P[2]])
    h = 1e-6
    Jfd = np.stack([(pi(X + h * e) - pi(X - h * e)) / (2 * h) for e in np.eye(3)], 1)
    x, y, z = X
    Jan = np.array([[fx / z, 0, -fx * x / z ** 2], [0, fy / z, -fy * y / z ** 2]])
    assert np.abs(Jfd - Jan).max() < 1e-6


# ------------------------------------------------------------------ blending, Eq. (1)

def test_two_gaussian_compositing_closed_form():
    """Two Gaussians at one pixel: C = c1 a1 + c2 a2 (1 - a1), front one first by depth."""
    sc = one_gaussian_scene([(0.0, 0.0, 0.5), (0.0, 0.0, -0.5)], log_scale=(-1.0, -1.0, -1.0),
                            opacity=0.3, decay=1e15, dc=(0.0, 0.0, 0.0))
    sc["sh"][0, :, 0] = np.array([1.0, -1.0, 0.2], np.float32)
    sc["sh"][0, :, 1] = np.array([-0.5, 0.8, 0.1], np.float32)
    v = synth.look_at((0, 0, -3), width=64, height=64)
    r = O.render32(sc, v)
    px, py = 32, 32
    rec = r["rec"].astype(np.float64)

    def a_of(g):
        dx, dy = rec[g, 0] - (px + 0.5), rec[g, 1] - (py + 0.5)
        pw = -0.5 * (rec[g, 3] * dx * dx + rec[g, 5] * dy * dy) - rec[g, 4] * dx * dy
        return min(0.99, rec[g, 6] * math.exp(pw))

    front, back = 1, 0                                    # Gaussian 1 is nearer the camera
    assert rec[front, 2] < rec[back, 2]
    a1, a2 = a_of(front), a_of(back)
    C = rec[front, 7:10] * a1 + rec[back, 7:10] * a2 * (1 - a1)
    np.testing.assert_allclose(r["rgb"][:, py, px], C, atol=2e-7)
    assert abs(r["T"][py, px] - (1 - a1) * (1 - a2)) < 2e-7
    assert r["last"][py, px] == 2


def test_white_on_white_telescopes_to_one():
    """All colours 1 and background 1: sum c a T + T_final = 1 for every pixel."""
    sc = synth.make_scene(3000, 0, "uniform", seed=2)
    sc["sh"][0] = 0.5 / (0.5 / math.sqrt(math.pi))        # degree-0 colour exactly 1.0 in FP64
    v = synth.look_at((0, 0, -3), width=96, height=64)
    r = O.render32(sc, v, dict(bg=(1.0, 1.0, 1.0)))
    assert np.all(r["rec"][r["flags"] & 4 > 0, 7:10] > 0.9999)
    assert np.abs(r["rgb"] - 1.0).max() < 1e-5
    assert r["last"].max() > 3


def test_termination_rule_closed_form():
    """Twenty identical opaque Gaussians stacked along the axis with alpha' = a at the
    centre pixel: T after k blends is (1-a)^k; blending stops before the first k with
    (1-a)^k < 1e-4, so last = that k - 1 entries."""
    m = [(0.0, 0.0, 0.01 * j) for j in range(20)]
    sc = one_gaussian_scene(m, log_scale=(0.0, 0.0, 0.0), opacity=0.0, decay=1e15, dc=(0.0, 0.0, 0.0))
    v = synth.look_at((0, 0, -3), width=32, height=32)
    r = O.render32(sc, v)
    a = float(r["rec"][0, 6])                             # 0.5, G ~ 1 at the centre pixel
    px = py = 16
    dx = r["rec"][0, 0] - (px + 0.5)
    g = math.exp(-0.5 * r["rec"][0, 3] * dx * dx * 2)
    a_eff = a * g
    k = next(k for k in range(1, 100) if (1 - a_eff) ** k < 1e-4)
    assert r["last"][py, px] == k - 1
    assert abs(r["T"][py, px] - (1 - a_eff) ** (k - 1)) < 1e-6


def test_skip_rule_drops_faint_contributions():
    """A Gaussian whose alpha' stays below 1/255 leaves the image untouched."""
    sc = one_gaussian_scene([(0.0, 0.0, 0.0)], log_scale=(0.0, 0.0, 0.0), opacity=-6.0, decay=1e15,
                            dc=(2.0, 2.0, 2.0))
    v = synth.look_at((0, 0, -3), width=32, height=32)
    r = O.render32(sc, v, dict(tau=0.0))
    assert r["rec"][0, 6] < 1.0 / 255.0 and r["counts"][2] == 1
    assert np.all(r["rgb"] == 0.0) and np.all(r["T"] == 1.0) and np.all(r["last"] == 0)


def test_permuting_gaussians_leaves_image_unchanged():
    sc = synth.make_scene(2000, 1, "uniform", seed=4)
    v = synth.look_at((0.5, 0.2, -3), width=80, height=64)
    r = O.render32(sc, v)
    perm = np.random.default_rng(1).permutation(sc["n"])
    sp = dict(sc)
    for k in ("mean", "log_scale", "quat", "sh"):
        sp[k] = np.ascontiguousarray(sc[k][..., perm])
    for k in ("opacity", "decay"):
        sp[k] = np.ascontiguousarray(sc[k][perm])
    rp = O.render32(sp, v)
    depths = r["rec"][r["flags"] & 4 > 0, 2]
    assert np.unique(depths).size == depths.size          # distinct depths: order is unique
    assert np.array_equal(r["rgb"], rp["rgb"]) and np.array_equal(r["last"], rp["last"])


@pytest.mark.parametrize("seed,deg", [(3, 1), (8, 3), (21, 0)])
def test_brute_force_no_tiles_matches_oracle(seed, deg):
    """No-tile FP64 brute force (per-pixel support set sorted by depth) vs the binary32
    tiled oracle: same per-tile lists, same last-contributor index, colour within 1e-5."""
    sc = synth.make_scene(48, deg, "uniform", seed=seed, log_scale_mean=-2.5)
    v = synth.look_at((0.2, -0.3, -3), width=48, height=40, s_v=1.5)
    r = O.render32(sc, v)
    b = brute.render(sc, v)
    assert b["min_margin"] > 1e-5, "seed lands near a decision threshold"
    assert np.array_equal(b["rendered"], (r["flags"] & 4) > 0)
    TW = (v.width + 15) // 16
    for (tx, ty), lst in b["tile_lists"].items():
        t = ty * TW + tx
        assert np.array_equal(lst, r["entries"][r["tile_off"][t]:r["tile_off"][t + 1]])
    assert np.array_equal(b["last"], r["last"])
    assert np.abs(b["rgb"] - r["rgb"]).max() < 1e-5
    assert np.abs(b["T"] - r["T"]).max() < 1e-5


def test_tile_lists_equal_stable_sort_of_emitted_keys():
    """Emitting one (tile, depth) key per covered tile in Gaussian index order and sorting
    stably gives the oracle's per-tile lists; the ranges partition [0, D) and depth is
    non-decreasing inside each tile."""
    sc = synth.make_scene(10000, 0, "uniform", seed=0)
    v = synth.look_at((0, 0, -3), width=256, height=256)
    r = O.render32(sc, v)
    TW = 16
    keys, vals = [], []
    for i in np.nonzero(r["flags"] & 4)[0]:
        x0, x1, y0, y1 = r["rect"][i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                keys.append(((ty * TW + tx) << 32) | int(r["rec"][i, 2:3].view(np.uint32)[0]))
                vals.append(i)
    keys = np.array(keys, np.uint64)
    vals = np.array(vals, np.int64)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(vals[order], r["entries"])
    assert np.array_equal(keys[order], O.sorted_keys(r))
    tiles_touched = ((r["rect"][:, 1] - r["rect"][:, 0]) * (r["rect"][:, 3] - r["rect"][:, 2]))[r["flags"] & 4 > 0]
    assert tiles_touched.sum() == r["entries"].size == r["tile_off"][-1]
    d = r["rec"][r["entries"], 2]
    for t in range(256):
        a, b = r["tile_off"][t], r["tile_off"][t + 1]
        assert np.all(np.diff(d[a:b]) >= 0)


# ------------------------------------------------------------------ FP64 path and gradients

def test_fp64_forward_matches_binary32_oracle():
    sc = synth.make_scene(3000, 3, "uniform", seed=9)
    v = synth.look_at((0.4, 0.3, -3), width=80, height=48, s_v=1.3)
    r = O.render32(sc, v)
    t = O.scene_to_torch64(sc, requires_grad=False)
    rgb, T, eta, a2 = O.fp64_view_forward(t, v, r)
    assert np.abs(rgb.numpy() - r["rgb"]).max() < 1e-5
    assert np.abs(T.numpy() - r["T"]).max() < 1e-5
    assert abs(float(eta) - r["counts"][1] / sc["n"]) < 1e-15
    # alpha'' = alpha exp(-q) inherits q's relative error times q: tight where it matters.
    big = r["rec"][:, 6] > 1e-3
    np.testing.assert_allclose(a2.numpy()[big], r["rec"][big, 6], rtol=2e-6)
    assert np.abs(a2.numpy() - r["rec"][:, 6]).max() < 5e-7


def test_fp64_autograd_matches_finite_differences():
    """Central differences of the FP64 forward (discrete decisions held fixed) agree with
    its autograd gradient, including the frustum-maximum path.  The point-count term has
    a constant value (n_M / N), so its straight-through gradient is checked separately
    against differences of the kept-primitive mass sum_i alpha''_i / N."""
    sc = synth.make_scene(40, 2, "uniform", seed=12, log_scale_mean=-2.5)
    sc["decay"] = np.abs(sc["decay"]) + np.float32(0.3)
    v = synth.look_at((0.3, -0.2, -3), width=32, height=32, s_v=1.4)
    r = O.render32(sc, v)
    rng = np.random.default_rng(0)
    g_rgb = rng.normal(size=(3, 32, 32))
    g_eta = 0.7
    grads_r = O.fp64_grads(sc, v, r, g_rgb, 0.0)
    grads_all = O.fp64_grads(sc, v, r, g_rgb, g_eta)
    t = O.scene_to_torch64(sc, requires_grad=False)

    def losses():
        rgb, _, _, a2 = O.fp64_view_forward(t, v, r)
        return float((rgb.numpy() * g_rgb).sum()), float(a2.sum()) / sc["n"]

    k = r["argmax"]
    checks = [("mean", (0, k)), ("mean", (2, k)), ("decay", (k,))]
    rend = np.nonzero(r["flags"] & 4)[0]
    for i in rend[:4]:
        checks += [("mean", (0, i)), ("mean", (1, i)), ("log_scale", (1, i)), ("quat", (2, i)),
                   ("opacity", (i,)), ("decay", (i,)), ("sh", (0, 1, i)), ("sh", (5, 2, i))]
    for name, idx in checks:
        base = t[name].detach().clone()
        h = 1e-6 * max(1.0, abs(float(base[idx])))
        t[name] = base.clone(); t[name][idx] += h
        lp, mp = losses()
        t[name] = base.clone(); t[name][idx] -= h
        lm, mm = losses()
        t[name] = base
        fd = (lp - lm) / (2 * h)
        an = grads_r[name][idx]
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (name, idx, fd, an)
        ste = grads_all[name][idx] - an
        fd_mass = g_eta * (mp - mm) / (2 * h)
        assert abs(fd_mass - ste) <= 1e-6 * max(1.0, abs(ste)), (name, idx, fd_mass, ste)


# ------------------------------------------------------------------ loss scalars, Eq. (3)-(5)

def test_loss_scalars_closed_form():
    assert O.eta_target(4.0) == 0.125
    assert abs(O.l_reg(4.0, 0.5) - 9 * 0.375 ** 2) < 1e-15 and abs(O.l_reg(4.0, 0.5) - 1.265625) < 1e-15
    assert O.l_reg(4.0, 0.1) == 0.0 and O.l_reg(1.0, 0.9) == 0.0
    assert O.w_s(4.0, 8.0) == 0.5625 and O.w_s(8.0, 8.0) == 0.25 and O.w_s(1.0, 1.0) == 0.25
    assert abs(O.total_loss(0.2, 4.0, 0.5, 8.0) - 0.5625 * (0.2 + 1.265625)) < 1e-15


def test_storage_overhead_matches_paper_table():
    """One extra float per Gaussian: 248 -> 252 bytes (Sec. 4.4), so the memory column of
    the main results table is #GS x 252 B / 2^20 for the CLoD models."""
    rows = json.load(open(os.path.join(GOLDEN, "paper_storage.json")))["rows"]
    for row in rows:
        # #GS is printed rounded to thousands: +-500 Gaussians = +-0.121 MB.
        mem = row["gaussians_k"] * 1000 * row["bytes_per_gaussian"] / 2 ** 20
        assert abs(mem - row["mem_mb"]) < 0.5e3 * row["bytes_per_gaussian"] / 2 ** 20, row
    assert round(4 / 248 * 100, 1) == 1.6


# ---------------------------------------------------------------------------------------
# Budgeted LoD selection (the Sec. 4 comparisons keep the Gaussians of highest attenuated
# opacity): pinned against a brute-force rank definition and against the threshold mask.
# ---------------------------------------------------------------------------------------

def _with_budget(view, k):
    import dataclasses
    return dataclasses.replace(view, budget=int(k))


def test_budget_mask_equals_brute_force_rank_with_ties():
    """Kept iff fewer than K Gaussians precede it in (alpha'' descending, index ascending),
    counted pair by pair; duplicated Gaussians make equal alpha'' values."""
    sc = synth.make_scene(300, 1, "uniform", seed=21)
    for dst, src in ((9, 5), (40, 5), (77, 120)):
        for key in ("mean", "log_scale", "quat", "sh"):
            sc[key][..., dst] = sc[key][..., src]
        sc["opacity"][dst] = sc["opacity"][src]
        sc["decay"][dst] = sc["decay"][src]
    view = synth.look_at((0.2, -0.1, -3.0), width=96, height=80, s_v=2.0)
    a2 = O.view_pass(sc, view)["rec"][:, 6].astype(np.float64)
    assert a2[9] == a2[5] == a2[40] and a2[77] == a2[120]
    n = sc["n"]
    before = np.array([np.sum((a2 > a2[i]) | ((a2 == a2[i]) & (np.arange(n) < i))) for i in range(n)])
    for k in (1, 2, 17, 150, int(before[9]), int(before[9]) + 1, n - 1, n, n + 5):
        vp = O.view_pass(sc, _with_budget(view, k))
        kept = (vp["flags"] & 2) > 0
        assert np.array_equal(kept, before < k), k
        assert vp["counts"][1] == min(k, n)


def test_budget_mask_equals_threshold_mask_between_consecutive_values():
    """With no tie at the cut, keeping the K largest alpha'' is the threshold mask for any
    tau * s_v strictly between the K-th and (K+1)-th largest values; every output agrees."""
    sc = synth.make_scene(2000, 3, "mixture", seed=22)
    view = synth.look_at((1.0, 0.5, -7.0), width=128, height=96, s_v=1.0)
    a2 = np.sort(O.view_pass(sc, view)["rec"][:, 6])[::-1]
    checked = 0
    for k in (50, 150, 300, 500, 800):   # 916 of the 2000 alpha'' are non-zero here
        hi, lo = a2[k - 1], a2[k]
        if not hi > lo:
            continue
        tau = np.float32((np.float64(hi) + np.float64(lo)) / 2)
        if not (lo < tau < hi):
            continue
        p = dict(tau=float(tau))
        a = O.render32(sc, view, p)
        b = O.render32(sc, _with_budget(view, k), p)
        assert np.array_equal(a["flags"], b["flags"]), k
        assert np.array_equal(a["rec"].view(np.uint32), b["rec"].view(np.uint32)), k
        assert np.array_equal(a["rgb"].view(np.uint32), b["rgb"].view(np.uint32)), k
        assert np.array_equal(a["last"], b["last"]), k
        checked += 1
    assert checked >= 3


def test_budget_masks_nest_as_the_budget_grows():
    sc = synth.make_scene(1500, 0, "uniform", seed=23)
    view = synth.look_at((0.0, 0.0, -3.0), width=64, height=64, s_v=3.0)
    prev = None
    for k in (0, 1, 10, 100, 700, 1499, 1500):
        if k == 0:
            continue
        kept = (O.view_pass(sc, _with_budget(view, k))["flags"] & 2) > 0
        assert kept.sum() == k
        if prev is not None:
            assert np.all(kept[prev])
        prev = kept


# ---------------------------------------------------------------------------------------
# Optimiser step (Sec. 4.1: 3DGS Adam recipe with the decay factor as one more parameter).
# ---------------------------------------------------------------------------------------

def test_adam_binary32_matches_textbook_fp64_within_rounding():
    from oracle import train_oracle as TO
    rng = np.random.default_rng(40)
    n = 20000
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    p64, m64, v64 = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    S = np.zeros(n)   # running sum of the magnitudes of the terms of m (its rounding scale)
    for t in range(1, 6):
        g = (rng.normal(size=n) * 10.0 ** rng.uniform(-6, 1, size=n)).astype(np.float32)
        p, m, v = TO.adam_step32(p, g, m, v, 1e-2, t)
        # The textbook update with the binary32 hyperparameters the binary32 step uses.
        f = lambda x: float(np.float32(x))
        p64, m64, v64 = TO.adam_step64(p64, g, m64, v64, f(1e-2), t, b1=f(0.9), b2=f(0.999), eps=f(1e-15))
        S = 0.9 * S + 0.1 * np.abs(g.astype(np.float64))
        # Each step moves p by at most lr (|m_hat| <= sqrt(v_hat)); binary32 adds a few ulps.
        assert np.max(np.abs(p - p64)) <= 1e-6 * t
        assert np.all(np.abs(m - m64) <= 2.0 ** -21 * t * S)
        assert np.all(np.abs(v - v64) <= 2.0 ** -20 * t * v64 + 1e-45)


def test_adam_first_step_is_lr_times_sign_and_zero_gradient_is_a_no_op():
    from oracle import train_oracle as TO
    g = np.array([3.0, -0.5, 1e-3, -2e-6, 0.0], np.float32)
    p = np.ones(5, np.float32)
    z = np.zeros(5, np.float32)
    p1, m1, v1 = TO.adam_step32(p, g, z, z, 0.01, 1)
    # t = 1: m_hat = g and v_hat = g^2, so the step is lr * g / (|g| + eps).
    want = 1.0 - 0.01 * g.astype(np.float64) / (np.abs(g.astype(np.float64)) + 1e-15)
    assert np.allclose(p1, want, rtol=0, atol=2e-7)
    assert p1[4] == 1.0 and m1[4] == 0.0 and v1[4] == 0.0


def test_position_lr_schedule_endpoints_and_log_linearity():
    from oracle import train_oracle as TO
    assert math.isclose(TO.position_lr(0), 1.6e-4, rel_tol=1e-12)
    assert math.isclose(TO.position_lr(30000), 1.6e-6, rel_tol=1e-12)
    assert math.isclose(TO.position_lr(15000), math.sqrt(1.6e-4 * 1.6e-6), rel_tol=1e-12)


# ---------------------------------------------------------------------------------------
# D-SSIM part of L_render (Eq. (5): the 3DGS weighted sum of L1 and D-SSIM).
# ---------------------------------------------------------------------------------------

def test_ssim_two_implementations_agree():
    from oracle import ssim_oracle as SO
    rng = np.random.default_rng(60)
    x = rng.uniform(size=(3, 37, 29))
    y = np.clip(x + rng.normal(scale=0.1, size=x.shape), 0, 1)
    a = SO.ssim64(x, y)
    b = 1.0 - float(SO.dssim_torch64(torch.from_numpy(x), torch.from_numpy(y)))
    assert abs(a - b) < 1e-12


def test_ssim_identical_images_is_one_and_constant_images_closed_form():
    from oracle import ssim_oracle as SO
    rng = np.random.default_rng(61)
    x = rng.uniform(size=(3, 24, 30))
    assert np.allclose(SO.ssim_map64(x, x), 1.0, atol=1e-12)
    # Constant images a and b: away from the zero padding every variance vanishes and
    # S = (2ab + C1) / (a^2 + b^2 + C1).
    a, b = 0.7, 0.2
    m = SO.ssim_map64(np.full((1, 30, 30), a), np.full((1, 30, 30), b))
    want = (2 * a * b + SO.C1) / (a * a + b * b + SO.C1)
    assert np.allclose(m[0, 5:-5, 5:-5], want, rtol=1e-12)
    assert abs(SO.window1d().sum() - 1.0) < 1e-15 and np.allclose(SO.window1d(), SO.window1d()[::-1])


def test_ssim_linear_ramp_closed_form_pins_c1_c2_and_window():
    """x = a + g1 i + g2 j and y = c + s x.  More than 5 px from the zero padding the
    window-weighted moments are exact: mean_x = x (the window is symmetric), var_x =
    (g1^2 + g2^2) m2, var_y = s^2 var_x, cov_xy = s var_x, with m2 = sum_k w_k k^2 the second
    moment of the normalised 11-tap Gaussian window of standard deviation 1.5 (the 3DGS rendering
    loss), so SSIM = (2 mx my + C1)(2 s var_x + C2) / ((mx^2 + my^2 + C1)((1 + s^2) var_x + C2))
    with C1 = 0.01^2 and C2 = 0.03^2.  Unlike constant images, the variances are not zero here,
    so C2 and the window width both enter (checked: other values move SSIM far outside the
    tolerance)."""
    from oracle import ssim_oracle as SO

    def closed_form(x, y, s, grad2, sigma, c1, c2):
        k = np.arange(-5, 6, dtype=np.float64)
        w = np.exp(-k * k / (2.0 * sigma * sigma))
        m2 = float((w * k * k).sum() / w.sum())
        var = grad2 * m2
        return (2 * x * y + c1) * (2 * s * var + c2) / ((x * x + y * y + c1) * ((1 + s * s) * var + c2))

    H, W = 40, 48
    i, j = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    g1, g2, a, c, s = 0.004, 0.011, 0.1, 0.95, -0.5
    x = a + g1 * i + g2 * j
    y = c + s * x
    got = SO.ssim_map64(x[None], y[None])[0][5:-5, 5:-5]
    inner = np.s_[5:-5, 5:-5]
    want = closed_form(x[inner], y[inner], s, g1 * g1 + g2 * g2, 1.5, 0.01 ** 2, 0.03 ** 2)
    assert np.allclose(got, want, rtol=1e-10, atol=0)
    # The same images under other constants: each differs from the oracle by far more than
    # the tolerance, so a wrong C1, C2 or window width fails the check above.
    for sigma, c1, c2 in ((1.0, 0.01 ** 2, 0.03 ** 2), (2.0, 0.01 ** 2, 0.03 ** 2),
                          (1.5, 0.01 ** 2, 0.02 ** 2), (1.5, 0.01 ** 2, 0.05 ** 2), (1.5, 0.02 ** 2, 0.03 ** 2)):
        other = closed_form(x[inner], y[inner], s, g1 * g1 + g2 * g2, sigma, c1, c2)
        assert np.abs(other - got).max() > 1e-4, (sigma, c1, c2)
    # The differentiable implementation gives the same mean over the whole image.
    d = float(SO.dssim_torch64(torch.from_numpy(x[None]), torch.from_numpy(y[None])))
    assert abs((1.0 - d) - SO.ssim_map64(x[None], y[None]).mean()) < 1e-12


def test_render_loss_gradient_matches_central_differences():
    from oracle import ssim_oracle as SO
    rng = np.random.default_rng(62)
    x = rng.uniform(0.1, 0.9, size=(3, 14, 17))
    y = rng.uniform(size=x.shape)
    _, g = SO.render_loss64(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 7, 8), (2, 13, 16), (0, 3, 12), (2, 9, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (SO.render_loss64(xp, y)[0] - SO.render_loss64(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), idx


# ---------------------------------------------------------------------------------------
# Viewports of a frame (spatially varying s_v, the strips of the Sec. 4 DLoD/CLoD comparison):
# a viewport renders exactly the frame's pixels under its own s_v.
# ---------------------------------------------------------------------------------------

def _crop(img, v):
    return img[..., v.vy:v.vy + v.height, v.vx:v.vx + v.width]


def test_viewport_strips_stitch_to_the_whole_frame_bit_exact():
    sc = synth.make_scene(4000, 1, "mixture", seed=80)
    frame = synth.look_at((2.0, 1.0, -9.0), width=200, height=130, s_v=2.0)
    full = O.render32(sc, frame)
    for v in synth.strips(frame, [2.0, 2.0, 2.0, 2.0]):
        r = O.render32(sc, v)
        assert np.array_equal(r["rgb"].view(np.uint32), _crop(full["rgb"], v).view(np.uint32))
        assert np.array_equal(r["T"].view(np.uint32), _crop(full["T"], v).view(np.uint32))
        assert np.array_equal(r["last"], _crop(full["last"], v))
        assert r["dmax"] == full["dmax"] and r["argmax"] == full["argmax"]
        assert np.array_equal(r["counts"][:2], full["counts"][:2])


def test_viewport_strips_at_different_sv_equal_uniform_renders_at_each_sv():
    sc = synth.make_scene(6000, 3, "mixture", seed=81)
    frame = synth.look_at((-3.0, 2.0, -8.0), width=160, height=96)
    svs = [8.0, 4.0, 2.0, 1.0]
    for v, s in zip(synth.strips(frame, svs), svs):
        import dataclasses
        uni = O.render32(sc, dataclasses.replace(frame, s_v=s))
        r = O.render32(sc, v)
        assert np.array_equal(r["rgb"].view(np.uint32), _crop(uni["rgb"], v).view(np.uint32)), s
        assert np.array_equal(r["last"], _crop(uni["last"], v)), s


def test_viewport_window_offset_on_both_axes():
    sc = synth.make_scene(3000, 0, "uniform", seed=82)
    frame = synth.look_at((0.2, -0.1, -3.0), width=150, height=120, s_v=1.5)
    full = O.render32(sc, frame)
    v = synth.viewport(frame, 32, 48, 70, 41)
    r = O.render32(sc, v)
    assert np.array_equal(r["rgb"].view(np.uint32), _crop(full["rgb"], v).view(np.uint32))
    assert np.array_equal(r["last"], _crop(full["last"], v))
