"""Shared test helpers: run the HIP path through the C ABI and the oracle on the same seeded
inputs, and compare them."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O
from paper_2510_09997_amd import _clod as C
from paper_2510_09997_amd.render import Batch, Scene


def params_struct(p: dict | None):
    p = {**O.DEFAULT_PARAMS, **(p or {})}
    return C.make_params(tau=p["tau"], eps=p["eps"], near=p["near"], guard=p["guard"],
                         dilation=p["dilation"], bg=p["bg"])


def gpu_forward(sc: dict, views, params: dict | None = None, dup_capacity=None, packed_sh: bool = False,
                scene: Scene | None = None):
    """Runs clod_project, clod_bin_sort and clod_render_fwd; returns host copies.  `scene`
    reuses a device-resident scene built from `sc`."""
    if scene is None:
        scene = Scene(sc, packed_sh=packed_sh)
    b = Batch(sc["n"], views, params_struct(params), dup_capacity=dup_capacity)
    b.project(scene)
    D = b.bin_sort()
    pairs = torch.zeros(3, dtype=torch.int64, device="cuda")
    rgb, T, last = b.render_fwd(pairs)
    torch.cuda.synchronize()
    out = dict(batch=b, scene=scene, D=D, counts=b.counts.cpu().numpy(), pairs=pairs.cpu().numpy(),
               rgb_flat=rgb, T_flat=T, last_flat=last)
    out["rgb"] = [t.cpu().numpy() for t in b.split(rgb, 3)]
    out["T"] = [t.cpu().numpy() for t in b.split(T, 1)]
    out["last"] = [t.cpu().numpy() for t in b.split(last, 1)]
    out["tile_ids"] = b.section(C.SEC_KEYS, D).cpu().numpy().view(np.uint32)
    out["vals"] = b.section(C.SEC_VALUES, D).cpu().numpy().view(np.uint32)
    out["ranges"] = b.section(C.SEC_RANGES).cpu().numpy().view(np.uint32)
    out["rec"] = b.section(C.SEC_REC).cpu().numpy()
    out["alpha"] = b.section(C.SEC_ALPHA).cpu().numpy()
    # Fourth quad of a record: depth, rectangle words, tiles touched.
    q3 = out["rec"][:, 3, :]
    out["depth"] = q3[:, 0].copy()
    # The sorted pairs as (tile << 32 | bits(depth)) keys, from the tile ids and the depth of
    # each pair's record.
    dbits = out["depth"].view(np.uint32).astype(np.uint64)
    out["keys"] = (out["tile_ids"].astype(np.uint64) << np.uint64(32)) | dbits[out["vals"].astype(np.int64)]
    out["flags"] = b.section(C.SEC_FLAGS).cpu().numpy()
    out["dmax"] = b.section(C.SEC_DMAX).cpu().numpy().view(np.uint64)
    out["rect"] = np.ascontiguousarray(q3[:, 1:3]).view(np.uint32)
    out["tiles_touched"] = np.ascontiguousarray(q3[:, 3]).view(np.uint32)
    return out


def stored_planes(scene: Scene) -> dict:
    """Host copies of a device scene's planes as stored (after any spatial reorder), in the
    layout of the synthetic scenes, for the oracle."""
    d = {k: v.cpu().numpy() for k, v in scene.t.items()}
    d["n"], d["sh_degree"] = scene.n, scene.sh_degree
    return d


def tile_bases(views):
    tb = [0]
    for v in views:
        tb.append(tb[-1] + ((v.width + 15) // 16) * ((v.height + 15) // 16))
    return tb


def compare_forward(g: dict, sc: dict, views, params: dict | None = None, fp64: bool = False,
                    check_records: bool = True):
    """Bit-exact comparison of everything integer (and the binary32 contract values) per view."""
    n = sc["n"]
    tb = tile_bases(views)
    all_keys, all_vals = [], []
    for v, view in enumerate(views):
        r = O.render32(sc, view, params)
        assert np.array_equal(g["counts"][v], r["counts"]), (v, g["counts"][v], r["counts"])
        key = int(g["dmax"][v])
        if r["argmax"] < 0:
            assert key == 0
        else:
            assert np.float32(r["dmax"]).view(np.uint32) == (key >> 32), v
            assert 0xFFFFFFFF - (key & 0xFFFFFFFF) == r["argmax"], v
        fl = g["flags"][v * n:(v + 1) * n]
        assert np.array_equal(fl, r["flags"]), v
        if check_records:
            rend = (r["flags"] & 4) > 0
            rec = g["rec"][v * n:(v + 1) * n][rend]
            depth = g["depth"][v * n:(v + 1) * n][rend]
            # alpha'' for every Gaussian, the rest for rendered ones.
            alpha = g["alpha"][v * n:(v + 1) * n]
            assert np.array_equal(alpha.view(np.uint32), r["rec"][:, 6].view(np.uint32)), v
            want = r["rec"][rend]
            got = np.stack([rec[:, 0, 0], rec[:, 0, 1], depth, rec[:, 1, 0], rec[:, 1, 1],
                            rec[:, 1, 2], rec[:, 0, 2], rec[:, 2, 0], rec[:, 2, 1], rec[:, 2, 2]], 1)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), v
            rc = g["rect"][v * n:(v + 1) * n][rend]
            rect = np.stack([rc[:, 0] & 0xFFFF, rc[:, 0] >> 16, rc[:, 1] & 0xFFFF, rc[:, 1] >> 16], 1)
            assert np.array_equal(rect.astype(np.int32), r["rect"][rend]), v
            tt = g["tiles_touched"][v * n:(v + 1) * n][rend].astype(np.int64)
            area = (rect[:, 1].astype(np.int64) - rect[:, 0]) * (rect[:, 3].astype(np.int64) - rect[:, 2])
            assert np.array_equal(tt, area), v
        # Keys, values and ranges of this view's tiles.
        all_keys.append(O.sorted_keys(r, tb[v]))
        all_vals.append(r["entries"].astype(np.uint64) + np.uint64(v * n))
        T_t = tb[v + 1] - tb[v]
        rg = g["ranges"][tb[v]:tb[v + 1]]
        off = r["tile_off"]
        base = int(sum(len(k) for k in all_keys[:-1]))
        for t in range(T_t):
            a, b = int(off[t]), int(off[t + 1])
            if b > a:
                assert rg[t, 0] == a + base and rg[t, 1] == b + base, (v, t)
            else:
                assert rg[t, 0] == 0 and rg[t, 1] == 0, (v, t)
        assert np.array_equal(g["last"][v].astype(np.int64), r["last"].astype(np.int64)), v
        assert np.array_equal(g["T"][v].view(np.uint32), r["T"].view(np.uint32)), v
        assert np.array_equal(g["rgb"][v].view(np.uint32), r["rgb"].view(np.uint32)), v
        if fp64:
            t = O.scene_to_torch64(sc, requires_grad=False)
            rgb64, T64, _, _ = O.fp64_view_forward(t, view, r, params)
            assert np.abs(g["rgb"][v] - rgb64.numpy()).max() <= 1e-5, v
    keys = np.concatenate(all_keys) if all_keys else np.zeros(0, np.uint64)
    vals = np.concatenate(all_vals) if all_vals else np.zeros(0, np.uint64)
    assert g["D"] == keys.size
    assert np.array_equal(g["keys"][:g["D"]], keys)
    assert np.array_equal(g["vals"][:g["D"]].astype(np.uint64), vals)


def _grad_case(sc, views, seed=0, dL_deta=None):
    """GPU gradients of sum(g * rgb) + sum_v dL_deta[v] eta_v for a random g, and the FP64
    oracle's gradients and absolute adjoints (per element, the magnitude of its terms) summed
    over the views.  Returns (got, want, S, vps)."""
    scene = Scene(sc)
    b = Batch(sc["n"], views, params_struct(None))
    b.project(scene)
    b.bin_sort()
    rgb, T, last = b.render_fwd()
    rng = np.random.default_rng(seed)
    g_rgb = rng.normal(size=3 * b.pixels).astype(np.float32)
    eta_g = None if dL_deta is None else torch.tensor(dL_deta, dtype=torch.float32, device="cuda")
    grads = b.render_bwd(scene, T, last, torch.from_numpy(g_rgb).cuda(), eta_g)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in grads.items()}
    want = {k: np.zeros(v.shape) for k, v in got.items()}
    S = {k: np.zeros(v.shape) for k, v in got.items()}
    vps = []
    for v, view in enumerate(views):
        r = O.render32(sc, view)
        vps.append(r)
        a = int(b.pix_base[v])
        h, w = view.height, view.width
        gv = g_rgb[3 * a:3 * a + 3 * h * w].reshape(3, h, w)
        ref = O.fp64_grads(sc, view, r, gv, 0.0 if dL_deta is None else float(dL_deta[v]), abs_terms=True)
        for k in want:
            want[k] += ref[k]
            S[k] += ref["abs"][k]
    return got, want, S, vps


def check_grads(got: dict, want: dict, S: dict, tol: float = 1e-4, log=print, argmaxes=()):
    """Element-wise gradient parity: |g_i - r_i| <= tol * S_i for every element of every plane
    (S_i = the magnitude of element i's chain-rule terms, = |r_i| where they do not cancel).
    Logs the bound's worst ratio, the floor-relative error max|g-r| / max(|r|, 1e-3 max|r|) and
    the L2 error for reference, and the element that is worst under the floor metric."""
    worst = {}
    for k in want:
        g = np.asarray(got[k], np.float64)
        r = np.asarray(want[k], np.float64)
        s = np.asarray(S[k], np.float64)
        e = O.grad_elem_error(g, r, s)
        fl = O.grad_floor_error(g, r)
        l2 = O.grad_l2_error(g, r)
        d = np.abs(g - r).ravel()
        den = np.maximum(np.abs(r).ravel(), 1e-3 * np.abs(r).max()) if r.size else d
        i = int(np.argmax(d / np.where(den > 0, den, 1.0))) if r.size else 0
        where = np.unravel_index(i, r.shape) if r.size else ()
        gauss = int(where[-1]) if r.size else -1
        note = " (frustum argmax)" if gauss in argmaxes else ""
        log(f"  {k}: elem/S {e:.3e}  floor-rel {fl:.3e}  l2 {l2:.3e}  worst-floor at {tuple(int(x) for x in where)}"
            f"{note}: got {g.ravel()[i]:.6e} want {r.ravel()[i]:.6e} S {s.ravel()[i]:.3e}" if r.size else f"  {k}: empty")
        if r.size:
            j = int(np.argmax(O.grad_elem_terms(g, r, s)))
            wj = np.unravel_index(j, r.shape)
            log(f"      worst elem/S at {tuple(int(x) for x in wj)}"
                f"{' (frustum argmax)' if int(wj[-1]) in argmaxes else ''}: got {g.ravel()[j]:.6e} "
                f"want {r.ravel()[j]:.6e} S {s.ravel()[j]:.3e}")
        worst[k] = e
    bad = {k: e for k, e in worst.items() if not e <= tol}
    assert not bad, bad
    return worst
