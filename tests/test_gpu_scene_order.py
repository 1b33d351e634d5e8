"""Spatial order of a scene (clod_scene_reorder: a preparation step outside the method, which
stores Gaussians that are close in space close in memory).

The permutation must equal a stable sort by the documented 30-bit Morton code, computed here
independently in float32 numpy; every plane must be the source plane gathered by it; and the
reordered scene, rendered through the C ABI, must be bit-identical to the oracle run on the
same stored planes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_09997_amd import _clod as C, synth
from paper_2510_09997_amd.render import Scene

from helpers import compare_forward, gpu_forward

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    C.load()


def log(*a):
    print(*a, flush=True)


def morton_codes(mean):
    """10 bits per axis over the box of the finite coordinates (float32 arithmetic), x lowest."""
    mean = np.asarray(mean, np.float32)
    code = np.zeros(mean.shape[1], np.uint64)
    for a in range(3):
        x = mean[a]
        fin = x[np.isfinite(x)]
        if fin.size:
            lo, hi = fin.min(), fin.max()
            ext = np.float32(hi - lo)
            sc = np.float32(1024.0) / ext if ext > 0 else np.float32(0.0)
        else:
            lo, sc = np.float32(0.0), np.float32(0.0)
        with np.errstate(invalid="ignore", over="ignore"):
            q = (x - np.float32(lo)) * np.float32(sc)
        q = np.where(np.isnan(q), np.float32(0.0), q)
        q = np.minimum(np.maximum(q, np.float32(0.0)), np.float32(1023.0)).astype(np.uint64)
        for b in range(10):
            code |= ((q >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return code


def reorder(sc):
    scene = Scene(sc, spatial_order=True)
    torch.cuda.synchronize()
    perm = scene.perm.cpu().numpy().astype(np.int64)
    planes = {k: v.cpu().numpy() for k, v in scene.t.items()}
    return scene, perm, planes


@pytest.mark.parametrize("n, kind, special, deg", [(100_003, "uniform", True, 3), (250_000, "mixture", False, 3),
                                                   (1, "uniform", False, 3), (4097, "uniform", "same", 3),
                                                   (30_001, "mixture", False, 0), (20_000, "uniform", False, 1),
                                                   (70_000, "mixture", True, 2)])
def test_permutation_is_the_stable_morton_order_and_planes_follow_it(n, kind, special, deg):
    log(f"case: reorder n={n} {kind} special={special} degree={deg}")
    sc = synth.make_scene(n, deg, kind, seed=5)
    if special is True:
        # Non-finite coordinates clamp to the box faces; they do not widen the box.
        rng = np.random.default_rng(3)
        idx = rng.choice(n, 40, replace=False)
        sc["mean"][0, idx[:10]] = np.nan
        sc["mean"][1, idx[10:20]] = np.inf
        sc["mean"][2, idx[20:30]] = -np.inf
        sc["mean"][:, idx[30:]] = np.float32(1e30)
    elif special == "same":
        sc["mean"][:] = np.float32(0.25)   # no extent: every code 0, the identity
    scene, perm, planes = reorder(sc)
    want = np.argsort(morton_codes(sc["mean"]), kind="stable")
    assert np.array_equal(perm, want)
    if special == "same":
        assert np.array_equal(perm, np.arange(n))
    for k in ("mean", "log_scale", "quat", "opacity", "decay", "sh"):
        src = np.asarray(sc[k], np.float32)
        assert np.array_equal(planes[k].view(np.uint32), src[..., perm].view(np.uint32)), k


def test_reordered_scene_renders_bitexact_to_the_oracle_on_its_stored_planes():
    log("case: reordered mixture scene, three views")
    sc = synth.make_scene(200_000, 3, "mixture", seed=11)
    scene, perm, planes = reorder(sc)
    stored = dict(planes, n=sc["n"], sh_degree=sc["sh_degree"])
    views = [synth.look_at((4.0, -2.0, -6.0), width=320, height=240, s_v=1.0),
             synth.look_at((-3.0, 1.0, 5.0), width=200, height=136, s_v=3.0)]
    g = gpu_forward(stored, views, scene=scene)
    compare_forward(g, stored, views)


def test_empty_scene_is_a_no_op():
    sc = synth.make_scene(0, 0, "uniform", seed=0)
    scene = Scene(sc, spatial_order=True)
    assert scene.perm is None and scene.n == 0
