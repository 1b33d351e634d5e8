"""The allocation-free LoD count (for callers that cannot allocate device memory), called through
the C ABI: its counts equal clod_lod_count's, bit for bit, on two calls in a row, the second with
a smaller input (fewer Gaussians and views: the library scratch still holds the first call's
contents), and inputs beyond its scratch are rejected before anything is launched."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2510_09997_amd import _clod as C, synth
from paper_2510_09997_amd.render import Batch, Scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def _both(scene, views):
    b = Batch(scene.n, views)
    want = b.lod_count(scene)
    got = torch.full((len(views), 3), -1, dtype=torch.int64, device="cuda")
    vh = C.make_views(views)
    vd = C.views_to_device(vh, "cuda")
    C.clod_lod_count_noalloc(scene.c_struct(), vh, vd, C.make_params(), got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), want.cpu().numpy()


def test_noalloc_lod_count_matches_workspace_entry_point_on_two_calls():
    log("case: no-alloc lod count, 1M x 33 views then 150k x 5 views")
    big = Scene(synth.make_scene(1_000_000, 3, "mixture", seed=21))
    ds = synth.sweep_distances(32, 2.0, 200.0)
    views = [synth.look_at((0.0, 0.0, -float(d)), width=1920, height=1080) for d in ds]
    views.append(dataclasses.replace(synth.look_at((3.0, 2.0, -9.0), width=1280, height=720, s_v=2.0), budget=40000))
    got, want = _both(big, views)
    log(f"  call 1: {got[:3].tolist()} ... budget view {got[-1].tolist()}")
    assert np.array_equal(got, want)
    assert got[-1, 1] == 40000
    small = Scene(synth.make_scene(150_000, 1, "uniform", seed=22))
    views2 = [synth.look_at((0.5, 0.2, -3.0), width=w, height=h, s_v=s)
              for w, h, s in ((256, 256, 1.0), (640, 480, 1.5), (100, 75, 3.0), (1920, 1080, 6.0), (64, 64, 12.0))]
    got2, want2 = _both(small, views2)
    log(f"  call 2: {got2.tolist()}")
    assert np.array_equal(got2, want2)


def test_noalloc_lod_count_rejects_oversize_input_before_launch():
    log("case: no-alloc lod count oversize")
    n = 17_000_000   # the work list alone (4 bytes per Gaussian) exceeds the 64 MiB scratch
    zeros = {k: torch.zeros(c * n, dtype=torch.float32, device="cuda") for k, c in
             (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity", 1), ("decay", 1), ("sh", 3))}
    scene = Scene(dict(zeros, n=n, sh_degree=0))
    views = [synth.look_at((0, 0, -3), width=16, height=16)]
    vh = C.make_views(views)
    vd = C.views_to_device(vh, "cuda")
    out = torch.zeros(len(views), 3, dtype=torch.int64, device="cuda")
    with pytest.raises(C.ClodError) as e:
        C.clod_lod_count_noalloc(scene.c_struct(), vh, vd, C.make_params(), out)
    assert e.value.status == C.CLOD_E_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(out.abs().sum()) == 0   # nothing was written
