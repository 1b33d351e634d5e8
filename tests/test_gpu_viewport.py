"""Viewports of a frame on the GPU (spatially varying s_v): bit-exact forward against the oracle
for a batch mixing strips at different s_v, an offset window and a whole frame; stitched strips
equal the whole-frame render at 1080p; gradients through viewport views match FP64 autograd."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2510_09997_amd import synth
from paper_2510_09997_amd.render import Batch, Scene

from helpers import _grad_case, check_grads, compare_forward, gpu_forward, params_struct

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def test_viewport_batch_forward_bitexact():
    log("case: viewport batch")
    sc = synth.make_scene(20000, 3, "mixture", seed=90)
    frame = synth.look_at((2.0, 1.0, -9.0), width=333, height=150, s_v=1.0)
    views = synth.strips(frame, [8.0, 4.0, 2.0, 1.0])
    views.append(synth.viewport(frame, 64, 32, 100, 77, s_v=3.0))
    views.append(synth.look_at((-3.0, 2.0, -8.0), width=120, height=90, s_v=2.0))
    g = gpu_forward(sc, views)
    compare_forward(g, sc, views)


def test_strips_stitch_to_whole_frame_at_1080p():
    log("case: strips 1080p")
    sc = synth.make_scene(300000, 3, "mixture", seed=91)
    frame = synth.look_at((3.0, 1.0, -8.0), width=1920, height=1080, s_v=2.0)
    strips = synth.strips(frame, [2.0] * 5)
    scene = Scene(sc)
    outs = []
    for views in ([frame], strips):
        b = Batch(sc["n"], views, params_struct(None))
        b.project(scene)
        b.bin_sort()
        rgb, T, last = b.render_fwd()
        torch.cuda.synchronize()
        outs.append((b, b.split(rgb, 3), b.split(last, 1)))
    _, frgb, flast = outs[0]
    _, srgb, slast = outs[1]
    full_rgb, full_last = frgb[0].cpu().numpy(), flast[0].cpu().numpy()
    for v, view in enumerate(strips):
        a = np.s_[..., view.vy:view.vy + view.height, view.vx:view.vx + view.width]
        assert np.array_equal(srgb[v].cpu().numpy().view(np.uint32), full_rgb[a].view(np.uint32)), v
        assert np.array_equal(slast[v].cpu().numpy(), full_last[a]), v


def test_gradients_through_viewports_match_fp64_oracle():
    log("case: viewport gradients")
    sc = synth.make_scene(3000, 3, "uniform", seed=92, log_scale_mean=-3.5)
    frame = synth.look_at((0.4, 0.3, -3.2), width=112, height=64, s_v=1.0)
    views = synth.strips(frame, [1.3, 2.0]) + [synth.viewport(frame, 32, 16, 48, 40, s_v=1.6)]
    got, want, S, vps = _grad_case(sc, views, seed=3, dL_deta=[0.3, -0.2, 0.1])
    check_grads(got, want, S, 1e-4, log=log, argmaxes={vp["argmax"] for vp in vps})
