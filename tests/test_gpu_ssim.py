"""The D-SSIM part of L_render (Eq. (5), the 3DGS rendering loss) on the GPU against the
float64 oracle: loss values and the gradient with respect to the rendered image, for views of
ragged sizes in one batch."""
import numpy as np
import pytest
import torch

from oracle import oracle as O, ssim_oracle as SO
from paper_2510_09997_amd import synth
from paper_2510_09997_amd.render import Batch, Scene

from helpers import params_struct

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_loss_with_dssim_matches_fp64_oracle(lam):
    log(f"case: dssim lambda {lam}")
    views = [synth.look_at((0.0, 0.0, -3.0), width=131, height=77, s_v=1.0),
             synth.look_at((1.0, 0.0, -3.0), width=64, height=48, s_v=3.0),
             synth.look_at((0.0, 1.0, -3.0), width=200, height=35, s_v=6.0)]
    sc = synth.make_scene(2000, 0, "uniform", seed=70)
    scene = Scene(sc)
    b = Batch(sc["n"], views, params_struct(None))
    b.project(scene)
    rng = np.random.default_rng(71)
    # A smooth target and a noisy rendering of it, so SSIM is far from both 0 and 1.
    xs, ys = [], []
    for v in views:
        yy = np.clip(0.5 + 0.3 * np.sin(np.linspace(0, 6, v.width))[None, None, :]
                     * np.cos(np.linspace(0, 4, v.height))[None, :, None] + np.zeros((3, 1, 1)), 0, 1)
        xx = np.clip(yy + rng.normal(scale=0.08, size=yy.shape), 0, 1)
        xs.append(xx.astype(np.float32))
        ys.append(yy.astype(np.float32))
    rgb = torch.from_numpy(np.concatenate([x.reshape(-1) for x in xs])).cuda()
    tgt = torch.from_numpy(np.concatenate([y.reshape(-1) for y in ys])).cuda()
    s_max = 8.0
    loss, dL, _ = b.loss(rgb, tgt, s_max, lambda_reg=0.0, lambda_dssim=lam)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    dLs = b.split(dL, 3)
    for v, view in enumerate(views):
        ref, g, terms = SO.render_loss64(xs[v], ys[v], lam, abs_terms=True)
        ws = O.w_s(view.s_v, s_max)
        assert abs(loss[v] - ws * ref) <= 2e-6 * max(1.0, abs(ws * ref)), (v, loss[v], ws * ref)
        got = dLs[v].cpu().numpy()
        # Every pixel's gradient within 1e-4 of the magnitude of its chain-rule terms (the
        # 11 x 11 window sums of the SSIM map's derivatives cancel strongly).
        err = O.grad_elem_error(got, ws * g, ws * terms)
        log(f"  view {v}: loss {loss[v]:.7f} ref {ws * ref:.7f}  grad elem/S {err:.2e}  "
            f"floor-rel {O.grad_floor_error(got, ws * g):.2e}")
        assert err <= 1e-4, (v, err)
