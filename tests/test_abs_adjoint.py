"""Pins of the oracle's absolute adjoint (the per-element scale of a gradient's chain-rule
terms that the gradient parity tests measure errors against).  No GPU needed.

* every intercepted primitive against the brute-force |J|^T |g| of its Jacobian;
* a differentiable operation without known absolute partials raises instead of silently
  propagating signed partials;
* on whole renders: S >= |gradient| everywhere (triangle inequality), and S = |gradient|
  exactly where no term can cancel (SH coefficients under a positive colour gradient: every
  term is the product of a positive upstream gradient, a positive blend weight and the same
  basis value Y_k)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle.abs_adjoint import AbsAdjointMode
from paper_2510_09997_amd import synth



def _abs_vjp(f, inputs, g):
    xs = [x.clone().requires_grad_(True) for x in inputs]
    with AbsAdjointMode():
        y = f(*xs)
    y.backward(g.abs())
    return [x.grad for x in xs]


def _brute(f, inputs, g):
    J = torch.autograd.functional.jacobian(f, tuple(inputs))
    out = []
    for x, Jx in zip(inputs, J):
        Jm = Jx.reshape(g.numel(), x.numel()).abs()
        out.append((Jm.T @ g.abs().reshape(-1)).reshape(x.shape))
    return out


rng = np.random.default_rng(5)


def T(*shape, positive=False):
    a = rng.normal(size=shape)
    if positive:
        a = np.abs(a) + 0.5
    return torch.from_numpy(a)   # float64 (numpy's default), no change to torch's defaults


CASES = [
    ("mul_broadcast", lambda a, b: a[:, None] * b[None, :], [T(4), T(3)]),
    ("mul_scalar_negative", lambda a: -2.5 * a, [T(5)]),
    ("mul_same_operand", lambda a: a * a, [T(6)]),
    ("matmul", lambda a, b: a @ b, [T(3, 4), T(4, 2)]),
    ("matmul_batched", lambda a, b: a @ b.transpose(1, 2), [T(2, 3, 4), T(2, 5, 4)]),
    ("einsum", lambda a, b: torch.einsum("mk,kcm->mc", a, b), [T(3, 4), T(4, 2, 3)]),
    ("cumprod", lambda a: torch.cumprod(a, dim=1), [T(3, 5)]),
    ("sub", lambda a, b: a - b[None, :], [T(3, 4), T(4)]),
    ("rsub", lambda a: 1.0 - a, [T(5)]),
    ("neg", lambda a: -a, [T(5)]),
    ("div", lambda a, b: a / b, [T(4), T(4, positive=True)]),
    ("rdiv_scalar", lambda b: -3.0 / b, [T(4, positive=True)]),
    ("div_by_scalar", lambda a: a / -7.0, [T(4)]),
    ("pow2", lambda a: a ** 2, [T(5)]),
    ("norm", lambda a: torch.linalg.norm(a, dim=0, keepdim=True), [T(4, 3)]),
    ("abs", lambda a: (a - 0.1).abs(), [T(6)]),
    ("conv2d", lambda x, w: torch.nn.functional.conv2d(x, w, padding=1, groups=2), [T(1, 2, 5, 6), T(2, 1, 3, 3)]),
]


@pytest.mark.parametrize("name,f,inputs", CASES, ids=[c[0] for c in CASES])
def test_primitive_absolute_vjp_equals_brute_force_absolute_jacobian(name, f, inputs):
    y = f(*inputs)
    g = torch.from_numpy(rng.normal(size=tuple(y.shape)))
    got = _abs_vjp(f, inputs, g)
    want = _brute(f, inputs, g)
    for a, b in zip(got, want):
        assert torch.allclose(a, b, rtol=1e-12, atol=1e-14), name


def test_passthrough_operations_keep_non_negative_partials():
    # sums, exp, sqrt, sigmoid, relu, where and indexing: the mode's result equals |J|^T |g|
    f = lambda a: torch.where(a > 0, torch.sqrt(a.abs() + 1.0), torch.exp(a)).sum() + torch.sigmoid(a)[1:3].sum()
    a = T(6)
    one = torch.ones(1, dtype=torch.float64)
    got = _abs_vjp(lambda x: f(x).reshape(1), [a], one)[0]
    want = _brute(lambda x: f(x).reshape(1), [a], one)[0]
    assert torch.allclose(got, want, rtol=1e-12, atol=0)


def test_unknown_differentiable_operation_raises():
    a = T(4).requires_grad_(True)
    with pytest.raises(NotImplementedError):
        with AbsAdjointMode():
            torch.sin(a)


def test_composite_sum_of_mixed_sign_terms():
    # L = sum_j c_j x: dL/dx = sum_j c_j, its terms' magnitudes sum to sum_j |c_j|.
    c = torch.tensor([3.0, -2.0, 0.5, -1.5], dtype=torch.float64)
    x = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    with AbsAdjointMode():
        L = (c * x).sum()
    L.backward()
    assert float(x.grad) == pytest.approx(7.0, rel=1e-15)


@pytest.mark.parametrize("deg", [0, 3])
def test_render_absolute_adjoint_bounds_gradient_and_is_tight_without_cancellation(deg):
    sc = synth.make_scene(400, deg, "uniform", seed=30 + deg, log_scale_mean=-3.0)
    view = synth.look_at((0.3, 0.2, -3.0), width=48, height=40, s_v=1.4)
    vp = O.render32(sc, view)
    g = np.random.default_rng(31).normal(size=(3, 40, 48))
    ref = O.fp64_grads(sc, view, vp, g, 0.25, abs_terms=True)
    for k in O.PLANES:
        S, r = ref["abs"][k], ref[k]
        assert np.all(S >= 0.0), k
        assert np.all(S >= np.abs(r) * (1.0 - 1e-12)), k
        assert np.any(S > 0.0), k
    # Positive upstream gradient, no regulariser term: SH terms share one sign per coefficient.
    gp = np.abs(g) + 0.1
    pos = O.fp64_grads(sc, view, vp, gp, 0.0, abs_terms=True)
    S, r = pos["abs"]["sh"], pos["sh"]
    assert np.any(r != 0.0)
    assert np.allclose(S, np.abs(r), rtol=1e-11, atol=0.0)
    # Rendered Gaussians' opacity gradients do cancel (an opaque Gaussian darkens what lies
    # behind it), so there S exceeds |gradient| somewhere.
    assert np.any(pos["abs"]["opacity"] > np.abs(pos["opacity"]) * (1 + 1e-6))
