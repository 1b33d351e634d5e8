"""Oracle for the optimiser step of CLoD-GS training.  TEST INFRASTRUCTURE ONLY: imported by
tests, the smoke check and the benchmark's CPU-baseline leg, never by the product path.

Sec. 4.1 (implementation details): training follows the 3DGS recipe (Adam over every
per-Gaussian parameter, a learning rate per parameter group) with the decay factor sigma_d of
Eq. (2) as one more per-Gaussian parameter, learning rate 1e-2, and the LoD mechanism (virtual
distance scale sampling, the decay and the regulariser of Sec. 3.3) switched on from iteration
5,000 of 30,000.

Adam (Kingma and Ba, 2015) per element, step t = 1, 2, ...:
    m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

`adam_step32` evaluates it in IEEE binary32 in this exact operation order (each numpy float32
operation is one correctly rounded binary32 operation, no fused multiply-add); b1, b2, lr and
eps are the binary32 roundings of the hyperparameters:
    c1 = 1 - b1, c2 = 1 - b2 (binary32);  bc1 = fl(1 - b1^t), bc2 = fl(1 - b2^t) (evaluated in
    float64 from the binary32 b1, b2, rounded once)
    m' = b1*m + c1*g;  v' = b2*v + c2*(g*g);  mh = m'/bc1;  vh = v'/bc2;
    p' = p - lr*(mh/(sqrt(vh) + eps)).
`adam_step64` is the textbook update in float64, the pin for the binary32 version.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32

# 3DGS per-group learning rates (positions decay exponentially over training) and the
# sigma_d rate of Sec. 4.1.  Groups: mean, log_scale, quat, opacity, decay, SH degree 0, SH
# degree >= 1.
GROUPS = ("mean", "log_scale", "quat", "opacity", "decay", "sh_dc", "sh_rest")


def bias_corrections(t: int, b1: float, b2: float):
    b1d, b2d = float(F32(b1)), float(F32(b2))
    return F32(1.0 - b1d ** t), F32(1.0 - b2d ** t)


def adam_step32(p, g, m, v, lr: float, t: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-15):
    """One binary32 Adam step on float32 arrays; returns (p', m', v')."""
    p, g, m, v = (np.asarray(a, dtype=F32) for a in (p, g, m, v))
    b1f, b2f, lrf, epsf = F32(b1), F32(b2), F32(lr), F32(eps)
    c1, c2 = F32(1.0) - b1f, F32(1.0) - b2f
    bc1, bc2 = bias_corrections(t, b1, b2)
    m2 = b1f * m + c1 * g
    v2 = b2f * v + c2 * (g * g)
    mh = m2 / bc1
    vh = v2 / bc2
    p2 = p - lrf * (mh / (np.sqrt(vh) + epsf))
    return p2.astype(F32), m2.astype(F32), v2.astype(F32)


def adam_step64(p, g, m, v, lr: float, t: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-15):
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m2 = b1 * m + (1 - b1) * g
    v2 = b2 * v + (1 - b2) * g * g
    p2 = p - lr * (m2 / (1 - b1 ** t)) / (np.sqrt(v2 / (1 - b2 ** t)) + eps)
    return p2, m2, v2


def scene_groups(scene: dict) -> dict:
    """The seven learning-rate groups as views into the scene's float32 planes."""
    K = (scene["sh_degree"] + 1) ** 2
    sh = scene["sh"].reshape(K, 3, -1)
    return dict(mean=scene["mean"], log_scale=scene["log_scale"], quat=scene["quat"],
                opacity=scene["opacity"], decay=scene["decay"], sh_dc=sh[:1], sh_rest=sh[1:])


def scene_adam_step32(scene: dict, grads: dict, m: dict, v: dict, lrs: dict, t: int, **hp):
    """Adam over every parameter plane of a scene (all arrays float32, same layout as the
    scene), each group with its own learning rate.  Updates the dicts in place."""
    out = {}
    for name, ps, gs, ms, vs in zip(GROUPS, scene_groups(scene).values(), scene_groups(grads).values(),
                                    scene_groups(m).values(), scene_groups(v).values()):
        p2, m2, v2 = adam_step32(ps, gs, ms, vs, lrs[name], t, **hp)
        ps[...] = p2
        ms[...] = m2
        vs[...] = v2
        out[name] = p2
    return out


def position_lr(step: int, lr_init: float = 1.6e-4, lr_final: float = 1.6e-6, max_steps: int = 30000,
                extent: float = 1.0) -> float:
    """Position learning rate of the 3DGS recipe: a geometric interpolation from lr_init to
    lr_final over max_steps (constant outside), i.e. lr_init (lr_final / lr_init)^t with
    t = step / max_steps clamped to [0, 1]; both ends scaled by the scene extent."""
    t = min(max(step / max_steps, 0.0), 1.0)
    return (lr_init * extent) * ((lr_final * extent) / (lr_init * extent)) ** t


def schedule_lrs(step: int, base: dict, enable_at: int, total: int) -> dict:
    """Learning rates of training iteration `step` (Sec. 4.1): the 3DGS per-group rates, the
    position rate decaying to 1/100 of its start over `total` iterations, and sigma_d frozen
    (rate 0) until the LoD mechanism is switched on at iteration `enable_at`."""
    out = dict(base)
    out["mean"] = position_lr(step, lr_init=base["mean"], lr_final=base["mean"] / 100.0, max_steps=total)
    if step < enable_at:
        out["decay"] = 0.0
    return out
