"""Absolute adjoint of the FP64 oracle's forward.  TEST INFRASTRUCTURE ONLY: imported by tests,
the smoke check and the benchmark's CPU-baseline leg, never by the product path.

A gradient dL/dtheta_i is, by the chain rule, a sum over every path from theta_i to the loss of
the product of the local partial derivatives along the path.  Its absolute adjoint

    S_i = sum over paths of the product of |local partial| (times |dL/d output|)

bounds |dL/dtheta_i| (triangle inequality) and is the scale against which the rounding of any
binary32 evaluation of that sum is measured: a sum of many terms of both signs, evaluated in
any order, has an error of a few units of roundoff times the sum of its terms' magnitudes, not
times its (possibly much smaller) value.  Where the terms do not cancel, S_i = |dL/dtheta_i|.

S is computed by running the unchanged oracle forward under ``AbsAdjointMode`` and calling
backward with |dL/d output|.  The mode intercepts every operation whose local partials can be
negative or mixed in sign and replaces its backward by the product of absolute partials:

* multilinear operations (elementwise product, matrix product, einsum, cumulative product):
  every entry of their Jacobian is a single monomial of the operands with coefficient +1, so the
  absolute Jacobian-vector product is the ordinary one evaluated at the operands' absolute
  values (constants included) with the absolute cotangent;
* subtraction and negation: partials +1 and -1 become 1;
* division a / b: partials 1/b and -a/b^2 become 1/|b| and |a|/b^2;
* a ** p (scalar p): |p| |a|^(p-1);
* the Euclidean norm: |x_j| / ||x||; the absolute value: |sign(x)|.

Convolution (conv2d without bias) is multilinear too.

Operations whose partials are never negative (addition, sums, exp, sqrt, sigmoid, relu, routing
and indexing: where, stack, cat, gathers and scatters, reshapes) keep their own backward,
which maps a non-negative cotangent to a non-negative one.  Any other operation on a tensor
that requires a gradient raises, so the mode never silently propagates a signed partial.
"""
from __future__ import annotations

import torch
from torch.overrides import TorchFunctionMode, resolve_name


def _abs_operand(x):
    if isinstance(x, torch.Tensor):
        return x.detach().abs()
    if isinstance(x, (int, float)):
        return abs(x)
    return x


def _unbroadcast(g: torch.Tensor, shape) -> torch.Tensor:
    """Sums a broadcast cotangent back to `shape` (all terms are non-negative here)."""
    shape = tuple(shape)
    while g.dim() > len(shape):
        g = g.sum(0)
    for d, s in enumerate(shape):
        if s == 1 and g.shape[d] != 1:
            g = g.sum(d, keepdim=True)
    return g


class _Multilinear(torch.autograd.Function):
    """y = fn(*operands) with fn linear in each tensor operand separately."""

    @staticmethod
    def forward(ctx, fn, nconst, *ops):
        ctx.fn = fn
        ctx.is_tensor = [isinstance(o, torch.Tensor) for o in ops]
        ctx.consts = [None if t else o for t, o in zip(ctx.is_tensor, ops)]
        ctx.save_for_backward(*[o for o in ops if isinstance(o, torch.Tensor)])
        with torch.no_grad():
            return fn(*ops)

    @staticmethod
    def backward(ctx, g):
        saved = iter(ctx.saved_tensors)
        ops = [next(saved) if t else c for t, c in zip(ctx.is_tensor, ctx.consts)]
        need = ctx.needs_input_grad[2:]
        absops = []
        for o, nd in zip(ops, need):
            a = _abs_operand(o)
            if isinstance(a, torch.Tensor):
                a = a.requires_grad_(bool(nd))
            absops.append(a)
        wanted = [a for a, nd in zip(absops, need) if nd and isinstance(a, torch.Tensor)]
        grads = iter(())
        if wanted:
            with torch.enable_grad():
                y = ctx.fn(*absops)
                grads = iter(torch.autograd.grad(y, wanted, g.abs(), allow_unused=True))
        out = []
        for a, nd in zip(absops, need):
            if nd and isinstance(a, torch.Tensor):
                gr = next(grads)
                out.append(torch.zeros_like(a) if gr is None else gr)
            else:
                out.append(None)
        return (None, None, *out)


class _Sub(torch.autograd.Function):
    """a - b (either may be a Python number); |partials| = 1."""

    @staticmethod
    def forward(ctx, a, b):
        ctx.sa = a.shape if isinstance(a, torch.Tensor) else None
        ctx.sb = b.shape if isinstance(b, torch.Tensor) else None
        with torch.no_grad():
            return a - b

    @staticmethod
    def backward(ctx, g):
        g = g.abs()
        ga = _unbroadcast(g, ctx.sa) if ctx.sa is not None and ctx.needs_input_grad[0] else None
        gb = _unbroadcast(g, ctx.sb) if ctx.sb is not None and ctx.needs_input_grad[1] else None
        return ga, gb


class _Neg(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a):
        with torch.no_grad():
            return -a

    @staticmethod
    def backward(ctx, g):
        return g.abs()


class _Div(torch.autograd.Function):
    """a / b: |d/da| = 1/|b|, |d/db| = |a| / b^2."""

    @staticmethod
    def forward(ctx, a, b):
        ctx.ta, ctx.tb = isinstance(a, torch.Tensor), isinstance(b, torch.Tensor)
        ctx.ca = None if ctx.ta else a
        ctx.cb = None if ctx.tb else b
        ctx.save_for_backward(*[x for x in (a, b) if isinstance(x, torch.Tensor)])
        with torch.no_grad():
            return a / b

    @staticmethod
    def backward(ctx, g):
        saved = list(ctx.saved_tensors)
        a = saved.pop(0) if ctx.ta else ctx.ca
        b = saved.pop(0) if ctx.tb else ctx.cb
        g = g.abs()
        A, B = _abs_operand(a), _abs_operand(b)
        ga = gb = None
        if ctx.ta and ctx.needs_input_grad[0]:
            ga = _unbroadcast(g / B, a.shape)
        if ctx.tb and ctx.needs_input_grad[1]:
            gb = _unbroadcast(g * A / (B * B), b.shape)
        return ga, gb


class _Pow(torch.autograd.Function):
    """a ** p for a Python number p: |p| |a|^(p - 1)."""

    @staticmethod
    def forward(ctx, a, p):
        ctx.p = p
        ctx.save_for_backward(a)
        with torch.no_grad():
            return a ** p

    @staticmethod
    def backward(ctx, g):
        (a,) = ctx.saved_tensors
        p = ctx.p
        return g.abs() * abs(p) * a.abs() ** (p - 1), None


class _Abs(torch.autograd.Function):
    """|a|: partial sign(a) (0 at a = 0) becomes |sign(a)|."""

    @staticmethod
    def forward(ctx, a):
        ctx.save_for_backward(a)
        with torch.no_grad():
            return a.abs()

    @staticmethod
    def backward(ctx, g):
        (a,) = ctx.saved_tensors
        return g.abs() * (a != 0).to(g.dtype)


class _Norm(torch.autograd.Function):
    """Euclidean norm over `dim`: |d||x||/dx_j| = |x_j| / ||x||."""

    @staticmethod
    def forward(ctx, x, dim):
        with torch.no_grad():
            y = torch.linalg.norm(x, dim=dim, keepdim=True)
        ctx.save_for_backward(x, y)
        return y

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        return g.abs() * x.abs() / y, None


# Operations whose local partials are never negative, or that do not propagate gradients.
_PASSTHROUGH = {
    "torch.Tensor.__add__", "torch.Tensor.__radd__", "torch.Tensor.add", "torch.add",
    "torch.Tensor.sum", "torch.sum", "torch.Tensor.mean", "torch.mean",
    "torch.exp", "torch.Tensor.exp", "torch.sqrt", "torch.Tensor.sqrt", "torch.sigmoid",
    "torch.Tensor.sigmoid", "torch.relu", "torch.Tensor.relu", "torch.nn.functional.relu",
    "torch.where", "torch.stack", "torch.cat", "torch.Tensor.__getitem__", "torch.Tensor.index_select",
    "torch.Tensor.index_copy", "torch.Tensor.reshape", "torch.Tensor.view", "torch.Tensor.transpose",
    "torch.Tensor.T.__get__", "torch.Tensor.contiguous", "torch.Tensor.expand", "torch.Tensor.unsqueeze",
    "torch.Tensor.squeeze", "torch.Tensor.clone", "torch.Tensor.detach", "torch.Tensor.shape.__get__",
    "torch.Tensor.dim", "torch.Tensor.size", "torch.Tensor.numel", "torch.Tensor.dtype.__get__",
    "torch.Tensor.device.__get__", "torch.Tensor.requires_grad.__get__", "torch.Tensor.grad.__get__",
    "torch.Tensor.grad_fn.__get__", "torch.Tensor.is_leaf.__get__", "torch.Tensor.__len__",
    "torch.zeros_like", "torch.ones_like", "torch.full_like", "torch.Tensor.__eq__", "torch.Tensor.__gt__",
    "torch.Tensor.__ge__", "torch.Tensor.__lt__", "torch.Tensor.__le__", "torch.Tensor.__ne__",
    "torch.Tensor.__bool__", "torch.Tensor.__float__", "torch.Tensor.item", "torch.Tensor.numpy",
    "torch.Tensor.tolist", "torch.Tensor.__format__", "torch.Tensor.__repr__", "torch.Tensor.layout.__get__",
    "torch.Tensor.requires_grad_", "torch.Tensor.__setitem__", "torch.Tensor.ndim.__get__",
    "torch.Tensor.is_sparse.__get__", "torch.Tensor.data_ptr", "torch.Tensor.stride",
    "torch.Tensor.storage_offset", "torch.Tensor.is_contiguous", "torch.Tensor.__index__",
    "torch.Tensor.__int__", "torch.Tensor.to", "torch.Tensor.double", "torch.Tensor.float",
    "torch.Tensor.long", "torch.Tensor.bool", "torch.Tensor.gt", "torch.Tensor.ge", "torch.Tensor.lt",
    "torch.Tensor.le", "torch.Tensor.eq", "torch.Tensor.ne", "torch.gt", "torch.ge", "torch.lt", "torch.le",
    "torch.eq", "torch.ne", "torch.Tensor.any", "torch.Tensor.all", "torch.isfinite",
}


def _multilinear(fn, *ops):
    return _Multilinear.apply(fn, 0, *ops)


class AbsAdjointMode(TorchFunctionMode):
    """Within this mode, backward through the recorded graph yields absolute adjoints (see the
    module docstring).  Differentiable operations outside the known set raise."""

    def __torch_function__(self, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        name = resolve_name(func) or getattr(func, "__name__", repr(func))
        if name in ("torch.Tensor.__mul__", "torch.Tensor.__rmul__", "torch.mul", "torch.Tensor.mul"):
            a, b = args[0], args[1]
            return _multilinear(lambda x, y: x * y, a, b)
        if name in ("torch.Tensor.__matmul__", "torch.matmul", "torch.Tensor.matmul", "torch.bmm"):
            return _multilinear(lambda x, y: torch.matmul(x, y), args[0], args[1])
        if name == "torch.Tensor.__rmatmul__":
            return _multilinear(lambda x, y: torch.matmul(x, y), args[1], args[0])
        if name in ("torch.einsum", "torch.functional.einsum"):
            spec, ops = args[0], args[1:]
            if len(ops) == 1 and isinstance(ops[0], (list, tuple)):
                ops = tuple(ops[0])
            return _multilinear(lambda *t: torch.einsum(spec, *t), *ops)
        if name in ("torch.conv2d", "torch.nn.functional.conv2d"):
            x, w = args[0], args[1]
            rest = dict(kwargs)
            for key, val in zip(("bias", "stride", "padding", "dilation", "groups"), args[2:]):
                rest[key] = val
            if rest.get("bias") is not None:
                raise NotImplementedError("AbsAdjointMode: conv2d with a bias")
            return _multilinear(lambda a, b: torch.nn.functional.conv2d(a, b, **rest), x, w)
        if name in ("torch.abs", "torch.Tensor.abs"):
            return _Abs.apply(args[0])
        if name in ("torch.cumprod", "torch.Tensor.cumprod"):
            dim = kwargs.get("dim", args[1] if len(args) > 1 else None)
            return _multilinear(lambda x: torch.cumprod(x, dim=dim), args[0])
        if name in ("torch.Tensor.__sub__", "torch.sub", "torch.Tensor.sub"):
            return _Sub.apply(args[0], args[1])
        if name == "torch.Tensor.__rsub__":
            return _Sub.apply(args[1], args[0])
        if name in ("torch.Tensor.__neg__", "torch.neg", "torch.Tensor.neg"):
            return _Neg.apply(args[0])
        if name in ("torch.Tensor.__truediv__", "torch.div", "torch.Tensor.div", "torch.true_divide"):
            return _Div.apply(args[0], args[1])
        if name == "torch.Tensor.__rtruediv__":
            return _Div.apply(args[1], args[0])
        if name in ("torch.Tensor.__pow__", "torch.pow", "torch.Tensor.pow"):
            if not isinstance(args[1], (int, float)):
                raise NotImplementedError("AbsAdjointMode: tensor exponents are not supported")
            return _Pow.apply(args[0], args[1])
        if name == "torch.linalg.norm":
            x = args[0]
            dim = kwargs.get("dim", args[2] if len(args) > 2 else None)
            keepdim = kwargs.get("keepdim", False)
            if dim is None or kwargs.get("ord") not in (None, 2) or len(args) > 1 and args[1] not in (None, 2):
                raise NotImplementedError("AbsAdjointMode: only the Euclidean norm over one dim")
            y = _Norm.apply(x, dim)
            return y if keepdim else y.squeeze(dim)
        if name in _PASSTHROUGH:
            return func(*args, **kwargs)
        flat = list(args) + list(kwargs.values())
        flat += [x for a in args if isinstance(a, (list, tuple)) for x in a]
        if any(isinstance(x, torch.Tensor) and x.requires_grad for x in flat):
            raise NotImplementedError(f"AbsAdjointMode: no absolute partials for {name}")
        return func(*args, **kwargs)
