"""torch.autograd binding of the summed bead energy E = sum_b V(x_b) (eq. PI_potential
without the 1/P) of a context.

``bead_energy(ctx, pos, charge, lj_epsilon, lj_sigma)`` returns E as a 0-d tensor. Its
gradient in positions is the library's forces (qhp_eval), its gradients in the charges and
per-type LJ parameters are qhp_param_grad, and the backward of the position gradient (a
second backward pass, ``create_graph=True``) is qhp_hvp: the exact Hessian-vector product
(the Hessian is symmetric, so the vector-Jacobian product of the gradient is H v) and the
mixed derivatives d(v . grad E)/d(q, epsilon, sigma), so a loss on forces can be
differentiated with respect to the parameters. This module only marshals tensors to the C
ABI: every derivative is computed by the library.

Tensors live on the context's device (``mem_kind`` device) or on the host (CPU tensors,
copied through host memory). The parameters are inputs so that autograd can route their
gradients; their values must equal the context's, which the library copied at creation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import MEM_DEVICE, MEM_HOST, NTERMS, _ptr


def _mem(t):
    return MEM_DEVICE if t.is_cuda else MEM_HOST


def _arg(t):
    return _ptr(t if t.is_cuda else t.numpy())


def _eval(context, pos):
    pos = pos.detach().contiguous().to(torch.float64)
    E = torch.zeros((context.P, NTERMS), dtype=torch.float64, device=pos.device)
    F = torch.zeros_like(pos)
    context._check(context._lib.qhp_eval(context._h, _arg(pos), None, _arg(E), _arg(F),
                                         _mem(pos)))
    if pos.is_cuda:
        context.sync()
    return E, F


def _hvp(context, pos, v, mixed=False):
    pos = pos.detach().contiguous().to(torch.float64)
    v = v.detach().contiguous().to(torch.float64)
    out = torch.zeros_like(pos)
    kw = dict(dtype=torch.float64, device=pos.device)
    m = ([torch.zeros(context.N, **kw), torch.zeros(context.n_types, **kw),
          torch.zeros(context.n_types, **kw)] if mixed else [None, None, None])
    args = [_arg(t) if t is not None else None for t in m]
    context._check(context._lib.qhp_hvp(context._h, _arg(pos), _arg(v), _arg(out), args[0],
                                        args[1], args[2], _mem(pos)))
    if pos.is_cuda:
        context.sync()
    return (out, *m) if mixed else out


def _param_grad(context, pos):
    pos = pos.detach().contiguous().to(torch.float64)
    kw = dict(dtype=torch.float64, device=pos.device)
    dq = torch.zeros(context.N, **kw)
    de = torch.zeros(context.n_types, **kw)
    ds = torch.zeros(context.n_types, **kw)
    context._check(context._lib.qhp_param_grad(context._h, _arg(pos), _arg(dq), _arg(de),
                                               _arg(ds), _mem(pos)))
    if pos.is_cuda:
        context.sync()
    return dq, de, ds


class _Gradient(torch.autograd.Function):
    """grad E in positions; its backward is the Hessian-vector product and the mixed
    parameter derivatives."""

    @staticmethod
    def forward(ctx, pos, charge, lj_epsilon, lj_sigma, context):
        ctx.context = context
        ctx.save_for_backward(pos)
        _, F = _eval(context, pos)
        return -F

    @staticmethod
    def backward(ctx, v):
        (pos,) = ctx.saved_tensors
        if any(ctx.needs_input_grad[1:4]):
            hv, dq, de, ds = _hvp(ctx.context, pos, v, mixed=True)
            return hv, dq, de, ds, None
        return _hvp(ctx.context, pos, v), None, None, None, None


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, charge, lj_epsilon, lj_sigma, context):
        ctx.context = context
        ctx.save_for_backward(pos, charge, lj_epsilon, lj_sigma)
        E, _ = _eval(context, pos)
        return E.sum()

    @staticmethod
    def backward(ctx, gE):
        pos, charge, lj_epsilon, lj_sigma = ctx.saved_tensors
        context = ctx.context
        grad_pos = gE * _Gradient.apply(pos, charge, lj_epsilon, lj_sigma, context)
        dq = de = ds = None
        if any(ctx.needs_input_grad[1:4]):
            dq, de, ds = _param_grad(context, pos)
            dq, de, ds = gE * dq, gE * de, gE * ds
        return grad_pos, dq, de, ds, None


def bead_energy(context, pos, charge=None, lj_epsilon=None, lj_sigma=None):
    """E = sum over beads and terms of the bead potentials at pos [P][N][3] (FP64 tensor)."""
    kw = dict(dtype=torch.float64, device=pos.device)
    p = context.params
    ref_q = np.ctypeslib.as_array(p.charge, shape=(context.N,))
    ref_e = np.ctypeslib.as_array(p.lj_epsilon, shape=(context.n_types,))
    ref_s = np.ctypeslib.as_array(p.lj_sigma, shape=(context.n_types,))
    out = []
    for t, ref in ((charge, ref_q), (lj_epsilon, ref_e), (lj_sigma, ref_s)):
        if t is None:
            t = torch.tensor(ref, **kw)
        elif not np.array_equal(t.detach().cpu().numpy(), ref):
            raise ValueError("parameter values must equal the context's (copied at creation)")
        out.append(t)
    return _Energy.apply(pos, out[0], out[1], out[2], context)


def forces(context, pos, charge=None, lj_epsilon=None, lj_sigma=None):
    """-grad E at pos, differentiable with respect to pos (H v) and the parameters."""
    E = bead_energy(context, pos, charge, lj_epsilon, lj_sigma)
    (g,) = torch.autograd.grad(E, pos, create_graph=True)
    return -g
