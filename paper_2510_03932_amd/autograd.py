"""PyTorch autograd over the transcribed Lagrangian L(z, y) = sigma f(z) + y^T c(z).

Forward and every derivative run in the library's HIP kernels (through the C
ABI); PyTorch supplies the tensors, streams and the autograd graph.

    L = lagrangian(prob, z, y, A, B, gamma, sigma)       # 0-dim tensor
    L.backward()   # z.grad = grad_z L, y.grad = c(z), A.grad = dL/dA, ...

Second order: grad_z L is itself differentiable in (z, y, A, B, gamma), so
``torch.autograd.grad(L, z, create_graph=True)`` followed by a backward with a
vector v gives the Hessian-vector product (Hessian of L) v for z, J v for y
and the mixed second derivatives d/dtheta (v^T grad_z L) for the
coefficients theta = (A, B, gamma) (library call ocp_eval_coef_mixed)::

    gz = lagrangian_grad(prob, z, y, A, B, gamma)
    hv, hA, hB, hg = torch.autograd.grad(gz, (z, A, B, gamma), v)

The coefficient gradient dL/dtheta is differentiable too: L is affine in
theta, so its derivative in theta is zero and its derivatives in z and y are
the coefficient parts of grad_z L and of c under the cotangent coefficients
(library call ocp_eval_coef_adjoint).  So ``torch.autograd.gradgradcheck`` of L passes over all of
(z, y, A, B, gamma).  Third derivatives raise NotImplementedError.
"""
from __future__ import annotations

import torch


def _coefficients(prob, A, B, gamma, key=None):
    """Make the handle hold the coefficient tensors (one stream-ordered kernel
    launch) and return the key of the upload that put them there; a model
    without coefficient arrays (the quadrotor) takes A = B = gamma = None.
    Each upload gets a fresh key.  A backward passes the key its forward got,
    and nothing is uploaded while that upload is still the handle's last one
    (the values are then exactly the forward's); inside _Lagrangian.backward,
    which uploads for the Functions it applies, nothing is uploaded either.
    Problem.set_coefficients clears the key, so an upload made any other way
    makes the next backward upload again.  (A cache keyed on the tensors'
    identity and version would not be safe: writes through ``.data``, as
    torch.autograd.gradcheck makes them, change values without a version
    bump.)"""
    if A is None and B is None and gamma is None:
        return None
    current = getattr(prob, "_coef_key", None)
    if getattr(prob, "_coef_uploaded", False) or (key is not None and current is key):
        return current
    prob.set_coefficients(A.detach(), B.detach(), gamma.detach())
    prob._coef_key = key = object()
    return key


class _LagGrad(torch.autograd.Function):
    """grad_z L as a function of (z, y, A, B, gamma); its backward gives
    (Hessian of L) v for z, J v for y and d/dtheta (v^T grad_z L) for the
    coefficients."""

    @staticmethod
    def forward(ctx, z, y, A, B, gamma, sigma, prob):
        ctx.coef_key = _coefficients(prob, A, B, gamma)
        ctx.save_for_backward(z, y, A, B, gamma)
        ctx.sigma, ctx.prob = sigma, prob
        return prob.lag_grad(z.detach().contiguous(), y.detach().contiguous(), sigma)

    @staticmethod
    def backward(ctx, v):
        z, y, A, B, gamma = ctx.saved_tensors
        prob = ctx.prob
        _coefficients(prob, A, B, gamma, ctx.coef_key)
        v = v.detach().contiguous()
        zd, yd = z.detach().contiguous(), y.detach().contiguous()
        gz = gy = gA = gB = gg = None
        if ctx.needs_input_grad[0]:
            gz = prob.hvp(zd, yd, v, ctx.sigma)
        if ctx.needs_input_grad[1]:
            gy = prob.jvp(zd, v)
        if any(ctx.needs_input_grad[2:5]):
            gA, gB, gg = prob.coef_mixed(zd, yd, v)
        return gz, gy, gA, gB, gg, None, None


class _Cons(torch.autograd.Function):
    """c(z) as a function of (z, A, B, gamma); its backward is the
    vector-Jacobian product: J^T w for z (grad_z of w^T c, i.e. grad_z L with
    sigma = 0 and multipliers w) and the coefficient gradient of w^T c."""

    @staticmethod
    def forward(ctx, z, A, B, gamma, prob):
        ctx.coef_key = _coefficients(prob, A, B, gamma)
        ctx.save_for_backward(z, A, B, gamma)
        ctx.prob = prob
        return prob.cons(z.detach().contiguous())

    @staticmethod
    def backward(ctx, w):
        z, A, B, gamma = ctx.saved_tensors
        prob = ctx.prob
        if torch.is_grad_enabled() and (w.requires_grad or z.requires_grad):
            raise NotImplementedError("third derivatives of the defects are not provided")
        _coefficients(prob, A, B, gamma, ctx.coef_key)
        zd, w = z.detach().contiguous(), w.detach().contiguous()
        gz = prob.lag_grad(zd, w, 0.0) if ctx.needs_input_grad[0] else None
        gA = gB = gg = None
        if any(ctx.needs_input_grad[1:4]):
            gA, gB, gg = prob.coef_grad(zd, w)
        return gz, gA, gB, gg, None


class _CoefGrad(torch.autograd.Function):
    """dL/d(A, B, gamma) as a function of (z, y, A, B, gamma).  Its backward
    uses that L is affine in theta = (A, B, gamma): for cotangents tb,
    tb . dL/dtheta = y^T (c(z; tb) - c(z; 0)), whose gradients in z and y
    (the coefficient parts of J^T y and of c under tb) one library call
    returns (ocp_eval_coef_adjoint, which reads tb from its arguments and
    leaves the handle alone); the gradient in theta is zero."""

    @staticmethod
    def forward(ctx, z, y, A, B, gamma, prob):
        _coefficients(prob, A, B, gamma)
        ctx.save_for_backward(z, y, A, B, gamma)
        ctx.prob = prob
        return prob.coef_grad(z.detach().contiguous(), y.detach().contiguous())

    @staticmethod
    def backward(ctx, tA, tB, tg):
        z, y, A, B, gamma = ctx.saved_tensors
        prob = ctx.prob
        if torch.is_grad_enabled() and any(t.requires_grad for t in (z, y, tA, tB, tg)):
            raise NotImplementedError("third derivatives of the Lagrangian are not provided")
        gz = gy = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            gz, gy = prob.coef_adjoint(z.detach().contiguous(), y.detach().contiguous(),
                                       *(t.detach().contiguous() for t in (tA, tB, tg)),
                                       want_z=ctx.needs_input_grad[0], want_y=ctx.needs_input_grad[1])
        return gz, gy, None, None, None, None


class _Lagrangian(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, y, A, B, gamma, sigma, prob):
        ctx.coef_key = _coefficients(prob, A, B, gamma)
        ctx.save_for_backward(z, y, A, B, gamma)
        ctx.sigma, ctx.prob = sigma, prob
        return prob.lagrangian(z.detach().contiguous(), y.detach().contiguous(), sigma)[0]

    @staticmethod
    def backward(ctx, gL):
        z, y, A, B, gamma = ctx.saved_tensors
        prob, sigma = ctx.prob, ctx.sigma
        gz = gy = gA = gB = gg = None
        # the forward's upload, if it is still the handle's last one, or one
        # upload now, serves the three Functions below (nothing else runs on
        # the handle in between)
        _coefficients(prob, A, B, gamma, ctx.coef_key)
        if not torch.is_grad_enabled():
            # a plain backward (no create_graph): one library call computes
            # every piece and scales it by the incoming gradient on the device
            want_z, want_y = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            want_coef = any(ctx.needs_input_grad[2:5])
            if not (want_z or want_y or want_coef):
                return gz, gy, gA, gB, gg, None, None
            gz, gy, coef = prob.lagrangian_backward(z.detach().contiguous(), y.detach().contiguous(), sigma,
                                                    gL.detach().contiguous(), want_z, want_y, want_coef)
            if coef is not None:
                gA, gB, gg = coef
            return gz, gy, gA, gB, gg, None, None
        prob._coef_uploaded = True
        try:
            # each piece goes through a Function of its own so that a
            # create_graph backward stays differentiable where it is defined
            if ctx.needs_input_grad[0]:
                gz = _LagGrad.apply(z, y, A, B, gamma, sigma, prob) * gL
            if ctx.needs_input_grad[1]:
                gy = _Cons.apply(z, A, B, gamma, prob) * gL
            if any(ctx.needs_input_grad[2:5]):
                dA, dB, dg = _CoefGrad.apply(z, y, A, B, gamma, prob)
                gA, gB, gg = dA * gL, dB * gL, dg * gL
        finally:
            prob._coef_uploaded = False
        return gz, gy, gA, gB, gg, None, None


def lagrangian(prob, z, y, A=None, B=None, gamma=None, sigma: float = 1.0):
    """L(z, y) = sigma f(z) + y^T c(z) with differentiable z, y, A (n, n),
    B (n, m) and gamma (n,) (float64 tensors on the problem's device);
    sigma is a plain number.  For the quadrotor model, which has no
    coefficient arrays, leave A, B and gamma out."""
    return _Lagrangian.apply(z, y, A, B, gamma, float(sigma), prob)


def lagrangian_grad(prob, z, y, A=None, B=None, gamma=None, sigma: float = 1.0):
    """grad_z L as a differentiable function of (z, y, A, B, gamma)."""
    return _LagGrad.apply(z, y, A, B, gamma, float(sigma), prob)


def constraints(prob, z, A=None, B=None, gamma=None):
    """c(z) as a differentiable function of (z, A, B, gamma)."""
    return _Cons.apply(z, A, B, gamma, prob)
