"""Differentiable soft-argmin disparity head (torch autograd binding).

``DcoSoftArgmin.apply(matcher, L, R, theta) -> dhat`` runs the library's
soft forward (Eq. 1 costs with theta = (lambda_AD, lambda_census, T), the
two-stage region means of Eq. 2, softmax over d) and, on ``backward``, its
hand-written backward kernels, which return d loss / d theta.  The backward
uses the aggregation the handle still holds from the forward (or recomputes
it when another soft call has replaced it).  Census codes and arm lengths are
integer and are not differentiated.
"""
from __future__ import annotations

import torch

from ._lib import check, lib
from .api import StereoMatcher, _need, _ptr


def _pairs(m: StereoMatcher, L, R):
    if L.dim() == 3:
        L, R = L.unsqueeze(0), R.unsqueeze(0)
    B = L.shape[0]
    _need(L, "L", torch.uint8, (B, m.H, m.W, 3))
    _need(R, "R", torch.uint8, (B, m.H, m.W, 3))
    return L, R, B


def soft_forward(m: StereoMatcher, L, R, theta):
    """(dhat, lse), each B x H x W float32."""
    L, R, B = _pairs(m, L, R)
    _need(theta, "theta", torch.float32, (3,))
    m._begin()
    dhat = m._empty((B, m.H, m.W), torch.float32)
    lse = m._empty((B, m.H, m.W), torch.float32)
    check(lib().dco_soft_forward(m._h, B, _ptr(L), _ptr(R), _ptr(theta), _ptr(dhat), _ptr(lse)))
    return dhat, lse


def soft_backward(m: StereoMatcher, L, R, theta, dhat, lse, grad_dhat, reuse=False):
    """d loss / d theta (3 float32) for grad_dhat = d loss / d dhat.  With
    reuse, the aggregation the handle holds from the forward on these same
    L, R, theta tensors (unchanged since) is used instead of recomputed."""
    L, R, B = _pairs(m, L, R)
    shape = (B, m.H, m.W)
    _need(theta, "theta", torch.float32, (3,))
    for t, n in ((dhat, "dhat"), (lse, "lse"), (grad_dhat, "grad_dhat")):
        _need(t, n, torch.float32, shape)
    m._begin()
    g = m._empty((3,), torch.float32)
    fn = lib().dco_soft_backward_reuse if reuse else lib().dco_soft_backward
    check(fn(m._h, B, _ptr(L), _ptr(R), _ptr(theta), _ptr(dhat), _ptr(lse), _ptr(grad_dhat),
             _ptr(g)))
    return g


class DcoSoftArgmin(torch.autograd.Function):
    """dhat = soft-argmin disparity of the left view; differentiable in theta."""

    @staticmethod
    def forward(ctx, matcher, L, R, theta):
        theta_c = theta.detach().contiguous()
        dhat, lse = soft_forward(matcher, L, R, theta_c)
        ctx.matcher = matcher
        ctx.save_for_backward(L, R, theta_c, dhat, lse)
        return dhat.reshape(L.shape[:-1])

    @staticmethod
    def backward(ctx, grad_dhat):
        # saved tensors cannot have changed in place since the forward
        # (autograd checks their versions), so the handle's aggregation of
        # that forward can be reused if nothing has replaced it
        L, R, theta, dhat, lse = ctx.saved_tensors
        g = soft_backward(ctx.matcher, L, R, theta, dhat, lse,
                          grad_dhat.reshape(dhat.shape).contiguous().float(), reuse=True)
        return None, None, None, g.to(theta.dtype)


def soft_argmin_disparity(matcher, L, R, theta):
    return DcoSoftArgmin.apply(matcher, L, R, theta)
