"""torch.autograd.Function wrappers around the library's forward and adjoint
entry points.  The tree and near lists are constants of the operator (the
binning is piecewise constant in the positions), so gradients flow through
the pairwise sums only.

GravityP2P.apply(x, y, z, m, tree, nbrs, eps) -> (phi, ax, ay, az)
    backward: p2p_adjoint(gravity): dL/dx, dL/dy, dL/dz, dL/dm (FP64).
HelmholtzP2P.apply(q, tree, nbrs, prec) -> u = A q
    backward: grad_q = A^H grad_u = conj(A^T conj(grad_u)), PyTorch's
    convention for complex inputs; A^T = A by reciprocity.

A contrast chi enters as q = chi * u_inc composed in PyTorch, and autograd
carries the product rule (the inverse-scattering gradient of a DBIM step).
"""
from __future__ import annotations

import torch

from . import api


class GravityP2P(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, m, tree: api.Tree, nbrs: api.Nbrs, eps: float):
        x, y, z, m = (t.contiguous() for t in (x, y, z, m))
        phi, ax, ay, az = api.gravity(tree, nbrs, eps, x=x, y=y, z=z, m=m, layout="gather",
                                      prec="fp64")
        ctx.save_for_backward(x, y, z, m)
        ctx.tree, ctx.nbrs, ctx.eps = tree, nbrs, eps
        return phi, ax, ay, az

    @staticmethod
    def backward(ctx, g_phi, g_ax, g_ay, g_az):
        x, y, z, m = ctx.saved_tensors
        dev = x.device
        gs = [g if g is not None else torch.zeros(x.numel(), dtype=torch.float64, device=dev)
              for g in (g_phi, g_ax, g_ay, g_az)]
        gs = [g.contiguous() for g in gs]
        gx, gy, gz, gm = api.gravity_adjoint(ctx.tree, ctx.nbrs, ctx.eps, x, y, z, m, *gs)
        return gx, gy, gz, gm, None, None, None


class HelmholtzP2P(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, tree: api.Tree, nbrs: api.Nbrs, prec: str = "fp64"):
        q = q.contiguous()
        ctx.tree, ctx.nbrs, ctx.prec = tree, nbrs, prec
        return api.helmholtz(tree, nbrs, q, layout="gather", prec=prec)

    @staticmethod
    def backward(ctx, g_u):
        g = api.helmholtz_adjoint(ctx.tree, ctx.nbrs, g_u.contiguous(), prec=ctx.prec,
                                  conjugate=True)
        return g, None, None, None


def gravity(x, y, z, m, tree, nbrs, eps):
    return GravityP2P.apply(x, y, z, m, tree, nbrs, eps)


def helmholtz(q, tree, nbrs, prec="fp64"):
    return HelmholtzP2P.apply(q, tree, nbrs, prec)
