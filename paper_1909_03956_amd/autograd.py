"""torch.autograd.Functions over the library's forward and adjoint kernels.

For a real loss L and complex visibilities V, torch hands the backward
g = dL/dRe V + i dL/dIm V; the gradient of a real parameter x is then
Re sum_j conj(g_j) dV_j/dx, which the library computes directly:
  * direct route (Eq. 12) with respect to flux, l, m: swv_grad_direct with
    y = g, alpha = 1;
  * tree route (Eqs. 16-17, linear in the leaf fluxes, V = sum_k F_k eta_k):
    dL/dF_k = Re sum_j conj(g_j) eta_jk = Re (A^H g)_k, the adjoint at the
    leaf centres.
"""
from __future__ import annotations

import torch

from . import api


class DirectPredict(torch.autograd.Function):
    """V = predict_direct(u, v, w, l, m, flux); differentiable in flux, l, m."""

    @staticmethod
    def forward(ctx, flux, l, m, u, v, w, sign=-1):
        V = api.predict_direct(u, v, w, l, m, flux, sign=sign)
        ctx.save_for_backward(flux, l, m, u, v, w)
        ctx.sign = sign
        return V

    @staticmethod
    def backward(ctx, g):
        flux, l, m, u, v, w = ctx.saved_tensors
        if g.dtype != torch.complex128:
            g = g.to(torch.complex128)
        d_flux, d_l, d_m = api.grad_direct(u, v, w, g.contiguous(), l, m, flux,
                                           sign=ctx.sign, alpha=1.0)
        return d_flux, d_l, d_m, None, None, None, None


class TreePredict(torch.autograd.Function):
    """V = tree route with the given leaf fluxes; differentiable in them.

    The tree's pixel set (its leaves) is fixed; forward loads the fluxes into
    the tree (recomputing its coefficients) before predicting."""

    @staticmethod
    def forward(ctx, leaf_flux, tree, u, v, w, sign=-1):
        tree.set_leaf_flux(leaf_flux)
        V = tree.predict(u, v, w, sign=sign)
        lv = tree.leaves()
        dev = u.device
        ctx.save_for_backward(u, v, w)
        ctx.leaves = tuple(torch.as_tensor(lv[k], device=dev) for k in ("l", "m", "nm1"))
        ctx.sign = sign
        return V

    @staticmethod
    def backward(ctx, g):
        u, v, w = ctx.saved_tensors
        l, m, nm1 = ctx.leaves
        if g.dtype != torch.complex128:
            g = g.to(torch.complex128)
        img = api.adjoint(u, v, w, g.contiguous(), l, m, nm1, sign=ctx.sign)
        return img.real.contiguous(), None, None, None, None, None


def predict_direct(u, v, w, l, m, flux, sign: int = -1):
    """Differentiable direct prediction (see DirectPredict)."""
    return DirectPredict.apply(flux, l, m, u, v, w, sign)


def predict_tree(tree, leaf_flux, u, v, w, sign: int = -1):
    """Differentiable tree prediction in the leaf fluxes (see TreePredict)."""
    return TreePredict.apply(leaf_flux, tree, u, v, w, sign)
