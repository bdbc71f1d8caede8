"""torch.autograd wrappers of the differentiable entry points.

``chi0(...)`` differentiates with respect to the valence energies, the column energies
(band energies or window energies E_i), the column multiplicities (the weights
g(E_i) dE_i of Eq. (energyintegration)) and, in the float64 mode, the wavefunction
coefficients; ``eps_inv(...)`` with respect to chi0.  Forward
and backward run in the library's kernels (gw_chi0_build / gw_chi0_backward,
gw_eps_inv / gw_eps_inv_backward); the pair densities are recomputed in the backward
pass, never stored.  Complex gradients follow torch's convention dL/dRe + i dL/dIm,
which is the ABI's.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import _lib as L


class _Chi0(torch.autograd.Function):
    @staticmethod
    def forward(ctx, e_v, e_col, n_col, gctx, geom, coef_v, coef_c, col_band, omegas, delta, prec):
        ev, ec, nc = e_v.detach().contiguous(), e_col.detach().contiguous(), n_col.detach().contiguous()
        coef_v, coef_c = coef_v.detach().contiguous(), coef_c.detach().contiguous()
        prob = L.make_problem(geom, coef_v, ev, coef_c, ec, nc, col_band)
        if geom.value not in _geom_ng:
            raise ValueError("geometry not registered: create it with autograd.geometry()")
        ng = _geom_ng[geom.value]
        out = L.gw_chi0_build(gctx, [prob], [ng], omegas, delta, prec)[0]
        ctx.save_for_backward(ev, ec, nc)
        ctx.meta = (gctx, geom, coef_v, coef_c, col_band, omegas, delta, prec, ng)
        return out

    @staticmethod
    def backward(ctx, gout):
        ev, ec, nc = ctx.saved_tensors
        gctx, geom, coef_v, coef_c, col_band, omegas, delta, prec, ng = ctx.meta
        prob = L.make_problem(geom, coef_v, ev, coef_c, ec, nc, col_band)
        want = tuple(ctx.needs_input_grad[:3])
        coef = tuple(ctx.needs_input_grad[5:7])
        g = L.gw_chi0_backward(gctx, [prob], omegas, delta, prec, gout.contiguous(), want=want, coef=coef)
        gcv = g[3].view(coef_v.shape) if any(coef) and g[3] is not None else None
        gcc = g[4].view(coef_c.shape) if any(coef) and g[4] is not None else None
        return g[0], g[1], g[2], None, None, gcv, gcc, None, None, None, None


class _EpsInv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, chi, vcoul, gctx, hermitian):
        z = L.gw_eps_inv(gctx, vcoul, chi.detach(), hermitian=hermitian)
        L.gw_eps_inv_status(gctx)
        ctx.save_for_backward(z, vcoul)
        ctx.gctx = gctx
        return z

    @staticmethod
    def backward(ctx, gz):
        z, v = ctx.saved_tensors
        return L.gw_eps_inv_backward(ctx.gctx, v, z, gz.contiguous()), None, None, None


_geom_ng = {}


def geometry(gctx, n_fft: Sequence[int], gvec_wf, gvec_chi, cell=None, q=None):
    """gw_geom_create, remembering the dielectric-sphere size for the autograd wrappers."""
    g = L.gw_geom_create(gctx, n_fft, gvec_wf, gvec_chi, cell, q)
    _geom_ng[g.value] = len(gvec_chi)
    return g


def chi0(gctx, geom, coef_v, e_v, coef_c, e_col, n_col: Optional[torch.Tensor] = None, col_band=None,
         omegas=(0.0,), delta: float = 0.0, prec: str = "fp64"):
    """Differentiable chi0 (nomega, ng, ng) complex128."""
    if n_col is None:
        n_col = torch.ones_like(e_col)
    return _Chi0.apply(e_v, e_col, n_col, gctx, geom, coef_v, coef_c, col_band, tuple(float(w) for w in omegas),
                       float(delta), L.PRECISIONS[prec])


def eps_inv(gctx, chi, vcoul, hermitian: bool = False):
    """Differentiable (I - diag(v) chi)^-1 in float64 (hermitian=True: the static route, for a
    Hermitian negative semidefinite chi and v > 0; the gradient is the same)."""
    return _EpsInv.apply(chi, vcoul, gctx, bool(hermitian))
