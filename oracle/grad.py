"""Oracle: closed-form gradients of the band sum and of the inverse (test infrastructure only).

Not in the paper: the derivatives follow from Eq. (chi0) and eps = 1 - v chi0 by
ordinary calculus.  Convention for a real loss L of a complex matrix X: the gradient
is Xbar = dL/dRe X + i dL/dIm X, so that dL = Re sum conj(Xbar) dX.

  * Z = (I - V chi0)^-1  =>  chi0bar = V Z^H Zbar Z^H            (V = diag v, real)
  * chi0(w) = sum_p w_p m_p m_p^H  =>  wbar_p = m_p^H chi0bar m_p
  * w_p = n_c/2 [1/(x - w + i d) + 1/(x + w + i d)], x = E_v - E_c:
      dL/dx = Re(conj(wbar) dw/dx),  dw/dx = -n_c/2 [(x - w + i d)^-2 + (x + w + i d)^-2]
      dL/dn = Re(conj(wbar) dw/dn),  dw/dn = 1/2 [(x - w + i d)^-1 + (x + w + i d)^-1]
    dL/dE_v = sum_c dL/dx, dL/dE_c = -sum_v dL/dx (this covers a window energy E_i too).
  * coefficients, back through the matrix element m_p = F(conj(u_v) u_c), F x (G) =
    (1/N) sum_r x(r) e^{iG.r}, u_n = B c_n, B c (r) = sum_g c(g) e^{ig.r}:
      mbar_p = sum_w [conj(w_p) chi0bar m_p + w_p chi0bar^H m_p]
      h_p = F^H mbar_p,  h_p(r) = (1/N) sum_G mbar_p(G) e^{-iG.r}
      ubar_c = sum_v h_vc u_v,  ubar_v = sum_c conj(h_vc) u_c
      cbar_n = B^H ubar_n,  cbar_n(g) = sum_r ubar_n(r) e^{-ig.r}
Every formula here is pinned against central finite differences of the oracle's
forward functions in tests/test_oracle.py.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import scipy.fft as sfft

from .chi0 import _workers, box_map, pair_density_fft, psi_real_space, weights


def head_block_loss(eps_inv_mat: np.ndarray, head: np.ndarray) -> float:
    """L = Re sum_{G in H} [eps^-1]_GG over a set H of G-vectors (the 'head block')."""
    return float(np.real(np.trace(eps_inv_mat[np.ix_(head, head)])))


def head_block_loss_grad(ng: int, head: np.ndarray) -> np.ndarray:
    g = np.zeros((ng, ng), dtype=np.complex128)
    g[head, head] = 1.0
    return g


def grad_eps_inv(z: np.ndarray, vcoul: np.ndarray, zbar: np.ndarray) -> np.ndarray:
    """chi0bar = V Z^H Zbar Z^H for Z = (I - V chi0)^-1."""
    zh = np.conj(z.T)
    return vcoul[:, None] * (zh @ zbar @ zh)


def grad_weights_dynamic(x: np.ndarray, n: np.ndarray, omega: float, delta: float):
    """(dw/dx, dw/dn) of w = n/2 [1/(x - w + i d) + 1/(x + w + i d)]."""
    a = 1.0 / (x - omega + 1j * delta)
    b = 1.0 / (x + omega + 1j * delta)
    return -0.5 * n * (a * a + b * b), 0.5 * (a + b)


def grad_chi0_energies(coef_v: np.ndarray, e_v: np.ndarray, coef_c: np.ndarray, e_col: np.ndarray,
                       gvec_wf: np.ndarray, gvec_chi: np.ndarray, nd: Sequence[int], chibar: np.ndarray,
                       omegas: Sequence[float] = (0.0,), delta: float = 0.0,
                       n_col: Optional[np.ndarray] = None, col_band: Optional[np.ndarray] = None):
    """(dL/dE_v, dL/dE_col, dL/dn_col) given chibar (nomega, ng, ng)."""
    if col_band is None:
        col_band = np.arange(coef_c.shape[0])
    n = np.ones(len(col_band)) if n_col is None else np.asarray(n_col, dtype=np.float64)
    psi_v = psi_real_space(coef_v, gvec_wf, nd)
    psi_c = psi_real_space(coef_c[col_band], gvec_wf, nd)
    m = pair_density_fft(psi_v, psi_c, gvec_chi)               # (nv, nc, ng)
    x = e_v[:, None] - e_col[None, :]
    gx = np.zeros_like(x)
    gn = np.zeros_like(x)
    for iw, om in enumerate(omegas):
        # wbar_p = m_p^H chibar m_p
        s = np.einsum("vcg,gh,vch->vc", np.conj(m), chibar[iw], m)
        dwdx, dwdn = grad_weights_dynamic(x, n[None, :], om, delta)
        gx += np.real(np.conj(s) * dwdx)
        gn += np.real(np.conj(s) * dwdn)
    return gx.sum(1), -gx.sum(0), gn.sum(0)


def grad_chi0_coefficients(coef_v: np.ndarray, e_v: np.ndarray, coef_c: np.ndarray, e_col: np.ndarray,
                           gvec_wf: np.ndarray, gvec_chi: np.ndarray, nd: Sequence[int], chibar: np.ndarray,
                           omegas: Sequence[float] = (0.0,), delta: float = 0.0,
                           n_col: Optional[np.ndarray] = None, col_band: Optional[np.ndarray] = None):
    """(dL/dcoef_v, dL/dcoef_c) given chibar (nomega, ng, ng), in the same convention
    (dL/dRe + i dL/dIm), shaped like coef_v and coef_c; several columns on one
    coefficient row add up."""
    if col_band is None:
        col_band = np.arange(coef_c.shape[0])
    n = np.ones(len(col_band)) if n_col is None else np.asarray(n_col, dtype=np.float64)
    nd = tuple(int(x) for x in nd)
    npts = nd[0] * nd[1] * nd[2]
    psi_v = psi_real_space(coef_v, gvec_wf, nd)
    psi_c = psi_real_space(coef_c[col_band], gvec_wf, nd)
    m = pair_density_fft(psi_v, psi_c, gvec_chi)                    # (nv, nc, ng)
    mbar = np.zeros_like(m)
    for iw, om in enumerate(omegas):
        w = weights(e_v, e_col, n, om, delta)                        # (nv, nc)
        gb = chibar[iw]
        mbar += np.conj(w)[:, :, None] * np.einsum("gh,vch->vcg", gb, m)
        mbar += w[:, :, None] * np.einsum("hg,vch->vcg", np.conj(gb), m)
    i1, i2, i3 = box_map(gvec_chi, nd)
    w1, w2, w3 = box_map(gvec_wf, nd)
    ubar_v = np.zeros_like(psi_v)
    ubar_c = np.zeros_like(psi_c)
    for v in range(psi_v.shape[0]):
        box = np.zeros((psi_c.shape[0],) + nd, dtype=np.complex128)
        box[:, i1, i2, i3] = mbar[v]
        h = sfft.fftn(box, axes=(1, 2, 3), workers=_workers()) / npts   # (nc, grid)
        ubar_c += h * psi_v[v][None]
        ubar_v[v] = np.sum(np.conj(h) * psi_c, axis=0)
    gv = sfft.fftn(ubar_v, axes=(1, 2, 3), workers=_workers())[:, w1, w2, w3]
    gcol = sfft.fftn(ubar_c, axes=(1, 2, 3), workers=_workers())[:, w1, w2, w3]
    gc = np.zeros_like(coef_c, dtype=np.complex128)
    np.add.at(gc, col_band, gcol)
    return gv, gc
