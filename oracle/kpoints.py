"""Oracle: the k-point sum of Eq. (chi0) with the k+q mapping (test infrastructure only).

Eq. (chi0) sums over k; the valence states enter at k+q.  With Bloch states
psi_nk(r) = sum_g c_nk(g) e^{i(k+g).r} (g over k's own wavefunction sphere), the matrix
element <v,k+q| e^{i(q+G).r} |c,k> is the convolution sum_g' conj(c_{v,k+q}(g' + G)) c_{c,k}(g').
When k+q leaves the k-point set, k+q = k'' + G0 with k'' in the set and G0 a reciprocal
lattice vector, and the state at k+q is the one at k'' relabelled:
c_{v,k+q}(g) = c_{v,k''}(g + G0), with E_{v,k+q} = E_{v,k''}.  Everything here is written
from that definition (dictionaries of Miller indices, no FFT), and pinned in
tests/test_oracle.py by momentum conservation for plane-wave states (which fixes the
direction of G0), the Gamma-only reduction to chi0_bands, and Hermiticity / negative
semidefiniteness of the static sum.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .chi0 import weights


def kq_map(kpts: np.ndarray, q: Sequence[float], tol: float = 1e-8):
    """For each k of the set (fractional, reciprocal-lattice units): (index of k'', G0) with
    k + q = k'' + G0, G0 integer.  ValueError if k + q is not a set point modulo G."""
    kpts = np.asarray(kpts, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    idx = np.zeros(len(kpts), dtype=np.int64)
    g0 = np.zeros((len(kpts), 3), dtype=np.int64)
    for i, k in enumerate(kpts):
        found = False
        for j, kk in enumerate(kpts):
            d = k + q - kk
            if np.all(np.abs(d - np.round(d)) < tol):
                idx[i], g0[i], found = j, np.round(d).astype(np.int64), True
                break
        if not found:
            raise ValueError("k + q is not on the k-point set")
    return idx, g0


def pair_density_kq(coef_v_kk: np.ndarray, gw_kk: np.ndarray, coef_c_k: np.ndarray, gw_k: np.ndarray,
                    g0: Sequence[int], gvec_chi: np.ndarray) -> np.ndarray:
    """M_vc(k, q, G) = sum_{g' in sphere(k)} conj(c_{v,k''}(g' + G + G0)) c_{c,k}(g'), (nv, nc, ng)."""
    index = {tuple(int(x) for x in g): i for i, g in enumerate(gw_kk)}
    ext = np.concatenate([coef_v_kk, np.zeros((coef_v_kk.shape[0], 1), dtype=coef_v_kk.dtype)], axis=1)
    g0 = np.asarray(g0, dtype=np.int64)
    m = np.zeros((coef_v_kk.shape[0], coef_c_k.shape[0], len(gvec_chi)), dtype=np.complex128)
    for a, G in enumerate(gvec_chi):
        j = np.array([index.get(tuple(int(x) for x in (g + G + g0)), -1) for g in gw_k])
        m[:, :, a] = np.conj(ext[:, j]) @ coef_c_k.T
    return m


def chi0_ksum(coef_v: Sequence[np.ndarray], e_v: Sequence[np.ndarray], coef_c: Sequence[np.ndarray],
              e_c: Sequence[np.ndarray], gw: Sequence[np.ndarray], kpts: np.ndarray, q: Sequence[float],
              gvec_chi: np.ndarray, omegas: Sequence[float] = (0.0,), delta: float = 0.0,
              n_col: Optional[Sequence[np.ndarray]] = None) -> np.ndarray:
    """(nomega, ng, ng) chi0 of Eq. (chi0) summed over the k-point set; per k: coefficients
    (rows on that k's sphere gw[k]), energies, optional column weights."""
    idx, g0 = kq_map(kpts, q)
    ng = len(gvec_chi)
    out = np.zeros((len(omegas), ng, ng), dtype=np.complex128)
    for k in range(len(kpts)):
        kk = idx[k]
        m = pair_density_kq(coef_v[kk], gw[kk], coef_c[k], gw[k], g0[k], gvec_chi)
        n = None if n_col is None else n_col[k]
        for iw, om in enumerate(omegas):
            w = weights(e_v[kk], e_c[k], n, om, delta)                     # E_{v,k+q} - E_{c,k}
            mw = m * w[:, :, None]
            out[iw] += np.einsum("vcg,vch->gh", mw, np.conj(m))
    return out


def grad_chi0_ksum_energies(coef_v: Sequence[np.ndarray], e_v: Sequence[np.ndarray], coef_c: Sequence[np.ndarray],
                            e_c: Sequence[np.ndarray], gw: Sequence[np.ndarray], kpts: np.ndarray, q: Sequence[float],
                            gvec_chi: np.ndarray, chibar: np.ndarray, omegas: Sequence[float] = (0.0,),
                            delta: float = 0.0):
    """Per k-point term of the sum: (dL/dE_v of the states at k + q, dL/dE_c at k) for a real
    loss with chibar = dL/dRe chi0 + i dL/dIm chi0 of the summed chi0.  A term's valence
    gradient belongs to k'' = k + q - G0; adding the terms with the same k'' gives dL/dE_{v,k''}."""
    from .grad import grad_weights_dynamic
    idx, g0 = kq_map(kpts, q)
    gv, gcl = [], []
    for k in range(len(kpts)):
        kk = idx[k]
        m = pair_density_kq(coef_v[kk], gw[kk], coef_c[k], gw[k], g0[k], gvec_chi)
        x = e_v[kk][:, None] - e_c[k][None, :]
        gx = np.zeros_like(x)
        for iw, om in enumerate(omegas):
            s = np.einsum("vcg,gh,vch->vc", np.conj(m), chibar[iw], m)
            dwdx, _ = grad_weights_dynamic(x, np.ones_like(x), om, delta)
            gx += np.real(np.conj(s) * dwdx)
        gv.append(gx.sum(1))
        gcl.append(-gx.sum(0))
    return gv, gcl
