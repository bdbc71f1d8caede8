"""Oracle: the COH self-energy of Eq. (sigmach) (test infrastructure only).

Two forms.  sigma_coh_gpp evaluates Eq. (sigmach) with the plasmon-pole eps^-1(w) of the
model the paper uses (oracle/gpp.py): each element of [eps^r]^-1 - [eps^a]^-1 on E' > 0 is
-i pi (Omega^2 / wt) delta(E' - wt) as the broadening of the pole goes to zero, so the
E' integral leaves one pole term per element,

    <n|Sigma_COH(E)|n'> = 1/2 sum_{n''} w_{n''} sum_{G G'} M_{n n''}(G)
                          Omega^2_{GG'} / (wt_{GG'} (E - E_{n''} - wt_{GG'} + i delta)) v(G')
                          conj(M_{n' n''}(G')),

with the band energy E_{n''} in the denominator (for a window column its energy E_i, weight
w = g(E_i) dE_i of Eq. (energyintegration)).  wt is the principal square root of wt^2 (for a
complex wt^2 of an off-diagonal element the expression is taken as written, its analytic
continuation); elements without a pole (unscreened) or without pole weight (Omega^2 = 0) add
nothing.  Pinned in
tests/test_oracle.py by a quadrature of Eq. (sigmach)'s E' integral as printed, by its
E - E_{n''} -> 0 limit (the static form below) and by the homogeneous electron gas.

sigma_coh_static is the static limit.

With the energy denominator of Eq. (sigmach) taken as -E' (the static limit), the
frequency integral of the retarded-minus-advanced inverse dielectric function gives, by
the Kramers-Kronig relation, half the static [eps^-1 - 1]:

    <n|Sigma_COH|n'> = 1/2 sum_{n''} w_{n''} sum_{G G'} M_{n n''}(G) [eps^-1 - I]_{G G'} v(G')
                       conj(M_{n' n''}(G'))

with M the matrix element of Eq. (chi0) between state n and band n'' (q -> 0, Gamma only)
and w_{n''} = 1 for a band, or the weight g(E_i) dE_i of Eq. (energyintegration) for a
window representative (the paper applies the same energy integration to the COH sum).
The band energies do not enter this limit.  Pinned in tests/test_oracle.py by the
completeness relation (summed over a complete set of bands the pair-density sum becomes a
plane-wave convolution of the two states' coefficients), Hermiticity and negative
semidefiniteness for a static eps^-1.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from .chi0 import pair_density_fft, psi_real_space


def coh_kernel(eps_inv_mat: np.ndarray, vcoul: np.ndarray) -> np.ndarray:
    """A = [eps^-1 - I] diag(v): the screened-minus-bare interaction of the static COH term."""
    ng = eps_inv_mat.shape[0]
    return (eps_inv_mat - np.eye(ng)) * vcoul[None, :]


def sigma_coh_static(coef_n: np.ndarray, coef_cols: np.ndarray, gvec_wf: np.ndarray, gvec_chi: np.ndarray,
                     nd: Sequence[int], eps_inv_mat: np.ndarray, vcoul: np.ndarray,
                     n_col: Optional[np.ndarray] = None) -> np.ndarray:
    """(Ns, Ns) matrix <n|Sigma_COH|n'> for the states coef_n over the bands (columns) coef_cols
    with weights n_col (default 1)."""
    nd = tuple(int(x) for x in nd)
    w = np.ones(coef_cols.shape[0]) if n_col is None else np.asarray(n_col, dtype=np.float64)
    psi_n = psi_real_space(coef_n, gvec_wf, nd)
    psi_c = psi_real_space(coef_cols, gvec_wf, nd)
    m = pair_density_fft(psi_n, psi_c, gvec_chi)                  # (Ns, Nc, ng): M_{n n''}(G)
    a = coh_kernel(eps_inv_mat, vcoul)
    # 1/2 sum_{n''} w_{n''} sum_{G G'} M_{n n''}(G) A_{G G'} conj(M_{n' n''}(G')), as written
    return 0.5 * np.einsum("c,ncg,gh,pch->np", w, m, a, np.conj(m), optimize=True)


def sigma_coh_complete_set(coef_n: np.ndarray, gvec_wf: np.ndarray, gvec_chi: np.ndarray, eps_inv_mat: np.ndarray,
                           vcoul: np.ndarray) -> np.ndarray:
    """The same matrix summed over a complete orthonormal set of bands of the wavefunction
    sphere, written without any band: sum_{n''} M_{n n''}(G) conj(M_{n' n''}(G')) =
    sum_g conj(c_n(g + G)) c_{n'}(g + G') (g and g + G, g + G' in the sphere)."""
    index = {tuple(int(x) for x in g): i for i, g in enumerate(gvec_wf)}
    npw, ng = gvec_wf.shape[0], gvec_chi.shape[0]
    # shifted[G][g] = index of g + G in the sphere, or -1
    shifted = np.full((ng, npw), -1, dtype=np.int64)
    for a, G in enumerate(gvec_chi):
        for i, g in enumerate(gvec_wf):
            shifted[a, i] = index.get((int(g[0] + G[0]), int(g[1] + G[1]), int(g[2] + G[2])), -1)
    ext = np.concatenate([coef_n, np.zeros((coef_n.shape[0], 1), dtype=coef_n.dtype)], axis=1)
    cs = ext[:, shifted]                                          # (Ns, ng, npw): c_n(g + G)
    corr = np.einsum("ngk,phk->npgh", np.conj(cs), cs)            # sum_g conj(c_n(g+G)) c_n'(g+G')
    a = coh_kernel(eps_inv_mat, vcoul)
    return 0.5 * np.einsum("gh,npgh->np", a, corr)


def gpp_coh_kernel(om2: np.ndarray, wt2: np.ndarray, vcoul: np.ndarray, x: complex) -> np.ndarray:
    """A_GG'(x) = Omega^2_GG' v(G') / (wt_GG' (x - wt_GG')), x = E - E_{n''} + i delta; zero where
    the element has no pole (wt^2 = inf) or no pole weight (Omega^2 = 0)."""
    pole = np.isfinite(wt2) & (om2 != 0)
    wt = np.sqrt(wt2[pole].astype(np.complex128))                  # principal branch
    a = np.zeros(om2.shape, dtype=np.complex128)
    a[pole] = om2[pole] / (wt * (x - wt))
    return a * vcoul[None, :]


def sigma_coh_gpp(coef_n: np.ndarray, coef_cols: np.ndarray, e_cols: np.ndarray, gvec_wf: np.ndarray,
                  gvec_chi: np.ndarray, nd: Sequence[int], om2: np.ndarray, wt2: np.ndarray, vcoul: np.ndarray,
                  energies: Sequence[float], delta: float = 0.0, n_col: Optional[np.ndarray] = None) -> np.ndarray:
    """(nE, Ns, Ns): <n|Sigma_COH(E)|n'> of Eq. (sigmach) with the plasmon-pole model, at each E of
    energies, for the states coef_n over the columns coef_cols (energies e_cols, weights n_col)."""
    nd = tuple(int(x) for x in nd)
    w = np.ones(coef_cols.shape[0]) if n_col is None else np.asarray(n_col, dtype=np.float64)
    m = pair_density_fft(psi_real_space(coef_n, gvec_wf, nd), psi_real_space(coef_cols, gvec_wf, nd), gvec_chi)
    ns = m.shape[0]
    out = np.zeros((len(energies), ns, ns), dtype=np.complex128)
    for j, e in enumerate(energies):
        for c in range(m.shape[1]):
            a = gpp_coh_kernel(om2, wt2, vcoul, e - e_cols[c] + 1j * delta)
            out[j] += 0.5 * w[c] * (m[:, c, :] @ a @ np.conj(m[:, c, :]).T)
    return out
