"""Oracle: the static limit of the COH self-energy of Eq. (sigmach) (test infrastructure only).

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
    z = np.conj(m) @ a.T                                          # z[n', n'', G] = sum_G' A_{GG'} conj(M_{n' n''}(G'))
    ns, nc, ng = m.shape
    x = (m * w[None, :, None]).reshape(ns, nc * ng)               # w_{n''} M_{n n''}(G), (n'', G) flattened
    return 0.5 * (x @ z.reshape(ns, nc * ng).T)


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
