"""Oracle: RPA dielectric matrix and its inverse (test infrastructure only).

The paper relates the dielectric function to the polarizability by eps = 1 - v chi0
(RPA, in the text before Eq. (chi0)), uses W = eps^-1 v, and reports the macroscopic
dielectric constant eps_inf = lim_{q->0} 1/[eps^-1]_{00}(q, 0) (Table 3).  In a
plane-wave basis v is diagonal, v(q+G).

Reading: eps is taken as I - diag(v) chi0, unsymmetrised, exactly as written.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def eps_matrix(chi0: np.ndarray, vcoul: np.ndarray) -> np.ndarray:
    """eps_GG' = delta_GG' - v(q+G) chi0_GG'."""
    ng = chi0.shape[-1]
    return np.eye(ng) - vcoul[:, None] * chi0


def eps_inv(chi0: np.ndarray, vcoul: np.ndarray) -> np.ndarray:
    """[I - diag(v) chi0]^-1 by LAPACK LU."""
    return np.linalg.inv(eps_matrix(chi0, vcoul))


def eps_inv_static_cholesky(chi0: np.ndarray, vcoul: np.ndarray) -> np.ndarray:
    """Same inverse by a different route, valid for a Hermitian, negative semidefinite
    static chi0: eps~ = I - v^1/2 chi0 v^1/2 is Hermitian positive definite, so
    eps^-1 = v^1/2 (eps~)^-1 v^-1/2 with (eps~)^-1 from a Cholesky factorisation."""
    s = np.sqrt(vcoul)
    et = np.eye(len(s)) - s[:, None] * chi0 * s[None, :]
    c = sla.cho_factor(et, lower=True)
    inv_t = sla.cho_solve(c, np.eye(len(s), dtype=et.dtype))
    return s[:, None] * inv_t / s[None, :]


def eps_inf(eps_inv_mat: np.ndarray, head: int = 0) -> float:
    """Table 3's macroscopic constant 1/[eps^-1]_00 (head = index of G = 0)."""
    return float(1.0 / eps_inv_mat[head, head].real)
