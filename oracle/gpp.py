"""Oracle: the generalized plasmon-pole extension of the static eps^-1 to real frequencies
(test infrastructure only).

The paper extends its static dielectric matrices to finite frequency with the Hybertsen-Louie
generalized plasmon-pole model.  Restated from that model (Hartree atomic units, e = m = 1):
  Omega^2_{GG'} = w_p^2 [(q+G).(q+G') / |q+G|^2] rho(G - G') / rho(0),   w_p^2 = 4 pi rho(0)
  wt^2_{GG'}    = Omega^2_{GG'} / (delta_{GG'} - [eps^-1]_{GG'}(q, 0))
  [eps^-1]_{GG'}(q, w) = delta_{GG'} + Omega^2_{GG'} / ((w + i eta)^2 - wt^2_{GG'})
with rho(G) the Fourier coefficients of the valence electron density (electrons per unit
volume; rho(0) the mean density).  An element with delta_{GG'} - eps^-1_{GG'}(0) = 0 exactly
(unscreened) has no pole: it keeps its static value at every frequency.  By construction w = 0 gives back the static matrix, and
each element is a single pole whose weight satisfies the f-sum rule
  -(2/pi) int_0^inf w Im[eps^-1]_{GG'}(w) dw = Omega^2_{GG'}
(for real positive wt^2, eta -> 0).  Pinned in tests/test_oracle.py by those two properties
and by the homogeneous electron gas, where Omega^2 is diagonal and equal to w_p^2.
"""
from __future__ import annotations

from typing import Callable, Sequence

import numpy as np


def gpp_modes(eps_inv_static: np.ndarray, gvec_chi: np.ndarray, q: Sequence[float], bvec: np.ndarray,
              rho: Callable[[np.ndarray], complex], rho0: float):
    """(Omega^2, wt^2) as (ng, ng) complex arrays; rho(n) = rho(G) for a Miller-index vector n."""
    ng = len(gvec_chi)
    k = (np.asarray(gvec_chi, dtype=np.float64) + np.asarray(q, dtype=np.float64)) @ bvec   # q + G (1/bohr)
    wp2 = 4.0 * np.pi * rho0
    om2 = np.zeros((ng, ng), dtype=np.complex128)
    for a in range(ng):
        for b in range(ng):
            om2[a, b] = wp2 * (k[a] @ k[b]) / (k[a] @ k[a]) * rho(gvec_chi[a] - gvec_chi[b]) / rho0
    den = np.eye(ng) - eps_inv_static
    wt2 = np.full((ng, ng), np.inf + 0j)
    nz = den != 0
    wt2[nz] = om2[nz] / den[nz]          # an unscreened element (den = 0) has no pole
    return om2, wt2


def gpp_eps_inv(om2: np.ndarray, wt2: np.ndarray, omegas: Sequence[float], eta: float) -> np.ndarray:
    """[eps^-1](w) for each real w: (nomega, ng, ng)."""
    ng = om2.shape[0]
    out = np.zeros((len(omegas), ng, ng), dtype=np.complex128)
    pole = np.isfinite(wt2)
    for i, w in enumerate(omegas):
        z = (w + 1j * eta) ** 2
        out[i] = np.eye(ng)
        out[i][pole] += om2[pole] / (z - wt2[pole])
    return out
