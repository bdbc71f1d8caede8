"""Oracle: pair densities and the polarizability band sum (test infrastructure only).

Paper passages (arXiv:1601.06767):
  * Eq. (chi0): chi0_GG'(q,w) = 1/2 sum_{c,v,k} M_vc(k,q,G) M*_vc(k,q,G')
    [1/(E_v,k+q - E_c,k - w + i delta) + 1/(E_v,k+q - E_c,k + w + i delta)],
    with M_vc(k,q,G) = <v,k+q| exp(i(q+G).r) |c,k>.
  * Eq. (chi02): static chi0 split into an explicit sum over c <= N_0 and an
    integral over E' > E_0 weighted by the DOS g(E') = Omega/pi^2 sqrt(2(E'-V_xc(0))).
  * Eq. (energyintegration): that integral as sum_i sum_v M_vEi M*_vEi /(E_v - E_i) g(E_i) dE_i.
  * Tables 1-2: the speed-up of the method is the band count ratio N_c/(N_0+N_E).

Readings (the paper is silent or garbled here):
  * The matrix element is printed exp(i(q+G)) without ".r"; read as exp(i(q+G).r).
    With Bloch states u_nk the phases cancel, so
    M_vc(G) = (1/N) sum_r conj(u_v(r)) u_c(r) exp(iG.r) on an N-point grid
            = sum_G' conj(c_v(G'+G)) c_c(G')   (exact when the grid is alias-free).
    The caller passes the valence set at k+q explicitly.
  * Eq. (chi0) is evaluated literally: prefactor 1/2, no spin factor, no 1/(N_k Omega);
    those constants belong to the Coulomb interaction that multiplies chi0.
  * Both terms carry +i delta, as printed.
  * Only one k-point (Gamma) is summed.
  * Window grouping: windows [E_0 + i dE, E_0 + (i+1) dE), the last one closed at its top;
    a band exactly at E_0 is explicit; the representative state of window i is the band
    nearest its midpoint E_i = E_0 + (i+1/2) dE (lower index on a tie); empty windows are
    dropped.  Weight g(E_i) dE_i is either the number of bands in the window ("count",
    exact for a DOS that is constant over a window) or A sqrt(E_i - V0) dE ("dos").
"""
from __future__ import annotations

import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft


def _workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def alias_free(gvec_wf: np.ndarray, gvec_chi: np.ndarray, nd: Sequence[int]) -> bool:
    """True when every product coefficient landing on a chi-sphere G is unaliased.

    conj(u_v) u_c has components G_c - G_v with |n_i| <= 2 R_wf,i; the grid folds
    G + m N_d onto G, so G in the chi sphere is clean when 2 R_wf,i + R_chi,i < N_d,i."""
    rw = np.abs(gvec_wf).max(0)
    rc = np.abs(gvec_chi).max(0)
    return bool(np.all(2 * rw + rc < np.asarray(nd)))


def box_map(gvec: np.ndarray, nd: Sequence[int]) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Grid indices n mod N_d of Miller indices."""
    nd = np.asarray(nd)
    m = np.mod(gvec, nd[None, :])
    return m[:, 0], m[:, 1], m[:, 2]


def psi_real_space(coef: np.ndarray, gvec_wf: np.ndarray, nd: Sequence[int]) -> np.ndarray:
    """u_n(r) = sum_G c_n(G) exp(iG.r) on the grid (unnormalised; (1/N) sum_r |u|^2 = sum_G |c|^2).

    Input to Eq. (chi0)'s matrix element.  coef: (nb, npw) -> (nb, N1, N2, N3)."""
    nd = tuple(int(x) for x in nd)
    i1, i2, i3 = box_map(gvec_wf, nd)
    box = np.zeros((coef.shape[0],) + nd, dtype=np.complex128)
    box[:, i1, i2, i3] = coef
    n = nd[0] * nd[1] * nd[2]
    # scipy's inverse FFT is sum_k X_k exp(+2 pi i k x / N) / N
    return sfft.ifftn(box, axes=(1, 2, 3), workers=_workers()) * n


def pair_density_fft(psi_v: np.ndarray, psi_c: np.ndarray, gvec_chi: np.ndarray) -> np.ndarray:
    """M_vc(G) = (1/N) sum_r conj(u_v(r)) u_c(r) exp(iG.r), Eq. (chi0) matrix element.

    psi_v: (nv, grid), psi_c: (nc, grid) -> (nv, nc, ng)."""
    nd = psi_v.shape[1:]
    i1, i2, i3 = box_map(gvec_chi, nd)
    out = np.empty((psi_v.shape[0], psi_c.shape[0], gvec_chi.shape[0]), dtype=np.complex128)
    for v in range(psi_v.shape[0]):
        prod = np.conj(psi_v[v])[None] * psi_c
        f = sfft.ifftn(prod, axes=(1, 2, 3), workers=_workers())
        out[v] = f[:, i1, i2, i3]
    return out


def pair_density_direct(coef_v: np.ndarray, coef_c: np.ndarray, gvec_wf: np.ndarray,
                        gvec_chi: np.ndarray) -> np.ndarray:
    """M_vc(G) = sum_G' conj(c_v(G'+G)) c_c(G'): the matrix element as a plane-wave
    convolution, with no grid at all.  Brute force; small inputs only."""
    index = {tuple(g): i for i, g in enumerate(gvec_wf.tolist())}
    out = np.zeros((coef_v.shape[0], coef_c.shape[0], gvec_chi.shape[0]), dtype=np.complex128)
    for ig, g in enumerate(gvec_chi.tolist()):
        src, dst = [], []
        for j, gp in enumerate(gvec_wf.tolist()):
            k = index.get((gp[0] + g[0], gp[1] + g[1], gp[2] + g[2]))
            if k is not None:
                src.append(k)
                dst.append(j)
        if src:
            out[:, :, ig] = np.conj(coef_v[:, src]) @ coef_c[:, dst].T
    return out


def weights(e_v: np.ndarray, e_col: np.ndarray, n_col: Optional[np.ndarray], omega: float,
            delta: float) -> np.ndarray:
    """Energy factor of Eq. (chi0) per pair, times the column multiplicity:
    w_vc = n_c * 1/2 [1/(E_v - E_c - w + i delta) + 1/(E_v - E_c + w + i delta)].  (nv, nc) complex."""
    n = np.ones_like(e_col) if n_col is None else n_col
    x = e_v[:, None] - e_col[None, :]
    return n[None, :] * 0.5 * (1.0 / (x - omega + 1j * delta) + 1.0 / (x + omega + 1j * delta))


def weights_static(e_v: np.ndarray, e_col: np.ndarray, n_col: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. (chi0) at w = 0, delta = 0: the two terms coincide and w_vc = n_c/(E_v - E_c)
    (the form printed in Eq. (chi02)).  (nv, nc) real."""
    n = np.ones_like(e_col) if n_col is None else n_col
    x = e_v[:, None] - e_col[None, :]
    return 0.5 * n[None, :] * (1.0 / x + 1.0 / x)


def chi0_from_pair_densities(m: np.ndarray, w: np.ndarray) -> np.ndarray:
    """chi0_GG' = sum_{v,c} w_vc M_vc(G) conj(M_vc(G')), Eq. (chi0). m: (nv, nc, ng), w: (nv, nc)."""
    ng = m.shape[-1]
    mm = m.reshape(-1, ng)
    ww = w.reshape(-1)
    return (mm.T * ww[None, :]) @ np.conj(mm)


def chi0_bands(coef_v: np.ndarray, e_v: np.ndarray, coef_c: np.ndarray, e_col: np.ndarray,
               gvec_wf: np.ndarray, gvec_chi: np.ndarray, nd: Sequence[int],
               omegas: Sequence[float] = (0.0,), delta: float = 0.0, n_col: Optional[np.ndarray] = None,
               col_band: Optional[np.ndarray] = None, c_chunk: int = 64) -> np.ndarray:
    """Eq. (chi0) on explicit columns: (nomega, ng, ng) complex128.

    Column j uses coefficient row col_band[j] (identity if None), energy e_col[j] and
    multiplicity n_col[j] (1 if None).  Conduction columns are processed in chunks to
    bound memory; the sum itself is the plain band sum."""
    if not alias_free(gvec_wf, gvec_chi, nd):
        raise ValueError("grid is not alias-free for these spheres")
    if col_band is None:
        col_band = np.arange(coef_c.shape[0])
    n = np.ones(len(col_band)) if n_col is None else np.asarray(n_col, dtype=np.float64)
    ng = gvec_chi.shape[0]
    psi_v = psi_real_space(coef_v, gvec_wf, nd)
    out = np.zeros((len(omegas), ng, ng), dtype=np.complex128)
    for c0 in range(0, len(col_band), c_chunk):
        cols = np.arange(c0, min(c0 + c_chunk, len(col_band)))
        psi_c = psi_real_space(coef_c[col_band[cols]], gvec_wf, nd)
        m = pair_density_fft(psi_v, psi_c, gvec_chi)
        for iw, om in enumerate(omegas):
            w = weights(e_v, e_col[cols], n[cols], om, delta)
            out[iw] += chi0_from_pair_densities(m, w)
    return out


def chi0_grouped_static(coef_v: np.ndarray, e_v: np.ndarray, coef_c: np.ndarray, e_c: np.ndarray,
                        gvec_wf: np.ndarray, gvec_chi: np.ndarray, nd: Sequence[int], e0: float,
                        de: float, nwin: int, mode: str = "count", dos_a: float = 0.0,
                        dos_v0: float = 0.0) -> np.ndarray:
    """Eqs. (chi02) + (energyintegration): explicit sum over bands with E_c <= E_0, plus
    sum_i sum_v M_vEi M*_vEi/(E_v - E_i) g(E_i) dE_i over the windows.  (ng, ng)."""
    col_band, e_col, n_col, n0 = group_windows(e_c, e0, de, nwin, mode, dos_a, dos_v0)
    explicit = chi0_bands(coef_v, e_v, coef_c[:n0], e_c[:n0], gvec_wf, gvec_chi, nd)[0] if n0 else 0.0
    ng = gvec_chi.shape[0]
    integral = np.zeros((ng, ng), dtype=np.complex128)
    if len(col_band) > n0:
        psi_v = psi_real_space(coef_v, gvec_wf, nd)
        reps = col_band[n0:]
        psi_e = psi_real_space(coef_c[reps], gvec_wf, nd)
        m = pair_density_fft(psi_v, psi_e, gvec_chi)           # M_vEi
        g_de = n_col[n0:]                                       # g(E_i) dE_i
        w = g_de[None, :] / (e_v[:, None] - e_col[n0:][None, :])
        integral = chi0_from_pair_densities(m, w)
    return explicit + integral


def free_electron_dos(e: np.ndarray, volume: float, v0: float = 0.0) -> np.ndarray:
    """g(E) = Omega/pi^2 sqrt(2(E - V_xc(0))), the free-electron DOS of Eq. (chi02) (both spins,
    Hartree atomic units); zero below V_xc(0)."""
    x = np.maximum(np.asarray(e, dtype=np.float64) - v0, 0.0)
    return volume / math.pi ** 2 * np.sqrt(2.0 * x)


def group_windows(e_c: np.ndarray, e0: float, de: float, nwin: int, mode: str = "count",
                  dos_a: float = 0.0, dos_v0: float = 0.0):
    """Columns of Eq. (energyintegration) from a sorted or unsorted conduction spectrum.

    Returns (col_band, e_col, n_col, n0): the explicit bands (E_c <= E_0, in index order,
    multiplicity 1), then one column per non-empty window: its representative band, its
    energy E_i (the window midpoint) and its weight g(E_i) dE (band count, or
    dos_a * sqrt(E_i - dos_v0) * dE)."""
    e_c = np.asarray(e_c, dtype=np.float64)
    top = e0 + nwin * de
    explicit = [i for i in range(len(e_c)) if e_c[i] <= e0]
    members = [[] for _ in range(nwin)]
    for i in range(len(e_c)):
        e = e_c[i]
        if e <= e0:
            continue
        k = int(math.floor((e - e0) / de))
        if k >= nwin:
            if e <= top:
                k = nwin - 1
            else:
                raise ValueError("band energy above the last window")
        members[k].append(i)
    col_band = list(explicit)
    e_col = [float(e_c[i]) for i in explicit]
    n_col = [1.0] * len(explicit)
    for k in range(nwin):
        if not members[k]:
            continue
        mid = e0 + (k + 0.5) * de
        best = min(members[k], key=lambda i: (abs(e_c[i] - mid), i))
        col_band.append(best)
        e_col.append(mid)
        if mode == "count":
            n_col.append(float(len(members[k])))
        elif mode == "dos":
            n_col.append(dos_a * math.sqrt(max(mid - dos_v0, 0.0)) * de)
        else:
            raise ValueError(mode)
    return (np.asarray(col_band, dtype=np.int64), np.asarray(e_col), np.asarray(n_col), len(explicit))


def group_edges(e_c: np.ndarray, edges: np.ndarray, mode: str = "count", rule: str = "midpoint",
                dos_a: float = 0.0, dos_v0: float = 0.0):
    """Columns of Eq. (energyintegration) on an arbitrary (uniform or non-uniform) energy grid.

    Window k is [edges[k], edges[k+1]) (the last one closed); bands at or below edges[0]
    (= E_0) are explicit columns.  Each window with at least one band gets integration
    nodes: rule "midpoint" one node at the window centre, rule "gauss2" the two
    Gauss-Legendre nodes centre -+ dE / (2 sqrt 3) (the higher-order rule the paper allows).
    A node's column is (the window's band nearest the node, lower index on a tie; the node
    energy; its weight).  Weights: mode "count" = the number of bands in the window (midpoint
    rule only: a count is exact, a quadrature rule does not apply to it); mode "dos" = the
    quadrature weight times g(E) = dos_a sqrt(E - dos_v0): dE for the midpoint, dE / 2 per
    Gauss node.  Returns (col_band, e_col, n_col, n0) like group_windows."""
    e_c = np.asarray(e_c, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.float64)
    nwin = len(edges) - 1
    if nwin < 0 or np.any(np.diff(edges) <= 0.0):
        raise ValueError("edges must increase strictly")
    if rule not in ("midpoint", "gauss2") or mode not in ("count", "dos"):
        raise ValueError((mode, rule))
    if rule == "gauss2" and mode == "count":
        raise ValueError("the two-point rule needs density weights")
    explicit = [i for i in range(len(e_c)) if e_c[i] <= edges[0]]
    members = [[] for _ in range(nwin)]
    for i in range(len(e_c)):
        e = e_c[i]
        if e <= edges[0]:
            continue
        if nwin == 0 or e > edges[-1]:
            raise ValueError("band energy above the last window")
        k = nwin - 1
        for j in range(nwin):
            if edges[j] < e < edges[j + 1] or (e == edges[j] and j > 0):
                k = j
                break
        members[k].append(i)
    col_band = list(explicit)
    e_col = [float(e_c[i]) for i in explicit]
    n_col = [1.0] * len(explicit)
    for k in range(nwin):
        if not members[k]:
            continue
        lo, hi = edges[k], edges[k + 1]
        de = hi - lo
        mid = 0.5 * (lo + hi)
        if rule == "midpoint":
            nodes = [(mid, de)]
        else:
            off = de / (2.0 * math.sqrt(3.0))
            nodes = [(mid - off, 0.5 * de), (mid + off, 0.5 * de)]
        for x, wq in nodes:
            best = min(members[k], key=lambda i: (abs(e_c[i] - x), i))
            col_band.append(best)
            e_col.append(x)
            if mode == "count":
                n_col.append(float(len(members[k])))
            else:
                n_col.append(dos_a * math.sqrt(max(x - dos_v0, 0.0)) * wq)
    return (np.asarray(col_band, dtype=np.int64), np.asarray(e_col), np.asarray(n_col), len(explicit))


def speedup_factor(n_c: float, n_0_plus_n_e: float) -> float:
    """Tables 1-2: speed-up of the method = conventional band count / (N_0 + N_E)."""
    return n_c / n_0_plus_n_e
