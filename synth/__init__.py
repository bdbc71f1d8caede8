"""Seeded synthetic inputs shaped like the MgO supercells of the paper.

The paper's runs (Tables 1-3) use DFT-LDA wavefunctions of MgO supercells with
2-256 atoms.  Those are not available here, so every input is drawn from a
seeded generator with the same shapes: plane-wave coefficient sets on a
wavefunction G-sphere, valence energies below a gap, conduction energies with a
free-electron-like sqrt(E) density (the observation behind Eq. (chi02)),
dielectric G-spheres ordered by |q+G|, frequencies and the bare Coulomb
interaction v(q+G).

This module holds none of the method's arithmetic (no pair densities, weights,
grouping, sums or inversions).  It feeds both the CPU oracle and the GPU
library, which share nothing else.

Random streams: numpy ``PCG64(SeedSequence([160106767, cfg, stream, index]))``.
Streams: 0 = coefficients (index = band), 1 = valence energies, 2 = conduction
energies, 10+iq = valence coefficients of q-point iq > 0, 20+iq = their
energies, 30 = extra test draws.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SEED_ROOT = 160106767
HARTREE_EV = 27.211386245988


def rng(cfg: int, stream: int, index: int = 0) -> np.random.Generator:
    """Counter-style generator: one independent stream per (config, stream, index)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, stream, index])))


# --------------------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Config:
    """One workload.  Energies in eV here; generators return Hartree."""
    index: int
    name: str
    nd: int                      # FFT grid N_d (cubic N_d^3)
    nv: int                      # valence bands per q
    nc: int                      # conduction bands generated
    ng: List[int]                # dielectric-sphere size per q-point
    a_bohr: float                # simple-cubic lattice constant
    qs: List[Sequence[float]]    # q-points in reciprocal-lattice units
    omegas_ev: List[float]       # real frequencies (eV); [0.0] = static
    delta_ev: float              # broadening (eV)
    e0_ev: Optional[float]       # grouping threshold E_0 (eV); None = exact band sum
    de_ev: float                 # window width (eV)
    emax_ev: float               # top of the generated conduction spectrum (eV)
    precision: str               # contraction mode the workload is quoted in

    @property
    def wf_radius(self) -> int:
        return self.nd // 4

    @property
    def cell(self) -> np.ndarray:
        return np.eye(3) * self.a_bohr

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.cell)))


_Q0 = (0.01, 0.0, 0.0)
_BATCHED_QS = [_Q0, (0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5), (0.5, 0.5, 0.5)]
_BATCHED_NG = [800, 1114, 1429, 1743, 2057, 2371, 2686, 3000]


def _a_for_atoms(atoms: int) -> float:
    # rock-salt MgO, 8 atoms per conventional cube of 8.4 bohr (simple-cubic stand-in cell)
    return 8.4 * (atoms / 8.0) ** (1.0 / 3.0)


WORKLOADS = [
    Config(0, "static-24^3-16x240-ng259-fp64", 24, 16, 240, [259], 8.4, [_Q0], [0.0], 0.0, None, 1.0, 60.0, "fp64"),
    Config(1, "mgo64-static-72^3-128x4000-ng2000", 72, 128, 4000, [2000], _a_for_atoms(64), [_Q0], [0.0], 0.0,
           None, 1.0, 60.0, "fp64+fp32"),
    Config(2, "mgo128-grouped-96^3-256x16000-ng4000", 96, 256, 16000, [4000], _a_for_atoms(128), [_Q0], [0.0], 0.0,
           30.0, 1.0, 60.0, "bf16x3"),
    Config(3, "batched-8q-16w-72^3-128x6000", 72, 128, 6000, list(_BATCHED_NG), _a_for_atoms(64), list(_BATCHED_QS),
           [40.0 * j / 15.0 for j in range(16)], 0.1, None, 1.0, 60.0, "fp32"),
    Config(4, "mgo256-grouped-128^3-512x25000-ng8000", 128, 512, 25000, [8000], _a_for_atoms(256), [_Q0], [0.0],
           0.0, 30.0, 1.0, 60.0, "bf16x3"),
]


def config(i: int) -> Config:
    return dataclasses.replace(WORKLOADS[i])


# --------------------------------------------------------------------------------------
# G-spheres (Miller indices)
# --------------------------------------------------------------------------------------
def _box(r: int) -> np.ndarray:
    a = np.arange(-r, r + 1)
    g = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3)
    return g


def wf_sphere(nd: int, radius: Optional[int] = None) -> np.ndarray:
    """Wavefunction sphere |n| <= radius (default nd/4), ordered by (|n|^2, n1, n2, n3). int32 (npw, 3)."""
    r = nd // 4 if radius is None else radius
    g = _box(r)
    g = g[(g * g).sum(1) <= r * r]
    key = (g * g).sum(1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], key))
    return np.ascontiguousarray(g[order].astype(np.int32))


def wf_sphere_k(k: Sequence[float], radius: float) -> np.ndarray:
    """Wavefunction sphere of a k-point (fractional, simple cubic): Miller indices g with
    |k + g| <= radius, ordered by (|k + g|^2, n1, n2, n3). int32 (npw, 3)."""
    k = np.asarray(k, dtype=np.float64)
    g = _box(int(math.ceil(radius)) + 1)
    d = ((g + k) ** 2).sum(1)
    g, d = g[d <= radius * radius + 1e-9], d[d <= radius * radius + 1e-9]
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], d))
    return np.ascontiguousarray(g[order].astype(np.int32))


def kpoint_grid(n: int) -> np.ndarray:
    """Gamma-centred n x n x n grid of fractional k-points in [0, 1), (n^3, 3)."""
    f = np.arange(n) / n
    return np.array([(a, b, c) for a in f for b in f for c in f], dtype=np.float64)


@dataclasses.dataclass
class KBands:
    """Per k-point: sphere (npw_k, 3), valence / conduction coefficient rows on it, energies (Hartree)."""
    gw: List[np.ndarray]
    coef_v: List[np.ndarray]
    e_v: List[np.ndarray]
    coef_c: List[np.ndarray]
    e_c: List[np.ndarray]


def make_kbands(cfg_index: int, kpts: np.ndarray, radius: float, nv: int, nc: int,
                emax_ev: float = 60.0) -> KBands:
    """Orthonormal random bands per k-point (stream 40 + k for the coefficients, 60 + k for
    the energies): valence E uniform in [-10, 0] eV, conduction with density ~ sqrt(E) on
    [5, emax] eV, each sorted."""
    out = KBands([], [], [], [], [])
    for ik, k in enumerate(kpts):
        gw = wf_sphere_k(k, radius)
        q = orthonormalize(gaussian_columns(cfg_index, 40 + ik, range(nv + nc), gw.shape[0]))
        r = rng(cfg_index, 60 + ik)
        ev = np.sort(r.uniform(-10.0, 0.0, nv)) / HARTREE_EV
        u = r.uniform(0.0, 1.0, nc)
        ec = np.sort((5.0 ** 1.5 + u * (emax_ev ** 1.5 - 5.0 ** 1.5)) ** (2.0 / 3.0)) / HARTREE_EV
        out.gw.append(gw)
        out.coef_v.append(q[:nv])
        out.e_v.append(ev)
        out.coef_c.append(q[nv:])
        out.e_c.append(ec)
    return out


def density_box(half: int, cell: np.ndarray, n_electrons: float, width: float = 0.6) -> np.ndarray:
    """Synthetic valence density rho(G) on the Miller box |n_i| <= half (complex128,
    (2 half + 1)^3, index (n1 + half, n2 + half, n3 + half)): electrons per bohr^3, a smooth
    real density rho(G) = rho0 exp(-|G|^2 width^2 / 2) with rho(-G) = conj(rho(G)), plus a
    seeded small phase so the off-diagonal structure is not symmetric in G."""
    b = recip(cell)
    vol = abs(np.linalg.det(cell))
    rho0 = n_electrons / vol
    a = np.arange(-half, half + 1)
    n = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1)
    gg = ((n @ b) ** 2).sum(-1)
    phase = rng(0, 77).uniform(-0.3, 0.3, n.shape[:3])
    phase = 0.5 * (phase - phase[::-1, ::-1, ::-1])             # odd in G: rho(-G) = conj(rho(G))
    box = rho0 * np.exp(-0.5 * gg * width * width) * np.exp(1j * phase)
    box[half, half, half] = rho0
    return box


def recip(cell: np.ndarray) -> np.ndarray:
    """Reciprocal lattice vectors (rows), b_i . a_j = 2 pi delta_ij."""
    return 2.0 * math.pi * np.linalg.inv(cell).T


SHELL_TOL = 1e-12   # |q+G|^2 values within this relative distance are one shell


def chi_sphere(ng: int, q: Sequence[float], cell: np.ndarray) -> np.ndarray:
    """First ng Miller indices in the order (|q+G|^2, n1, n2, n3); int32 (ng, 3).

    Keys that agree to a relative SHELL_TOL are one shell (equal |q+G| computed in another
    summation order can differ in the last bit), ordered by the Miller indices."""
    q = np.asarray(q, dtype=np.float64)
    b = recip(cell)
    r = 1
    while True:
        g = _box(r)
        k = ((g + q) @ b)
        key = (k * k).sum(1)
        # every point of the box whose key is below the smallest key outside the box is final
        outside_min = ((r + 1 - np.abs(q).max()) * np.linalg.svd(b, compute_uv=False).min()) ** 2
        inside = key < outside_min
        if inside.sum() >= ng:
            by_key = np.argsort(key, kind="stable")
            ks = key[by_key]
            new_shell = np.concatenate([[True], ks[1:] - ks[:-1] > SHELL_TOL * np.maximum(ks[1:], ks[:-1])])
            shell = np.empty(len(key), dtype=np.int64)
            shell[by_key] = np.cumsum(new_shell)
            order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], shell))
            sel = order[:ng]
            if key[sel].max() < outside_min:
                return np.ascontiguousarray(g[sel].astype(np.int32))
        r += 1


def coulomb(gvec: np.ndarray, q: Sequence[float], cell: np.ndarray, prefactor: Optional[float] = None) -> np.ndarray:
    """Bare Coulomb interaction v(q+G) = f * 4 pi / |q+G|^2 (Hartree atomic units).

    f defaults to 2/Omega: spin degeneracy 2, one k-point, and the cell volume that
    a literal band sum leaves out."""
    b = recip(cell)
    k = (gvec.astype(np.float64) + np.asarray(q, dtype=np.float64)) @ b
    k2 = (k * k).sum(1)
    if prefactor is None:
        prefactor = 2.0 / abs(np.linalg.det(cell))
    return prefactor * 4.0 * math.pi / k2


# --------------------------------------------------------------------------------------
# energies
# --------------------------------------------------------------------------------------
def valence_energies(cfg: Config, iq: int = 0) -> np.ndarray:
    """E_v ~ U(-10, 0) eV, sorted ascending; Hartree."""
    stream = 1 if iq == 0 else 20 + iq
    e = np.sort(rng(cfg.index, stream).uniform(-10.0, 0.0, cfg.nv))
    return e / HARTREE_EV


def conduction_energies(cfg: Config, nc: Optional[int] = None) -> np.ndarray:
    """E_c with density ~ sqrt(E) on [5, emax] eV, sorted ascending; Hartree."""
    nc = cfg.nc if nc is None else nc
    u = rng(cfg.index, 2).uniform(0.0, 1.0, cfg.nc)[:nc]
    lo, hi = 5.0 ** 1.5, cfg.emax_ev ** 1.5
    e = np.sort((lo + u * (hi - lo)) ** (2.0 / 3.0))
    return e / HARTREE_EV


# --------------------------------------------------------------------------------------
# coefficients
# --------------------------------------------------------------------------------------
def gaussian_columns(cfg_index: int, stream: int, bands: Sequence[int], npw: int) -> np.ndarray:
    """Complex Gaussian rows (re, im ~ N(0, 1/2)), one independent draw per band index."""
    out = np.empty((len(bands), npw), dtype=np.complex128)
    for i, b in enumerate(bands):
        g = rng(cfg_index, stream, int(b))
        x = g.standard_normal(2 * npw).reshape(npw, 2) * math.sqrt(0.5)
        out[i] = x[:, 0] + 1j * x[:, 1]
    return out


def gaussian_columns_threaded(cfg_index: int, stream: int, bands: Sequence[int], npw: int,
                              workers: int = 16, out: Optional[np.ndarray] = None) -> np.ndarray:
    """gaussian_columns with the bands split over threads (each band keeps its own generator,
    so the rows are the same bits)."""
    from concurrent.futures import ThreadPoolExecutor
    bands = np.asarray(bands)
    if out is None:
        out = np.empty((len(bands), npw), dtype=np.complex128)
    step = max(1, -(-len(bands) // (4 * workers)))

    def job(k):
        out[k:k + step] = gaussian_columns(cfg_index, stream, bands[k:k + step], npw)
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(job, range(0, len(bands), step)))
    return out


def orthonormalize_on_device(rows: np.ndarray, device: str = "cuda"):
    """orthonormalize() run by torch on the GPU, the result left there (a torch tensor of rows):
    input preparation only, for workloads whose coefficient sets are only needed on the GPU."""
    import torch  # local: only used to speed up input preparation
    t = torch.from_numpy(rows).to(device).T
    q, r = torch.linalg.qr(t)
    del t
    d = torch.diagonal(r)
    q.mul_(torch.conj(d / d.abs())[None, :])
    del r
    return q.T.contiguous()


def orthonormalize(rows: np.ndarray, device: Optional[str] = None) -> np.ndarray:
    """Householder QR of the stacked rows (as columns), phases fixed so diag(R) > 0.

    With ``device`` set (e.g. "cuda"), torch's QR runs there: input preparation only."""
    a = rows.T
    if device is None:
        q, r = np.linalg.qr(a)
        d = np.diagonal(r)
    else:
        import torch  # local: only used to speed up input preparation
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device)
        qt, rt = torch.linalg.qr(t)
        d = torch.diagonal(rt).cpu().numpy()
        q = qt.cpu().numpy()
    ph = d / np.abs(d)
    q = q * np.conj(ph)[None, :]
    return np.ascontiguousarray(q.T)


@dataclasses.dataclass
class Bands:
    """Coefficient rows (band, npw) complex128 and energies (Hartree)."""
    coef_v: np.ndarray
    e_v: np.ndarray
    coef_c: np.ndarray
    e_c: np.ndarray
    v_index: np.ndarray
    c_index: np.ndarray


def make_bands(cfg: Config, v_index: Optional[Sequence[int]] = None, c_index: Optional[Sequence[int]] = None,
               gvec_wf: Optional[np.ndarray] = None, iq: int = 0, device: Optional[str] = None,
               e_c_all: Optional[np.ndarray] = None) -> Bands:
    """Orthonormal coefficient sets for the selected valence / conduction bands.

    Valence and conduction rows are stacked [valence | conduction] and
    orthonormalised together (iq = 0).  For iq > 0 the valence set is the one at
    k+q: its own draw (stream 10+iq), orthonormalised on its own.
    """
    if gvec_wf is None:
        gvec_wf = wf_sphere(cfg.nd)
    npw = gvec_wf.shape[0]
    v_index = np.arange(cfg.nv) if v_index is None else np.asarray(v_index)
    c_index = np.arange(cfg.nc) if c_index is None else np.asarray(c_index)
    ev_all = valence_energies(cfg, iq)
    ec_all = conduction_energies(cfg) if e_c_all is None else e_c_all
    if iq == 0:
        rows = np.concatenate([gaussian_columns(cfg.index, 0, v_index, npw),
                               gaussian_columns(cfg.index, 0, cfg.nv + c_index, npw)])
        q = orthonormalize(rows, device)
        cv, cc = q[: len(v_index)], q[len(v_index):]
    else:
        cv = orthonormalize(gaussian_columns(cfg.index, 10 + iq, v_index, npw), device)
        cc = orthonormalize(np.concatenate([gaussian_columns(cfg.index, 0, v_index, npw),
                                            gaussian_columns(cfg.index, 0, cfg.nv + c_index, npw)]),
                            device)[len(v_index):]
    return Bands(cv, ev_all[v_index], cc, ec_all[c_index], v_index, c_index)


def omegas(cfg: Config) -> np.ndarray:
    return np.asarray(cfg.omegas_ev) / HARTREE_EV


def delta(cfg: Config) -> float:
    return cfg.delta_ev / HARTREE_EV


def plane_wave_bands(gvec_wf: np.ndarray, picks: Sequence[int]) -> np.ndarray:
    """Unit coefficient rows e_{G_pick}: the plane-wave states of a free-electron gas."""
    out = np.zeros((len(picks), gvec_wf.shape[0]), dtype=np.complex128)
    for i, p in enumerate(picks):
        out[i, p] = 1.0
    return out


def loss_head_block(gvec_chi: np.ndarray) -> np.ndarray:
    """Indices of the 27 G with n in {-1,0,1}^3 (the 'head block' of eps^-1)."""
    m = np.all(np.abs(gvec_chi) <= 1, axis=1)
    return np.nonzero(m)[0]
