"""Full-size parity for the 72^3 grid / 128 x 4000 bands / NG 2000 static workload, run
the way the benchmark runs it (all 512,000 pairs in one build call).  The oracle cannot
form the whole 2000 x 2000 matrix, but it can form any entries: it computes the pair
densities of all pairs at a few G by its plane-wave convolution (one GEMM per G over the
wavefunction sphere) and contracts them with its static weights (Eq. (chi0) at w = 0)."""
import numpy as np
import pytest

import oracle
import synth
from cases import Gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    cfg = synth.config(1)
    gw = synth.wf_sphere(cfg.nd)
    gc = synth.chi_sphere(cfg.ng[0], cfg.qs[0], cfg.cell)
    bands = synth.make_bands(cfg, gvec_wf=gw, device="cuda")
    # the head, a few low and high |q+G| entries of the sphere order, and the last one
    sample = np.array([0, 1, 2, 37, 500, 1234, len(gc) - 1])
    m = oracle.pair_density_direct(bands.coef_v, bands.coef_c, gw, gc[sample])
    w = oracle.weights_static(bands.e_v, bands.e_c)
    ref = oracle.chi0_from_pair_densities(m, w)
    return cfg, gw, gc, bands, sample, ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)])
def test_full_size_sampled_entries(gpu, full, prec, tol):
    cfg, gw, gc, bands, sample, ref = full
    g = Gpu()
    p = g.p
    geom = p.gw_geom_create(g.ctx, (cfg.nd,) * 3, gw, gc, cfg.cell, cfg.qs[0])
    prob = p.make_problem(geom, g.t(bands.coef_v), g.t(bands.e_v), g.t(bands.coef_c), g.t(bands.e_c))
    chi = p.gw_chi0_build(g.ctx, [prob], [len(gc)], [0.0], 0.0, p.PRECISIONS[prec])[0][0]
    g.torch.cuda.synchronize()
    got = chi.cpu().numpy()
    sub = got[np.ix_(sample, sample)]
    scale = np.abs(ref).max()
    err = np.abs(sub - ref).max() / scale
    assert err <= tol, (prec, err)
    # properties of the whole matrix: Hermitian, negative semidefinite (static weights < 0)
    herm = np.abs(got - got.conj().T).max() / np.abs(got).max()
    assert herm <= (1e-14 if prec == "fp64" else 1e-6), herm
    ev = np.linalg.eigvalsh(0.5 * (got + got.conj().T))
    assert ev.max() <= tol * np.abs(ev).max(), (ev.max(), np.abs(ev).max())
    p.gw_geom_destroy(geom)


@pytest.fixture(scope="module")
def grouped():
    # 96^3 grid, 256 valence bands, 16,000 conduction bands grouped above E0 = 30 eV into
    # 1 eV windows (Eq. (energyintegration)), NG 4000: only the explicit bands and the
    # window representatives need coefficients
    cfg = synth.config(2)
    gw = synth.wf_sphere(cfg.nd)
    gc = synth.chi_sphere(cfg.ng[0], cfg.qs[0], cfg.cell)
    e_all = synth.conduction_energies(cfg)
    ev = synth.HARTREE_EV
    nwin = int(round((cfg.emax_ev - cfg.e0_ev) / cfg.de_ev))
    col, e_col, n_col, n0 = oracle.group_windows(e_all, cfg.e0_ev / ev, cfg.de_ev / ev, nwin)
    bands = synth.make_bands(cfg, c_index=col, gvec_wf=gw, device="cuda")
    sample = np.array([0, 1, 5, 222, 1500, len(gc) - 1])
    m = oracle.pair_density_direct(bands.coef_v, bands.coef_c, gw, gc[sample])
    w = oracle.weights_static(bands.e_v, e_col, n_col)
    ref = oracle.chi0_from_pair_densities(m, w)
    return cfg, gw, gc, bands, e_col, n_col, n0, sample, ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 1e-4)])
def test_full_size_grouped_sampled_entries(gpu, grouped, prec, tol):
    cfg, gw, gc, bands, e_col, n_col, n0, sample, ref = grouped
    assert 0 < n0 < len(e_col) <= n0 + int(round((cfg.emax_ev - cfg.e0_ev) / cfg.de_ev))
    g = Gpu()
    p = g.p
    geom = p.gw_geom_create(g.ctx, (cfg.nd,) * 3, gw, gc, cfg.cell, cfg.qs[0])
    prob = p.make_problem(geom, g.t(bands.coef_v), g.t(bands.e_v), g.t(bands.coef_c), g.t(e_col), g.t(n_col))
    chi = p.gw_chi0_build(g.ctx, [prob], [len(gc)], [0.0], 0.0, p.PRECISIONS[prec])[0][0]
    g.torch.cuda.synchronize()
    sub = chi.cpu().numpy()[np.ix_(sample, sample)]
    err = np.abs(sub - ref).max() / np.abs(ref).max()
    assert err <= tol, (prec, err)
    p.gw_geom_destroy(geom)
