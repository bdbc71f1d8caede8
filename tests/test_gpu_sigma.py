"""GPU parity of the static COH self-energy (gw_sigma_coh_static) against the oracle,
with band columns, weighted window columns and several conduction chunks."""
import numpy as np
import pytest

import oracle
import synth
from cases import Gpu, make_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


@pytest.fixture(scope="module")
def screened():
    # a static eps^-1 from the oracle's chi0 of the 24^3 workload
    case = make_case(0)
    chi = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    v = synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell)
    return case, oracle.eps_inv(chi, v), v


def run(g, case, states, coef_cols, z, v, col=None, w=None):
    torch = g.torch
    p = g.p
    geom = g.geom(case)
    ncol = len(col) if col is not None else coef_cols.shape[0]
    e_dummy = np.zeros(max(ncol, states.shape[0]))
    prob = p.make_problem(geom, g.t(states), g.t(e_dummy[: states.shape[0]]), g.t(coef_cols),
                          g.t(e_dummy[:ncol]), None if w is None else g.t(w),
                          None if col is None else g.t(np.asarray(col, dtype=np.int32)))
    s = p.gw_sigma_coh_static(g.ctx, prob, g.t(v), g.t(z))
    torch.cuda.synchronize()
    return s.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_sigma_coh_all_bands_matches_oracle(g, screened):
    case, z, v = screened
    states = np.concatenate([case.coef_v[-3:], case.coef_c[:3]])        # band edges
    cols = np.concatenate([case.coef_v, case.coef_c])                   # every band
    got = run(g, case, states, cols, z, v)
    want = oracle.sigma_coh_static(states, cols, case.gw, case.gc, (case.nd,) * 3, z, v)
    assert rel(got, want) <= 1e-10, rel(got, want)
    assert np.abs(got - got.conj().T).max() <= 1e-12 * np.abs(got).max()
    assert np.linalg.eigvalsh(0.5 * (got + got.conj().T)).max() <= 0.0


def test_sigma_coh_weighted_columns_in_several_chunks(g, screened):
    # 8 states make a chunk of 4096 columns; 9000 columns reuse the 240 conduction rows
    # with window-like weights, so three chunks are summed
    case, z, v = screened
    r = np.random.default_rng(3)
    states = np.concatenate([case.coef_v[-4:], case.coef_c[:4]])
    col = r.integers(0, len(case.e_c), 9000)
    w = r.uniform(0.5, 4.0, 9000)
    got = run(g, case, states, case.coef_c, z, v, col=col, w=w)
    want = oracle.sigma_coh_static(states, case.coef_c[col], case.gw, case.gc, (case.nd,) * 3, z, v, n_col=w)
    assert rel(got, want) <= 1e-10, rel(got, want)


def test_sigma_coh_argument_errors(g, screened):
    case, z, v = screened
    p = g.p
    states = np.concatenate([case.coef_v, case.coef_c[:17]])            # 33 states: one too many
    with pytest.raises(p.GwError):
        run(g, case, states, case.coef_c, z, v)


# ---------------------------------------------------------------- plasmon-pole COH
@pytest.fixture(scope="module")
def gpp_modes(screened):
    # the oracle's plasmon-pole modes of the oracle's static eps^-1 (one unscreened element)
    case, z, v = screened
    z = z.copy()
    z[5, 5] = 1.0
    half = int((case.gc.max(0) - case.gc.min(0)).max())
    box = synth.density_box(half, case.cfg.cell, 2.0 * case.cfg.nv)
    rho = lambda n: box[n[0] + half, n[1] + half, n[2] + half]
    om2, wt2 = oracle.gpp_modes(z, case.gc, case.cfg.qs[0], synth.recip(case.cfg.cell), rho,
                                box[half, half, half].real)
    return z, om2, wt2


def run_gpp(g, problems):
    """problems: (case, states, coef_cols, e_cols, w or None, col or None, v, om2, wt2) per q."""
    p = g.p
    probs, vs, ms = [], [], []
    for case, states, cols, e_cols, w, col, v, om2, wt2 in problems:
        ncol = len(col) if col is not None else cols.shape[0]
        probs.append(p.make_problem(g.geom(case), g.t(states), g.t(np.zeros(states.shape[0])), g.t(cols),
                                    g.t(e_cols[:ncol]), None if w is None else g.t(w),
                                    None if col is None else g.t(np.asarray(col, dtype=np.int32))))
        vs.append(g.t(v))
        ms.append(g.t(np.concatenate([om2.reshape(-1), wt2.reshape(-1)])))
    return probs, vs, ms


@pytest.mark.parametrize("nstates,energies,delta", [(8, [-0.1, 0.05, 0.3], 0.0), (5, [0.2], 0.01),
                                                    (12, [-0.3, -0.2, 0.0, 0.1, 0.15, 0.2, 0.25, 0.3, 0.5], 0.004)],
                         ids=["8states-3E", "5states-1E", "12states-9E"])
def test_sigma_coh_gpp_matches_oracle(g, screened, gpp_modes, nstates, energies, delta):
    # every band (valence and conduction) as a column with its energy; states around the gap;
    # 12 states and 9 energies take two state blocks and two energy passes
    case, _, v = screened
    z, om2, wt2 = gpp_modes
    states = np.concatenate([case.coef_v[-(nstates // 2):], case.coef_c[:nstates - nstates // 2]])
    cols = np.concatenate([case.coef_v, case.coef_c])
    e_cols = np.concatenate([case.e_v, case.e_c])
    probs, vs, ms = run_gpp(g, [(case, states, cols, e_cols, None, None, v, om2, wt2)])
    got = g.p.gw_sigma_coh_gpp(g.ctx, probs, vs, ms, energies, delta).cpu().numpy()
    want = oracle.sigma_coh_gpp(states, cols, e_cols, case.gw, case.gc, (case.nd,) * 3, om2, wt2, v, energies, delta)
    assert got.shape == want.shape
    err = rel(got, want)
    print(f"{nstates} states, {len(energies)} energies: max|S - S_oracle| / max|S_oracle| = {err:.2e}")
    assert err <= 1e-10, err


def test_sigma_coh_gpp_grouped_columns_chunks_and_q_sum(g, screened, gpp_modes):
    # window columns (several on one band, weights g(E_i) dE_i) over 9000 columns (three chunks of
    # 4096), and a sum over two q-point problems (the second with its own modes and Coulomb
    # factors on the first 150 G-vectors, a smaller sphere)
    case, _, v = screened
    z, om2, wt2 = gpp_modes
    r = np.random.default_rng(5)
    states = np.concatenate([case.coef_v[-4:], case.coef_c[:4]])
    col = r.integers(0, len(case.e_c), 9000)
    w = r.uniform(0.5, 4.0, 9000)
    e_cols = case.e_c[col] + r.uniform(-0.01, 0.01, 9000)
    import dataclasses
    small = dataclasses.replace(case, gc=case.gc[:150])
    v2 = 0.7 * v[:150]
    om2b = 1.3 * om2[:150, :150]
    wt2b = np.where(np.isfinite(wt2[:150, :150]), 0.8 * np.where(np.isfinite(wt2), wt2, 0)[:150, :150],
                    wt2[:150, :150])
    col2 = col[:700]
    energies = [0.0, 0.25]
    probs, vs, ms = run_gpp(g, [(case, states, case.coef_c, e_cols, w, col, v, om2, wt2),
                                (small, states, case.coef_c, e_cols[:700], w[:700], col2, v2, om2b, wt2b)])
    got = g.p.gw_sigma_coh_gpp(g.ctx, probs, vs, ms, energies, 0.002).cpu().numpy()
    want = oracle.sigma_coh_gpp(states, case.coef_c[col], e_cols, case.gw, case.gc, (case.nd,) * 3, om2, wt2, v,
                                energies, 0.002, n_col=w)
    want += oracle.sigma_coh_gpp(states, case.coef_c[col2], e_cols[:700], case.gw, small.gc, (case.nd,) * 3, om2b,
                                 wt2b, v2, energies, 0.002, n_col=w[:700])
    err = rel(got, want)
    print(f"grouped, 3 chunks, 2 q: {err:.2e}")
    assert err <= 1e-10, err


def test_sigma_coh_gpp_zero_energy_transfer_is_the_static_gpu_result(g, screened, gpp_modes):
    # every column at the evaluation energy, no broadening: the GPU's plasmon-pole form equals
    # the GPU's static form (same pair densities, different kernels)
    case, _, v = screened
    z, om2, wt2 = gpp_modes
    states = np.concatenate([case.coef_v[-2:], case.coef_c[:2]])
    e = 0.123
    probs, vs, ms = run_gpp(g, [(case, states, case.coef_c, np.full(len(case.e_c), e), None, None, v, om2, wt2)])
    got = g.p.gw_sigma_coh_gpp(g.ctx, probs, vs, ms, [e], 0.0).cpu().numpy()[0]
    stat = run(g, case, states, case.coef_c, z, v)
    assert rel(got, stat) <= 1e-11, rel(got, stat)
