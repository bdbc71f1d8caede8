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
