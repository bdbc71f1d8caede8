"""GPU parity of the plasmon-pole extension (gw_gpp_eps_inv) against the oracle."""
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
def inputs():
    case = make_case(0)
    chi = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    v = synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell)
    z = oracle.eps_inv(chi, v)
    half = int((case.gc.max(0) - case.gc.min(0)).max())
    box = synth.density_box(half, case.cfg.cell, 2.0 * case.cfg.nv)
    return case, z, half, box


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_gpp_matches_oracle(g, inputs):
    case, z, half, box = inputs
    z = z.copy()
    z[7, 7] = 1.0                                     # one unscreened element: no pole
    b = synth.recip(case.cfg.cell)
    q = case.cfg.qs[0]
    om = np.array([0.0, 0.05, 0.3, 1.2])
    rho = lambda n: box[n[0] + half, n[1] + half, n[2] + half]
    om2, wt2 = oracle.gpp_modes(z, case.gc, q, b, rho, box[half, half, half].real)
    want = oracle.gpp_eps_inv(om2, wt2, om, 0.01)
    got, modes = g.p.gw_gpp_eps_inv(g.ctx, case.gc, q, b, g.t(box), g.t(z), om, 0.01, want_modes=True)
    got, modes = got.cpu().numpy(), modes.cpu().numpy()
    assert rel(got, want) <= 1e-12, rel(got, want)
    assert rel(modes[0], om2) <= 1e-13
    fin = np.isfinite(wt2)
    assert np.array_equal(np.isfinite(modes[1]), fin) and rel(modes[1][fin], wt2[fin]) <= 1e-12
    # static limit (no broadening): the pole form gives back eps^-1(0)
    e0 = g.p.gw_gpp_eps_inv(g.ctx, case.gc, q, b, g.t(box), g.t(z), [0.0], 0.0).cpu().numpy()[0]
    assert np.abs(e0 - z).max() <= 1e-12 * np.abs(z).max()


def test_gpp_argument_errors(g, inputs):
    case, z, half, box = inputs
    b = synth.recip(case.cfg.cell)
    small = synth.density_box(half - 1, case.cfg.cell, 2.0 * case.cfg.nv)
    with pytest.raises(g.p.GwError):
        g.p.gw_gpp_eps_inv(g.ctx, case.gc, case.cfg.qs[0], b, g.t(small), g.t(z), [0.1], 0.01)
    with pytest.raises(g.p.GwError):                  # q + G = 0 for G = 0 at q = 0
        g.p.gw_gpp_eps_inv(g.ctx, case.gc, (0.0, 0.0, 0.0), b, g.t(box), g.t(z), [0.1], 0.01)
