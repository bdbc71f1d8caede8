"""GPU parity of the wavefunction-coefficient gradients of gw_chi0_backward (float64)
against the oracle's adjoint (itself pinned by finite differences), and of the autograd
wrapper's coefficient gradients against central finite differences of the GPU loss."""
import numpy as np
import pytest

import synth
from oracle import grad as og
from cases import Gpu, make_case, many_valence_rows

pytestmark = pytest.mark.gpu
EV = synth.HARTREE_EV


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def rand_gbar(ng, nw, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal((nw, ng, ng)) + 1j * r.standard_normal((nw, ng, ng))


def grouped_columns(case, seed):
    """Columns that reuse coefficient rows (a window representative standing for several
    energies) and leave one row unused, with multiplicities n >= 1."""
    r = np.random.default_rng(seed)
    nb = len(case.e_c)
    col = np.concatenate([np.arange(nb), r.integers(0, nb, nb // 3)])
    col = col[col != nb // 2]
    case.col_band = col.astype(np.int32)
    case.e_col = case.e_c[col] + r.uniform(0.0, 0.02, len(col))
    case.n_col = r.uniform(1.0, 4.0, len(col))


def run(g, case, gbar, omegas, delta, prec="fp64", want=(True, True, True)):
    torch = g.torch
    prob = g.problem(case)
    out = g.p.gw_chi0_backward(g.ctx, [prob], omegas, delta, g.p.PRECISIONS[prec],
                               torch.from_numpy(np.ascontiguousarray(gbar)).to(g.dev), want=want,
                               coef=(True, True))
    torch.cuda.synchronize()
    return [None if x is None else x.cpu().numpy() for x in out]


def want_coef(case, gbar, omegas, delta):
    col, e_col, n_col = case.columns()
    return og.grad_chi0_coefficients(case.coef_v, case.e_v, case.coef_c, e_col, case.gw, case.gc,
                                     (case.nd,) * 3, gbar, omegas, delta, n_col=n_col, col_band=col)


def err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    # (config, nv, nc, ng override, omegas eV, delta eV, grouped)
    pytest.param(0, 6, 21, None, (0.0,), 0.0, False, id="24cube-static"),
    pytest.param(0, 6, 21, None, (0.0, 0.3, 9.0), 0.1, True, id="24cube-dynamic-grouped"),
    # 144 valence rows make the conduction chunk 224 columns: two chunks, so the valence
    # gradient is summed over chunks
    pytest.param(0, -144, 240, None, (0.0,), 0.0, False, id="24cube-two-chunks"),
    pytest.param(1, 4, 10, 300, (0.0, 0.5), 0.05, True, id="72cube"),
    # the pair kernels at 96^3 and 128^3 are built for dielectric spheres of half-width 8..13
    pytest.param(2, 4, 10, 2600, (0.0,), 0.0, False, id="96cube"),
    pytest.param(4, 4, 10, 6500, (0.5,), 0.05, False, id="128cube"),
]


@pytest.mark.parametrize("cfg,nv,nc,ng,omegas,delta,grouped", CASES)
def test_coefficient_gradients_match_oracle(g, cfg, nv, nc, ng, omegas, delta, grouped):
    if nv > 0:
        case = make_case(cfg, nv=nv, nc=nc, ng=ng)
    else:
        case = many_valence_rows(make_case(cfg, nc=nc, ng=ng), -nv)
        nv = -nv
    if grouped:
        grouped_columns(case, 11)
    om = np.asarray(omegas) / EV
    gbar = rand_gbar(len(case.gc), len(om), 5)
    got = run(g, case, gbar, om, delta / EV)
    gv, gc = want_coef(case, gbar, om, delta / EV)
    assert got[3].shape == (nv * len(case.gw),) and got[4].shape == (nc * len(case.gw),)
    ev, ec = err(got[3].reshape(gv.shape), gv), err(got[4].reshape(gc.shape), gc)
    assert ev <= 1e-10 and ec <= 1e-10, (ev, ec)
    if grouped:
        # the row no column refers to gets no gradient
        assert np.abs(got[4].reshape(gc.shape)[nc // 2]).max() == 0.0


def test_coefficient_gradients_without_energy_gradients(g):
    # only the coefficient gradients asked for: same values
    case = make_case(0, nv=5, nc=13)
    gbar = rand_gbar(len(case.gc), 1, 6)
    a = run(g, case, gbar, [0.0], 0.0)
    b = run(g, case, gbar, [0.0], 0.0, want=(False, False, False))
    assert b[0] is None and b[1] is None and b[2] is None
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])


def test_coefficient_gradients_need_fp64(g):
    import paper_1601_06767_amd as p
    case = make_case(0, nv=4, nc=8)
    gbar = rand_gbar(len(case.gc), 1, 7)
    for prec in ("fp32", "bf16x3"):
        with pytest.raises(p.GwError, match="float64"):
            run(g, case, gbar, [0.0], 0.0, prec)


def _loss(g, A, geom, cv, cc, ev, ec, v, hd):
    chi = A.chi0(g.ctx, geom, cv, ev, cc, ec)[0]
    z = A.eps_inv(g.ctx, chi, v)
    return z[hd, hd].real.sum()


def test_autograd_coefficient_gradients_match_finite_differences(g):
    import paper_1601_06767_amd.autograd as A
    torch = g.torch
    case = make_case(0, nv=8, nc=24)
    geom = A.geometry(g.ctx, (case.nd,) * 3, case.gw, case.gc)
    v = g.t(synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell))
    hd = torch.from_numpy(synth.loss_head_block(case.gc)).to(g.dev)
    ev, ec = g.t(case.e_v), g.t(case.e_c)
    cv = torch.from_numpy(case.coef_v.copy()).to(g.dev).requires_grad_(True)
    cc = torch.from_numpy(case.coef_c.copy()).to(g.dev).requires_grad_(True)
    _loss(g, A, geom, cv, cc, ev, ec, v, hd).backward()
    grads = {"v": cv.grad.cpu().numpy(), "c": cc.grad.cpu().numpy()}
    base = {"v": case.coef_v, "c": case.coef_c}
    # the largest coefficient of a few bands (where the loss moves most) and a small one
    picks = []
    for name, rows in (("v", (0, 7)), ("c", (0, 13, 23))):
        for r in rows:
            k = int(np.argmax(np.abs(base[name][r])))
            picks += [(name, r, k), (name, r, (k + 100) % base[name].shape[1])]
    h = 1e-5
    scale = max(np.abs(grads["v"]).max(), np.abs(grads["c"]).max())
    for name, r, k in picks:
        for unit in (1.0, 1j):
            vals = []
            for sgn in (1, -1):
                arr = {n: x.copy() for n, x in base.items()}
                arr[name][r, k] += sgn * h * unit
                with torch.no_grad():
                    vals.append(float(_loss(g, A, geom, torch.from_numpy(arr["v"]).to(g.dev),
                                            torch.from_numpy(arr["c"]).to(g.dev), ev, ec, v, hd)))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = grads[name][r, k].real if unit == 1.0 else grads[name][r, k].imag
            # the gradients here are ~1e-3 and the difference quotient's rounding ~1e-10
            assert abs(fd - an) <= 1e-6 * scale, (name, r, k, unit, fd, an, scale)
