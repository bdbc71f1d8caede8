"""GPU parity of the adjoint (gw_chi0_backward, gw_eps_inv_backward and the autograd
wrappers) against the oracle's closed-form gradients and central finite differences."""
import numpy as np
import pytest

import oracle
import synth
from oracle import grad as og
from cases import Gpu, make_case

pytestmark = pytest.mark.gpu
EV = synth.HARTREE_EV


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def rand_gbar(ng, nw, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal((nw, ng, ng)) + 1j * r.standard_normal((nw, ng, ng))


def gpu_backward(g, case, gbar, omegas, delta, prec="fp64"):
    torch = g.torch
    prob = g.problem(case)
    out = g.p.gw_chi0_backward(g.ctx, [prob], omegas, delta, g.p.PRECISIONS[prec],
                               torch.from_numpy(np.ascontiguousarray(gbar)).to(g.dev))
    return [x.cpu().numpy() for x in out]


def ref_backward(case, gbar, omegas, delta):
    col, e_col, n_col = case.columns()
    return og.grad_chi0_energies(case.coef_v, case.e_v, case.coef_c, e_col, case.gw, case.gc, (case.nd,) * 3, gbar,
                                 omegas, delta, n_col=n_col, col_band=col)


def close(a, b, tol):
    return np.abs(a - b).max() <= tol * max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("omegas,delta", [((0.0,), 0.0), ((0.0, 0.3, 9.0), 0.1)])
def test_backward_matches_oracle_fp64(g, omegas, delta):
    case = make_case(0, nv=6, nc=21)
    case.e_col = case.e_c.copy()
    case.n_col = np.random.default_rng(1).uniform(0.5, 3.0, len(case.e_c))
    case.col_band = np.arange(len(case.e_c))
    om = np.asarray(omegas) / EV
    gbar = rand_gbar(len(case.gc), len(om), 3)
    got = gpu_backward(g, case, gbar, om, delta / EV)
    want = ref_backward(case, gbar, om, delta / EV)
    for a, b in zip(got, want):
        assert close(a, b, 1e-10)


def test_backward_fp32_and_bf16x3_modes(g):
    case = make_case(0, nv=8, nc=40)
    gbar = rand_gbar(len(case.gc), 1, 4)
    want = ref_backward(case, gbar, [0.0], 0.0)
    for prec in ("fp32", "bf16x3"):
        got = gpu_backward(g, case, gbar, [0.0], 0.0, prec)
        for a, b in zip(got, want):
            assert close(a, b, 1e-5), prec


@pytest.mark.parametrize("cfg,nv,nc,ng", [(0, 6, 21, None), (1, 8, 40, 300)], ids=["24cube", "72cube"])
def test_backward_mixed_modes_dynamic(g, cfg, nv, nc, ng):
    # frequencies with broadening and grouped columns, in float32 and on the split-bf16
    # adjoint kernel (128 x 128 tiles: the 72^3 sphere of 300 G spans three G tiles with a
    # ragged last one)
    case = make_case(cfg, nv=nv, nc=nc, ng=ng)
    r = np.random.default_rng(8)
    case.col_band = np.concatenate([np.arange(nc), r.integers(0, nc, nc // 3)]).astype(np.int32)
    case.e_col = case.e_c[case.col_band] + r.uniform(0.0, 0.02, len(case.col_band))
    case.n_col = r.uniform(1.0, 4.0, len(case.col_band))
    om = np.array([0.0, 0.3, 9.0]) / EV
    gbar = rand_gbar(len(case.gc), len(om), 9)
    want = ref_backward(case, gbar, om, 0.1 / EV)
    for prec in ("fp32", "bf16x3"):
        got = gpu_backward(g, case, gbar, om, 0.1 / EV, prec)
        for a, b in zip(got, want):
            assert close(a, b, 1e-5), prec


def _loss_gpu(g, geom, tensors, e_v, e_col, n_col, v, head, prec="fp64"):
    import paper_1601_06767_amd.autograd as A
    chi = A.chi0(g.ctx, geom, tensors[0], e_v, tensors[1], e_col, n_col, prec=prec)[0]
    z = A.eps_inv(g.ctx, chi, v)
    return z[head, head].real.sum()


def _fd_check(g, case, head, n_col, comps, h, tol, mixed=()):
    """dL/d(E_v, E_col, n_col) from the autograd chain against central finite differences of the
    float64 loss, fourth order (Richardson: (4 D(h) - D(2h)) / 3, so that the step can stay large
    beside the rounding noise of L), on the listed components.  The error is relative to the
    largest tested component: max |fd - g| <= tol * max |g|.  mixed: (precision, tolerance)
    pairs whose gradients are checked against the same differences at their own tolerance."""
    import paper_1601_06767_amd.autograd as A
    torch = g.torch
    geom = A.geometry(g.ctx, (case.nd,) * 3, case.gw, case.gc, case.cfg.cell, case.cfg.qs[0])
    tens = (g.t(case.coef_v), g.t(case.coef_c))
    v = g.t(synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell))
    hd = torch.from_numpy(head).to(g.dev)
    base = {"ev": case.e_v, "ec": case.e_c, "n": n_col}

    def grads(prec):
        ev = torch.from_numpy(case.e_v.copy()).to(g.dev).requires_grad_(True)
        ec = torch.from_numpy(case.e_c.copy()).to(g.dev).requires_grad_(True)
        nc = torch.from_numpy(n_col.copy()).to(g.dev).requires_grad_(True)
        _loss_gpu(g, geom, tens, ev, ec, nc, v, hd, prec).backward()
        out = {"ev": ev.grad.cpu().numpy(), "ec": ec.grad.cpu().numpy(), "n": nc.grad.cpu().numpy()}
        return np.array([out[name][i] for name, i in comps])

    def loss_at(name, i, step):
        arrs = {k: x.copy() for k, x in base.items()}
        arrs[name][i] += step
        with torch.no_grad():
            return float(_loss_gpu(g, geom, tens, torch.from_numpy(arrs["ev"]).to(g.dev),
                                   torch.from_numpy(arrs["ec"]).to(g.dev), torch.from_numpy(arrs["n"]).to(g.dev),
                                   v, hd))

    fd = []
    for name, i in comps:
        d1 = (loss_at(name, i, h) - loss_at(name, i, -h)) / (2 * h)
        d2 = (loss_at(name, i, 2 * h) - loss_at(name, i, -2 * h)) / (4 * h)
        fd.append((4.0 * d1 - d2) / 3.0)
    fd = np.array(fd)
    errs = {}
    for prec, t in (("fp64", tol),) + tuple(mixed):
        an = grads(prec)
        scale = np.abs(an).max()
        errs[prec] = float(np.abs(fd - an).max() / scale)
        print(f"{prec}: max|fd - g| / max|g| = {errs[prec]:.2e} over {len(comps)} components "
              f"(max|g| = {scale:.2e}; tolerance {t:g})")
        assert errs[prec] <= t, (prec, errs[prec], fd, an)
    return errs


def test_autograd_chain_matches_finite_differences_c1(g):
    case = make_case(0, nv=8, nc=24)
    head = synth.loss_head_block(case.gc)
    n_col = np.random.default_rng(2).uniform(0.5, 2.0, len(case.e_c))
    comps = [("ev", 0), ("ev", 7), ("ec", 0), ("ec", 11), ("ec", 23), ("n", 3), ("n", 20)]
    _fd_check(g, case, head, n_col, comps, 1e-3, 1e-6)


def test_autograd_chain_matches_oracle_gradients(g):
    # same chain through the oracle: eps^-1 adjoint then the band-sum adjoint
    import paper_1601_06767_amd.autograd as A
    torch = g.torch
    case = make_case(0, nv=5, nc=17)
    head = synth.loss_head_block(case.gc)
    v = synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell)
    chi = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    z = oracle.eps_inv(chi, v)
    gchi = og.grad_eps_inv(z, v, og.head_block_loss_grad(len(v), head))
    want = og.grad_chi0_energies(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3,
                                 gchi[None])
    geom = A.geometry(g.ctx, (case.nd,) * 3, case.gw, case.gc)
    ev = torch.from_numpy(case.e_v.copy()).to(g.dev).requires_grad_(True)
    ec = torch.from_numpy(case.e_c.copy()).to(g.dev).requires_grad_(True)
    loss = _loss_gpu(g, geom, (g.t(case.coef_v), g.t(case.coef_c)), ev, ec, None, g.t(v),
                     torch.from_numpy(head).to(g.dev))
    loss.backward()
    assert close(ev.grad.cpu().numpy(), want[0], 1e-9)
    assert close(ec.grad.cpu().numpy(), want[1], 1e-9)


def test_adjoint_grouped_128_grid_ng8000_finite_differences(g):
    # 256-atom-shaped geometry (128^3 grid, 8000 G), reduced to 16 valence bands and 48
    # columns: 40 explicit bands and 8 energy-window representatives (count weights)
    cfg = synth.config(4)
    e_all = synth.conduction_energies(cfg)
    col, e_col, n_col, n0 = g.p.gw_group_windows(e_all, 30.0 / EV, 1.0 / EV, 30)
    pick = np.concatenate([np.arange(40) * (n0 // 40), n0 + np.arange(8) * 3])
    gw = synth.wf_sphere(cfg.nd)
    gc = synth.chi_sphere(cfg.ng[0], cfg.qs[0], cfg.cell)
    b = synth.make_bands(cfg, v_index=np.arange(16) * 32, c_index=col[pick], gvec_wf=gw, e_c_all=e_all)
    from cases import Case
    case = Case(cfg, cfg.nd, gw, gc, b.coef_v, b.e_v, b.coef_c, e_col[pick].copy())
    head = synth.loss_head_block(gc)
    comps = [("ev", 0), ("ev", 15), ("ec", 5), ("ec", 39), ("ec", 41), ("ec", 47), ("n", 42), ("n", 46)]
    # the configuration's mixed precision against the same float64 differences, at the
    # tolerances of its modes (float32 contraction, split-bf16 x3)
    _fd_check(g, case, head, n_col[pick].copy(), comps, 1e-3, 1e-6, mixed=(("fp32", 2e-5), ("bf16x3", 1e-4)))
