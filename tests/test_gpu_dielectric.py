"""GPU parity of eps^-1 = (I - diag(v) chi0)^-1 and its adjoint against the FP64 oracle
(LAPACK inverse; closed-form adjoint pinned by finite differences in test_oracle)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import grad as og
from cases import Gpu, make_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def gpu_eps_inv(g, chi, v):
    torch = g.torch
    c = torch.from_numpy(np.ascontiguousarray(chi)).to(g.dev)
    vv = torch.from_numpy(np.ascontiguousarray(v)).to(g.dev)
    z = g.p.gw_eps_inv(g.ctx, vv, c)
    g.p.gw_eps_inv_status(g.ctx)
    return z.cpu().numpy()


def random_chi(n, seed, hermitian):
    r = np.random.default_rng(seed)
    a = (r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) / np.sqrt(n)
    if hermitian:
        a = -(a @ a.conj().T) / 4.0          # negative semidefinite like a static chi0
    return a


@pytest.mark.parametrize("n,herm", [(1, True), (27, True), (64, False), (259, True), (300, False), (1000, False)])
def test_eps_inv_matches_lapack(g, n, herm):
    chi = random_chi(n, n, herm)
    v = np.random.default_rng(n + 1).uniform(0.5, 3.0, n)
    z = gpu_eps_inv(g, chi, v)
    ref = oracle.eps_inv(chi, v)
    err = np.abs(z - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, err
    eps = oracle.eps_matrix(chi, v)
    assert np.abs(eps @ z - np.eye(n)).max() <= 1e-10


def test_eps_inv_needs_pivoting(g):
    # eps with a zero leading diagonal entry: Gauss-Jordan without row interchanges breaks down
    n = 130
    r = np.random.default_rng(4)
    eps = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    eps[0, 0] = 0.0
    v = np.ones(n)
    chi = np.eye(n) - eps                      # so that I - v chi = eps
    z = gpu_eps_inv(g, chi, v)
    assert np.abs(z - np.linalg.inv(eps)).max() <= 1e-10 * np.abs(np.linalg.inv(eps)).max()


def test_eps_inv_of_static_chi0_c1(g):
    case = make_case(0)
    chi = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    v = synth.coulomb(case.gc, case.cfg.qs[0], case.cfg.cell)
    z = gpu_eps_inv(g, chi, v)
    ref = oracle.eps_inv(chi, v)
    assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()
    assert oracle.eps_inf(z) == pytest.approx(oracle.eps_inf(ref), rel=1e-12)


def test_eps_inv_singular_is_reported(g):
    n = 70
    chi = np.eye(n, dtype=np.complex128)
    v = np.ones(n)                              # eps = I - I = 0
    torch = g.torch
    c = torch.from_numpy(chi).to(g.dev)
    vv = torch.from_numpy(v).to(g.dev)
    g.p.gw_eps_inv(g.ctx, vv, c)
    with pytest.raises(g.p.GwError) as e:
        g.p.gw_eps_inv_status(g.ctx)
    assert e.value.status == g.p.GW_ESINGULAR
    # a later good inversion clears the flag
    gpu_eps_inv(g, random_chi(40, 3, True), np.ones(40))


def test_eps_inv_batched(g):
    n, nb = 100, 3
    chis = np.stack([random_chi(n, 10 + i, i % 2 == 0) for i in range(nb)])
    vs = np.random.default_rng(9).uniform(0.5, 2.0, (nb, n))
    torch = g.torch
    z = g.p.gw_eps_inv(g.ctx, torch.from_numpy(vs).to(g.dev), torch.from_numpy(chis).to(g.dev)).cpu().numpy()
    for i in range(nb):
        ref = oracle.eps_inv(chis[i], vs[i])
        assert np.abs(z[i] - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("n", [27, 200])
def test_eps_inv_backward_matches_oracle(g, n):
    chi = random_chi(n, 5 * n, False)
    v = np.random.default_rng(2).uniform(0.5, 2.0, n)
    zbar = random_chi(n, 7 * n, False)
    ref_z = oracle.eps_inv(chi, v)
    ref = og.grad_eps_inv(ref_z, v, zbar)
    torch = g.torch
    out = g.p.gw_eps_inv_backward(g.ctx, torch.from_numpy(v).to(g.dev), torch.from_numpy(ref_z).to(g.dev),
                                  torch.from_numpy(zbar).to(g.dev)).cpu().numpy()
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
