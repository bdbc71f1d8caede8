"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 mode 1e-10 relative (Frobenius and max-abs over max |chi0|);
pair densities 1e-12 relative; FP32 mode 2e-5 relative (float32 pair transform,
float32 MFMA accumulation within a chunk of pairs); split-bf16 x3 mode 1e-4
(each product keeps about 16 bits of mantissa)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from cases import Case, Gpu, make_case, rel_err

pytestmark = pytest.mark.gpu

EV = synth.HARTREE_EV


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def ref_chi0(case: Case, omegas=(0.0,), delta=0.0):
    col, e_col, n_col = case.columns()
    return oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, e_col, case.gw, case.gc, (case.nd,) * 3,
                             omegas, delta, n_col=n_col, col_band=col)


def ref_m(case: Case, v0, nvs, c0, ncs):
    col, _, _ = case.columns()
    pv = oracle.psi_real_space(case.coef_v[v0:v0 + nvs], case.gw, (case.nd,) * 3)
    pc = oracle.psi_real_space(case.coef_c[col[c0:c0 + ncs]], case.gw, (case.nd,) * 3)
    return oracle.pair_density_fft(pv, pc, case.gc)


def test_pair_density_c1_fp64(g):
    case = make_case(0)
    m = g.pair_density(case, 0, 16, 0, 40)
    ref = ref_m(case, 0, 16, 0, 40)
    assert np.abs(m - ref).max() <= 1e-12 * np.abs(ref).max()
    # orthogonality: M_vc(G = 0) = <v|c> = 0
    assert np.abs(m[:, :, 0]).max() < 1e-14


def test_pair_density_ragged_block_fp64_fp32(g):
    case = make_case(0)
    ref = ref_m(case, 3, 5, 101, 13)
    m64 = g.pair_density(case, 3, 5, 101, 13, "fp64")
    m32 = g.pair_density(case, 3, 5, 101, 13, "fp32")
    assert np.abs(m64 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(m32 - ref).max() <= 1e-5 * np.abs(ref).max()


def test_pair_density_plane_waves_closed_form(g):
    # c_v = e_{G_a}, c_c = e_{G_b}  =>  M(G) = delta_{G, G_a - G_b}
    base = make_case(0, nv=4, nc=8)
    pa, pb = [0, 7, 40, 77], [3, 19, 33, 60, 101, 150, 200, 500]
    case = Case(base.cfg, base.nd, base.gw, base.gc, synth.plane_wave_bands(base.gw, pa), base.e_v,
                synth.plane_wave_bands(base.gw, pb), base.e_c)
    m = g.pair_density(case, 0, 4, 0, 8)
    gl = {tuple(x): i for i, x in enumerate(base.gc.tolist())}
    want = np.zeros_like(m)
    for i, a in enumerate(pa):
        for j, b in enumerate(pb):
            k = gl.get(tuple(base.gw[a] - base.gw[b]))
            if k is not None:
                want[i, j, k] = 1.0
    assert np.abs(m - want).max() < 1e-14


def test_chi0_c1_fp64(g):
    case = make_case(0)
    chi = g.chi0(case)[0]
    ref = ref_chi0(case)[0]
    fro, mx = rel_err(chi, ref)
    assert fro <= 1e-10 and mx <= 1e-10, (fro, mx)
    assert np.abs(chi - chi.conj().T).max() <= 1e-14 * np.abs(chi).max()
    assert np.linalg.eigvalsh(chi).max() <= 1e-12 * np.abs(chi).max()
    assert np.abs(chi[0]).max() <= 1e-13 * np.abs(chi).max()


def test_chi0_c1_fp32(g):
    case = make_case(0)
    chi = g.chi0(case, prec="fp32")[0]
    ref = ref_chi0(case)[0]
    fro, mx = rel_err(chi, ref)
    assert fro <= 2e-5 and mx <= 2e-5, (fro, mx)


def test_chi0_c1_bf16x3(g):
    # split-bf16 x3 products carry ~2^-16 relative error each; float32 accumulation
    case = make_case(0)
    chi = g.chi0(case, prec="bf16x3")[0]
    ref = ref_chi0(case)[0]
    fro, mx = rel_err(chi, ref)
    assert fro <= 1e-4 and mx <= 1e-4, (fro, mx)
    assert np.abs(chi - chi.conj().T).max() <= 1e-14 * np.abs(chi).max()


def test_chi0_dynamic_bf16x3(g):
    case = make_case(0, nv=8, nc=60)
    om = np.array([0.0, 7.0]) / EV
    d = 0.1 / EV
    chi = g.chi0(case, omegas=om, delta=d, prec="bf16x3")
    ref = ref_chi0(case, om, d)
    for i in range(len(om)):
        fro, mx = rel_err(chi[i], ref[i])
        assert fro <= 1e-4 and mx <= 1e-4, (i, fro, mx)


@pytest.mark.parametrize("nv,nc", [(1, 1), (5, 13), (7, 65)])
def test_chi0_ragged_fp64(g, nv, nc):
    case = make_case(0, nv=nv, nc=nc)
    chi = g.chi0(case)[0]
    ref = ref_chi0(case)[0]
    fro, mx = rel_err(chi, ref)
    assert fro <= 1e-10 and mx <= 1e-10, (fro, mx)


def test_chi0_dynamic_fp64(g):
    case = make_case(0, nv=8, nc=60)
    om = np.array([0.0, 0.3, 7.0, 25.0]) / EV
    d = 0.1 / EV
    chi = g.chi0(case, omegas=om, delta=d)
    ref = ref_chi0(case, om, d)
    for i in range(len(om)):
        fro, mx = rel_err(chi[i], ref[i])
        assert fro <= 1e-10 and mx <= 1e-10, (i, fro, mx)
    # delta = 0 below the gap: Hermitian
    chi0 = g.chi0(case, omegas=[0.5 / EV], delta=0.0)[0]
    assert np.abs(chi0 - chi0.conj().T).max() <= 1e-14 * np.abs(chi0).max()


def test_chi0_grouped_fp64(g):
    # the 24^3 workload's spectrum [5, 60] eV grouped above E_0 = 30 eV in 1 eV windows (count weights)
    case = make_case(0, nv=16, nc=240)
    e0, de, nwin = 30.0 / EV, 1.0 / EV, 30
    col, e_col, n_col, n0 = g.p.gw_group_windows(case.e_c, e0, de, nwin)
    want = oracle.group_windows(case.e_c, e0, de, nwin)
    assert np.array_equal(col, want[0]) and np.array_equal(n_col, want[2]) and n0 == want[3]
    case.col_band, case.e_col, case.n_col = col, e_col, n_col
    chi = g.chi0(case)[0]
    ref = oracle.chi0_grouped_static(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc,
                                     (case.nd,) * 3, e0, de, nwin)
    fro, mx = rel_err(chi, ref)
    assert fro <= 1e-10 and mx <= 1e-10, (fro, mx)


@pytest.mark.parametrize("cfg,prec,tol", [(1, "fp64", 1e-10), (1, "fp32", 2e-5), (2, "fp32", 2e-5),
                                          (4, "fp32", 2e-5), (1, "bf16x3", 1e-4), (2, "bf16x3", 1e-4),
                                          (4, "bf16x3", 1e-4)])
def test_chi0_config_geometry_subset(g, cfg, prec, tol):
    # the configs' grids and dielectric spheres (72^3 / NG 2000, 96^3 / 4000, 128^3 / 8000)
    # on a few bands the oracle finishes in seconds
    case = make_case(cfg, nv=4, nc=12)
    chi = g.chi0(case, prec=prec)[0]
    ref = ref_chi0(case)[0]
    fro, mx = rel_err(chi, ref)
    assert fro <= tol and mx <= tol, (fro, mx)


@pytest.mark.parametrize("iq", [0, 3, 7])
def test_chi0_batched_config_q_points(g, iq):
    # q-points and dielectric spheres of the batched workload (NG 800 ... 3000), dynamic
    case = make_case(3, nv=4, nc=8, iq=iq)
    om = np.array([0.0, 10.0]) / EV
    d = 0.1 / EV
    chi = g.chi0(case, omegas=om, delta=d, prec="fp32")
    ref = ref_chi0(case, om, d)
    for i in range(2):
        fro, mx = rel_err(chi[i], ref[i])
        assert fro <= 2e-5 and mx <= 2e-5, (iq, i, fro, mx)


def test_chi0_deterministic(g):
    case = make_case(0, nv=8, nc=100)
    a = g.chi0(case)
    b = g.chi0(case)
    assert np.array_equal(a, b)


def test_invalid_arguments_raise(g):
    case = make_case(0, nv=2, nc=3)
    p = g.p
    prob = g.problem(case)
    with pytest.raises(p.GwError):
        p.gw_chi0_build(g.ctx, [prob], [len(case.gc)], [0.0], -1.0, p.GW_FP64)
    with pytest.raises(p.GwError):
        p.gw_pair_density(g.ctx, prob, 0, 3, 0, 1, len(case.gc), p.GW_FP64)
    # not alias-free: 24^3 grid, wavefunction half-width 10, dielectric half-width 4 (2*10 + 4 = 24)
    with pytest.raises(p.GwError):
        p.gw_geom_create(g.ctx, (24, 24, 24), synth.wf_sphere(24, 10), case.gc)
    # workspace too small
    import torch
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(p.GwError):
        p.gw_chi0_build(g.ctx, [prob], [len(case.gc)], [0.0], 0.0, p.GW_FP64, workspace=ws)


# (workload, NG, smaller grid): the spheres of the 72^3 workload (wavefunction radius 18,
# chi radius 7 at NG 2000) are alias-free on 48^3 (2 * 18 + 7 < 48), those of the 96^3 one
# (24, 9) on 64^3, those of the 128^3 one (32, 12) on 96^3
@pytest.mark.parametrize("cfg,ng,small_nd", [(1, 2000, 48), (2, 4000, 64), (4, 8000, 96)],
                         ids=["72cube-on-48", "96cube-on-64", "128cube-on-96"])
def test_reduced_alias_free_grid_gives_the_same_chi0(g, cfg, ng, small_nd):
    # the build on the smaller grid reproduces the oracle's chi0 on the stated grid, in
    # every precision
    import dataclasses
    case = make_case(cfg, nv=4, nc=13, ng=ng)
    small = dataclasses.replace(case, nd=small_nd)
    assert 2 * np.abs(case.gw).max() + np.abs(case.gc).max() < small_nd
    ref = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)):
        chi = g.chi0(small, prec=prec)[0]
        fro, mx = rel_err(chi, ref)
        assert fro <= tol and mx <= tol, (prec, fro, mx)
    # a 32^3 grid is refused (the wavefunction sphere already folds onto itself there)
    with pytest.raises(g.p.GwError, match="collide|alias"):
        g.p.gw_geom_create(g.ctx, (32,) * 3, case.gw, case.gc)


def test_values_and_spheres_are_checked(g):
    # the band-sum entry points check the values behind the device pointers (one synchronising
    # read): a column row outside the coefficient rows, a negative multiplicity or a non-finite
    # energy is GW_EINVAL; the geometry checks the dielectric sphere's order when given cell and q
    case = make_case(0, nv=2, nc=5)
    p = g.p
    cases = []
    bad_row = dataclasses.replace(case, col_band=np.array([0, 1, 5, 2], dtype=np.int32), e_col=case.e_c[:4].copy(),
                                  n_col=np.ones(4))
    bad_n = dataclasses.replace(case, col_band=np.arange(4, dtype=np.int32), e_col=case.e_c[:4].copy(),
                                n_col=np.array([1.0, -0.5, 1.0, 1.0]))
    e_nan = case.e_c.copy()
    e_nan[2] = np.nan
    bad_e = dataclasses.replace(case, e_c=e_nan)
    for c, what in ((bad_row, "col_band"), (bad_n, "n_col"), (bad_e, "energy")):
        with pytest.raises(p.GwError, match=what):
            g.chi0(c)
        with pytest.raises(p.GwError, match=what):
            p.gw_chi0_backward(g.ctx, [g.problem(c)], [0.0], 0.0, p.GW_FP64,
                               g.t(np.zeros((1, len(c.gc), len(c.gc)), dtype=np.complex128)))
    # a good call afterwards still works
    ref = oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3)[0]
    assert np.abs(g.chi0(case)[0] - ref).max() <= 1e-10 * np.abs(ref).max()
    # sphere order: a swapped pair, or the sphere of another q
    swapped = case.gc.copy()
    swapped[[3, 30]] = swapped[[30, 3]]
    with pytest.raises(p.GwError, match="not ordered"):
        p.gw_geom_create(g.ctx, (24,) * 3, case.gw, swapped, case.cfg.cell, case.q)
    with pytest.raises(p.GwError):
        p.gw_geom_create(g.ctx, (24,) * 3, case.gw, case.gc, case.cfg.cell, (0.5, 0.0, 0.0))
    geom = p.gw_geom_create(g.ctx, (24,) * 3, case.gw, swapped)     # no cell and q: not checked
    p.gw_geom_destroy(geom)


# Grids and dielectric spheres without a compiled pair-transform instance run the generic
# kernel (run-time N and K): N = 40 and 56 split 8 x 5 and 8 x 7 (odd S: the second half of
# each line has one chunk fewer), 48 with K = 17 (the instance there is K = 15), 80 = 16 x 5.
@pytest.mark.parametrize("nd,ng", [(40, 500), (56, 1500), (48, 2600), (80, 3000)],
                         ids=["40cube-K11", "56cube-K15", "48cube-K17", "80cube-K19"])
def test_generic_pair_kernel_shapes_match_oracle(g, nd, ng):
    cfg = synth.config(1)
    gw = synth.wf_sphere(nd)
    gc = synth.chi_sphere(ng, cfg.qs[0], cfg.cell)
    assert 2 * int(np.abs(gw).max()) + int(np.abs(gc).max()) < nd
    b = synth.make_bands(cfg, v_index=np.arange(4), c_index=np.arange(13), gvec_wf=gw)
    case = Case(cfg, nd, gw, gc, b.coef_v, b.e_v, b.coef_c, b.e_c, q=tuple(cfg.qs[0]))
    ref = ref_chi0(case)[0]
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)):
        chi = g.chi0(case, prec=prec)[0]
        fro, mx = rel_err(chi, ref)
        print(f"N = {nd}, NG = {ng}, {prec}: {fro:.2e} / {mx:.2e}")
        assert fro <= tol and mx <= tol, (prec, fro, mx)
    # the coefficient gradients need a compiled instance: refused, not approximated
    p = g.p
    gb = g.torch.zeros((1, len(gc), len(gc)), dtype=g.torch.complex128, device=g.dev)
    with pytest.raises(p.GwError) as e:
        p.gw_chi0_backward(g.ctx, [g.problem(case)], [0.0], 0.0, p.GW_FP64, gb, coef=(True, False))
    assert e.value.status == p.GW_EUNSUPPORTED
