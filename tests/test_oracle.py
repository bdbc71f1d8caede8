"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a brute-force plane-wave
convolution, a closed form, an invariant of Eq. (chi0), the exact band sum that
Eqs. (chi02)/(energyintegration) reduce to, the paper's printed tables, the
free-electron state count, a second factorisation, or finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import grad as og

HERE = os.path.dirname(os.path.abspath(__file__))


def assert_fd(pairs, label, tol=1e-6):
    """Central differences against analytic gradients, relative to the largest tested component
    of the gradient (no absolute floor): max_i |fd_i - g_i| <= tol * max_i |g_i|."""
    fd = np.array([a for a, _ in pairs], dtype=np.float64)
    g = np.array([b for _, b in pairs], dtype=np.float64)
    scale = np.abs(g).max()
    err = float(np.abs(fd - g).max() / scale)
    print(f"{label}: max|fd - g| / max|g| = {err:.1e} over {len(g)} components (max|g| = {scale:.2e})")
    assert scale > 0 and err <= tol, (label, err, fd, g)
    return err


def tiny(nd=12, rw=3, ng=27, nv=3, nc=5, seed=7):
    gw = synth.wf_sphere(nd, rw)
    cell = np.eye(3) * 7.0
    gc = synth.chi_sphere(ng, (0.01, 0, 0), cell)
    rows = synth.gaussian_columns(99, 30 + seed, range(nv + nc), gw.shape[0])
    q = synth.orthonormalize(rows)
    r = np.random.default_rng(seed)
    e_v = np.sort(r.uniform(-0.4, -0.05, nv))
    e_c = np.sort(r.uniform(0.2, 1.5, nc))
    return dict(gw=gw, gc=gc, cv=q[:nv], cc=q[nv:], e_v=e_v, e_c=e_c, nd=(nd, nd, nd), cell=cell)


# ---------------------------------------------------------------- matrix element
def test_pair_density_fft_equals_direct_convolution():
    t = tiny()
    pv = oracle.psi_real_space(t["cv"], t["gw"], t["nd"])
    pc = oracle.psi_real_space(t["cc"], t["gw"], t["nd"])
    m_fft = oracle.pair_density_fft(pv, pc, t["gc"])
    m_dir = oracle.pair_density_direct(t["cv"], t["cc"], t["gw"], t["gc"])
    assert np.abs(m_fft - m_dir).max() < 1e-14


def test_pair_density_plane_wave_closed_form():
    # c_v = e_{G_a}, c_c = e_{G_b}  =>  M(G) = 1 if G = G_a - G_b else 0
    gw = synth.wf_sphere(12, 3)
    gc = synth.chi_sphere(27, (0.01, 0, 0), np.eye(3) * 7.0)
    pa, pb = [5, 17, 40], [2, 9, 33, 60]
    cv = synth.plane_wave_bands(gw, pa)
    cc = synth.plane_wave_bands(gw, pb)
    m = oracle.pair_density_fft(oracle.psi_real_space(cv, gw, (12,) * 3),
                                oracle.psi_real_space(cc, gw, (12,) * 3), gc)
    for i, a in enumerate(pa):
        for j, b in enumerate(pb):
            want = np.array([1.0 if tuple(g) == tuple(gw[a] - gw[b]) else 0.0 for g in gc.tolist()])
            assert np.abs(m[i, j] - want).max() < 1e-14


def test_pair_density_head_is_overlap():
    # M_nm(G=0) = <n|m>: identity for an orthonormal set
    t = tiny()
    allc = np.concatenate([t["cv"], t["cc"]])
    p = oracle.psi_real_space(allc, t["gw"], t["nd"])
    g0 = np.array([[0, 0, 0]], dtype=np.int32)
    m = oracle.pair_density_fft(p, p, g0)[:, :, 0]
    assert np.abs(m - np.eye(len(allc))).max() < 1e-14


def test_pair_density_parseval():
    t = tiny()
    nd = t["nd"][0]
    a = np.arange(-nd // 2, nd // 2)
    full = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    pv = oracle.psi_real_space(t["cv"][:1], t["gw"], t["nd"])
    pc = oracle.psi_real_space(t["cc"][:2], t["gw"], t["nd"])
    m = oracle.pair_density_fft(pv, pc, full)
    lhs = (np.abs(m[0]) ** 2).sum(1)
    rhs = (np.abs(pv[0])[None] ** 2 * np.abs(pc) ** 2).reshape(2, -1).sum(1) / nd ** 3
    assert np.allclose(lhs, rhs, rtol=1e-13)


def test_alias_free_bound():
    gw = synth.wf_sphere(12, 3)
    gc = synth.chi_sphere(27, (0.01, 0, 0), np.eye(3) * 7.0)
    assert oracle.alias_free(gw, gc, (12, 12, 12))
    assert not oracle.alias_free(gw, gc, (7, 12, 12))


# ---------------------------------------------------------------- weights
def test_weights_static_limit_and_symmetry():
    r = np.random.default_rng(3)
    e_v = -r.uniform(0.05, 0.5, 4)
    e_c = r.uniform(0.2, 2.0, 6)
    n = r.uniform(0.5, 3, 6)
    ws = oracle.weights_static(e_v, e_c, n)
    assert np.allclose(ws, n[None] / (e_v[:, None] - e_c[None]), rtol=1e-15)
    assert np.all(ws < 0)
    w0 = oracle.weights(e_v, e_c, n, 0.0, 0.0)
    assert np.abs(w0 - ws).max() == 0.0
    for om in (0.01, 0.2, 1.3):
        wp = oracle.weights(e_v, e_c, n, om, 0.004)
        wm = oracle.weights(e_v, e_c, n, -om, 0.004)
        assert np.allclose(wp, wm, rtol=1e-14, atol=0)


def test_weights_below_gap_closed_form():
    # |w| below the gap, delta = 0: n/2 (1/(x-w) + 1/(x+w)) = n x/(x^2 - w^2) < 0
    e_v = np.array([-0.3, -0.1])
    e_c = np.array([0.25, 0.6])
    x = e_v[:, None] - e_c[None]
    for om in (0.05, 0.2, 0.3):
        w = oracle.weights(e_v, e_c, None, om, 0.0)
        assert np.allclose(w.real, x / (x * x - om * om), rtol=1e-14)
        assert np.all(w.imag == 0) and np.all(w.real < 0)


# ---------------------------------------------------------------- chi0
def test_chi0_static_hermitian_negative_semidefinite():
    t = tiny(nv=4, nc=9)
    chi = oracle.chi0_bands(t["cv"], t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    assert np.abs(chi - chi.conj().T).max() < 1e-15 * np.abs(chi).max() * 10
    ev = np.linalg.eigvalsh(chi)
    assert ev.max() <= 1e-13 * np.abs(ev).max()
    # head row and column vanish: M_vc(G=0) = <v|c> = 0
    assert np.abs(chi[0]).max() < 1e-14 and np.abs(chi[:, 0]).max() < 1e-14


def test_chi0_plane_waves_is_lindhard_sum():
    # plane-wave states: chi0_GG' = delta_GG' sum_{v,c: G_v - G_c = G} w_vc (discrete Lindhard sum)
    gw = synth.wf_sphere(12, 3)
    gc = synth.chi_sphere(27, (0.01, 0, 0), np.eye(3) * 7.0)
    pv, pc = [0, 1, 2, 3], [7, 8, 9, 10, 20, 30]
    e_v = np.array([-0.5, -0.4, -0.35, -0.2])
    e_c = np.array([0.3, 0.31, 0.5, 0.9, 1.1, 1.7])
    n_c = np.array([1.0, 2.0, 1.0, 0.5, 1.0, 3.0])
    for om, d in ((0.0, 0.0), (0.15, 0.01)):
        chi = oracle.chi0_bands(synth.plane_wave_bands(gw, pv), e_v, synth.plane_wave_bands(gw, pc), e_c,
                                gw, gc, (12,) * 3, omegas=(om,), delta=d, n_col=n_c)[0]
        want = np.zeros(len(gc), dtype=np.complex128)
        gl = [tuple(g) for g in gc.tolist()]
        for i, a in enumerate(pv):
            for j, b in enumerate(pc):
                dg = tuple(gw[a] - gw[b])
                if dg in gl:
                    x = e_v[i] - e_c[j]
                    want[gl.index(dg)] += n_c[j] * 0.5 * (1 / (x - om + 1j * d) + 1 / (x + om + 1j * d))
        assert np.abs(chi - np.diag(want)).max() < 1e-14


def test_chi0_dynamic_symmetries():
    t = tiny(nv=3, nc=6)
    args = (t["cv"], t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])
    om = [0.07, -0.07]
    chi = oracle.chi0_bands(*args, omegas=om, delta=0.003)
    assert np.abs(chi[0] - chi[1]).max() < 1e-14 * np.abs(chi).max()
    # below the gap with delta = 0 the dynamic chi0 is Hermitian and NSD
    gap = t["e_c"].min() - t["e_v"].max()
    chi_b = oracle.chi0_bands(*args, omegas=[0.5 * gap], delta=0.0)[0]
    assert np.abs(chi_b - chi_b.conj().T).max() < 1e-14 * np.abs(chi_b).max()
    assert np.linalg.eigvalsh(chi_b).max() <= 1e-13 * np.abs(chi_b).max()


def test_chi0_linear_in_column_chunks():
    t = tiny(nv=3, nc=8)
    args = (t["cv"], t["e_v"])
    whole = oracle.chi0_bands(*args, t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    a = oracle.chi0_bands(*args, t["cc"][:3], t["e_c"][:3], t["gw"], t["gc"], t["nd"])[0]
    b = oracle.chi0_bands(*args, t["cc"][3:], t["e_c"][3:], t["gw"], t["gc"], t["nd"])[0]
    assert np.abs(whole - a - b).max() < 1e-15 * np.abs(whole).max() * 10
    # chunk size of the internal loop does not matter
    c = oracle.chi0_bands(*args, t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"], c_chunk=1)[0]
    assert np.abs(whole - c).max() < 1e-15 * np.abs(whole).max() * 10


def test_chi0_trace_identity():
    # Tr chi0 = sum_p w_p ||m_p||^2
    t = tiny(nv=2, nc=4)
    chi = oracle.chi0_bands(t["cv"], t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    m = oracle.pair_density_direct(t["cv"], t["cc"], t["gw"], t["gc"])
    w = t["e_v"][:, None] - t["e_c"][None]
    assert np.isclose(np.trace(chi).real, ((np.abs(m) ** 2).sum(-1) / w).sum(), rtol=1e-13)


# ---------------------------------------------------------------- grouping
def test_grouping_one_band_per_window_reproduces_exact_sum():
    t = tiny(nv=3, nc=7)
    e0, de, nwin = 0.5, 0.1, 4
    # 3 explicit bands below E_0, then exactly one band at each window midpoint
    e_c = np.concatenate([[0.2, 0.3, 0.5], [e0 + (k + 0.5) * de for k in range(nwin)]])
    col, e_col, n_col, n0 = oracle.group_windows(e_c, e0, de, nwin)
    assert n0 == 3 and list(col) == list(range(7)) and np.all(n_col == 1.0)
    assert np.all(e_col == e_c)
    exact = oracle.chi0_bands(t["cv"], t["e_v"], t["cc"], e_c, t["gw"], t["gc"], t["nd"])[0]
    grouped = oracle.chi0_grouped_static(t["cv"], t["e_v"], t["cc"], e_c, t["gw"], t["gc"], t["nd"], e0, de, nwin)
    assert np.abs(grouped - exact).max() < 1e-14 * np.abs(exact).max()


def test_grouping_counts_and_representatives():
    r = np.random.default_rng(11)
    e_c = r.uniform(0.1, 2.0, 500)
    e0, de, nwin = 1.1, 0.09, 10   # top = 2.0
    col, e_col, n_col, n0 = oracle.group_windows(e_c, e0, de, nwin)
    assert n0 == int((e_c <= e0).sum())
    assert list(col[:n0]) == [i for i in range(500) if e_c[i] <= e0]
    assert n_col[n0:].sum() == 500 - n0
    for j in range(n0, len(col)):
        k = int(round((e_col[j] - e0) / de - 0.5))
        lo, hi = e0 + k * de, e0 + (k + 1) * de
        mem = [i for i in range(500) if lo < e_c[i] and (e_c[i] < hi or (k == nwin - 1 and e_c[i] <= hi))]
        assert len(mem) == n_col[j]
        d = [abs(e_c[i] - e_col[j]) for i in mem]
        assert abs(e_c[col[j]] - e_col[j]) == min(d)
    # no windows: explicit columns only; everything above the last window is rejected
    col2, _, _, n02 = oracle.group_windows(e_c[e_c <= e0], e0, de, nwin)
    assert n02 == len(col2)
    with pytest.raises(ValueError):
        oracle.group_windows(np.array([0.5, 2.5]), e0, de, nwin)


def test_group_edges_on_a_uniform_grid_is_group_windows():
    r = np.random.default_rng(12)
    e_c = r.uniform(0.1, 2.0, 400)
    e0, de, nwin = 1.1, 0.09, 10
    edges = e0 + de * np.arange(nwin + 1)
    for mode in ("count", "dos"):
        a = oracle.group_windows(e_c, e0, de, nwin, mode, dos_a=3.0, dos_v0=0.05)
        b = oracle.group_edges(e_c, edges, mode, "midpoint", dos_a=3.0, dos_v0=0.05)
        assert a[3] == b[3] and np.array_equal(a[0], b[0])
        assert np.allclose(a[1], b[1], rtol=0, atol=1e-15) and np.allclose(a[2], b[2], rtol=1e-14, atol=0)


def test_group_edges_quadrature_orders():
    # density weights summed over the windows integrate g(E) = A sqrt(E - V0) over
    # [E0, Emax]: the midpoint rule with error O(h^2), the two-point Gauss rule O(h^4)
    A, v0, e0, emax = 2.5, 0.2, 1.0, 3.0
    e_c = np.linspace(e0 + 1e-9, emax, 4001)        # every window holds bands
    exact = 2.0 * A / 3.0 * ((emax - v0) ** 1.5 - (e0 - v0) ** 1.5)
    errs = {}
    for rule in ("midpoint", "gauss2"):
        for nwin in (4, 8):
            edges = np.linspace(e0, emax, nwin + 1)
            col, e_col, n_col, n0 = oracle.group_edges(e_c, edges, "dos", rule, dos_a=A, dos_v0=v0)
            assert n0 == 0 and len(col) == nwin * (1 if rule == "midpoint" else 2)
            errs[rule, nwin] = abs(n_col.sum() - exact)
    assert 3.5 < errs["midpoint", 4] / errs["midpoint", 8] < 4.5
    assert 13.0 < errs["gauss2", 4] / errs["gauss2", 8] < 19.0
    assert errs["gauss2", 8] < 1e-2 * errs["midpoint", 8]


def test_group_edges_non_uniform_counts_and_representatives():
    r = np.random.default_rng(13)
    e_c = r.uniform(0.1, 2.0, 500)
    edges = 1.0 + np.cumsum(np.concatenate([[0.0], 0.02 * 1.3 ** np.arange(9)]))
    edges[-1] = 2.0
    col, e_col, n_col, n0 = oracle.group_edges(e_c, edges, "count")
    assert n0 == int((e_c <= edges[0]).sum())
    assert n_col[n0:].sum() == 500 - n0
    for j in range(n0, len(col)):
        k = int(np.searchsorted(edges, e_col[j]) - 1)
        assert abs(e_col[j] - 0.5 * (edges[k] + edges[k + 1])) < 1e-15
        mem = [i for i in range(500) if edges[k] < e_c[i] and (e_c[i] < edges[k + 1] or
                                                                (k == len(edges) - 2 and e_c[i] <= edges[k + 1]))]
        assert len(mem) == n_col[j] and col[j] in mem
        assert abs(e_c[col[j]] - e_col[j]) == min(abs(e_c[i] - e_col[j]) for i in mem)
    # two Gauss nodes per window, each inside its window and represented by a member
    col, e_col, n_col, n0 = oracle.group_edges(e_c, edges, "dos", "gauss2", dos_a=1.0)
    assert len(col) - n0 == 2 * (len(edges) - 1)
    with pytest.raises(ValueError):
        oracle.group_edges(e_c, edges, "count", "gauss2")
    with pytest.raises(ValueError):
        oracle.group_edges(e_c, edges[::-1], "count")
    with pytest.raises(ValueError):
        oracle.group_edges(np.array([2.5]), edges, "count")


def test_speedup_matches_printed_tables():
    with open(os.path.join(HERE, "golden", "paper_tables.json")) as f:
        tab = json.load(f)
    t1 = tab["table1"]
    for n, s in zip(t1["n0_plus_ne"], t1["speedup"]):
        assert round(oracle.speedup_factor(t1["n_c"], n), 1) == s
    t2 = tab["table2"]
    for nc, n, s in zip(t2["n_c"], t2["n0_plus_ne"], t2["speedup"]):
        assert round(oracle.speedup_factor(nc, n), 1) == s


def test_free_electron_dos_counts_plane_waves():
    # integral_0^E g = number of spin-degenerate plane-wave states with |G|^2/2 <= E
    a = 40.0
    b = 2 * math.pi / a
    r = 22
    n = np.arange(-r, r + 1)
    n1, n2, n3 = np.meshgrid(n, n, n, indexing="ij")
    kin = 0.5 * b * b * (n1 ** 2 + n2 ** 2 + n3 ** 2)
    for e in (2.0, 3.0, 4.5):
        count = 2 * int((kin <= e).sum())
        es = np.linspace(0, e, 20001)
        integ = np.trapezoid(oracle.free_electron_dos(es, a ** 3), es)
        assert abs(integ - count) / count < 0.01
        assert np.isclose(integ, a ** 3 * (2 * e) ** 1.5 / (3 * math.pi ** 2), rtol=1e-6)


# ---------------------------------------------------------------- dielectric
def test_eps_inv_routes_agree_and_properties():
    t = tiny(nv=4, nc=9)
    chi = oracle.chi0_bands(t["cv"], t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    v = synth.coulomb(t["gc"], (0.01, 0, 0), t["cell"])
    z = oracle.eps_inv(chi, v)
    z2 = oracle.eps_inv_static_cholesky(chi, v)
    assert np.abs(z - z2).max() < 1e-12 * np.abs(z).max()
    eps = oracle.eps_matrix(chi, v)
    assert np.abs(eps @ z - np.eye(len(v))).max() < 1e-12
    assert np.abs(np.diagonal(z).imag).max() < 1e-14
    s = np.sqrt(v)
    zt = z * s[None] / s[:, None]          # symmetrised inverse (eps~)^-1
    ev = np.linalg.eigvalsh(0.5 * (zt + zt.conj().T))
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12
    assert np.abs(oracle.eps_inv(np.zeros_like(chi), v) - np.eye(len(v))).max() == 0
    assert oracle.eps_inf(z) == pytest.approx(1.0)       # head row/column of chi0 vanish


def _chi0_with_head(mix=0.05, seed=7):
    # valence states at k+q that are not orthogonal to the conduction states at k (their own
    # set, as at a q-point away from Gamma): M_vc(G=0) = <v,k+q|c,k> != 0, so the head row and
    # column of chi0 do not vanish and [eps^-1]_00 differs from 1
    t = tiny(nv=4, nc=9, seed=seed)
    cvq = synth.orthonormalize(t["cv"] + mix * t["cc"][:4])
    chi = oracle.chi0_bands(cvq, t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    return chi, synth.coulomb(t["gc"], (0.01, 0, 0), t["cell"])


def test_eps_inf_is_the_reciprocal_of_the_inverse_head():
    # Table 3's eps_inf = 1/[eps^-1]_00.  The (0,0) entry of an inverse is the reciprocal of the
    # Schur complement eps_00 - eps_0R eps_RR^-1 eps_R0 (block elimination), computed here by a
    # linear solve on the remaining block, without forming eps^-1
    chi, v = _chi0_with_head()
    assert abs(chi[0, 0]) > 1e-3 * np.abs(chi).max() and np.abs(chi[0, 1:]).max() > 0
    eps = oracle.eps_matrix(chi, v)
    schur = eps[0, 0] - eps[0, 1:] @ np.linalg.solve(eps[1:, 1:], eps[1:, 0])
    assert abs(schur.imag) < 1e-12 * abs(schur)
    for z in (oracle.eps_inv(chi, v), oracle.eps_inv_static_cholesky(chi, v)):
        assert oracle.eps_inf(z) == pytest.approx(schur.real, rel=1e-12)
    # eps~ = I - v^1/2 chi0 v^1/2 >= I and the Schur complement of a block never exceeds the
    # diagonal entry: 1 < eps_inf < eps_00 = 1 - v_0 chi0_00 (the head couples to the rest)
    einf = oracle.eps_inf(oracle.eps_inv(chi, v))
    assert 1.0 < einf < eps[0, 0].real and einf < 0.999 * eps[0, 0].real
    # a head decoupled from the other G-vectors: eps_inf is exactly the scalar 1 - v_0 chi0_00
    chi_d = chi.copy()
    chi_d[0, 1:] = 0.0
    chi_d[1:, 0] = 0.0
    assert oracle.eps_inf(oracle.eps_inv(chi_d, v)) == pytest.approx(1.0 - v[0] * chi_d[0, 0].real, rel=1e-13)
    # head index other than 0: a permuted sphere gives the same value
    perm = np.roll(np.arange(len(v)), 3)
    zp = oracle.eps_inv(chi[np.ix_(perm, perm)], v[perm])
    assert oracle.eps_inf(zp, head=int(np.nonzero(perm == 0)[0][0])) == pytest.approx(einf, rel=1e-12)


# ---------------------------------------------------------------- gradients
def _loss_static(t, v, head, e_v, e_c, n_c):
    chi = oracle.chi0_bands(t["cv"], e_v, t["cc"], e_c, t["gw"], t["gc"], t["nd"], n_col=n_c)[0]
    return og.head_block_loss(oracle.eps_inv(chi, v), head)


def test_gradients_static_match_finite_differences():
    t = tiny(nv=3, nc=5)
    v = synth.coulomb(t["gc"], (0.01, 0, 0), t["cell"])
    head = synth.loss_head_block(t["gc"])
    e_v, e_c, n_c = t["e_v"], t["e_c"], np.array([1.0, 2.0, 1.5, 1.0, 0.7])
    chi = oracle.chi0_bands(t["cv"], e_v, t["cc"], e_c, t["gw"], t["gc"], t["nd"], n_col=n_c)[0]
    z = oracle.eps_inv(chi, v)
    gchi = og.grad_eps_inv(z, v, og.head_block_loss_grad(len(v), head))
    gv, gc, gn = og.grad_chi0_energies(t["cv"], e_v, t["cc"], e_c, t["gw"], t["gc"], t["nd"], gchi[None],
                                       n_col=n_c)
    h = 1e-5
    for arr, g, name in ((e_v, gv, "ev"), (e_c, gc, "ec"), (n_c, gn, "n")):
        pairs = []
        for i in range(len(arr)):
            p, m = arr.copy(), arr.copy()
            p[i] += h
            m[i] -= h
            kw = dict(e_v=e_v, e_c=e_c, n_c=n_c)
            key = {"ev": "e_v", "ec": "e_c", "n": "n_c"}[name]
            lp = _loss_static(t, v, head, **{**kw, key: p})
            lm = _loss_static(t, v, head, **{**kw, key: m})
            pairs.append(((lp - lm) / (2 * h), g[i]))
        assert_fd(pairs, f"static dL/d{name}")


def test_gradients_dynamic_match_finite_differences():
    t = tiny(nv=2, nc=4)
    r = np.random.default_rng(5)
    ng = len(t["gc"])
    bmat = r.standard_normal((2, ng, ng)) + 1j * r.standard_normal((2, ng, ng))
    om, d = [0.05, 0.4], 0.01

    def loss(e_v, e_c):
        chi = oracle.chi0_bands(t["cv"], e_v, t["cc"], e_c, t["gw"], t["gc"], t["nd"], omegas=om, delta=d)
        return float(np.real(np.sum(np.conj(bmat) * chi)))

    gv, gc, _ = og.grad_chi0_energies(t["cv"], t["e_v"], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"], bmat,
                                      omegas=om, delta=d)
    h = 1e-6
    pairs = []
    for i in range(2):
        p, m = t["e_v"].copy(), t["e_v"].copy()
        p[i] += h
        m[i] -= h
        pairs.append(((loss(p, t["e_c"]) - loss(m, t["e_c"])) / (2 * h), gv[i]))
    assert_fd(pairs, "dynamic dL/dE_v")
    pairs = []
    for i in range(4):
        p, m = t["e_c"].copy(), t["e_c"].copy()
        p[i] += h
        m[i] -= h
        pairs.append(((loss(t["e_v"], p) - loss(t["e_v"], m)) / (2 * h), gc[i]))
    assert_fd(pairs, "dynamic dL/dE_c")


def test_grad_eps_inv_general_matches_finite_differences():
    r = np.random.default_rng(8)
    ng = 6
    chi = 0.05 * (r.standard_normal((ng, ng)) + 1j * r.standard_normal((ng, ng)))
    v = r.uniform(0.5, 2.0, ng)
    bmat = r.standard_normal((ng, ng)) + 1j * r.standard_normal((ng, ng))

    def loss(c):
        return float(np.real(np.sum(np.conj(bmat) * oracle.eps_inv(c, v))))

    g = og.grad_eps_inv(oracle.eps_inv(chi, v), v, bmat)
    h = 1e-6
    pairs = []
    for (i, j) in ((0, 0), (1, 4), (5, 2)):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            p, m = chi.copy(), chi.copy()
            p[i, j] += unit * h
            m[i, j] -= unit * h
            pairs.append(((loss(p) - loss(m)) / (2 * h), part(g[i, j])))
    assert_fd(pairs, "dL/dchi0 through eps^-1")


@pytest.mark.parametrize("om,d", [([0.0], 0.0), ([0.05, 0.4], 0.01)])
def test_coefficient_gradients_match_finite_differences(om, d):
    # both terms of the matrix element (the valence set enters conjugated, the conduction
    # set plainly), a grouped column layout with two columns on one coefficient row
    t = tiny(nv=2, nc=4)
    r = np.random.default_rng(11)
    ng = len(t["gc"])
    bmat = r.standard_normal((len(om), ng, ng)) + 1j * r.standard_normal((len(om), ng, ng))
    col = np.array([0, 1, 3, 1])
    e_col = t["e_c"][col] + np.array([0.0, 0.0, 0.0, 0.07])
    n_col = np.array([1.0, 1.0, 2.0, 0.5])

    def loss(cv, cc):
        chi = oracle.chi0_bands(cv, t["e_v"], cc, e_col, t["gw"], t["gc"], t["nd"], omegas=om, delta=d,
                                n_col=n_col, col_band=col)
        return float(np.real(np.sum(np.conj(bmat) * chi)))

    gv, gcc = og.grad_chi0_coefficients(t["cv"], t["e_v"], t["cc"], e_col, t["gw"], t["gc"], t["nd"], bmat,
                                        omegas=om, delta=d, n_col=n_col, col_band=col)
    assert gv.shape == t["cv"].shape and gcc.shape == t["cc"].shape
    assert np.all(gcc[2] == 0)          # row 2 feeds no column
    h = 1e-6
    pairs = []
    for which, idx in (("v", (0, 3)), ("v", (1, 20)), ("c", (1, 0)), ("c", (3, 11)), ("c", (0, 7))):
        for unit, part in ((1.0, np.real), (1j, np.imag)):
            cv_p, cv_m, cc_p, cc_m = t["cv"].copy(), t["cv"].copy(), t["cc"].copy(), t["cc"].copy()
            if which == "v":
                cv_p[idx] += unit * h
                cv_m[idx] -= unit * h
                want = part(gv[idx])
            else:
                cc_p[idx] += unit * h
                cc_m[idx] -= unit * h
                want = part(gcc[idx])
            pairs.append(((loss(cv_p, cc_p) - loss(cv_m, cc_m)) / (2 * h), want))
    assert_fd(pairs, "dL/dcoefficients")


# ---------------------------------------------------------------- static COH self-energy
def _static_eps_inv(t, nv=3):
    chi = oracle.chi0_bands(t["cv"][:nv], t["e_v"][:nv], t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"])[0]
    v = synth.coulomb(t["gc"], (0.01, 0, 0), t["cell"])
    return oracle.eps_inv(chi, v), v


def test_sigma_coh_over_a_complete_set_is_the_plane_wave_convolution():
    # every orthonormal band of the 7^3-box wavefunction sphere (npw of them): the band sum
    # equals the band-free closed form of the completeness relation
    t = tiny(nd=12, rw=2, ng=19, nv=3, nc=5)
    z, v = _static_eps_inv(t)
    npw = t["gw"].shape[0]
    full = synth.orthonormalize(synth.gaussian_columns(98, 3, range(npw), npw))
    states = t["cv"][:2]
    got = oracle.sigma_coh_static(states, full, t["gw"], t["gc"], t["nd"], z, v)
    want = oracle.sigma_coh_complete_set(states, t["gw"], t["gc"], z, v)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # a truncated band sum does not reach it (the slow convergence the grouping addresses)
    part = oracle.sigma_coh_static(states, full[: npw // 2], t["gw"], t["gc"], t["nd"], z, v)
    assert np.abs(part - want).max() > 1e-2 * np.abs(want).max()


def test_sigma_coh_is_hermitian_and_negative_semidefinite():
    t = tiny(nd=12, rw=3, ng=27, nv=3, nc=8)
    z, v = _static_eps_inv(t)
    states = np.concatenate([t["cv"], t["cc"][:2]])
    w = np.random.default_rng(4).uniform(0.5, 3.0, len(t["cc"]))
    s = oracle.sigma_coh_static(states, t["cc"], t["gw"], t["gc"], t["nd"], z, v, n_col=w)
    assert np.abs(s - s.conj().T).max() < 1e-13 * np.abs(s).max()
    ev = np.linalg.eigvalsh(0.5 * (s + s.conj().T))
    assert ev.max() <= 1e-12 * np.abs(ev).max() and ev.min() < 0
    # weights enter linearly: doubling every weight doubles Sigma
    s2 = oracle.sigma_coh_static(states, t["cc"], t["gw"], t["gc"], t["nd"], z, v, n_col=2 * w)
    assert np.abs(s2 - 2 * s).max() < 1e-13 * np.abs(s).max()


# ---------------------------------------------------------------- k-point sum
def test_kq_map_folds_k_plus_q_onto_the_grid():
    k = synth.kpoint_grid(2)
    idx, g0 = oracle.kq_map(k, (0.5, 0.0, 0.0))
    for i in range(len(k)):
        assert np.allclose(k[i] + (0.5, 0, 0), k[idx[i]] + g0[i])
    assert any(np.abs(g0).sum(1) > 0)                       # some k + q leave the cell
    with pytest.raises(ValueError):
        oracle.kq_map(k, (0.25, 0.0, 0.0))


def test_pair_density_kq_conserves_crystal_momentum():
    # plane waves psi_c = e^{i(k + gb).r} at k = (1/2, 0, 0) and psi_v = e^{i(k'' + ga).r} at
    # k'' = 0 = k + q - G0 with q = (1/2, 0, 0), G0 = (1, 0, 0): the matrix element is 1
    # exactly at G = ga - gb - G0 (momentum conservation) and 0 elsewhere
    k, kk, q = np.array([0.5, 0, 0]), np.zeros(3), np.array([0.5, 0, 0])
    idx, g0 = oracle.kq_map(np.array([kk, k]), q)
    assert idx[1] == 0 and tuple(g0[1]) == (1, 0, 0)
    gw_k, gw_kk = synth.wf_sphere_k(k, 2.2), synth.wf_sphere_k(kk, 2.2)
    gc = synth.chi_sphere(57, (0.5, 0, 0), np.eye(3) * 7.0)
    ga_i, gb_i = 5, 9
    cv = np.zeros((1, len(gw_kk)), dtype=np.complex128)
    cc = np.zeros((1, len(gw_k)), dtype=np.complex128)
    cv[0, ga_i] = 1.0
    cc[0, gb_i] = 1.0
    m = oracle.pair_density_kq(cv, gw_kk, cc, gw_k, g0[1], gc)[0, 0]
    want = gw_kk[ga_i] - gw_k[gb_i] - g0[1]
    for a, G in enumerate(gc):
        assert m[a] == (1.0 if np.array_equal(G, want) else 0.0)
    assert any(np.array_equal(G, want) for G in gc)


def test_chi0_ksum_gamma_only_is_chi0_bands():
    t = tiny(nv=3, nc=6)
    gw = t["gw"]
    got = oracle.chi0_ksum([t["cv"]], [t["e_v"]], [t["cc"]], [t["e_c"]], [gw], np.zeros((1, 3)), (0, 0, 0),
                           t["gc"], omegas=(0.0, 0.3), delta=0.02)
    want = oracle.chi0_bands(t["cv"], t["e_v"], t["cc"], t["e_c"], gw, t["gc"], t["nd"], (0.0, 0.3), 0.02)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_chi0_ksum_static_is_hermitian_nsd_and_label_free():
    kp = synth.kpoint_grid(2)
    b = synth.make_kbands(5, kp, 2.2, nv=3, nc=6)
    gc = synth.chi_sphere(27, (0.5, 0, 0), np.eye(3) * 7.0)
    chi = oracle.chi0_ksum(b.coef_v, b.e_v, b.coef_c, b.e_c, b.gw, kp, (0.5, 0, 0), gc)[0]
    assert np.abs(chi - chi.conj().T).max() < 1e-14 * np.abs(chi).max()
    ev = np.linalg.eigvalsh(chi)
    assert ev.max() <= 1e-12 * np.abs(ev).max()
    perm = np.random.default_rng(0).permutation(len(kp))
    sel = lambda x: [x[i] for i in perm]
    chi2 = oracle.chi0_ksum(sel(b.coef_v), sel(b.e_v), sel(b.coef_c), sel(b.e_c), sel(b.gw), kp[perm], (0.5, 0, 0),
                            gc)[0]
    assert np.abs(chi2 - chi).max() < 1e-13 * np.abs(chi).max()


# ---------------------------------------------------------------- plasmon-pole extension
def _gpp_inputs(ng=27):
    t = tiny(nd=12, rw=3, ng=ng, nv=3, nc=6)
    z, v = _static_eps_inv(t)
    half = 2 * int(np.abs(t["gc"]).max())
    box = synth.density_box(half, t["cell"], 8.0)
    rho = lambda n: box[n[0] + half, n[1] + half, n[2] + half]
    b = synth.recip(t["cell"])
    return t, z, b, rho, box[half, half, half].real


def test_gpp_static_limit_and_hermitian_density_weights():
    t, z, b, rho, rho0 = _gpp_inputs()
    om2, wt2 = oracle.gpp_modes(z, t["gc"], (0.01, 0, 0), b, rho, rho0)
    e0 = oracle.gpp_eps_inv(om2, wt2, [0.0], 0.0)[0]
    assert np.abs(e0 - z).max() < 1e-12 * np.abs(z).max()
    # the density factor is Hermitian: rho(G - G') = conj(rho(G' - G))
    r = np.array([[rho(ga - gb) for gb in t["gc"]] for ga in t["gc"]])
    assert np.abs(r - r.conj().T).max() < 1e-15


def test_gpp_homogeneous_gas_is_a_single_plasmon():
    # no density modulation: Omega^2 = w_p^2 on the diagonal and 0 elsewhere
    t, z, b, _, _ = _gpp_inputs()
    rho0 = 0.05
    om2, wt2 = oracle.gpp_modes(z, t["gc"], (0.01, 0, 0), b, lambda n: rho0 if not np.any(n) else 0.0, rho0)
    assert np.allclose(om2, 4 * np.pi * rho0 * np.eye(len(t["gc"])), rtol=1e-14, atol=1e-16)


def test_gpp_f_sum_rule():
    # -(2/pi) int_0^inf w Im eps^-1(w) dw = Omega^2 for an element with real wt^2 > 0
    t, z, b, rho, rho0 = _gpp_inputs()
    om2, wt2 = oracle.gpp_modes(z, t["gc"], (0.01, 0, 0), b, rho, rho0)
    # the most screened diagonal element (the head is unscreened here: its row of chi0 is 0)
    a = int(np.argmax((np.eye(len(z)) - z).diagonal().real))
    wt = np.sqrt(wt2[a, a].real)
    assert abs(wt2[a, a].imag) < 1e-12 * abs(wt2[a, a]) and wt2[a, a].real > 0
    eta = 1e-3 * wt
    w = np.linspace(0.0, 40.0 * wt, 400001)
    f = oracle.gpp_eps_inv(om2[a:a + 1, a:a + 1], wt2[a:a + 1, a:a + 1], w, eta)[:, 0, 0]
    integral = -(2.0 / np.pi) * np.trapezoid(w * f.imag, w)
    assert abs(integral - om2[a, a].real) < 2e-2 * abs(om2[a, a].real), (integral, om2[a, a])


def _double_commutator_weights(cell, q, gc, coef, gw):
    """Brute-force <[[T, rho_k], rho_k'^+]> (k = q+G, k' = q+G', rho_k = sum_i e^{-i k.r_i}) for
    doubly occupied orbitals phi_v = sum_g c_v(g) e^{i g.r} / sqrt(Omega), with the kinetic
    energy T, e^{-i k.r} and e^{i k'.r} as explicit sparse matrices on a plane-wave basis that
    holds the Gamma, +q and -q sectors of a Miller box around the orbitals."""
    import scipy.sparse as sp
    b = synth.recip(cell)
    q = np.asarray(q, dtype=np.float64)
    rad = int(np.abs(gw).max() + np.abs(gc).max() + 1)
    a = np.arange(-rad, rad + 1)
    box = np.stack(np.meshgrid(a, a, a, indexing="ij"), -1).reshape(-1, 3)
    nb = len(box)
    shift = {0: np.zeros(3), 1: q, -1: -q}                       # sector s holds wavevectors (m + s q) b
    key = {(s, tuple(m)): s_i * nb + i for s_i, s in enumerate((0, 1, -1)) for i, m in enumerate(box.tolist())}
    kvec = np.concatenate([(box + shift[s]) @ b for s in (0, 1, -1)])
    tmat = sp.diags(0.5 * (kvec * kvec).sum(1))

    def plane_wave_factor(frac):
        # e^{i frac.b.r} maps |(m + s q) b> to |(m + s q + frac) b>; frac = +-(q + G)
        rows, cols = [], []
        for (s, m), i in key.items():
            t = np.asarray(m, dtype=np.float64) + s * q + frac
            for s_try in (0, 1, -1):
                mm = t - s_try * q
                if np.allclose(mm, np.rint(mm), atol=1e-9):
                    j = key.get((s_try, tuple(int(x) for x in np.rint(mm))))
                    if j is not None:
                        rows.append(j)
                        cols.append(i)
                    break
        return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(3 * nb, 3 * nb))

    phis = np.zeros((coef.shape[0], 3 * nb), dtype=np.complex128)
    for j, g in enumerate(gw.tolist()):
        phis[:, key[(0, tuple(g))]] = coef[:, j]
    ng = len(gc)
    out = np.zeros((ng, ng), dtype=np.complex128)
    amat = [plane_wave_factor(-(q + g)) for g in gc.astype(np.float64)]      # e^{-i k.r}
    bmat = [plane_wave_factor(q + g) for g in gc.astype(np.float64)]         # e^{+i k'.r}
    for i in range(ng):
        for j in range(ng):
            A, B = amat[i], bmat[j]
            c = tmat @ A @ B - A @ tmat @ B - B @ tmat @ A + B @ A @ tmat
            out[i, j] = 2.0 * np.einsum("vi,vi->", np.conj(phis), (c @ phis.T).T)   # both spins
    return out


def test_gpp_weights_are_the_f_sum_double_commutator():
    # The model's pole weights come from the f-sum rule: for electrons with kinetic energy T and
    # a local potential, Omega^2_GG' = -(4 pi / |q+G|^2) <[[T, rho_{q+G}], rho_{q+G'}^+]> / Omega.
    # The double commutator is evaluated by brute force for three random orthonormal orbitals in
    # a sheared cell at a general q, and the density handed to the model is their |phi|^2
    # sampled on a real-space grid and Fourier transformed.  This fixes the off-diagonal
    # structure: which of q+G, q+G' normalises, the dot product, and G - G' against G' - G.
    cell = np.array([[7.0, 0.0, 0.0], [0.6, 7.6, 0.0], [0.0, -0.4, 8.1]])
    q = (0.13, -0.07, 0.21)
    gc = synth.chi_sphere(9, q, cell)
    gw = synth.wf_sphere(8, 2)
    coef = synth.orthonormalize(synth.gaussian_columns(99, 31, range(3), len(gw)))
    vol = abs(np.linalg.det(cell))
    nd = 12
    u = oracle.psi_real_space(coef, gw, (nd,) * 3)                 # sum_g c(g) e^{ig.r}
    rho_r = 2.0 * (np.abs(u) ** 2).sum(0) / vol
    rho_g = np.fft.fftn(rho_r) / nd ** 3                           # rho(r) = sum_K rho(K) e^{iK.r}
    rho = lambda n: rho_g[n[0] % nd, n[1] % nd, n[2] % nd]
    rho0 = rho_g[0, 0, 0].real
    assert rho0 == pytest.approx(6.0 / vol, rel=1e-13)
    z = np.eye(len(gc)) * 0.5                                       # wt^2 is not compared here
    om2, _ = oracle.gpp_modes(z, gc, q, synth.recip(cell), rho, rho0)
    dc = _double_commutator_weights(cell, q, gc, coef, gw)
    k = (gc + np.asarray(q)) @ synth.recip(cell)
    want = -4.0 * np.pi / (k * k).sum(1)[:, None] * dc / vol
    scale = np.abs(want).max()
    assert np.abs(om2 - want).max() < 1e-12 * scale
    off = ~np.eye(len(gc), dtype=bool)
    assert np.abs(want[off]).max() > 0.05 * scale                  # the off-diagonal part is tested
    # the pin separates the plausible mistakes: a transposed density, or |q+G||q+G'| in place
    # of the dot product, miss it by far more than the tolerance
    kn = np.sqrt((k * k).sum(1))
    alt = want * (kn[:, None] * kn[None, :]) / (k @ k.T)
    assert np.abs(alt - want).max() > 1e-3 * scale
    assert np.abs(want - want.T * (k * k).sum(1)[None, :] / (k * k).sum(1)[:, None]).max() > 1e-3 * scale


def test_gpp_unscreened_element_keeps_its_static_value():
    t, z, b, rho, rho0 = _gpp_inputs()
    z = z.copy()
    z[3, 3] = 1.0                                          # delta - eps^-1 = 0 exactly
    om2, wt2 = oracle.gpp_modes(z, t["gc"], (0.01, 0, 0), b, rho, rho0)
    e = oracle.gpp_eps_inv(om2, wt2, [0.0, 0.2, 1.0], 1e-3)
    assert np.all(e[:, 3, 3] == 1.0) and np.all(np.isfinite(e))


def test_chi0_ksum_energy_gradients_match_finite_differences():
    kp = synth.kpoint_grid(2)
    q = (0.5, 0.0, 0.0)
    b = synth.make_kbands(6, kp, 2.2, nv=2, nc=4)
    gc = synth.chi_sphere(19, q, np.eye(3) * 7.0)
    om, d = (0.0, 0.4), 0.05
    r = np.random.default_rng(9)
    gbar = r.standard_normal((2, 19, 19)) + 1j * r.standard_normal((2, 19, 19))

    def loss(ev, ec):
        chi = oracle.chi0_ksum(b.coef_v, ev, b.coef_c, ec, b.gw, kp, q, gc, om, d)
        return float(np.real(np.sum(np.conj(gbar) * chi)))

    gv, gcl = oracle.grad_chi0_ksum_energies(b.coef_v, b.e_v, b.coef_c, b.e_c, b.gw, kp, q, gc, gbar, om, d)
    idx, _ = oracle.kq_map(kp, q)
    h = 1e-5
    pairs = []
    for kk, i in ((0, 0), (3, 1), (6, 1)):            # valence energy of state i at k-point kk
        plus = [e.copy() for e in b.e_v]
        minus = [e.copy() for e in b.e_v]
        plus[kk][i] += h
        minus[kk][i] -= h
        fd = (loss(plus, b.e_c) - loss(minus, b.e_c)) / (2 * h)
        pairs.append((fd, sum(gv[k][i] for k in range(len(kp)) if idx[k] == kk)))
    assert_fd(pairs, "k-sum dL/dE_v")
    pairs = []
    for k, j in ((1, 0), (5, 3)):                     # conduction energy j at k-point k
        plus = [e.copy() for e in b.e_c]
        minus = [e.copy() for e in b.e_c]
        plus[k][j] += h
        minus[k][j] -= h
        pairs.append(((loss(b.e_v, plus) - loss(b.e_v, minus)) / (2 * h), gcl[k][j]))
    assert_fd(pairs, "k-sum dL/dE_c")


def test_chi0_is_the_same_on_every_alias_free_grid():
    # Eq. (chi0)'s matrix element needs only the product's components on the chi sphere to
    # be unaliased.  On the 24^3 workload (wavefunction radius 6, chi radius 4) every grid
    # with N > 2*6 + 4 gives the same chi0 up to rounding; on N = 16 the components G +- 16
    # of the product fold onto the sphere and M changes.
    from oracle import chi0 as oc
    cfg = synth.config(0)
    gw = synth.wf_sphere(cfg.nd)
    gc = synth.chi_sphere(cfg.ng[0], cfg.qs[0], cfg.cell)
    b = synth.make_bands(cfg, v_index=np.arange(4), c_index=np.arange(10), gvec_wf=gw)
    assert 2 * np.abs(gw).max() + np.abs(gc).max() == 16
    assert oc.alias_free(gw, gc, (17,) * 3) and not oc.alias_free(gw, gc, (16,) * 3)
    ref = oracle.chi0_bands(b.coef_v, b.e_v, b.coef_c, b.e_c, gw, gc, (24,) * 3)[0]
    for n in (17, 18, 20):
        got = oracle.chi0_bands(b.coef_v, b.e_v, b.coef_c, b.e_c, gw, gc, (n,) * 3)[0]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), n
    m = {n: oc.pair_density_fft(oc.psi_real_space(b.coef_v, gw, (n,) * 3),
                                oc.psi_real_space(b.coef_c, gw, (n,) * 3), gc) for n in (16, 17, 24)}
    assert np.abs(m[17] - m[24]).max() <= 1e-12 * np.abs(m[24]).max()
    assert np.abs(m[16] - m[24]).max() > 1e-3 * np.abs(m[24]).max()


# ---------------------------------------------------------------- COH self-energy with the plasmon pole
def test_sigma_coh_gpp_at_zero_energy_transfer_is_the_static_limit():
    # E - E_{n''} -> 0 (every column at the evaluation energy, no broadening): each pole term
    # becomes -Omega^2/wt^2 = eps^-1(0) - delta (the model's definition of wt^2), which is the
    # static COH term; unscreened elements (no pole) add nothing on either side
    t, z, b, rho, rho0 = _gpp_inputs()
    om2, wt2 = oracle.gpp_modes(z, t["gc"], (0.01, 0, 0), b, rho, rho0)
    v = synth.coulomb(t["gc"], (0.01, 0, 0), t["cell"])
    states = np.concatenate([t["cv"][:2], t["cc"][:1]])
    w = np.random.default_rng(2).uniform(0.5, 2.0, len(t["cc"]))
    e = 0.37
    got = oracle.sigma_coh_gpp(states, t["cc"], np.full(len(t["cc"]), e), t["gw"], t["gc"], t["nd"], om2, wt2, v,
                               [e], 0.0, n_col=w)[0]
    want = oracle.sigma_coh_static(states, t["cc"], t["gw"], t["gc"], t["nd"], z, v, n_col=w)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # away from that limit the band energies enter
    far = oracle.sigma_coh_gpp(states, t["cc"], t["e_c"], t["gw"], t["gc"], t["nd"], om2, wt2, v, [e], 0.0,
                               n_col=w)[0]
    assert np.abs(far - want).max() > 1e-2 * np.abs(want).max()


def _coh_energy_integral(om2, wt2, x, delta, eta):
    """(i / 2 pi) int_0^inf dE' ([eps^r]^-1 - [eps^a]^-1)(E') / (x - E' + i delta) for one element
    of the plasmon-pole eps^-1 with broadening eta, by adaptive quadrature (Eq. (sigmach) as
    printed, without the Coulomb factor)."""
    from scipy.integrate import quad
    wt = math.sqrt(wt2)

    def f(ep):
        ret = om2 / ((ep + 1j * eta) ** 2 - wt2)
        adv = om2 / ((ep - 1j * eta) ** 2 - wt2)
        return 1j / (2 * math.pi) * (ret - adv) / (x - ep + 1j * delta)

    pts = [wt] + ([x] if 0 < x < 200 * wt else [])
    re = quad(lambda e: f(e).real, 0.0, 200 * wt, points=pts, limit=2000, epsabs=1e-13, epsrel=1e-11)[0]
    im = quad(lambda e: f(e).imag, 0.0, 200 * wt, points=pts, limit=2000, epsabs=1e-13, epsrel=1e-11)[0]
    return re + 1j * im


def test_sigma_coh_gpp_pole_term_is_the_energy_integral():
    # the pole term per element against Eq. (sigmach)'s E' integral evaluated by quadrature with
    # the model's eps^-1 at a small broadening eta: (i/2pi) int = 1/2 A_GG'(x) (the 1/2 of the
    # self-energy's prefactor); the difference vanishes linearly with eta
    r = np.random.default_rng(21)
    om2 = r.uniform(-0.6, 0.9, (3, 3))
    wt2 = r.uniform(0.2, 1.4, (3, 3))
    v = np.ones(3)
    errs = {}
    for eta in (1e-3, 1e-4):
        worst = 0.0
        for x, delta in ((-0.4, 0.0), (-1.3, 0.0), (-0.05, 0.02), (0.35, 0.05)):
            a = oracle.gpp_coh_kernel(om2, wt2, v, x + 1j * delta)
            for i in range(3):
                for j in range(3):
                    q = _coh_energy_integral(om2[i, j], wt2[i, j], x, delta, eta)
                    worst = max(worst, abs(q - 0.5 * a[i, j]) / abs(a[i, j]))
        errs[eta] = worst
    assert errs[1e-4] < 2e-3, errs
    assert 5.0 < errs[1e-3] / errs[1e-4] < 20.0, errs


def test_sigma_coh_gpp_homogeneous_gas_closed_form():
    # plane-wave states and columns, Omega^2 = w_p^2 on the diagonal, eps^-1(0) diagonal: only
    # the column at g_n - G reaches G, so Sigma is diagonal with
    # Sigma_nn(E) = 1/2 sum_G w_{g_n - G} w_p^2 v(G) / (wt_G (E - E_{g_n - G} - wt_G))
    gw = synth.wf_sphere(12, 3)
    cell = np.eye(3) * 7.0
    gc = synth.chi_sphere(27, (0.01, 0, 0), cell)
    v = synth.coulomb(gc, (0.01, 0, 0), cell)
    ng = len(gc)
    wp2 = 4 * np.pi * 0.03
    einv = np.random.default_rng(5).uniform(0.2, 0.9, ng)
    om2 = np.full((ng, ng), 0.0, dtype=np.complex128)
    np.fill_diagonal(om2, wp2)
    z = np.diag(einv).astype(np.complex128)
    wt2 = np.full((ng, ng), np.inf + 0j)
    np.fill_diagonal(wt2, wp2 / (1.0 - einv))
    ps, pc = [0, 3, 8], [1, 2, 5, 9, 14, 20, 33, 40]
    e_cols = np.linspace(0.3, 1.4, len(pc))
    wcol = np.linspace(1.0, 2.0, len(pc))
    energies = [-0.2, 0.1]
    got = oracle.sigma_coh_gpp(synth.plane_wave_bands(gw, ps), synth.plane_wave_bands(gw, pc), e_cols, gw, gc,
                               (12,) * 3, om2, wt2, v, energies, 0.0, n_col=wcol)
    gl = [tuple(g) for g in gc.tolist()]
    for j, e in enumerate(energies):
        want = np.zeros((len(ps), len(ps)), dtype=np.complex128)
        for a, sa in enumerate(ps):
            for c, sc in enumerate(pc):
                G = tuple(gw[sa] - gw[sc])
                if G in gl:
                    k = gl.index(G)
                    wt = math.sqrt(wp2 / (1.0 - einv[k]))
                    want[a, a] += 0.5 * wcol[c] * wp2 * v[k] / (wt * (e - e_cols[c] - wt))
        assert np.abs(want).max() > 0
        assert np.abs(got[j] - want).max() < 1e-13 * np.abs(want).max()
