"""GPU parity of the k-point sum of Eq. (chi0) (gw_chi0_build_ksum with the k+q mapping)
against the oracle's plane-wave convolution over each k-point's own sphere."""
import numpy as np
import pytest

import oracle
import synth
from cases import Gpu

pytestmark = pytest.mark.gpu
EV = synth.HARTREE_EV


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def union_sphere(spheres):
    u = np.unique(np.concatenate(spheres), axis=0)
    d = (u * u).sum(1)
    return np.ascontiguousarray(u[np.lexsort((u[:, 2], u[:, 1], u[:, 0], d))].astype(np.int32))


def embed(rows, gw, u):
    pos = {tuple(x): i for i, x in enumerate(u.tolist())}
    out = np.zeros((rows.shape[0], len(u)), dtype=np.complex128)
    out[:, [pos[tuple(x)] for x in gw.tolist()]] = rows
    return out


def ksum_case(g, n, q, ng, radius=5.0, nv=4, nc=12, seed=7, relabel=False):
    """One problem per k: valence rows of k'' = k + q - G0 either relabelled to k + q (one
    geometry, dielectric sphere G) or as stored (dielectric sphere shifted to G + G0)."""
    kp = synth.kpoint_grid(n)
    b = synth.make_kbands(seed, kp, radius, nv, nc)
    gc = synth.chi_sphere(ng, q, np.eye(3) * 8.4)
    idx, g0 = g.p.gw_kq_map(kp, q)
    vsph = [b.gw[idx[k]] - g0[k] if relabel else b.gw[idx[k]] for k in range(len(kp))]
    u = union_sphere(list(b.gw) + vsph)
    geoms = {}
    probs = []
    for k in range(len(kp)):
        key = () if relabel else tuple(g0[k])
        if key not in geoms:
            sphere = gc if relabel else gc + g0[k]
            geoms[key] = g.p.gw_geom_create(g.ctx, (24, 24, 24), u, sphere.astype(np.int32))
        kk = idx[k]
        probs.append(g.p.make_problem(geoms[key], g.t(embed(b.coef_v[kk], vsph[k], u)), g.t(b.e_v[kk]),
                                      g.t(embed(b.coef_c[k], b.gw[k], u)), g.t(b.e_c[k])))
    return kp, b, gc, probs, geoms


@pytest.mark.parametrize("n,q,omegas,delta,relabel", [(2, (0.5, 0.0, 0.0), (0.0,), 0.0, False),
                                                      (2, (0.5, 0.5, 0.0), (0.0, 6.0), 0.1, False),
                                                      (3, (1 / 3, 0.0, 0.0), (0.0,), 0.0, False),
                                                      (2, (0.5, 0.5, 0.0), (0.0, 6.0), 0.1, True),
                                                      (3, (1 / 3, 2 / 3, 0.0), (0.0,), 0.0, True)],
                         ids=["2cube-static", "2cube-dynamic", "3cube-27k-two-batches", "2cube-dynamic-relabelled",
                              "3cube-relabelled"])
def test_ksum_matches_oracle(g, n, q, omegas, delta, relabel):
    kp, b, gc, probs, geoms = ksum_case(g, n, q, 59, relabel=relabel)
    om = np.asarray(omegas) / EV
    got = g.p.gw_chi0_build_ksum(g.ctx, probs, len(gc), om, delta / EV, g.p.GW_FP64)
    g.torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle.chi0_ksum(b.coef_v, b.e_v, b.coef_c, b.e_c, b.gw, kp, q, gc, om, delta / EV)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-10, err
    if delta == 0.0 and len(omegas) == 1:
        assert np.linalg.eigvalsh(0.5 * (got[0] + got[0].conj().T)).max() <= 1e-12 * np.abs(got).max()
    for gm in geoms.values():
        g.p.gw_geom_destroy(gm)


def test_ksum_of_one_problem_is_the_build(g):
    kp, b, gc, probs, geoms = ksum_case(g, 2, (0.5, 0.0, 0.0), 59)
    one = g.p.gw_chi0_build_ksum(g.ctx, probs[:1], len(gc), [0.0], 0.0, g.p.GW_FP64)
    ref = g.p.gw_chi0_build(g.ctx, probs[:1], [len(gc)], [0.0], 0.0, g.p.GW_FP64)[0]
    g.torch.cuda.synchronize()
    assert g.torch.equal(one, ref)
    other = g.p.gw_geom_create(g.ctx, (24, 24, 24), union_sphere(b.gw), gc[:50])
    bad = g.p.make_problem(other, g.t(embed(b.coef_v[0], b.gw[0], union_sphere(b.gw))), g.t(b.e_v[0]),
                           g.t(embed(b.coef_c[0], b.gw[0], union_sphere(b.gw))), g.t(b.e_c[0]))
    with pytest.raises(g.p.GwError):
        g.p.gw_chi0_build_ksum(g.ctx, [probs[0], bad], len(gc), [0.0], 0.0, g.p.GW_FP64)
    for gm in list(geoms.values()) + [other]:
        g.p.gw_geom_destroy(gm)


@pytest.mark.parametrize("omegas,delta", [((0.0,), 0.0), ((0.0, 6.0), 0.1)], ids=["static", "dynamic"])
def test_ksum_backward_matches_oracle(g, omegas, delta):
    q = (0.5, 0.0, 0.0)
    kp, b, gc, probs, geoms = ksum_case(g, 2, q, 59)
    om = np.asarray(omegas) / EV
    r = np.random.default_rng(8)
    gbar = r.standard_normal((len(om), len(gc), len(gc))) + 1j * r.standard_normal((len(om), len(gc), len(gc)))
    gev, gec, _ = g.p.gw_chi0_backward(g.ctx, probs, om, delta / EV, g.p.GW_FP64,
                                       g.torch.from_numpy(gbar).to(g.dev), ksum=True)
    g.torch.cuda.synchronize()
    gv, gcl = oracle.grad_chi0_ksum_energies(b.coef_v, b.e_v, b.coef_c, b.e_c, b.gw, kp, q, gc, gbar, om, delta / EV)
    want_v, want_c = np.concatenate(gv), np.concatenate(gcl)
    got_v, got_c = gev.cpu().numpy(), gec.cpu().numpy()
    assert np.abs(got_v - want_v).max() <= 1e-10 * np.abs(want_v).max()
    assert np.abs(got_c - want_c).max() <= 1e-10 * np.abs(want_c).max()
    for gm in geoms.values():
        g.p.gw_geom_destroy(gm)
