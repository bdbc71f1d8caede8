"""Batched q-points / frequencies in one persistent contraction launch, graph capture and
replay, and the launch-shape tuner -- all checked against the oracle and against
separate eager calls."""
import numpy as np
import pytest

import oracle
import synth
from cases import Gpu, make_case, many_valence_rows, rel_err

pytestmark = pytest.mark.gpu
EV = synth.HARTREE_EV


@pytest.fixture(scope="module")
def g(gpu):
    return Gpu()


def ref_chi0(case, om, d):
    return oracle.chi0_bands(case.coef_v, case.e_v, case.coef_c, case.e_c, case.gw, case.gc, (case.nd,) * 3, om, d)


def test_batched_q_points_uneven_spheres_match_oracle_and_single_calls(g):
    # the batched workload's q-points (NG 800 ... 3000), 3 frequencies with broadening
    cases = [make_case(3, nv=4, nc=10, iq=iq) for iq in (0, 2, 5, 7)]
    om = np.array([0.0, 12.0, 33.0]) / EV
    d = 0.1 / EV
    p = g.p
    probs = [g.problem(c) for c in cases]
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5)):
        got = p.gw_chi0_build(g.ctx, probs, [len(c.gc) for c in cases], om, d, p.PRECISIONS[prec])
        g.torch.cuda.synchronize()
        for c, x in zip(cases, got):
            x = x.cpu().numpy()
            ref = ref_chi0(c, om, d)
            single = g.chi0(c, om, d, prec)
            for i in range(len(om)):
                fro, mx = rel_err(x[i], ref[i])
                assert fro <= tol and mx <= tol, (prec, len(c.gc), i, fro, mx)
                assert rel_err(x[i], single[i])[1] <= (1e-13 if prec == "fp64" else 1e-6)


def test_more_than_sixteen_problems(g):
    # 18 problems run as two batches of the persistent launch
    base = make_case(0, nv=2, nc=3)
    cases = [base] * 18
    p = g.p
    got = p.gw_chi0_build(g.ctx, [g.problem(c) for c in cases], [len(base.gc)] * 18, [0.0], 0.0, p.GW_FP64)
    ref = ref_chi0(base, [0.0], 0.0)[0]
    for x in got:
        assert rel_err(x[0].cpu().numpy(), ref)[0] <= 1e-10


def test_graph_capture_replays_match_eager(g):
    torch = g.torch
    p = g.p
    case = make_case(0, nv=6, nc=30)
    stream = torch.cuda.Stream()
    ctx = p.gw_ctx_create(0, stream)
    geom = p.gw_geom_create(ctx, (case.nd,) * 3, case.gw, case.gc, case.cfg.cell, case.q)
    cv, cc = g.t(case.coef_v), g.t(case.coef_c)
    ev, ec = g.t(case.e_v.copy()), g.t(case.e_c.copy())
    prob = p.make_problem(geom, cv, ev, cc, ec)
    ng = len(case.gc)
    om = [0.0, 5.0 / EV]
    ws = torch.empty(p.gw_chi0_workspace_size(ctx, [prob], 2, p.GW_FP64), dtype=torch.uint8, device=g.dev)
    out = torch.empty(2 * ng * ng, dtype=torch.complex128, device=g.dev)
    with torch.cuda.stream(stream):
        eager = p.gw_chi0_build(ctx, [prob], [ng], om, 0.05 / EV, p.GW_FP64, workspace=ws, out=out)[0].clone()
        p.gw_ctx_set_graph(ctx, True)
        for rep in range(3):
            if rep == 2:
                ec.add_(0.01)        # new data behind the same pointers: the replay must see it
            got = p.gw_chi0_build(ctx, [prob], [ng], om, 0.05 / EV, p.GW_FP64, workspace=ws, out=out)[0].clone()
            torch.cuda.synchronize()
            # eager work between replays
            _ = (got.abs() ** 2).sum().item()
            if rep < 2:
                assert torch.equal(got, eager)
        p.gw_ctx_set_graph(ctx, False)
        again = p.gw_chi0_build(ctx, [prob], [ng], om, 0.05 / EV, p.GW_FP64, workspace=ws, out=out)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(got, again)
    assert not torch.equal(got, eager)
    p.gw_geom_destroy(geom)
    p.gw_ctx_destroy(ctx)


def test_tuner_choices_keep_parity(g):
    p = g.p
    case = make_case(1, nv=8, nc=24)
    prob = g.problem(case)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)):
        p.gw_tune(g.ctx, [prob], 1, p.PRECISIONS[prec])
        chi = g.chi0(case, prec=prec)[0]
        ref = ref_chi0(case, [0.0], 0.0)[0]
        fro, mx = rel_err(chi, ref)
        assert fro <= tol and mx <= tol, (prec, fro, mx)


# 72^3 with NG 2600 / 3600 gives K = 17 / 19, where the lean split-line form (5) is built;
# 128^3 with NG 8000 is the 256-atom workload's K = 25 (the direct-load forms 6 and 7); the
# last three run a workload's spheres on its smaller alias-free grid (the instances (48, K 15),
# (64, K 19) and (96, K 25)) against the oracle on the stated grid
@pytest.mark.parametrize("cfg,ng,grid", [(0, None, None), (1, 300, None), (1, 2600, None), (1, 3600, None),
                                         (2, 2600, None), (4, 6500, None), (4, 8000, None), (1, 2000, 48),
                                         (2, 4000, 64), (4, 8000, 96)],
                         ids=["24cube", "72cube", "72cube-K17", "72cube-K19", "96cube", "128cube", "128cube-K25",
                              "72cube-on-48", "96cube-on-64", "128cube-on-96"])
def test_every_pair_kernel_form_matches_oracle(g, cfg, ng, grid):
    # each form of the pair kernel forced through gw_tune_set, float64 and float32, on a
    # conduction count that is not a multiple of the workgroup's 8 columns
    import dataclasses
    p = g.p
    case = make_case(cfg, nv=4, nc=13, ng=ng)
    ref = ref_chi0(case, [0.0], 0.0)[0]
    if grid is not None:
        case = dataclasses.replace(case, nd=grid)
    prob = g.problem(case)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5)):
        for form in (1, 2, 3, 4, 5, 6, 7):
            p.gw_tune_set(g.ctx, prob, p.PRECISIONS[prec], form, 0)
            assert p.gw_tune_get(g.ctx, prob, p.PRECISIONS[prec]) == (form, 0)
            chi = g.chi0(case, prec=prec)[0]
            fro, mx = rel_err(chi, ref)
            assert fro <= tol and mx <= tol, (prec, form, fro, mx)
        p.gw_tune_set(g.ctx, prob, p.PRECISIONS[prec], 0, 0)
        assert p.gw_tune_get(g.ctx, prob, p.PRECISIONS[prec]) == (0, 0)
    with pytest.raises(p.GwError):
        p.gw_tune_set(g.ctx, prob, p.GW_FP64, 8, 0)
    with pytest.raises(p.GwError):
        p.gw_tune_set(g.ctx, prob, p.GW_FP64, 1, 33)


@pytest.mark.parametrize("om,d", [((0.0,), 0.0), ((0.0, 7.0), 0.1)], ids=["static", "dynamic"])
def test_contraction_splits_keep_parity(g, om, d):
    # the pair range of each contraction tile split 1..32 ways (ranges are whole 16-pair
    # stages, so the larger splits leave empty ranges), in every precision
    p = g.p
    case = make_case(0, nv=6, nc=21)
    prob = g.problem(case)
    om = np.asarray(om) / EV
    ref = ref_chi0(case, om, d / EV)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)):
        for ks in (1, 3, 7, 32):
            p.gw_tune_set(g.ctx, prob, p.PRECISIONS[prec], 0, ks)
            chi = g.chi0(case, om, d / EV, prec)
            for i in range(len(om)):
                fro, mx = rel_err(chi[i], ref[i])
                assert fro <= tol and mx <= tol, (prec, ks, i, fro, mx)
        p.gw_tune_set(g.ctx, prob, p.PRECISIONS[prec], 0, 0)


def _build(g, ctx, probs, ngs, om, d, prec, ws):
    p = g.p
    out = p.gw_chi0_build(ctx, probs, ngs, om, d, p.PRECISIONS[prec], workspace=ws)
    g.torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


@pytest.mark.parametrize("om,d", [((0.0,), 0.0), ((0.0, 7.0), 0.1)], ids=["static", "dynamic"])
def test_chunk_overlap_is_bitwise_neutral_and_matches_oracle(g, om, d):
    # 400 valence rows make the conduction chunk 80 columns: three chunks of 240, so the
    # contraction of one chunk overlaps the transforms of the next and a buffer is reused
    p = g.p
    torch = g.torch
    case = many_valence_rows(make_case(0), 400)
    prob = g.problem(case)
    ng = len(case.gc)
    om = np.asarray(om) / EV
    ref = ref_chi0(case, om, d / EV)
    for prec, tol in (("fp64", 1e-10), ("fp32", 2e-5), ("bf16x3", 1e-4)):
        ws = torch.empty(p.gw_chi0_workspace_size(g.ctx, [prob], len(om), p.PRECISIONS[prec]), dtype=torch.uint8,
                         device=g.dev)
        p.gw_ctx_set_overlap(g.ctx, 0)
        seq = _build(g, g.ctx, [prob], [ng], om, d / EV, prec, ws)[0]
        p.gw_ctx_set_overlap(g.ctx, 2)
        ovl = _build(g, g.ctx, [prob], [ng], om, d / EV, prec, ws)[0]
        p.gw_ctx_set_overlap(g.ctx, 1)
        auto = _build(g, g.ctx, [prob], [ng], om, d / EV, prec, ws)[0]
        assert np.array_equal(seq, ovl) and np.array_equal(seq, auto), prec
        for iw in range(len(om)):
            fro, mx = rel_err(ovl[iw], ref[iw])
            assert fro <= tol and mx <= tol, (prec, iw, fro, mx)


def test_chunk_overlap_with_several_problems_and_graph_replay(g):
    # two q-points with different dielectric spheres, three chunks each, in eager mode and
    # replayed from a captured graph (with eager work between the replays)
    p = g.p
    torch = g.torch
    cases = [many_valence_rows(make_case(0, ng=ng), 400) for ng in (259, 150)]
    stream = torch.cuda.Stream()
    ctx = p.gw_ctx_create(0, stream)
    geoms = [p.gw_geom_create(ctx, (c.nd,) * 3, c.gw, c.gc, c.cfg.cell, c.q) for c in cases]
    probs = [p.make_problem(gm, g.t(c.coef_v), g.t(c.e_v), g.t(c.coef_c), g.t(c.e_c)) for gm, c in zip(geoms, cases)]
    ngs = [len(c.gc) for c in cases]
    om = [0.0, 3.0 / EV]
    d = 0.1 / EV
    ws = torch.empty(p.gw_chi0_workspace_size(ctx, probs, 2, p.GW_FP64), dtype=torch.uint8, device=g.dev)
    with torch.cuda.stream(stream):
        p.gw_ctx_set_overlap(ctx, 0)
        seq = _build(g, ctx, probs, ngs, om, d, "fp64", ws)
        p.gw_ctx_set_overlap(ctx, 2)
        eager = _build(g, ctx, probs, ngs, om, d, "fp64", ws)
        for a, b in zip(seq, eager):
            assert np.array_equal(a, b)
        out = torch.empty(sum(2 * n * n for n in ngs), dtype=torch.complex128, device=g.dev)
        p.gw_ctx_set_graph(ctx, True)
        for rep in range(3):
            got = p.gw_chi0_build(ctx, probs, ngs, om, d, p.GW_FP64, workspace=ws, out=out)
            torch.cuda.synchronize()
            _ = (out.abs() ** 2).sum().item()
            for a, b in zip(got, eager):
                assert np.array_equal(a.cpu().numpy(), b), rep
        p.gw_ctx_set_graph(ctx, False)
    for c, e in zip(cases, eager):
        ref = ref_chi0(c, om, d)
        for iw in range(2):
            fro, mx = rel_err(e[iw], ref[iw])
            assert fro <= 1e-10 and mx <= 1e-10, (iw, fro, mx)
    with pytest.raises(p.GwError):
        p.gw_ctx_set_overlap(ctx, 3)
    for gm in geoms:
        p.gw_geom_destroy(gm)
    p.gw_ctx_destroy(ctx)


def test_graph_cache_drops_the_graphs_of_a_destroyed_geometry(g):
    # graph mode keys a capture by its arguments; a geometry destroyed and recreated (possibly at
    # the same host address) with another sphere size must get a capture of its own
    torch = g.torch
    p = g.p
    case = make_case(0, nv=6, nc=30)
    small = make_case(0, nv=6, nc=30, ng=150)
    stream = torch.cuda.Stream()
    ctx = p.gw_ctx_create(0, stream)
    cv, cc = g.t(case.coef_v), g.t(case.coef_c)
    ev, ec = g.t(case.e_v.copy()), g.t(case.e_c.copy())
    ng = len(case.gc)
    out = torch.zeros(ng * ng, dtype=torch.complex128, device=g.dev)
    results = []
    with torch.cuda.stream(stream):
        p.gw_ctx_set_graph(ctx, True)
        for c in (case, small, case):
            geom = p.gw_geom_create(ctx, (c.nd,) * 3, c.gw, c.gc, c.cfg.cell, c.q)
            prob = p.make_problem(geom, cv, ev, cc, ec)
            ws = torch.empty(p.gw_chi0_workspace_size(ctx, [prob], 1, p.GW_FP64), dtype=torch.uint8, device=g.dev)
            n = len(c.gc)
            for _ in range(2):   # capture, then replay
                chi = p.gw_chi0_build(ctx, [prob], [n], [0.0], 0.0, p.GW_FP64, workspace=ws, out=out)[0][0]
                results.append(chi.clone())
            torch.cuda.synchronize()
            p.gw_geom_destroy(geom)
        p.gw_ctx_set_graph(ctx, False)
    torch.cuda.synchronize()
    p.gw_ctx_destroy(ctx)
    for i, c in enumerate((case, small, case)):
        ref = ref_chi0(c, [0.0], 0.0)[0]
        for r in results[2 * i: 2 * i + 2]:
            assert r.shape == ref.shape
            assert rel_err(r.cpu().numpy(), ref)[0] <= 1e-10
