"""Failure paths of the set-up calls, forced from the host: GW_FAULT=alloc:N makes the N-th
device allocation of a gw_ctx_create or gw_geom_create call fail.  Each such call must return
GW_ENOMEM with a message, leave nothing behind, and leave the context usable."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def fault_env():
    old = os.environ.get("GW_FAULT")
    yield
    if old is None:
        os.environ.pop("GW_FAULT", None)
    else:
        os.environ["GW_FAULT"] = old


def test_geometry_allocation_failures_are_reported(gpu, fault_env):
    import paper_1601_06767_amd as p
    cfg = synth.config(0)
    gw = synth.wf_sphere(cfg.nd)
    gc = synth.chi_sphere(cfg.ng[0], cfg.qs[0], cfg.cell)
    ctx = p.gw_ctx_create(0)
    try:
        for n in range(1, 7):   # the six device tables of a geometry
            os.environ["GW_FAULT"] = f"alloc:{n}"
            with pytest.raises(p.GwError) as ei:
                p.gw_geom_create(ctx, (cfg.nd,) * 3, gw, gc, cfg.cell, cfg.qs[0])
            assert ei.value.status == p.GW_ENOMEM, (n, str(ei.value))
            print(f"alloc {n}: {ei.value}", flush=True)
        os.environ["GW_FAULT"] = "alloc:7"   # past the last allocation: no failure
        geom = p.gw_geom_create(ctx, (cfg.nd,) * 3, gw, gc, cfg.cell, cfg.qs[0])
        p.gw_geom_destroy(geom)
        os.environ.pop("GW_FAULT")
        geom = p.gw_geom_create(ctx, (cfg.nd,) * 3, gw, gc, cfg.cell, cfg.qs[0])
        p.gw_geom_destroy(geom)
    finally:
        p.gw_ctx_destroy(ctx)


def test_context_allocation_failures_are_reported(gpu, fault_env):
    import paper_1601_06767_amd as p
    for n in (1, 2):   # the two device flags of a context
        os.environ["GW_FAULT"] = f"alloc:{n}"
        with pytest.raises(p.GwError) as ei:
            p.gw_ctx_create(0)
        assert ei.value.status == p.GW_ENOMEM, (n, str(ei.value))
    os.environ.pop("GW_FAULT")
    ctx = p.gw_ctx_create(0)
    p.gw_ctx_destroy(ctx)
