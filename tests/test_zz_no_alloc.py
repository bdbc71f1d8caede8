"""The allocation-free inverse (gw_eps_inv_noalloc) against the workspace entry point
(gw_eps_inv): the same kernels, so the same bits; two calls in a row, the second smaller, a
batched call, and the size limit.  Collected last (a failure here must not hide the others)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _chi(n, seed, herm):
    r = np.random.default_rng(seed)
    a = (r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))) / np.sqrt(n)
    return -(a @ a.conj().T) / 4.0 if herm else a


def test_eps_inv_noalloc_matches_the_workspace_entry_point(gpu):
    import torch
    import paper_1601_06767_amd as p
    dev = torch.device("cuda", 0)
    ctx = p.gw_ctx_create(0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    cfg = synth.config(4)
    try:
        # the largest size, then smaller ones, with both routes of the inverse
        for n, herm, route in ((2048, True, True), (2048, True, False), (700, False, False), (500, True, True)):
            chi = _chi(n, n, herm)
            v = synth.coulomb(synth.chi_sphere(n, cfg.qs[0], cfg.cell), cfg.qs[0], cfg.cell) if herm else \
                np.random.default_rng(n).uniform(0.5, 3.0, n)
            vd, cd = t(v), t(chi)
            want = p.gw_eps_inv(ctx, vd, cd, hermitian=route)
            out = torch.full((n, n), np.nan, dtype=torch.complex128, device=dev)
            got = p.gw_eps_inv_noalloc(ctx, vd, cd, out, hermitian=route)
            p.gw_eps_inv_status(ctx)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (n, route)
            ref = oracle.eps_inv(chi, v)
            err = float(np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max())
            print(f"n={n} hermitian={route}: identical to gw_eps_inv; {err:.1e} from LAPACK")
            assert err <= 1e-11
        # a batch of three in one call reuses the scratch for each matrix
        chis = np.stack([_chi(300, 40 + i, i % 2 == 0) for i in range(3)])
        vs = np.random.default_rng(3).uniform(0.5, 2.0, (3, 300))
        want = p.gw_eps_inv(ctx, t(vs), t(chis))
        out = torch.empty((3, 300, 300), dtype=torch.complex128, device=dev)
        got = p.gw_eps_inv_noalloc(ctx, t(vs), t(chis), out)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        # beyond the static scratch: refused before any launch
        big = torch.zeros((2049, 2049), dtype=torch.complex128, device=dev)
        with pytest.raises(p.GwError, match="allocation-free maximum"):
            p.gw_eps_inv_noalloc(ctx, torch.ones(2049, dtype=torch.float64, device=dev), big, torch.empty_like(big))
    finally:
        p.gw_ctx_destroy(ctx)
