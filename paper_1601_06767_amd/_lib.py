"""ctypes binding of libgwchi0.so (argument marshalling only).

The functions keep the names of the C ABI in include/gwchi0.h and take torch
tensors for device buffers; every computation runs in the library's HIP kernels.
The library must have been built (``python paper_1601_06767_amd/build.py``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwchi0.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE, GW_ESINGULAR, GW_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GW_FP64, GW_FP32, GW_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "bf16x3": GW_BF16X3}
STATUS_NAMES = {0: "GW_OK", -1: "GW_EINVAL", -2: "GW_ENOMEM", -3: "GW_EDEVICE", -4: "GW_ESINGULAR",
                -5: "GW_EUNSUPPORTED"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1601_06767_amd/build.py`")
lib = C.CDLL(LIB_PATH)

vp = C.c_void_p
i32p = C.POINTER(C.c_int32)
dp = C.POINTER(C.c_double)


class gw_chi0_problem(C.Structure):
    _fields_ = [("geom", vp), ("nv", C.c_int), ("coef_v", vp), ("e_v", vp), ("nband", C.c_int), ("coef_c", vp),
                ("ncol", C.c_int), ("col_band", vp), ("e_col", vp), ("n_col", vp)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("gw_version", C.c_char_p, [])
_sig("gw_ctx_create", C.c_int, [C.c_int, vp, C.POINTER(vp)])
_sig("gw_ctx_destroy", C.c_int, [vp])
_sig("gw_last_error", C.c_char_p, [vp])
_sig("gw_geom_create", C.c_int, [vp, C.POINTER(C.c_int), dp, dp, C.c_int, i32p, C.c_int, i32p, C.POINTER(vp)])
_sig("gw_geom_destroy", C.c_int, [vp])
_sig("gw_sphere_check", C.c_int, [dp, dp, C.c_int, i32p, C.c_char_p, C.c_size_t])
_sig("gw_chi0_workspace_size", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, C.c_int,
                                         C.POINTER(C.c_size_t)])
_sig("gw_chi0_build", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, dp, C.c_double, C.c_int, vp,
                                C.c_size_t, vp])
_sig("gw_chi0_backward", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, dp, C.c_double, C.c_int,
                                   vp, C.c_size_t, vp, vp, vp, vp, vp, vp])
_sig("gw_chi0_backward_ksum", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, dp, C.c_double, C.c_int,
                                   vp, C.c_size_t, vp, vp, vp, vp, vp, vp])
_sig("gw_pair_density_workspace_size", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, C.c_int,
                                                 C.POINTER(C.c_size_t)])
_sig("gw_pair_density", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                  vp, C.c_size_t, vp])
_sig("gw_eps_inv_workspace_size", C.c_int, [vp, C.c_int, C.c_int, C.POINTER(C.c_size_t)])
_sig("gw_eps_inv", C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, C.c_size_t, vp])
_sig("gw_eps_inv_status", C.c_int, [vp])
_sig("gw_eps_inv_noalloc", C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp])
_sig("gw_eps_inv_backward", C.c_int, [vp, C.c_int, C.c_int, vp, vp, vp, vp, C.c_size_t, vp])
_sig("gw_group_windows", C.c_int, [C.c_int, dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                   i32p, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_int)])
_sig("gw_group_windows_edges", C.c_int, [C.c_int, dp, C.c_int, dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                          i32p, dp, dp, C.POINTER(C.c_int), C.POINTER(C.c_int)])

_sig("gw_ctx_set_timing", C.c_int, [vp, C.c_int])
_sig("gw_ctx_set_graph", C.c_int, [vp, C.c_int])
_sig("gw_tune", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, C.c_int, vp, C.c_size_t])
_sig("gw_tune_get", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)])
_sig("gw_tune_set", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, C.c_int])
_sig("gw_ctx_set_overlap", C.c_int, [vp, C.c_int])
_sig("gw_sigma_coh_workspace_size", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.POINTER(C.c_size_t)])
_sig("gw_chi0_build_ksum", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int, dp, C.c_double, C.c_int, vp,
                                     C.c_size_t, vp])
_sig("gw_kq_map", C.c_int, [C.c_int, dp, dp, C.c_double, i32p, i32p])
_sig("gw_gpp_workspace_size", C.c_int, [vp, C.c_int, C.c_int, C.POINTER(C.c_size_t)])
_sig("gw_gpp_eps_inv", C.c_int, [vp, C.c_int, i32p, dp, dp, C.c_int, vp, vp, C.c_int, dp, C.c_double, vp, C.c_size_t,
                                 vp, vp])
_sig("gw_sigma_coh_static", C.c_int, [vp, C.POINTER(gw_chi0_problem), vp, vp, vp, C.c_size_t, vp])
_sig("gw_ctx_stage_times", C.c_int, [vp, dp, C.POINTER(C.c_longlong), C.c_int])
_sig("gw_sigma_coh_gpp_workspace_size", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.c_int,
                                                  C.POINTER(C.c_size_t)])
_sig("gw_sigma_coh_gpp", C.c_int, [vp, C.POINTER(gw_chi0_problem), C.c_int, C.POINTER(vp), C.POINTER(vp), C.c_int, dp,
                                   C.c_double, vp, C.c_size_t, vp])

STAGES = ["band", "planes", "finish", "weights", "contract", "finalize", "eps_inv", "backward"]

EXPORTED = ["gw_ctx_set_timing", "gw_ctx_stage_times", "gw_ctx_set_graph", "gw_tune", "gw_tune_get", "gw_tune_set", "gw_ctx_set_overlap", "gw_group_windows_edges",
            "gw_sigma_coh_workspace_size", "gw_sigma_coh_static", "gw_chi0_build_ksum", "gw_chi0_backward_ksum", "gw_kq_map",
            "gw_gpp_workspace_size", "gw_gpp_eps_inv",
            "gw_version", "gw_ctx_create", "gw_ctx_destroy", "gw_last_error", "gw_geom_create", "gw_geom_destroy",
            "gw_chi0_workspace_size", "gw_chi0_build", "gw_chi0_backward", "gw_pair_density_workspace_size", "gw_pair_density",
            "gw_eps_inv_workspace_size", "gw_eps_inv", "gw_eps_inv_status", "gw_eps_inv_backward",
            "gw_group_windows", "gw_sphere_check", "gw_sigma_coh_gpp_workspace_size", "gw_sigma_coh_gpp", "gw_eps_inv_noalloc"]


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, ctx=None):
    if status != GW_OK:
        m = lib.gw_last_error(ctx)
        raise GwError(status, m.decode() if m else "")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def gw_version() -> str:
    return lib.gw_version().decode()


# ---------------------------------------------------------------- context / geometry
def gw_ctx_create(device: int = 0, stream=None):
    """Context on `device` enqueueing on `stream` (a torch.cuda.Stream; default: torch's current stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    out = vp()
    _check(lib.gw_ctx_create(device, vp(stream.cuda_stream), C.byref(out)), None)
    return out


def gw_ctx_destroy(ctx) -> None:
    _check(lib.gw_ctx_destroy(ctx))


def gw_last_error(ctx=None) -> str:
    return lib.gw_last_error(ctx).decode()


def gw_ctx_set_timing(ctx, enable: bool) -> None:
    _check(lib.gw_ctx_set_timing(ctx, 1 if enable else 0), ctx)


def gw_ctx_set_graph(ctx, enable: bool) -> None:
    _check(lib.gw_ctx_set_graph(ctx, 1 if enable else 0), ctx)


def gw_tune(ctx, problems, nomega: int, prec: int, workspace=None) -> None:
    import torch
    arr = _probs(problems)
    if workspace is None:
        workspace = torch.empty(gw_chi0_workspace_size(ctx, arr, nomega, prec), dtype=torch.uint8,
                                device=torch.device("cuda", torch.cuda.current_device()))
    _check(lib.gw_tune(ctx, arr, len(arr), nomega, prec, _ptr(workspace), workspace.numel()), ctx)


def gw_ctx_set_overlap(ctx, mode: int) -> None:
    """Chunk overlap of gw_chi0_build on a second stream: 0 off, 1 where it pays (default,
    dynamic split-BF16x3 builds at NG <= 2048), 2 always."""
    _check(lib.gw_ctx_set_overlap(ctx, int(mode)), ctx)


def gw_tune_set(ctx, problem, prec: int, pair_variant: int, ksplit: int) -> None:
    """Sets the tuned shapes for this problem's shape (0 = automatic; both 0 forgets it)."""
    _check(lib.gw_tune_set(ctx, C.byref(problem), prec, int(pair_variant), int(ksplit)), ctx)


def gw_tune_get(ctx, problem, prec: int):
    """(pair-kernel form, contraction splits) tuned for this problem's shape, (0, 0) if untuned."""
    a, b = C.c_int(), C.c_int()
    _check(lib.gw_tune_get(ctx, C.byref(problem), prec, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def gw_ctx_stage_times(ctx, reset: bool = False) -> dict:
    """{stage: (milliseconds, launch groups)} accumulated while timing was on."""
    ms = (C.c_double * 8)()
    n = (C.c_longlong * 8)()
    _check(lib.gw_ctx_stage_times(ctx, ms, n, 1 if reset else 0), ctx)
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


def gw_geom_create(ctx, n_fft: Sequence[int], gvec_wf: np.ndarray, gvec_chi: np.ndarray, cell=None, q=None):
    """Geometry of one q-point; with cell (3 x 3, rows = lattice vectors, bohr) and q (reciprocal-lattice
    units) the library checks that gvec_chi is the sphere ordered by (|q+G|^2, n1, n2, n3)."""
    gw_ = np.ascontiguousarray(gvec_wf, dtype=np.int32)
    gc = np.ascontiguousarray(gvec_chi, dtype=np.int32)
    nf = (C.c_int * 3)(*[int(x) for x in n_fft])
    if (cell is None) != (q is None):
        raise ValueError("give both cell and q, or neither")
    cl = None if cell is None else np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    qq = None if q is None else np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(3))
    out = vp()
    _check(lib.gw_geom_create(ctx, nf, None if cl is None else cl.ctypes.data_as(dp),
                              None if qq is None else qq.ctypes.data_as(dp), gw_.shape[0], gw_.ctypes.data_as(i32p),
                              gc.shape[0], gc.ctypes.data_as(i32p), C.byref(out)), ctx)
    _npw[out.value] = int(gw_.shape[0])
    return out


_npw = {}   # wavefunction-sphere size per geometry handle


def _geom_npw(geom) -> int:
    return _npw[geom if isinstance(geom, int) else geom.value]


def gw_sphere_check(cell, q, gvec_chi: np.ndarray) -> str:
    """'' if gvec_chi is the sphere ordered by (|q+G|^2, n1, n2, n3) for this cell and q, else the reason."""
    cl = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    qq = np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(3))
    gc = np.ascontiguousarray(gvec_chi, dtype=np.int32)
    buf = C.create_string_buffer(256)
    st = lib.gw_sphere_check(cl.ctypes.data_as(dp), qq.ctypes.data_as(dp), gc.shape[0], gc.ctypes.data_as(i32p), buf,
                             256)
    if st == GW_OK:
        return ""
    if st != GW_EINVAL or not buf.value:
        raise GwError(st, "bad arguments")
    return buf.value.decode()


def gw_geom_destroy(geom) -> None:
    _check(lib.gw_geom_destroy(geom))


# ---------------------------------------------------------------- problems
def make_problem(geom, coef_v, e_v, coef_c, e_col, n_col=None, col_band=None) -> gw_chi0_problem:
    """Problem record over torch device tensors (complex128 coefficients, float64 energies, int32 col_band)."""
    for t in (coef_v, coef_c):
        assert t.dtype.is_complex and t.element_size() == 16 and t.is_contiguous()
    rec = gw_chi0_problem(geom, coef_v.shape[0], _ptr(coef_v), _ptr(e_v), coef_c.shape[0], _ptr(coef_c),
                          e_col.shape[0], _ptr(col_band), _ptr(e_col), _ptr(n_col))
    # the record holds raw device pointers: keep the tensors alive as long as the record
    rec._tensors = (coef_v, e_v, coef_c, e_col, n_col, col_band)
    return rec


def _probs(problems) -> "C.Array":
    if isinstance(problems, gw_chi0_problem):
        problems = [problems]
    arr = (gw_chi0_problem * len(problems))(*problems)
    return arr


def gw_chi0_workspace_size(ctx, problems, nomega: int, prec: int) -> int:
    arr = _probs(problems)
    n = C.c_size_t()
    _check(lib.gw_chi0_workspace_size(ctx, arr, len(arr), nomega, prec, C.byref(n)), ctx)
    return n.value


def gw_chi0_build(ctx, problems, ngs: Sequence[int], omegas: Sequence[float], delta: float, prec: int,
                  workspace=None, out=None):
    """chi0 for each problem: returns a list of (nomega, ng, ng) complex128 tensors (views of one buffer)."""
    import torch
    arr = _probs(problems)
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        workspace = torch.empty(gw_chi0_workspace_size(ctx, arr, len(om), prec), dtype=torch.uint8, device=dev)
    total = sum(len(om) * g * g for g in ngs)
    if out is None:
        out = torch.empty(total, dtype=torch.complex128, device=dev)
    _check(lib.gw_chi0_build(ctx, arr, len(arr), len(om), om.ctypes.data_as(dp), float(delta), prec,
                             _ptr(workspace), workspace.numel(), _ptr(out)), ctx)
    res, o = [], 0
    for g in ngs:
        res.append(out[o: o + len(om) * g * g].view(len(om), g, g))
        o += len(om) * g * g
    return res


def gw_chi0_build_ksum(ctx, problems, ng: int, omegas: Sequence[float], delta: float, prec: int, workspace=None,
                       out=None):
    """k-point sum of chi0 over the problems (one per k, same ng): (nomega, ng, ng) complex128."""
    import torch
    arr = _probs(problems)
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        workspace = torch.empty(gw_chi0_workspace_size(ctx, arr, len(om), prec), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((len(om), ng, ng), dtype=torch.complex128, device=dev)
    _check(lib.gw_chi0_build_ksum(ctx, arr, len(arr), len(om), om.ctypes.data_as(dp), float(delta), prec,
                                  _ptr(workspace), workspace.numel(), _ptr(out)), ctx)
    return out


def gw_gpp_eps_inv(ctx, gvec_chi: np.ndarray, q, bvec: np.ndarray, rho_box, eps_inv_static, omegas, eta: float,
                   want_modes: bool = False):
    """Plasmon-pole eps^-1(w) (nomega, ng, ng) from the static eps^-1 and the density box
    rho_box (device complex128 (2h+1)^3); with want_modes also (Omega^2, wt^2)."""
    import torch
    g = np.ascontiguousarray(gvec_chi, dtype=np.int32)
    ng = g.shape[0]
    qq = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
    b = np.ascontiguousarray(bvec, dtype=np.float64).reshape(9)
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    w = rho_box.shape[0]
    dev = torch.device("cuda", torch.cuda.current_device())
    n = C.c_size_t()
    _check(lib.gw_gpp_workspace_size(ctx, ng, len(om), C.byref(n)), ctx)
    ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
    out = torch.empty((len(om), ng, ng), dtype=torch.complex128, device=dev)
    modes = torch.empty((2, ng, ng), dtype=torch.complex128, device=dev) if want_modes else None
    _check(lib.gw_gpp_eps_inv(ctx, ng, g.ctypes.data_as(i32p), qq.ctypes.data_as(dp), b.ctypes.data_as(dp), (w - 1) // 2,
                              _ptr(rho_box.contiguous()), _ptr(eps_inv_static.contiguous()), len(om),
                              om.ctypes.data_as(dp), float(eta), _ptr(ws), ws.numel(), _ptr(modes), _ptr(out)), ctx)
    return (out, modes) if want_modes else out


def gw_kq_map(kpts: np.ndarray, q, tol: float = 1e-8):
    """(kq_index int32 (nk,), g0 int32 (nk, 3)) with k + q = kpts[kq_index] + g0."""
    k = np.ascontiguousarray(kpts, dtype=np.float64).reshape(-1, 3)
    qq = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
    idx = np.zeros(len(k), dtype=np.int32)
    g0 = np.zeros((len(k), 3), dtype=np.int32)
    st = lib.gw_kq_map(len(k), k.ctypes.data_as(dp), qq.ctypes.data_as(dp), float(tol), idx.ctypes.data_as(i32p),
                       g0.ctypes.data_as(i32p))
    if st != GW_OK:
        raise GwError(st, "gw_kq_map: some k + q is not on the k-point set")
    return idx, g0


def gw_chi0_backward(ctx, problems, omegas: Sequence[float], delta: float, prec: int, grad_chi0, workspace=None,
                     want=(True, True, True), coef=(False, False), ksum: bool = False):
    """(dL/dE_v, dL/dE_col, dL/dn_col[, dL/dcoef_v, dL/dcoef_c]) over all problems
    (concatenated tensors, None where not wanted) from grad_chi0 in gw_chi0_build's output
    layout (with ksum: gw_chi0_build_ksum's single block, shared by every problem).  The coefficient gradients (float64 mode) are complex128, shaped like the
    concatenated coefficient rows (sum of nv x npw, sum of nband x npw) and returned only
    when one of them is asked for."""
    import torch
    arr = _probs(problems)
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        workspace = torch.empty(gw_chi0_workspace_size(ctx, arr, len(om), prec), dtype=torch.uint8, device=dev)
    nv = sum(p.nv for p in arr)
    nc = sum(p.ncol for p in arr)
    g = [torch.zeros(n, dtype=torch.float64, device=dev) if w else None for n, w in zip((nv, nc, nc), want)]
    gcoef = [None, None]
    if any(coef):
        npw = [_geom_npw(p.geom) for p in arr]
        rows = (sum(p.nv * n for p, n in zip(arr, npw)), sum(p.nband * n for p, n in zip(arr, npw)))
        gcoef = [torch.empty(r, dtype=torch.complex128, device=dev) if w else None for r, w in zip(rows, coef)]
    gc = grad_chi0.contiguous()
    fn = lib.gw_chi0_backward_ksum if ksum else lib.gw_chi0_backward
    _check(fn(ctx, arr, len(arr), len(om), om.ctypes.data_as(dp), float(delta), prec, _ptr(workspace),
              workspace.numel(), _ptr(gc), _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(gcoef[0]), _ptr(gcoef[1])), ctx)
    if any(coef):
        return tuple(g) + tuple(gcoef)
    return tuple(g)


def gw_pair_density_workspace_size(ctx, problem, nvs: int, ncs: int, prec: int) -> int:
    n = C.c_size_t()
    _check(lib.gw_pair_density_workspace_size(ctx, C.byref(problem), nvs, ncs, prec, C.byref(n)), ctx)
    return n.value


def gw_pair_density(ctx, problem, v0: int, nvs: int, c0: int, ncs: int, ng: int, prec: int, workspace=None):
    """M_vc(G) for v in [v0, v0+nvs), columns [c0, c0+ncs): (nvs, ncs, ng) complex128 tensor."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        workspace = torch.empty(gw_pair_density_workspace_size(ctx, problem, nvs, ncs, prec), dtype=torch.uint8,
                                device=dev)
    out = torch.empty((nvs, ncs, ng), dtype=torch.complex128, device=dev)
    _check(lib.gw_pair_density(ctx, C.byref(problem), v0, nvs, c0, ncs, prec, _ptr(workspace), workspace.numel(),
                               _ptr(out)), ctx)
    return out


# ---------------------------------------------------------------- COH self-energy
def gw_sigma_coh_workspace_size(ctx, problem) -> int:
    n = C.c_size_t()
    _check(lib.gw_sigma_coh_workspace_size(ctx, C.byref(problem), C.byref(n)), ctx)
    return n.value


def gw_sigma_coh_static(ctx, problem, vcoul, eps_inv, workspace=None, out=None):
    """Static COH self-energy <n|Sigma_COH|n'> (nv x nv complex128) of the problem's states
    (coef_v rows) over its weighted columns, from a static eps^-1 (ng x ng) and v(q+G)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        workspace = torch.empty(gw_sigma_coh_workspace_size(ctx, problem), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty((problem.nv, problem.nv), dtype=torch.complex128, device=dev)
    z = eps_inv.contiguous()
    v = vcoul.contiguous()
    _check(lib.gw_sigma_coh_static(ctx, C.byref(problem), _ptr(v), _ptr(z), _ptr(workspace),
                                   workspace.numel(), _ptr(out)), ctx)
    return out


# ---------------------------------------------------------------- dielectric

def gw_sigma_coh_gpp(ctx, problems, vcouls, modes, energies: Sequence[float], delta: float = 0.0, workspace=None,
                     out=None):
    """COH self-energy of Eq. (sigmach) with the plasmon-pole eps^-1: one problem per q (states
    coef_v, columns coef_c with energies e_col and weights n_col), each with its Coulomb factors
    (ng tensor) and modes (2 ng^2 complex128: Omega^2 then wt^2); returns (nenergy, nv, nv) complex128."""
    import torch
    arr = _probs(problems)
    nq = len(arr)
    if len(vcouls) != nq or len(modes) != nq:
        raise ValueError("one Coulomb vector and one mode array per problem")
    en = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
    vv = [v.contiguous() for v in vcouls]
    mm = [m.contiguous() for m in modes]
    vp_arr = (vp * nq)(*[vp(_ptr(v)) for v in vv])
    mp_arr = (vp * nq)(*[vp(_ptr(m)) for m in mm])
    dev = torch.device("cuda", torch.cuda.current_device())
    if workspace is None:
        n = C.c_size_t()
        _check(lib.gw_sigma_coh_gpp_workspace_size(ctx, arr, nq, len(en), C.byref(n)), ctx)
        workspace = torch.empty(n.value, dtype=torch.uint8, device=dev)
    ns = arr[0].nv
    if out is None:
        out = torch.empty((len(en), ns, ns), dtype=torch.complex128, device=dev)
    _check(lib.gw_sigma_coh_gpp(ctx, arr, nq, vp_arr, mp_arr, len(en), en.ctypes.data_as(dp), float(delta),
                                _ptr(workspace), workspace.numel(), _ptr(out)), ctx)
    return out

def gw_eps_inv_workspace_size(ctx, ng: int, nbatch: int) -> int:
    n = C.c_size_t()
    _check(lib.gw_eps_inv_workspace_size(ctx, ng, nbatch, C.byref(n)), ctx)
    return n.value


def gw_eps_inv(ctx, vcoul, chi0, workspace=None, out=None, hermitian=False):
    """(I - diag(v) chi0)^-1 for chi0 of shape (nbatch, ng, ng) (or (ng, ng)), vcoul (nbatch, ng) or (ng,);
    hermitian=True for a static (Hermitian negative semidefinite) chi0 and v > 0."""
    import torch
    squeeze = chi0.dim() == 2
    c = chi0.reshape(-1, chi0.shape[-1], chi0.shape[-1]).contiguous()
    nb, ng = c.shape[0], c.shape[-1]
    v = vcoul.reshape(-1, ng).expand(nb, ng).contiguous()
    if workspace is None:
        workspace = torch.empty(max(1, gw_eps_inv_workspace_size(ctx, ng, nb)),
                                dtype=torch.uint8, device=c.device)
    if out is None:
        out = torch.empty_like(c)
    _check(lib.gw_eps_inv(ctx, ng, nb, 1 if hermitian else 0, _ptr(v), _ptr(c), _ptr(workspace), workspace.numel(),
                          _ptr(out)), ctx)
    return out[0] if squeeze else out


def gw_eps_inv_noalloc(ctx, vcoul, chi0, out, hermitian=False):
    """gw_eps_inv without allocation: the library's static scratch (ng <= 2048); the caller passes
    the output (same shape as chi0, complex128)."""
    nb = 1 if chi0.dim() == 2 else chi0.shape[0]
    ng = chi0.shape[-1]
    _check(lib.gw_eps_inv_noalloc(ctx, ng, nb, 1 if hermitian else 0, _ptr(vcoul), _ptr(chi0), _ptr(out)), ctx)
    return out


def gw_eps_inv_status(ctx) -> None:
    _check(lib.gw_eps_inv_status(ctx), ctx)


def gw_eps_inv_backward(ctx, vcoul, eps_inv, grad_eps_inv, workspace=None, out=None):
    """chi0bar = diag(v) Z^H Zbar Z^H for Z = eps^-1 (shapes as in gw_eps_inv)."""
    import torch
    squeeze = eps_inv.dim() == 2
    z = eps_inv.reshape(-1, eps_inv.shape[-1], eps_inv.shape[-1]).contiguous()
    zb = grad_eps_inv.reshape(z.shape).contiguous()
    nb, ng = z.shape[0], z.shape[-1]
    v = vcoul.reshape(-1, ng).expand(nb, ng).contiguous()
    if workspace is None:
        workspace = torch.empty(gw_eps_inv_workspace_size(ctx, ng, nb), dtype=torch.uint8, device=z.device)
    if out is None:
        out = torch.empty_like(z)
    _check(lib.gw_eps_inv_backward(ctx, ng, nb, _ptr(v), _ptr(z), _ptr(zb), _ptr(workspace), workspace.numel(),
                                   _ptr(out)), ctx)
    return out[0] if squeeze else out


# ---------------------------------------------------------------- grouping (host)
def gw_group_windows_edges(e_band: np.ndarray, edges: np.ndarray, mode: int = 0, rule: int = 0, dos_a: float = 0.0,
                           dos_v0: float = 0.0):
    """Columns of Eq. (energyintegration) on window edges (uniform or not), rule 0 midpoint or
    1 two-point Gauss: (col_band int32, e_col, n_col, n0) as numpy arrays."""
    e = np.ascontiguousarray(e_band, dtype=np.float64)
    ed = np.ascontiguousarray(edges, dtype=np.float64)
    nwin = len(ed) - 1
    cap = len(e) + 2 * max(nwin, 0)
    col = np.zeros(cap, dtype=np.int32)
    ec = np.zeros(cap)
    nc = np.zeros(cap)
    ncol, n0 = C.c_int(), C.c_int()
    st = lib.gw_group_windows_edges(len(e), e.ctypes.data_as(dp), nwin, ed.ctypes.data_as(dp), mode, rule, dos_a,
                                    dos_v0, col.ctypes.data_as(i32p), ec.ctypes.data_as(dp), nc.ctypes.data_as(dp),
                                    C.byref(ncol), C.byref(n0))
    if st != GW_OK:
        raise GwError(st, "gw_group_windows_edges: edges not increasing, a band above the last edge, or a bad "
                          "mode / rule")
    k = ncol.value
    return col[:k].copy(), ec[:k].copy(), nc[:k].copy(), n0.value


def gw_group_windows(e_band: np.ndarray, e0: float, de: float, nwin: int, mode: int = 0, dos_a: float = 0.0,
                     dos_v0: float = 0.0):
    """Columns of Eq. (energyintegration): (col_band int32, e_col, n_col, n0) as numpy arrays."""
    e = np.ascontiguousarray(e_band, dtype=np.float64)
    cap = len(e) + nwin
    col = np.zeros(cap, dtype=np.int32)
    ec = np.zeros(cap)
    nc = np.zeros(cap)
    ncol, n0 = C.c_int(), C.c_int()
    st = lib.gw_group_windows(len(e), e.ctypes.data_as(dp), e0, de, nwin, mode, dos_a, dos_v0, col.ctypes.data_as(i32p),
                              ec.ctypes.data_as(dp), nc.ctypes.data_as(dp), C.byref(ncol), C.byref(n0))
    if st != GW_OK:
        raise GwError(st, "gw_group_windows: invalid arguments or a band above the last window")
    k = ncol.value
    return col[:k].copy(), ec[:k].copy(), nc[:k].copy(), n0.value
