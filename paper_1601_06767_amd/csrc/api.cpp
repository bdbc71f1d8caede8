// Host side of the gwchi0 C ABI: argument checks, geometry set-up, workspace
// layout and the launch sequence of the band sum of Eq. (chi0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"

using gw::Geom;

struct gw_geom {
  gw_ctx* ctx = nullptr;
  Geom g;
};

namespace {

std::string g_create_error;

gw_status fail(gw_ctx* ctx, gw_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

#define GW_HIP(ctx, expr)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail((ctx), GW_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));           \
  } while (0)

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Workspace layout of one chi0 problem (reused problem after problem).
struct ChiPlan {
  bool fp64 = true;
  size_t csz = 16;
  int nvs = 0;      // valence slots (multiple of 4)
  int cc = 0;       // columns per chunk (multiple of 8)
  int npair = 0;    // nvs * cc
  int ksplit = 1;
  int nparts = 1;   // 1 (real weights) or 2 (complex weights)
  int nomega = 1;
  int band_batch = 32;
  size_t off_psiv = 0, off_psic = 0, off_scr = 0, off_q = 0, off_m = 0, off_w = 0, off_acc = 0, total = 0;
  size_t off_part = 0, off_dx = 0, off_dn = 0;   // backward only
};

constexpr int kPairTarget = 32768;

ChiPlan make_plan(const Geom& g, int nv, int ncol, int nomega, bool complex_w, gw_precision prec) {
  ChiPlan p;
  p.fp64 = prec == GW_FP64;
  p.csz = p.fp64 ? 16 : 8;
  p.nvs = (int)round_up(nv, 4);
  int cc = std::max(8, (kPairTarget / p.nvs) / 8 * 8);
  cc = std::min<int>(cc, (int)round_up(ncol, 8));
  p.cc = cc;
  p.npair = p.nvs * cc;
  const int nt = g.ngp / gw::kTile;
  const int ntl = nt * (nt + 1) / 2;
  p.ksplit = std::max(1, std::min(32, (2048 + ntl - 1) / ntl));
  p.ksplit = std::min(p.ksplit, std::max(1, p.npair / 64));
  p.nparts = complex_w ? 2 : 1;
  p.nomega = nomega;
  const size_t npts = (size_t)g.nd * g.nd * g.nd;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  p.off_psiv = take((size_t)p.nvs * npts * p.csz);
  p.off_psic = take((size_t)cc * npts * p.csz);
  p.off_scr = take(gw::band_scratch_bytes(g, p.band_batch, p.fp64));
  p.off_q = take((size_t)p.npair * g.nd * g.K * g.K * p.csz);
  p.off_m = take((size_t)p.npair * g.ngp * p.csz);
  p.off_w = take((size_t)2 * p.npair * sizeof(double));
  p.off_acc = take((size_t)nomega * p.nparts * p.ksplit * g.ngp * g.ngp * sizeof(double2));
  p.off_part = take(gw::adjoint_partial_bytes(p.npair, g.ngp));
  p.off_dx = take((size_t)p.npair * sizeof(double));
  p.off_dn = take((size_t)p.npair * sizeof(double));
  p.total = o;
  return p;
}

gw_status band_to_real(gw_ctx* ctx, const ChiPlan& pl, const Geom& g, const double2* coef, int nrows, const int32_t* band_idx,
                       int band0, int nvalid, int nslot, char* ws, char* psi) {
  const size_t npts = (size_t)g.nd * g.nd * g.nd;
  const size_t scr_a = (size_t)pl.band_batch * g.W * g.W * g.nd * pl.csz;
  for (int s0 = 0; s0 < nslot; s0 += pl.band_batch) {
    const int ns = std::min(pl.band_batch, nslot - s0);
    void* tA = ws + pl.off_scr;
    void* tB = ws + pl.off_scr + scr_a;
    void* out = psi + (size_t)s0 * npts * pl.csz;
    gw::StageScope sc(ctx, gw::kStageBand);
    hipError_t e = pl.fp64 ? gw::launch_band_to_real<double>(g, coef, nrows, band_idx, band0 + s0, nvalid, ns, tA, tB, out,
                                                             ctx->stream)
                           : gw::launch_band_to_real<float>(g, coef, nrows, band_idx, band0 + s0, nvalid, ns, tA, tB, out,
                                                            ctx->stream);
    GW_HIP(ctx, e);
  }
  return GW_OK;
}

gw_status pair_block(gw_ctx* ctx, const ChiPlan& pl, const Geom& g, char* ws, int nvs, int ncs) {
  hipError_t e;
  {
    gw::StageScope sc(ctx, gw::kStagePlanes);
    e = pl.fp64 ? gw::launch_pair_planes<double>(g, ws + pl.off_psiv, ws + pl.off_psic, nvs, ncs,
                                                          ws + pl.off_q, ctx->stream)
                         : gw::launch_pair_planes<float>(g, ws + pl.off_psiv, ws + pl.off_psic, nvs, ncs,
                                                         ws + pl.off_q, ctx->stream);
  }
  GW_HIP(ctx, e);
  {
    gw::StageScope sc(ctx, gw::kStageFinish);
    e = pl.fp64 ? gw::launch_pair_finish<double>(g, ws + pl.off_q, nvs * ncs, ws + pl.off_m, ctx->stream)
                : gw::launch_pair_finish<float>(g, ws + pl.off_q, nvs * ncs, ws + pl.off_m, ctx->stream);
  }
  GW_HIP(ctx, e);
  return GW_OK;
}

gw_status check_problem(gw_ctx* ctx, const gw_chi0_problem& p) {
  if (!p.geom) return fail(ctx, GW_EINVAL, "problem without geometry");
  if (p.nv < 1 || p.ncol < 1 || p.nband < 1) return fail(ctx, GW_EINVAL, "nv, nband and ncol must be >= 1");
  if (!p.coef_v || !p.e_v || !p.coef_c || !p.e_col) return fail(ctx, GW_EINVAL, "NULL band data pointer");
  if (!p.col_band && p.ncol > p.nband) return fail(ctx, GW_EINVAL, "ncol > nband without col_band");
  return GW_OK;
}

}  // namespace

namespace gw {

bool line_split(int nd, LineSplit* out) {
  switch (nd) {
    case 24: *out = {8, 3}; return true;
    case 32: *out = {8, 4}; return true;
    case 48: *out = {16, 3}; return true;
    case 64: *out = {16, 4}; return true;
    case 72: *out = {8, 9}; return true;
    case 96: *out = {16, 6}; return true;
    case 128: *out = {16, 8}; return true;
    default: return false;
  }
}

}  // namespace gw

extern "C" {

const char* gw_version(void) { return "gwchi0 0.1 gfx950"; }

gw_status gw_ctx_create(int device, void* hip_stream, gw_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return GW_EINVAL;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    g_create_error = "no such HIP device";
    return GW_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return GW_EDEVICE;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("kernels are built for gfx950, device is ") + prop.gcnArchName;
    return GW_EUNSUPPORTED;
  }
  gw_ctx* c = new (std::nothrow) gw_ctx();
  if (!c) {
    g_create_error = "out of host memory";
    return GW_ENOMEM;
  }
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(device);
  hipError_t e = hipMalloc(&c->d_pivot_flag, sizeof(int));
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    delete c;
    g_create_error = "hipMalloc of the context flag failed";
    return GW_ENOMEM;
  }
  *out = c;
  return GW_OK;
}

gw_status gw_ctx_destroy(gw_ctx* ctx) {
  if (!ctx) return GW_EINVAL;
  if (ctx->d_pivot_flag) (void)hipFree(ctx->d_pivot_flag);
  delete ctx;
  return GW_OK;
}

const char* gw_last_error(const gw_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

gw_status gw_geom_create(gw_ctx* ctx, const int n_fft[3], int npw, const int32_t* gvec_wf, int ng,
                         const int32_t* gvec_chi, gw_geom** out) {
  if (!ctx) return GW_EINVAL;
  if (!out || !n_fft || !gvec_wf || !gvec_chi) return fail(ctx, GW_EINVAL, "NULL argument");
  *out = nullptr;
  if (npw < 1 || ng < 1) return fail(ctx, GW_EINVAL, "npw and ng must be >= 1");
  for (int i = 0; i < 3; ++i)
    if (n_fft[i] < 1) return fail(ctx, GW_EINVAL, "FFT grid must be positive");
  const int nd = n_fft[0];
  gw::LineSplit ls;
  if (n_fft[1] != nd || n_fft[2] != nd || !gw::line_split(nd, &ls))
    return fail(ctx, GW_EUNSUPPORTED, "FFT grid must be cubic with N in {24,32,48,64,72,96,128}");
  int rw = 0, rc = 0;
  std::unordered_set<long long> seen;
  auto key = [nd](const int32_t* n) {
    long long k = 0;
    for (int i = 0; i < 3; ++i) k = k * nd + ((n[i] % nd) + nd) % nd;
    return k;
  };
  for (int i = 0; i < npw; ++i) {
    for (int d = 0; d < 3; ++d) rw = std::max(rw, std::abs(gvec_wf[3 * i + d]));
    if (!seen.insert(key(gvec_wf + 3 * i)).second)
      return fail(ctx, GW_EINVAL, "wavefunction G-vectors collide modulo the grid");
  }
  seen.clear();
  for (int i = 0; i < ng; ++i) {
    for (int d = 0; d < 3; ++d) rc = std::max(rc, std::abs(gvec_chi[3 * i + d]));
    if (!seen.insert(key(gvec_chi + 3 * i)).second)
      return fail(ctx, GW_EINVAL, "dielectric G-vectors collide modulo the grid");
  }
  if (2 * rw + rc >= nd)
    return fail(ctx, GW_EINVAL,
                "grid is not alias-free: 2*max|n_wf| + max|n_chi| = " + std::to_string(2 * rw + rc) +
                    " >= N = " + std::to_string(nd));
  Geom g;
  g.nd = nd;
  g.npw = npw;
  g.ng = ng;
  g.rw = rw;
  g.W = 2 * rw + 1;
  g.rchi = rc;
  g.K = 2 * rc + 1;
  g.ngp = (int)round_up(ng, gw::kTile);
  g.line = ls;
  if (g.W > 2 * 64 + 1) return fail(ctx, GW_EUNSUPPORTED, "wavefunction sphere too wide");
  if (!gw::pair_supported(nd, g.K))
    return fail(ctx, GW_EUNSUPPORTED,
                "no pair kernel for N = " + std::to_string(nd) + ", K = " + std::to_string(g.K) +
                    " (dielectric sphere half-width " + std::to_string(rc) + ")");
  std::vector<int32_t> wf_map((size_t)g.W * g.W * g.W, -1);
  for (int i = 0; i < npw; ++i) {
    const int32_t* n = gvec_wf + 3 * i;
    wf_map[((size_t)(n[0] + rw) * g.W + (n[1] + rw)) * g.W + (n[2] + rw)] = i;
  }
  std::vector<int32_t> chi_map((size_t)g.K * g.K * g.K, -1);
  for (int i = 0; i < ng; ++i) {
    const int32_t* n = gvec_chi + 3 * i;
    chi_map[((size_t)(n[0] + rc) * g.K + (n[1] + rc)) * g.K + (n[2] + rc)] = i;
  }
  std::vector<double2> tw64(nd);
  std::vector<float2> tw32(nd);
  for (int j = 0; j < nd; ++j) {
    const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)nd;
    tw64[j] = double2{(double)cosl(a), (double)sinl(a)};
    tw32[j] = float2{(float)cosl(a), (float)sinl(a)};
  }
  gw_geom* gg = new (std::nothrow) gw_geom();
  if (!gg) return fail(ctx, GW_ENOMEM, "out of host memory");
  gg->ctx = ctx;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipSuccess;
  e = e == hipSuccess ? hipMalloc(&g.d_wf_map, wf_map.size() * 4) : e;
  e = e == hipSuccess ? hipMalloc(&g.d_chi_map, chi_map.size() * 4) : e;
  e = e == hipSuccess ? hipMalloc(&g.d_tw64, nd * sizeof(double2)) : e;
  e = e == hipSuccess ? hipMalloc(&g.d_tw32, nd * sizeof(float2)) : e;
  if (e == hipSuccess) e = hipMemcpy(g.d_wf_map, wf_map.data(), wf_map.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_chi_map, chi_map.data(), chi_map.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_tw64, tw64.data(), nd * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_tw32, tw32.data(), nd * sizeof(float2), hipMemcpyHostToDevice);
  (void)hipSetDevice(prev);
  gg->g = g;
  if (e != hipSuccess) {
    gw_geom_destroy(gg);
    return fail(ctx, GW_ENOMEM, std::string("geometry upload failed: ") + hipGetErrorString(e));
  }
  *out = gg;
  return GW_OK;
}

gw_status gw_geom_destroy(gw_geom* geom) {
  if (!geom) return GW_EINVAL;
  Geom& g = geom->g;
  if (g.d_wf_map) (void)hipFree(g.d_wf_map);
  if (g.d_chi_map) (void)hipFree(g.d_chi_map);
  if (g.d_tw64) (void)hipFree(g.d_tw64);
  if (g.d_tw32) (void)hipFree(g.d_tw32);
  delete geom;
  return GW_OK;
}

gw_status gw_chi0_workspace_size(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega,
                                 gw_precision prec, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!probs || nprob < 1 || nomega < 1 || !bytes) return fail(ctx, GW_EINVAL, "bad arguments");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(ctx, GW_EINVAL, "bad precision");
  size_t mx = 0;
  for (int i = 0; i < nprob; ++i) {
    gw_status s = check_problem(ctx, probs[i]);
    if (s != GW_OK) return s;
    const ChiPlan pl = make_plan(probs[i].geom->g, probs[i].nv, probs[i].ncol, nomega, true, prec);
    mx = std::max(mx, pl.total);
  }
  *bytes = mx;
  return GW_OK;
}

gw_status gw_chi0_build(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                        double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0) {
  if (!ctx) return GW_EINVAL;
  if (!probs || nprob < 1 || nomega < 1 || !omega || !chi0 || !workspace)
    return fail(ctx, GW_EINVAL, "bad arguments");
  if (!(delta >= 0.0)) return fail(ctx, GW_EINVAL, "delta must be >= 0");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(ctx, GW_EINVAL, "bad precision");
  for (int i = 0; i < nprob; ++i) {
    gw_status s = check_problem(ctx, probs[i]);
    if (s != GW_OK) return s;
    for (int w = 0; w < nomega; ++w)
      if (!std::isfinite(omega[w])) return fail(ctx, GW_EINVAL, "non-finite frequency");
  }
  const bool complex_w = delta > 0.0;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  char* ws = (char*)workspace;
  char* out = (char*)chi0;
  gw_status st = GW_OK;
  for (int ip = 0; ip < nprob && st == GW_OK; ++ip) {
    const gw_chi0_problem& p = probs[ip];
    const Geom& g = p.geom->g;
    const ChiPlan pl = make_plan(g, p.nv, p.ncol, nomega, complex_w, prec);
    if (pl.total > ws_bytes) {
      st = fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(pl.total) + " bytes");
      break;
    }
    const size_t acc_one = (size_t)pl.ksplit * g.ngp * g.ngp * sizeof(double2);
    auto run = [&]() -> gw_status {
      GW_HIP(ctx, gw::launch_zero(ws + pl.off_acc, acc_one * nomega * pl.nparts, ctx->stream));
      gw_status s = band_to_real(ctx, pl, g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, pl.nvs, ws,
                                 ws + pl.off_psiv);
      if (s != GW_OK) return s;
      for (int c0 = 0; c0 < p.ncol; c0 += pl.cc) {
        s = band_to_real(ctx, pl, g, (const double2*)p.coef_c, p.nband, p.col_band, c0, p.ncol, pl.cc, ws, ws + pl.off_psic);
        if (s != GW_OK) return s;
        s = pair_block(ctx, pl, g, ws, pl.nvs, pl.cc);
        if (s != GW_OK) return s;
        for (int iw = 0; iw < nomega; ++iw) {
          double* w = (double*)(ws + pl.off_w);
          {
            gw::StageScope scw(ctx, gw::kStageWeights);
            GW_HIP(ctx, gw::launch_weights(p.e_v, 0, p.nv, pl.nvs, p.e_col, p.n_col, c0, p.ncol, pl.cc, omega, iw,
                                           delta, w, ctx->stream));
          }
          for (int part = 0; part < pl.nparts; ++part) {
            double2* acc = (double2*)(ws + pl.off_acc + acc_one * ((size_t)iw * pl.nparts + part));
            gw::StageScope sc(ctx, gw::kStageContract);
            const double* wp = w + (size_t)part * pl.npair;
            hipError_t e =
                pl.fp64 ? gw::launch_contract<double>(ws + pl.off_m, wp, pl.npair, g.ngp, pl.ksplit, acc, ctx->stream)
                : prec == GW_BF16X3
                    ? gw::launch_contract_bf16x3(ws + pl.off_m, wp, pl.npair, g.ngp, pl.ksplit, acc, ctx->stream)
                    : gw::launch_contract<float>(ws + pl.off_m, wp, pl.npair, g.ngp, pl.ksplit, acc, ctx->stream);
            GW_HIP(ctx, e);
          }
        }
      }
      for (int iw = 0; iw < nomega; ++iw) {
        const double2* accA = (const double2*)(ws + pl.off_acc + acc_one * ((size_t)iw * pl.nparts));
        const double2* accB = pl.nparts == 2 ? accA + acc_one / sizeof(double2) : nullptr;
        gw::StageScope sc(ctx, gw::kStageFinalize);
        GW_HIP(ctx, gw::launch_finalize(accA, accB, pl.ksplit, g.ng, g.ngp, (double2*)out, ctx->stream));
        out += (size_t)g.ng * g.ng * sizeof(double2);
      }
      return GW_OK;
    };
    st = run();
  }
  (void)hipSetDevice(prev);
  return st;
}

gw_status gw_chi0_backward(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                           double delta, gw_precision prec, void* workspace, size_t ws_bytes, const void* grad_chi0,
                           double* grad_e_v, double* grad_e_col, double* grad_n_col, void* grad_coef_v,
                           void* grad_coef_c) {
  if (!ctx) return GW_EINVAL;
  if (!probs || nprob < 1 || nomega < 1 || !omega || !grad_chi0 || !workspace)
    return fail(ctx, GW_EINVAL, "bad arguments");
  if (!(delta >= 0.0)) return fail(ctx, GW_EINVAL, "delta must be >= 0");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(ctx, GW_EINVAL, "bad precision");
  if (grad_coef_v || grad_coef_c)
    return fail(ctx, GW_EUNSUPPORTED, "gradients with respect to the coefficients are not built");
  for (int i = 0; i < nprob; ++i) {
    gw_status s = check_problem(ctx, probs[i]);
    if (s != GW_OK) return s;
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  char* ws = (char*)workspace;
  const char* gin = (const char*)grad_chi0;
  size_t off_ev = 0, off_ec = 0;
  gw_status st = GW_OK;
  for (int ip = 0; ip < nprob && st == GW_OK; ++ip) {
    const gw_chi0_problem& p = probs[ip];
    const Geom& g = p.geom->g;
    const ChiPlan pl = make_plan(g, p.nv, p.ncol, nomega, delta > 0.0, prec);
    if (pl.total > ws_bytes) {
      st = fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(pl.total) + " bytes");
      break;
    }
    double* gev = grad_e_v ? grad_e_v + off_ev : nullptr;
    double* gec = grad_e_col ? grad_e_col + off_ec : nullptr;
    double* gn = grad_n_col ? grad_n_col + off_ec : nullptr;
    auto run = [&]() -> gw_status {
      gw::StageScope sc(ctx, gw::kStageBackward);
      if (gev) GW_HIP(ctx, gw::launch_fill_f64(gev, p.nv, 0.0, ctx->stream));
      gw_status s = band_to_real(ctx, pl, g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, pl.nvs, ws,
                                 ws + pl.off_psiv);
      if (s != GW_OK) return s;
      double* dx = (double*)(ws + pl.off_dx);
      double* dn = (double*)(ws + pl.off_dn);
      double2* part = (double2*)(ws + pl.off_part);
      for (int c0 = 0; c0 < p.ncol; c0 += pl.cc) {
        s = band_to_real(ctx, pl, g, (const double2*)p.coef_c, p.nband, p.col_band, c0, p.ncol, pl.cc, ws,
                         ws + pl.off_psic);
        if (s != GW_OK) return s;
        s = pair_block(ctx, pl, g, ws, pl.nvs, pl.cc);
        if (s != GW_OK) return s;
        GW_HIP(ctx, gw::launch_fill_f64(dx, pl.npair, 0.0, ctx->stream));
        GW_HIP(ctx, gw::launch_fill_f64(dn, pl.npair, 0.0, ctx->stream));
        for (int iw = 0; iw < nomega; ++iw) {
          const double2* gb = (const double2*)gin + (size_t)iw * g.ng * g.ng;
          hipError_t e = pl.fp64 ? gw::launch_adjoint<double>(ws + pl.off_m, pl.npair, g.ng, g.ngp, gb, part,
                                                              ctx->stream)
                                 : gw::launch_adjoint<float>(ws + pl.off_m, pl.npair, g.ng, g.ngp, gb, part,
                                                             ctx->stream);
          GW_HIP(ctx, e);
          GW_HIP(ctx, gw::launch_adjoint_pairs(part, g.ngp, p.e_v, p.nv, pl.nvs, p.e_col, p.n_col, c0, p.ncol, pl.cc,
                                               omega[iw], delta, dx, dn, ctx->stream));
        }
        GW_HIP(ctx, gw::launch_adjoint_reduce(dx, dn, p.nv, pl.cc, c0, p.ncol, gev, gec, gn, ctx->stream));
      }
      return GW_OK;
    };
    st = run();
    gin += (size_t)nomega * g.ng * g.ng * sizeof(double2);
    off_ev += p.nv;
    off_ec += p.ncol;
  }
  (void)hipSetDevice(prev);
  return st;
}

gw_status gw_pair_density_workspace_size(gw_ctx* ctx, const gw_chi0_problem* prob, int nvs, int ncs,
                                         gw_precision prec, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !bytes || nvs < 1 || ncs < 1) return fail(ctx, GW_EINVAL, "bad arguments");
  gw_status s = check_problem(ctx, *prob);
  if (s != GW_OK) return s;
  ChiPlan pl = make_plan(prob->geom->g, nvs, ncs, 1, false, prec);
  *bytes = pl.total;
  return GW_OK;
}

gw_status gw_pair_density(gw_ctx* ctx, const gw_chi0_problem* prob, int v0, int nvs, int c0, int ncs,
                          gw_precision prec, void* workspace, size_t ws_bytes, void* m_out) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !workspace || !m_out) return fail(ctx, GW_EINVAL, "NULL argument");
  gw_status s = check_problem(ctx, *prob);
  if (s != GW_OK) return s;
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return fail(ctx, GW_EINVAL, "bad precision");
  if (nvs < 1 || ncs < 1 || v0 < 0 || c0 < 0 || v0 + nvs > prob->nv || c0 + ncs > prob->ncol)
    return fail(ctx, GW_EINVAL, "pair block out of range");
  const Geom& g = prob->geom->g;
  ChiPlan pl = make_plan(g, nvs, ncs, 1, false, prec);
  if (pl.cc < (int)round_up(ncs, 8)) return fail(ctx, GW_EINVAL, "pair block too large for one pass");
  if (pl.total > ws_bytes) return fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(pl.total));
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  char* ws = (char*)workspace;
  auto run = [&]() -> gw_status {
    gw_status r = band_to_real(ctx, pl, g, (const double2*)prob->coef_v, prob->nv, nullptr, v0, v0 + nvs, pl.nvs, ws,
                               ws + pl.off_psiv);
    if (r != GW_OK) return r;
    r = band_to_real(ctx, pl, g, (const double2*)prob->coef_c, prob->nband, prob->col_band, c0, c0 + ncs, pl.cc, ws,
                     ws + pl.off_psic);
    if (r != GW_OK) return r;
    r = pair_block(ctx, pl, g, ws, pl.nvs, pl.cc);
    if (r != GW_OK) return r;
    GW_HIP(ctx, gw::launch_copy_m(ws + pl.off_m, nvs, ncs, pl.cc, g.ng, g.ngp, pl.fp64, (double2*)m_out,
                                  ctx->stream));
    return GW_OK;
  };
  s = run();
  (void)hipSetDevice(prev);
  return s;
}

gw_status gw_group_windows(int nband, const double* e_band, double e0, double de, int nwin, int mode, double dos_a,
                           double dos_v0, int32_t* col_band, double* e_col, double* n_col, int* ncol_out,
                           int* n0_out) {
  if (nband < 0 || (nband > 0 && !e_band) || !col_band || !e_col || !n_col || !ncol_out || !n0_out) return GW_EINVAL;
  if (!(de > 0.0) || nwin < 0 || (mode != 0 && mode != 1) || !std::isfinite(e0)) return GW_EINVAL;
  const double top = e0 + nwin * de;
  std::vector<int> win(nband, -1);
  int ncol = 0;
  for (int i = 0; i < nband; ++i) {
    const double e = e_band[i];
    if (!std::isfinite(e)) return GW_EINVAL;
    if (e <= e0) {
      col_band[ncol] = i;
      e_col[ncol] = e;
      n_col[ncol] = 1.0;
      ++ncol;
      continue;
    }
    int k = (int)std::floor((e - e0) / de);
    if (k >= nwin) {
      if (e <= top && nwin > 0)
        k = nwin - 1;
      else
        return GW_EINVAL;
    }
    win[i] = k;
  }
  *n0_out = ncol;
  std::vector<int> count(nwin, 0), best(nwin, -1);
  for (int i = 0; i < nband; ++i) {
    const int k = win[i];
    if (k < 0) continue;
    ++count[k];
    const double mid = e0 + (k + 0.5) * de;
    if (best[k] < 0 || std::fabs(e_band[i] - mid) < std::fabs(e_band[best[k]] - mid)) best[k] = i;
  }
  for (int k = 0; k < nwin; ++k) {
    if (count[k] == 0) continue;
    const double mid = e0 + (k + 0.5) * de;
    col_band[ncol] = best[k];
    e_col[ncol] = mid;
    n_col[ncol] = mode == 0 ? (double)count[k] : dos_a * std::sqrt(std::max(mid - dos_v0, 0.0)) * de;
    ++ncol;
  }
  *ncol_out = ncol;
  return GW_OK;
}

gw_status gw_ctx_set_timing(gw_ctx* ctx, int enable) {
  if (!ctx) return GW_EINVAL;
  ctx->timing = enable != 0;
  return GW_OK;
}

gw_status gw_ctx_stage_times(gw_ctx* ctx, double* ms, long long* counts, int reset) {
  if (!ctx) return GW_EINVAL;
  if (!ms || !counts) return fail(ctx, GW_EINVAL, "NULL argument");
  for (const gw_ctx::Mark& m : ctx->marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.b) == hipSuccess && hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
      ctx->stage_ms[m.stage] += t;
      ctx->stage_n[m.stage] += 1;
    }
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  ctx->marks.clear();
  for (int i = 0; i < gw::kNumStages; ++i) {
    ms[i] = ctx->stage_ms[i];
    counts[i] = ctx->stage_n[i];
    if (reset) {
      ctx->stage_ms[i] = 0.0;
      ctx->stage_n[i] = 0;
    }
  }
  return GW_OK;
}

gw_status gw_eps_inv_workspace_size(gw_ctx* ctx, int ng, int nbatch, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !bytes) return fail(ctx, GW_EINVAL, "bad arguments");
  *bytes = std::max(gw::eps_inv_workspace(ng), gw::eps_inv_backward_workspace(ng));
  return GW_OK;
}

gw_status gw_eps_inv(gw_ctx* ctx, int ng, int nbatch, const double* vcoul, const void* chi0, void* workspace,
                     size_t ws_bytes, void* eps_inv) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !vcoul || !chi0 || !workspace || !eps_inv) return fail(ctx, GW_EINVAL, "bad arguments");
  if (chi0 == eps_inv) return fail(ctx, GW_EINVAL, "eps_inv may not alias chi0");
  if (ws_bytes < gw::eps_inv_workspace(ng))
    return fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(gw::eps_inv_workspace(ng)));
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  auto run = [&]() -> gw_status {
    GW_HIP(ctx, gw::launch_flag_clear(ctx->d_pivot_flag, ctx->stream));
    gw::StageScope sc(ctx, gw::kStageEpsInv);
    const size_t nn = (size_t)ng * ng;
    for (int b = 0; b < nbatch; ++b)
      GW_HIP(ctx, gw::launch_eps_inv(ng, vcoul + (size_t)b * ng, (const double2*)chi0 + b * nn,
                                     (double2*)eps_inv + b * nn, workspace, ctx->d_pivot_flag, ctx->stream));
    return GW_OK;
  };
  gw_status s = run();
  (void)hipSetDevice(prev);
  return s;
}

gw_status gw_eps_inv_status(gw_ctx* ctx) {
  if (!ctx) return GW_EINVAL;
  int flag = 0;
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GW_HIP(ctx, hipMemcpy(&flag, ctx->d_pivot_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(ctx, GW_ESINGULAR, "zero or non-finite pivot in eps = I - v chi0");
  return GW_OK;
}

gw_status gw_eps_inv_backward(gw_ctx* ctx, int ng, int nbatch, const double* vcoul, const void* eps_inv,
                              const void* grad_eps_inv, void* workspace, size_t ws_bytes, void* grad_chi0) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !vcoul || !eps_inv || !grad_eps_inv || !workspace || !grad_chi0)
    return fail(ctx, GW_EINVAL, "bad arguments");
  if (ws_bytes < gw::eps_inv_backward_workspace(ng)) return fail(ctx, GW_EINVAL, "workspace too small");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  auto run = [&]() -> gw_status {
    gw::StageScope sc(ctx, gw::kStageBackward);
    const size_t nn = (size_t)ng * ng;
    for (int b = 0; b < nbatch; ++b)
      GW_HIP(ctx, gw::launch_eps_inv_backward(ng, vcoul + (size_t)b * ng, (const double2*)eps_inv + b * nn,
                                              (const double2*)grad_eps_inv + b * nn, (double2*)grad_chi0 + b * nn,
                                              workspace, ctx->stream));
    return GW_OK;
  };
  gw_status s = run();
  (void)hipSetDevice(prev);
  return s;
}

}  // extern "C"
