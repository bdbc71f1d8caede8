// Host side of the gwchi0 C ABI: contexts, stage timers, geometry set-up, window
// grouping and the dielectric inverse.  The band sum itself is driven from
// chi0_driver.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"

using gw::Geom;

namespace {

std::string g_create_error;
std::atomic<unsigned long long> g_geom_ids{0};

// Device allocation of the set-up calls.  GW_FAULT=alloc:N in the environment makes the N-th
// such allocation of the call fail (counted from 1 within each gw_ctx_create or gw_geom_create
// call), so that tests reach every failure path of set-up without exhausting the device.
int fault_alloc_index() {
  const char* f = std::getenv("GW_FAULT");
  if (!f || std::strncmp(f, "alloc:", 6) != 0) return 0;
  return std::atoi(f + 6);
}
hipError_t setup_alloc(void** p, size_t bytes, int* count, int fail_at) {
  if (++*count == fail_at) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Reciprocal lattice vectors as rows, b_i . a_j = 2 pi delta_ij, of a cell with the lattice
// vectors as rows; false for a singular cell.
bool reciprocal(const double* a, double* b) {
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  const double f = 2.0 * 3.141592653589793238462643383279502884 / det;
  // b = 2 pi (a^-1)^T: rows are the cofactor rows of a over det
  b[0] = f * (a[4] * a[8] - a[5] * a[7]);
  b[1] = f * (a[5] * a[6] - a[3] * a[8]);
  b[2] = f * (a[3] * a[7] - a[4] * a[6]);
  b[3] = f * (a[2] * a[7] - a[1] * a[8]);
  b[4] = f * (a[0] * a[8] - a[2] * a[6]);
  b[5] = f * (a[1] * a[6] - a[0] * a[7]);
  b[6] = f * (a[1] * a[5] - a[2] * a[4]);
  b[7] = f * (a[2] * a[3] - a[0] * a[5]);
  b[8] = f * (a[0] * a[4] - a[1] * a[3]);
  return true;
}

// |q + G|^2 in bohr^-2 for Miller indices n
double qg2(const double* b, const double* q, const int32_t* n) {
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    double x = 0.0;
    for (int e = 0; e < 3; ++e) x += ((double)n[e] + q[e]) * b[3 * e + d];
    s += x * x;
  }
  return s;
}

// The dielectric sphere must be the first ng G-vectors in the order (|q+G|^2, n1, n2, n3):
// ascending keys (keys equal within a relative 1e-12 count as a tie, decided by the Miller
// indices), and no G outside the list with a key below the list's largest (a cut through a
// shell keeps the lower Miller indices).  Returns "" or the reason.
std::string check_sphere_order(const double* cell, const double* q, int ng, const int32_t* gvec) {
  double b[9];
  if (!reciprocal(cell, b)) return "singular cell";
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(q[d])) return "non-finite q";
  const double tol = 1e-12;
  std::vector<double> key(ng);
  for (int i = 0; i < ng; ++i) key[i] = qg2(b, q, gvec + 3 * i);
  auto before = [&](int i, int j) {   // strictly before in the sphere order
    const double a = key[i], c = key[j];
    if (c - a > tol * std::max(a, c)) return true;
    if (a - c > tol * std::max(a, c)) return false;
    for (int d = 0; d < 3; ++d)
      if (gvec[3 * i + d] != gvec[3 * j + d]) return gvec[3 * i + d] < gvec[3 * j + d];
    return false;
  };
  for (int i = 0; i + 1 < ng; ++i)
    if (!before(i, i + 1))
      return "dielectric sphere not ordered by (|q+G|^2, n1, n2, n3) at entry " + std::to_string(i + 1);
  // completeness: |n + q| <= |q + G| ||a||_F / (2 pi) bounds every Miller index below the cut
  double fro = 0.0;
  for (int i = 0; i < 9; ++i) fro += cell[i] * cell[i];
  const double kmax = key[ng - 1];
  const int last = ng - 1;
  const double rad = std::sqrt(kmax) * std::sqrt(fro) / (2.0 * 3.141592653589793);
  int lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = (int)std::floor(-q[d] - rad) - 1;
    hi[d] = (int)std::ceil(-q[d] + rad) + 1;
    if (hi[d] - lo[d] > 4096) return "dielectric sphere too large to check";
  }
  std::unordered_set<long long> in;
  auto pack = [](long long a, long long c, long long e) { return ((a + 2048) * 4096 + (c + 2048)) * 4096 + (e + 2048); };
  for (int i = 0; i < ng; ++i) {
    for (int d = 0; d < 3; ++d)
      if (gvec[3 * i + d] < -2047 || gvec[3 * i + d] > 2047) return "Miller index out of range";
    in.insert(pack(gvec[3 * i], gvec[3 * i + 1], gvec[3 * i + 2]));
  }
  std::vector<int32_t> lastv(gvec + 3 * last, gvec + 3 * last + 3);
  for (int n1 = lo[0]; n1 <= hi[0]; ++n1)
    for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
      for (int n3 = lo[2]; n3 <= hi[2]; ++n3) {
        const int32_t n[3] = {n1, n2, n3};
        const double k = qg2(b, q, n);
        if (k > kmax * (1.0 + tol)) continue;
        bool below = k < kmax * (1.0 - tol);
        if (!below) {   // a tie with the last entry: below it if its Miller indices are lower
          for (int d = 0; d < 3; ++d)
            if (n[d] != lastv[d]) {
              below = n[d] < lastv[d];
              break;
            }
        }
        if (below && !in.count(pack(n1, n2, n3)))
          return "dielectric sphere misses G = (" + std::to_string(n1) + "," + std::to_string(n2) + "," +
                 std::to_string(n3) + ") below its cut";
      }
  return "";
}

}  // namespace

namespace gw {

// Line split N = R S of the band and pair transforms: radix 16 from N = 64 on where 16 divides N
// (64, 80, 96, 112, 128), else radix 8; N a multiple of 8 (the pair kernel's x2 row groups) from
// 16 to 128 (the band transform's LDS line buffer).
bool line_split(int nd, LineSplit* out) {
  if (nd < 16 || nd > 128 || nd % 8 != 0) return false;
  const int R = nd >= 64 && nd % 16 == 0 ? 16 : 8;
  *out = {R, nd / R};
  return true;
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
  // the scratch of the allocation-free inverse: its address on this device, looked up once
  hipError_t e = gw::noalloc_scratch_init(device);
  int nalloc = 0;
  const int fail_at = fault_alloc_index();
  if (e == hipSuccess) e = setup_alloc((void**)&c->d_pivot_flag, sizeof(int), &nalloc, fail_at);
  if (e == hipSuccess) e = setup_alloc((void**)&c->d_check_flag, sizeof(int), &nalloc, fail_at);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->h_check_flag, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&c->ev_ready[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_free[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    gw_ctx_destroy(c);
    g_create_error = "context set-up failed (device flag, side stream or events)";
    return GW_ENOMEM;
  }
  *out = c;
  return GW_OK;
}

gw_status gw_ctx_destroy(gw_ctx* ctx) {
  if (!ctx) return GW_EINVAL;
  if (ctx->d_pivot_flag) (void)hipFree(ctx->d_pivot_flag);
  if (ctx->d_check_flag) (void)hipFree(ctx->d_check_flag);
  if (ctx->h_check_flag) (void)hipHostFree(ctx->h_check_flag);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  for (int i = 0; i < 2; ++i) {
    if (ctx->ev_ready[i]) (void)hipEventDestroy(ctx->ev_ready[i]);
    if (ctx->ev_free[i]) (void)hipEventDestroy(ctx->ev_free[i]);
  }
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  for (auto& ge : ctx->graphs) {
    (void)hipGraphExecDestroy(ge.exec);
    (void)hipGraphDestroy(ge.graph);
  }
  for (auto& m : ctx->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (gw_geom* gg : ctx->geoms) gg->ctx = nullptr;
  delete ctx;
  return GW_OK;
}

const char* gw_last_error(const gw_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

gw_status gw_geom_create(gw_ctx* ctx, const int n_fft[3], const double* cell, const double* q, int npw,
                         const int32_t* gvec_wf, int ng, const int32_t* gvec_chi, gw_geom** out) {
  if (!ctx) return GW_EINVAL;
  if (!out || !n_fft || !gvec_wf || !gvec_chi) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  *out = nullptr;
  if (npw < 1 || ng < 1) return gw::fail(ctx, GW_EINVAL, "npw and ng must be >= 1");
  if ((cell == nullptr) != (q == nullptr)) return gw::fail(ctx, GW_EINVAL, "give both cell and q, or neither");
  if (cell) {
    const std::string why = check_sphere_order(cell, q, ng, gvec_chi);
    if (!why.empty()) return gw::fail(ctx, GW_EINVAL, why);
  }
  for (int i = 0; i < 3; ++i)
    if (n_fft[i] < 1) return gw::fail(ctx, GW_EINVAL, "FFT grid must be positive");
  const int nd = n_fft[0];
  gw::LineSplit ls;
  if (n_fft[1] != nd || n_fft[2] != nd || !gw::line_split(nd, &ls))
    return gw::fail(ctx, GW_EUNSUPPORTED, "FFT grid must be cubic with N a multiple of 8 from 16 to 128");
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
      return gw::fail(ctx, GW_EINVAL, "wavefunction G-vectors collide modulo the grid");
  }
  seen.clear();
  for (int i = 0; i < ng; ++i) {
    for (int d = 0; d < 3; ++d) rc = std::max(rc, std::abs(gvec_chi[3 * i + d]));
    if (!seen.insert(key(gvec_chi + 3 * i)).second)
      return gw::fail(ctx, GW_EINVAL, "dielectric G-vectors collide modulo the grid");
  }
  if (2 * rw + rc >= nd)
    return gw::fail(ctx, GW_EINVAL,
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
  if (cell) {
    g.has_q = true;
    for (int d = 0; d < 3; ++d) g.q[d] = q[d];
    for (int d = 0; d < 9; ++d) g.cell[d] = cell[d];
  }
  if (g.W > 2 * 64 + 1) return gw::fail(ctx, GW_EUNSUPPORTED, "wavefunction sphere too wide");
  // the pair kernels read the planes in the band transform's split order: same radix
  if (gw::pair_supported(nd, g.K) && gw::pair_radix(nd, g.K) != ls.R)
    return gw::fail(ctx, GW_EUNSUPPORTED, "pair kernel radix differs from the band transform's split");
  if (!gw::pair_supported(nd, g.K))
    return gw::fail(ctx, GW_EUNSUPPORTED,
                "no pair kernel for N = " + std::to_string(nd) + ", K = " + std::to_string(g.K) +
                    " (dielectric sphere half-width " + std::to_string(rc) + "; at most " +
                    std::to_string((gw::kPairGenKMax - 1) / 2) + ")");
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
  // the twiddles of the pruned outputs per chunk index b: kernels index them by (b, j) alone
  const size_t ntwk = (size_t)nd * g.K;
  std::vector<double2> twk64(ntwk);
  std::vector<float2> twk32(ntwk);
  for (int b = 0; b < nd; ++b)
    for (int j = 0; j < g.K; ++j) {
      const int k = (((j - rc) * b) % nd + nd) % nd;
      twk64[(size_t)b * g.K + j] = tw64[k];
      twk32[(size_t)b * g.K + j] = tw32[k];
    }
  gw_geom* gg = new (std::nothrow) gw_geom();
  if (!gg) return gw::fail(ctx, GW_ENOMEM, "out of host memory");
  gg->ctx = ctx;
  gg->id = ++g_geom_ids;
  ctx->geoms.push_back(gg);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipSuccess;
  int nalloc = 0;
  const int fail_at = fault_alloc_index();
  e = e == hipSuccess ? setup_alloc((void**)&g.d_wf_map, wf_map.size() * 4, &nalloc, fail_at) : e;
  e = e == hipSuccess ? setup_alloc((void**)&g.d_chi_map, chi_map.size() * 4, &nalloc, fail_at) : e;
  e = e == hipSuccess ? setup_alloc((void**)&g.d_tw64, nd * sizeof(double2), &nalloc, fail_at) : e;
  e = e == hipSuccess ? setup_alloc((void**)&g.d_tw32, nd * sizeof(float2), &nalloc, fail_at) : e;
  e = e == hipSuccess ? setup_alloc((void**)&g.d_twk64, ntwk * sizeof(double2), &nalloc, fail_at) : e;
  e = e == hipSuccess ? setup_alloc((void**)&g.d_twk32, ntwk * sizeof(float2), &nalloc, fail_at) : e;
  if (e == hipSuccess) e = hipMemcpy(g.d_wf_map, wf_map.data(), wf_map.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_chi_map, chi_map.data(), chi_map.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_tw64, tw64.data(), nd * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_tw32, tw32.data(), nd * sizeof(float2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_twk64, twk64.data(), ntwk * sizeof(double2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g.d_twk32, twk32.data(), ntwk * sizeof(float2), hipMemcpyHostToDevice);
  (void)hipSetDevice(prev);
  gg->g = g;
  if (e != hipSuccess) {
    gw_geom_destroy(gg);
    return gw::fail(ctx, GW_ENOMEM, std::string("geometry upload failed: ") + hipGetErrorString(e));
  }
  *out = gg;
  return GW_OK;
}

gw_status gw_sphere_check(const double* cell, const double* q, int ng, const int32_t* gvec_chi, char* msg,
                          size_t msg_len) {
  if (!cell || !q || ng < 1 || !gvec_chi) return GW_EINVAL;
  const std::string why = check_sphere_order(cell, q, ng, gvec_chi);
  if (msg && msg_len > 0) {
    const size_t n = std::min(msg_len - 1, why.size());
    std::memcpy(msg, why.data(), n);
    msg[n] = '\0';
  }
  return why.empty() ? GW_OK : GW_EINVAL;
}

gw_status gw_geom_destroy(gw_geom* geom) {
  if (!geom) return GW_EINVAL;
  // captured graphs that read this geometry's tables are dropped with it
  if (gw_ctx* ctx = geom->ctx) {
    std::vector<gw_ctx::GraphEntry> keep;
    for (auto& ge : ctx->graphs) {
      if (std::find(ge.geoms.begin(), ge.geoms.end(), geom->id) != ge.geoms.end()) {
        (void)hipGraphExecDestroy(ge.exec);
        (void)hipGraphDestroy(ge.graph);
      } else {
        keep.push_back(ge);
      }
    }
    ctx->graphs.swap(keep);
    ctx->geoms.erase(std::remove(ctx->geoms.begin(), ctx->geoms.end(), geom), ctx->geoms.end());
  }
  Geom& g = geom->g;
  if (g.d_wf_map) (void)hipFree(g.d_wf_map);
  if (g.d_chi_map) (void)hipFree(g.d_chi_map);
  if (g.d_tw64) (void)hipFree(g.d_tw64);
  if (g.d_tw32) (void)hipFree(g.d_tw32);
  if (g.d_twk64) (void)hipFree(g.d_twk64);
  if (g.d_twk32) (void)hipFree(g.d_twk32);
  delete geom;
  return GW_OK;
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

gw_status gw_group_windows_edges(int nband, const double* e_band, int nwin, const double* edges, int mode, int rule,
                                 double dos_a, double dos_v0, int32_t* col_band, double* e_col, double* n_col,
                                 int* ncol_out, int* n0_out) {
  if (nband < 0 || (nband > 0 && !e_band) || nwin < 0 || !edges || !col_band || !e_col || !n_col || !ncol_out ||
      !n0_out)
    return GW_EINVAL;
  if ((mode != 0 && mode != 1) || (rule != 0 && rule != 1) || (rule == 1 && mode == 0)) return GW_EINVAL;
  for (int k = 0; k <= nwin; ++k)
    if (!std::isfinite(edges[k]) || (k > 0 && !(edges[k] > edges[k - 1]))) return GW_EINVAL;
  std::vector<int> win(nband, -1);
  int ncol = 0;
  for (int i = 0; i < nband; ++i) {
    const double e = e_band[i];
    if (!std::isfinite(e)) return GW_EINVAL;
    if (e <= edges[0]) {
      col_band[ncol] = i;
      e_col[ncol] = e;
      n_col[ncol] = 1.0;
      ++ncol;
      continue;
    }
    if (nwin == 0 || e > edges[nwin]) return GW_EINVAL;
    // window k with edges[k] <= e < edges[k+1]; a band on the top edge joins the last window
    const int k = (int)(std::upper_bound(edges, edges + nwin + 1, e) - edges) - 1;
    win[i] = std::min(k, nwin - 1);
  }
  *n0_out = ncol;
  std::vector<std::vector<int>> members(nwin);
  for (int i = 0; i < nband; ++i)
    if (win[i] >= 0) members[win[i]].push_back(i);
  const double goff = 0.5 / std::sqrt(3.0);
  for (int k = 0; k < nwin; ++k) {
    if (members[k].empty()) continue;
    const double de = edges[k + 1] - edges[k];
    const double mid = 0.5 * (edges[k] + edges[k + 1]);
    double node[2];
    double wq;
    int nnode;
    if (rule == 0) {
      node[0] = mid;
      wq = de;
      nnode = 1;
    } else {
      node[0] = mid - goff * de;
      node[1] = mid + goff * de;
      wq = 0.5 * de;
      nnode = 2;
    }
    for (int t = 0; t < nnode; ++t) {
      int best = -1;
      for (int i : members[k])   // index order: a tie keeps the lower index
        if (best < 0 || std::fabs(e_band[i] - node[t]) < std::fabs(e_band[best] - node[t])) best = i;
      col_band[ncol] = best;
      e_col[ncol] = node[t];
      n_col[ncol] = mode == 0 ? (double)members[k].size() : dos_a * std::sqrt(std::max(node[t] - dos_v0, 0.0)) * wq;
      ++ncol;
    }
  }
  *ncol_out = ncol;
  return GW_OK;
}

gw_status gw_kq_map(int nk, const double* kpts, const double* q, double tol, int32_t* kq_index, int32_t* g0) {
  if (nk < 1 || !kpts || !q || !kq_index || !g0 || !(tol > 0.0) || !(tol < 0.5)) return GW_EINVAL;
  for (int i = 0; i < nk; ++i) {
    int found = -1;
    double d[3];
    for (int j = 0; j < nk && found < 0; ++j) {
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        d[a] = kpts[3 * i + a] + q[a] - kpts[3 * j + a];
        if (!std::isfinite(d[a]) || std::fabs(d[a] - std::nearbyint(d[a])) >= tol) ok = false;
      }
      if (ok) found = j;
    }
    if (found < 0) return GW_EINVAL;
    kq_index[i] = found;
    for (int a = 0; a < 3; ++a) g0[3 * i + a] = (int32_t)std::nearbyint(d[a]);
  }
  return GW_OK;
}

namespace {
size_t gpp_ws(int ng, int nomega) {
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r((size_t)ng * 3 * sizeof(double)) + r((size_t)ng * 3 * sizeof(int32_t)) +
         r((size_t)std::max(nomega, 1) * sizeof(double));
}
}  // namespace

gw_status gw_gpp_workspace_size(gw_ctx* ctx, int ng, int nomega, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nomega < 0 || !bytes) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  *bytes = gpp_ws(ng, nomega);
  return GW_OK;
}

gw_status gw_gpp_eps_inv(gw_ctx* ctx, int ng, const int32_t* gvec_chi, const double* q, const double* bvec,
                         int rho_half, const void* rho, const void* eps_inv_static, int nomega, const double* omega,
                         double eta, void* workspace, size_t ws_bytes, void* modes, void* eps_inv_omega) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nomega < 0 || !gvec_chi || !q || !bvec || !rho || !eps_inv_static || !workspace ||
      (nomega > 0 && (!omega || !eps_inv_omega)) || rho_half < 0 || !(eta >= 0.0) || !std::isfinite(eta))
    return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (ws_bytes < gpp_ws(ng, nomega)) return gw::fail(ctx, GW_EINVAL, "workspace too small");
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  std::vector<double> kv((size_t)ng * 3);
  for (int a = 0; a < ng; ++a) {
    double k2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], gvec_chi[3 * a + d]);
      hi[d] = std::max(hi[d], gvec_chi[3 * a + d]);
      double x = 0.0;
      for (int e = 0; e < 3; ++e) x += (gvec_chi[3 * a + e] + q[e]) * bvec[3 * e + d];
      kv[3 * a + d] = x;
      k2 += x * x;
    }
    if (!(k2 > 0.0) || !std::isfinite(k2)) return gw::fail(ctx, GW_EINVAL, "q + G = 0 or not finite");
  }
  for (int d = 0; d < 3; ++d)
    if (hi[d] - lo[d] > rho_half) return gw::fail(ctx, GW_EINVAL, "density box does not cover every G - G'");
  for (int i = 0; i < nomega; ++i)
    if (!std::isfinite(omega[i])) return gw::fail(ctx, GW_EINVAL, "non-finite frequency");
  char* ws = (char*)workspace;
  double* d_k = (double*)ws;
  int32_t* d_g = (int32_t*)(ws + ((size_t)ng * 3 * sizeof(double) + 255) / 256 * 256);
  double* d_w = (double*)((char*)d_g + ((size_t)ng * 3 * sizeof(int32_t) + 255) / 256 * 256);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipMemcpyAsync(d_k, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_g, gvec_chi, (size_t)ng * 3 * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && nomega > 0)
    e = hipMemcpyAsync(d_w, omega, (size_t)nomega * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = gw::launch_gpp(eps_inv_static, ng, d_k, d_g, rho, rho_half, d_w, nomega, eta, modes, eps_inv_omega,
                       ctx->stream);
  // the host arrays are staged before the copies return; the kernel reads the device copies
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return gw::fail(ctx, GW_EDEVICE, std::string("plasmon-pole launch: ") + hipGetErrorString(e));
  return GW_OK;
}

gw_status gw_ctx_set_timing(gw_ctx* ctx, int enable) {
  if (!ctx) return GW_EINVAL;
  ctx->timing = enable != 0;
  return GW_OK;
}

gw_status gw_ctx_set_overlap(gw_ctx* ctx, int mode) {
  if (!ctx) return GW_EINVAL;
  if (mode < 0 || mode > 2) return gw::fail(ctx, GW_EINVAL, "overlap mode must be 0, 1 or 2");
  ctx->overlap = mode;
  return GW_OK;
}

gw_status gw_ctx_stage_times(gw_ctx* ctx, double* ms, long long* counts, int reset) {
  if (!ctx) return GW_EINVAL;
  if (!ms || !counts) return gw::fail(ctx, GW_EINVAL, "NULL argument");
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
  if (ng < 1 || nbatch < 1 || !bytes) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  *bytes = std::max(gw::eps_inv_workspace(ng), gw::eps_inv_backward_workspace(ng));
  return GW_OK;
}

}  // extern "C"

namespace {
// nbatch inverses on the context's stream: the pivoted Gauss-Jordan route, or the block sweeps
// of the static (Hermitian) form
gw_status eps_inv_batch(gw_ctx* ctx, int ng, int nbatch, int hermitian, const double* vcoul, const void* chi0,
                        void* ws, void* eps_inv) {
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  auto run = [&]() -> gw_status {
    GW_HIP(ctx, gw::launch_flag_clear(ctx->d_pivot_flag, ctx->stream));
    gw::StageScope sc(ctx, gw::kStageEpsInv);
    const size_t nn = (size_t)ng * ng;
    for (int b = 0; b < nbatch; ++b) {
      const double* v = vcoul + (size_t)b * ng;
      const double2* c = (const double2*)chi0 + b * nn;
      double2* z = (double2*)eps_inv + b * nn;
      GW_HIP(ctx, hermitian ? gw::launch_eps_inv_sweep(ng, v, c, z, ws, ctx->d_pivot_flag, ctx->stream)
                            : gw::launch_eps_inv(ng, v, c, z, ws, ctx->d_pivot_flag, ctx->stream));
    }
    return GW_OK;
  };
  gw_status s = run();
  (void)hipSetDevice(prev);
  return s;
}
}  // namespace

extern "C" {

gw_status gw_eps_inv(gw_ctx* ctx, int ng, int nbatch, int hermitian, const double* vcoul, const void* chi0,
                     void* workspace, size_t ws_bytes, void* eps_inv) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !vcoul || !chi0 || !workspace || !eps_inv) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (hermitian != 0 && hermitian != 1) return gw::fail(ctx, GW_EINVAL, "hermitian must be 0 or 1");
  if (chi0 == eps_inv) return gw::fail(ctx, GW_EINVAL, "eps_inv may not alias chi0");
  if (ws_bytes < gw::eps_inv_workspace(ng))
    return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(gw::eps_inv_workspace(ng)));
  return eps_inv_batch(ctx, ng, nbatch, hermitian, vcoul, chi0, workspace, eps_inv);
}

gw_status gw_eps_inv_noalloc(gw_ctx* ctx, int ng, int nbatch, int hermitian, const double* vcoul, const void* chi0,
                             void* eps_inv) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !vcoul || !chi0 || !eps_inv) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (hermitian != 0 && hermitian != 1) return gw::fail(ctx, GW_EINVAL, "hermitian must be 0 or 1");
  if (chi0 == eps_inv) return gw::fail(ctx, GW_EINVAL, "eps_inv may not alias chi0");
  if (ng > gw::kNoAllocMaxNg)
    return gw::fail(ctx, GW_EINVAL, "ng = " + std::to_string(ng) + " exceeds the allocation-free maximum of " +
                                        std::to_string(gw::kNoAllocMaxNg) + " (use gw_eps_inv with a workspace)");
  void* scratch = gw::noalloc_scratch(ctx->device);
  if (!scratch) return gw::fail(ctx, GW_EDEVICE, "allocation-free scratch not set up on this device");
  return eps_inv_batch(ctx, ng, nbatch, hermitian, vcoul, chi0, scratch, eps_inv);
}

gw_status gw_eps_inv_status(gw_ctx* ctx) {
  if (!ctx) return GW_EINVAL;
  int flag = 0;
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  GW_HIP(ctx, hipMemcpy(&flag, ctx->d_pivot_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag)
    return gw::fail(ctx, GW_ESINGULAR,
                    "zero or non-finite pivot in eps = I - v chi0 (hermitian = 1: I - V^1/2 chi0 V^1/2 not positive "
                    "definite, or v <= 0)");
  return GW_OK;
}

gw_status gw_eps_inv_backward(gw_ctx* ctx, int ng, int nbatch, const double* vcoul, const void* eps_inv,
                              const void* grad_eps_inv, void* workspace, size_t ws_bytes, void* grad_chi0) {
  if (!ctx) return GW_EINVAL;
  if (ng < 1 || nbatch < 1 || !vcoul || !eps_inv || !grad_eps_inv || !workspace || !grad_chi0)
    return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (ws_bytes < gw::eps_inv_backward_workspace(ng)) return gw::fail(ctx, GW_EINVAL, "workspace too small");
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
