// Host driver of the band sum of Eq. (chi0): workspace layout, the launch sequence
// of gw_chi0_build / gw_chi0_backward / gw_pair_density, the launch-shape tuner and
// the graph cache.
//
// A build processes up to kMaxBatch q-points together.  Each q-point keeps its
// real-space valence bands, its pair densities of the current conduction chunk, its
// weights for every frequency and its float64 partial sums resident; the conduction
// chunks, the band-transform scratch and the pair-transform intermediate are shared
// and reused q-point after q-point.  After the pair densities of chunk j exist for
// every q-point, one persistent contraction launch covers all (q, frequency, part,
// tile, pair range) items of that chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using gw::Geom;

namespace {

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

constexpr int kPairTarget = 32768;   // band pairs per conduction chunk
constexpr int kBandBatch = 32;       // bands per band-transform launch group

int mode_of(gw_precision p) { return p == GW_FP64 ? 0 : (p == GW_FP32 ? 1 : 2); }

std::string shape_key(const Geom& g, int nv, int ncol, gw_precision prec) {
  char b[160];
  snprintf(b, sizeof b, "nd%d_K%d_ngp%d_nv%d_nc%d_p%d", g.nd, g.K, g.ngp, nv, ncol, (int)prec);
  return b;
}

struct ProbPlan {
  const gw_chi0_problem* p = nullptr;
  int nvs = 0, cc = 0, npair = 0, ksplit = 1, ntl = 0, minb = 0;
  size_t off_psiv = 0, off_m = 0, off_w = 0, off_acc = 0, acc_one = 0;
  size_t off_m2 = 0, off_w2 = 0;   // second pair-density / weight buffers of the forward build
  size_t off_img = 0, off_img2 = 0;   // static split-bf16 x3: bf16 row images of M and w M per buffer
};

struct Layout {
  bool fp64 = true;
  size_t csz = 16;
  int nparts = 1, nomega = 1, mode = 0;
  bool images = false;   // static split-bf16 x3 forward: the contraction reads split row images (mode 3)
  std::vector<ProbPlan> pp;
  size_t off_psic = 0, off_scr = 0, off_q = 0, off_part = 0, off_dx = 0, off_dn = 0, off_counter = 0, total = 0;
  size_t off_gsplit = 0;   // backward, split-bf16 mode: chibar split into bf16 row images
  size_t off_msplit = 0;   // and the chunk's pair densities, split the same way
  // coefficient gradients (backward, float64): mbar and a weighted copy of M per chunk,
  // ubar of the chunk's columns and of the valence slots, column gradients of a chunk
  size_t off_mbar = 0, off_atmp = 0, off_ubarc = 0, off_ubarv = 0, off_cbar = 0;
  int max_cc = 0;
};

// Contraction work items of one problem per job (frequency, part).
int items_per_job(const ProbPlan& q) { return q.ntl * q.ksplit; }

Layout make_layout(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, bool complex_w, gw_precision prec,
                   bool backward, int force_ksplit = 0) {
  Layout L;
  L.fp64 = prec == GW_FP64;
  L.csz = L.fp64 ? 16 : 8;
  L.nparts = complex_w ? 2 : 1;
  L.nomega = nomega;
  L.mode = mode_of(prec);
  L.images = !backward && L.mode == 2 && nomega == 1 && !complex_w;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  long long items = 0;
  for (int i = 0; i < nprob; ++i) {
    const Geom& g = probs[i].geom->g;
    ProbPlan q;
    q.p = &probs[i];
    q.nvs = (int)round_up(probs[i].nv, 4);
    int cc = std::max(8, (kPairTarget / q.nvs) / 8 * 8);
    q.cc = std::min<int>(cc, (int)round_up(probs[i].ncol, 8));
    q.npair = q.nvs * q.cc;
    const int nt = g.ngp / gw::contract_tile(L.mode);
    q.ntl = nt * (nt + 1) / 2;
    items += (long long)q.ntl * nomega * L.nparts;
    L.pp.push_back(q);
  }
  // Split the pair ranges so that (a) the batch has about 8 items per CU and (b) for a
  // single job, the rows of M that the items in flight share (one pair range) stay near
  // 32 MB, so they are served from cache instead of HBM (with several jobs the items of one
  // range already share their rows).  Every split costs a float64 partial NG^2 per job, so
  // the splits are capped to keep the partials within 16 GB (or their unsplit size).  A
  // tuned choice overrides.
  // The row-image contraction (static split-BF16x3) runs a static grid of two workgroups per
  // CU and reads its operands through L2 in tile order, so it wants only about two items per
  // workgroup and no cache-sized ranges: every split adds a float64 read-modify-write of a
  // 256 KB partial per item (one 128^3 / NG 8000 chunk of 32k pairs: 21.1 ms unsplit, 21.8 with
  // 4 splits, 25.6 with 32).
  const long long want = L.images ? 4LL * 256 : 8LL * 256;
  const int ks_par = items >= want ? 1 : (int)std::min<long long>(32, (want + items - 1) / items);
  const int njobs = nomega * L.nparts;
  size_t acc1 = 0;   // partials of all problems with one split each
  for (const auto& q : L.pp) acc1 += (size_t)q.p->geom->g.ngp * q.p->geom->g.ngp * sizeof(double2) * njobs;
  const int ks_mem = (int)std::max<size_t>(1, (size_t(16) << 30) / std::max<size_t>(acc1, 1));
  for (auto& q : L.pp) {
    const size_t mbytes = (size_t)q.npair * q.p->geom->g.ngp * L.csz;
    const int ks_cache = njobs > 1 || L.images ? 1 : (int)std::min<size_t>(32, (mbytes + (32u << 20) - 1) / (32u << 20));
    int k = std::min(std::max(ks_par, ks_cache), ks_mem);
    auto it = ctx->tune.find(shape_key(q.p->geom->g, q.p->nv, q.p->ncol, prec));
    if (it != ctx->tune.end()) {
      q.minb = it->second.first;
      if (it->second.second > 0) k = it->second.second;
    }
    if (force_ksplit) k = force_ksplit;
    q.ksplit = std::max(1, std::min(k, std::max(1, q.npair / 64)));
  }
  size_t max_psic = 0, max_scr = 0, max_q = 0, max_part = 0, max_np = 0;
  for (auto& q : L.pp) {
    const Geom& g = q.p->geom->g;
    const size_t npts = (size_t)g.nd * g.nd * g.nd;
    q.off_psiv = take((size_t)q.nvs * npts * L.csz);
    q.off_m = take((size_t)q.npair * g.ngp * L.csz);
    q.off_w = take((size_t)nomega * L.nparts * q.npair * sizeof(double));
    // the forward build alternates two buffers between consecutive conduction chunks
    q.off_m2 = backward ? q.off_m : take((size_t)q.npair * g.ngp * L.csz);
    q.off_w2 = backward ? q.off_w : take((size_t)nomega * L.nparts * q.npair * sizeof(double));
    q.acc_one = (size_t)q.ksplit * g.ngp * g.ngp * sizeof(double2);
    q.off_acc = backward ? 0 : take(q.acc_one * nomega * L.nparts);
    if (L.images) {
      q.off_img = take(gw::split_image_bytes(q.npair, g.ngp));
      q.off_img2 = take(gw::split_image_bytes(q.npair, g.ngp));
    }
    max_psic = std::max(max_psic, (size_t)q.cc * npts * L.csz);
    max_scr = std::max(max_scr, gw::band_scratch_bytes(g, kBandBatch, L.fp64));
    max_q = std::max(max_q, (size_t)q.npair * g.nd * g.K * g.K * L.csz);
    max_part = std::max(max_part, gw::adjoint_partial_bytes(q.npair, g.ngp));
    max_np = std::max(max_np, (size_t)q.npair);
    L.max_cc = std::max(L.max_cc, q.cc);
  }
  L.off_psic = take(max_psic);
  L.off_scr = take(max_scr);
  L.off_q = take(max_q);
  if (backward) {
    L.off_part = take(max_part);
    if (L.mode == 2) {
      size_t gs = 0;
      size_t ms = 0;
      for (const auto& q : L.pp) {
        gs = std::max(gs, gw::gbar_split_bytes(q.p->geom->g.ng));
        ms = std::max(ms, gw::m_split_bytes(q.npair, q.p->geom->g.ng));
      }
      L.off_gsplit = take(gs);
      L.off_msplit = take(ms);
    }
    L.off_dx = take(max_np * sizeof(double));
    L.off_dn = take(max_np * sizeof(double));
    if (L.fp64) {
      size_t mb = 0, uc = 0, uv = 0, cb = 0;
      for (const auto& q : L.pp) {
        const Geom& g = q.p->geom->g;
        const size_t npts = (size_t)g.nd * g.nd * g.nd;
        mb = std::max(mb, (size_t)q.npair * g.ngp * sizeof(double2));
        uc = std::max(uc, (size_t)q.cc * npts * sizeof(double2));
        uv = std::max(uv, (size_t)q.nvs * npts * sizeof(double2));
        cb = std::max(cb, (size_t)std::max(q.cc, kBandBatch) * g.npw * sizeof(double2));
      }
      L.off_mbar = take(mb);
      L.off_atmp = take(mb);
      L.off_ubarc = take(uc);
      L.off_ubarv = take(uv);
      L.off_cbar = take(cb);
    }
  }
  L.off_counter = take(256);
  L.total = o;
  return L;
}

gw_status band_to_real(gw_ctx* ctx, const Layout& L, const Geom& g, const double2* coef, int nrows,
                       const int32_t* band_idx, int band0, int nvalid, int nslot, char* ws, char* psi) {
  const size_t npts = (size_t)g.nd * g.nd * g.nd;
  for (int s0 = 0; s0 < nslot; s0 += kBandBatch) {
    const int ns = std::min(kBandBatch, nslot - s0);
    void* tB = ws + L.off_scr;
    void* out = psi + (size_t)s0 * npts * L.csz;
    gw::StageScope sc(ctx, gw::kStageBand);
    hipError_t e = L.fp64 ? gw::launch_band_to_real<double>(g, coef, nrows, band_idx, band0 + s0, nvalid, ns, tB,
                                                            out, ctx->stream)
                          : gw::launch_band_to_real<float>(g, coef, nrows, band_idx, band0 + s0, nvalid, ns, tB,
                                                           out, ctx->stream);
    GW_HIP(ctx, e);
  }
  return GW_OK;
}

// pair densities of problem q for the conduction chunk already in the shared psi_c
gw_status pair_block(gw_ctx* ctx, const Layout& L, const ProbPlan& q, char* ws) {
  const Geom& g = q.p->geom->g;
  hipError_t e;
  {
    gw::StageScope sc(ctx, gw::kStagePlanes);
    e = L.fp64 ? gw::launch_pair_planes<double>(g, ws + q.off_psiv, ws + L.off_psic, q.nvs, q.cc, ws + L.off_q, q.minb,
                                                ctx->stream)
               : gw::launch_pair_planes<float>(g, ws + q.off_psiv, ws + L.off_psic, q.nvs, q.cc, ws + L.off_q, q.minb,
                                               ctx->stream);
  }
  GW_HIP(ctx, e);
  {
    gw::StageScope sc(ctx, gw::kStageFinish);
    e = L.fp64 ? gw::launch_pair_finish<double>(g, ws + L.off_q, q.npair, ws + q.off_m, ctx->stream)
               : gw::launch_pair_finish<float>(g, ws + L.off_q, q.npair, ws + q.off_m, ctx->stream);
  }
  GW_HIP(ctx, e);
  return GW_OK;
}

gw_status check_problem(gw_ctx* ctx, const gw_chi0_problem& p) {
  if (!p.geom) return gw::fail(ctx, GW_EINVAL, "problem without geometry");
  if (p.nv < 1 || p.ncol < 1 || p.nband < 1) return gw::fail(ctx, GW_EINVAL, "nv, nband and ncol must be >= 1");
  if (!p.coef_v || !p.e_v || !p.coef_c || !p.e_col) return gw::fail(ctx, GW_EINVAL, "NULL band data pointer");
  if (!p.col_band && p.ncol > p.nband) return gw::fail(ctx, GW_EINVAL, "ncol > nband without col_band");
  return GW_OK;
}

// Checks the values behind the problems' device pointers (finite energies, multiplicities
// >= 0, column rows in range) with one small kernel and a synchronising read of its flag.
// Skipped while the context's stream is being captured into a graph (a synchronisation is
// not allowed there): the kernels then never read or write outside the coefficient rows
// (column rows are clamped on reads and skipped on writes), and only the result is undefined.
gw_status check_values(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob) {
  if (ctx->stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GW_HIP(ctx, hipStreamIsCapturing(ctx->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return GW_OK;
  }
  GW_HIP(ctx, gw::launch_flag_clear(ctx->d_check_flag, ctx->stream));
  for (int i = 0; i < nprob; ++i) {
    const gw_chi0_problem& p = probs[i];
    GW_HIP(ctx, gw::launch_check_columns(p.e_v, p.nv, p.e_col, p.n_col, p.col_band, p.ncol, p.nband,
                                         ctx->d_check_flag, ctx->stream));
  }
  GW_HIP(ctx, hipMemcpyAsync(ctx->h_check_flag, ctx->d_check_flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  GW_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int f = *ctx->h_check_flag;
  if (f & 4) return gw::fail(ctx, GW_EINVAL, "a col_band entry is outside [0, nband)");
  if (f & 2) return gw::fail(ctx, GW_EINVAL, "a column multiplicity n_col is negative or not finite");
  if (f & 1) return gw::fail(ctx, GW_EINVAL, "a band or column energy is not finite");
  return GW_OK;
}

gw_status check_common(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                       double delta, gw_precision prec) {
  if (!probs || nprob < 1 || nomega < 1 || !omega) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return gw::fail(ctx, GW_EINVAL, "delta must be finite and >= 0");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return gw::fail(ctx, GW_EINVAL, "bad precision");
  for (int w = 0; w < nomega; ++w)
    if (!std::isfinite(omega[w])) return gw::fail(ctx, GW_EINVAL, "non-finite frequency");
  for (int i = 0; i < nprob; ++i) {
    gw_status s = check_problem(ctx, probs[i]);
    if (s != GW_OK) return s;
  }
  return GW_OK;
}

struct DeviceScope {
  int prev = 0;
  explicit DeviceScope(int dev) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
  }
  ~DeviceScope() { (void)hipSetDevice(prev); }
};

// Enqueue one batch (<= kMaxBatch problems) of the forward band sum.
// ksum: every problem's chi0 goes into the same output (a k-point sum), added in problem
// order after the first (or after earlier batches, with acc_out).
gw_status enqueue_build(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                        double delta, gw_precision prec, char* ws, size_t ws_bytes, char* out, bool ksum = false,
                        bool acc_out = false) {
  const Layout L = make_layout(ctx, probs, nprob, nomega, delta > 0.0, prec, false);
  if (L.total > ws_bytes)
    return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(L.total) + " bytes");
  for (const ProbPlan& q : L.pp) {
    GW_HIP(ctx, gw::launch_zero(ws + q.off_acc, q.acc_one * nomega * L.nparts, ctx->stream));
    gw_status s = band_to_real(ctx, L, q.p->geom->g, (const double2*)q.p->coef_v, q.p->nv, nullptr, 0, q.p->nv, q.nvs,
                               ws, ws + q.off_psiv);
    if (s != GW_OK) return s;
  }
  int nchunk = 0;
  for (const ProbPlan& q : L.pp) nchunk = std::max(nchunk, (q.p->ncol + q.cc - 1) / q.cc);
  // Chunk j uses buffer set j % 2.  With overlap, its contraction runs on the side stream:
  // ev_ready[b] (main) -> contraction j (side) -> ev_free[b] (side) -> transforms of
  // chunk j + 2 (main), and ev_join before the finalisation.
  // Overlap pays where the contraction leaves registers for a pair-kernel workgroup on the
  // same CU and is small beside the transforms: the split-BF16x3 form at one 512-thread
  // workgroup per CU (146 VGPRs) with dielectric spheres up to 2048 (measured 214.7 ms per
  // 72^3 / 512k-pair / NG 2000 step, against 221.4 ms without overlap, where the contraction
  // alone runs two workgroups per CU at 128 VGPRs).  With larger spheres the contraction
  // alone is the faster choice (96^3 / NG 4000 grouped step: 1.599 s alone, 1.632 s
  // overlapped).  The float64 and float32 contractions fill the register file, so the next
  // chunk's transforms queue behind them (no gain measured; capping the contraction at one
  // workgroup per CU made float64 slower, 519 -> 558 ms).  The static split-BF16x3 build reads
  // row images with workgroups that fill each CU's LDS (measured with two 80 KB workgroups per
  // CU; the current form takes 120 KB in one), which leave nothing for the transforms: no gain
  // either (72^3, 8 chunks of 32k pairs: 101.2 ms overlapped, 100.9 alone; 128^3, 4 chunks:
  // 473 / 475 ms), so overlap is left to the register-staged form.
  int max_ngp = 0;
  for (const ProbPlan& q : L.pp) max_ngp = std::max(max_ngp, q.p->geom->g.ngp);
  const bool ovl =
      nchunk > 1 && (ctx->overlap == 2 || (ctx->overlap == 1 && L.mode == 2 && !L.images && max_ngp <= 2048));
  hipStream_t cs = ovl ? ctx->side : ctx->stream;
  auto chunk = [&](int j) -> gw_status {
    const int buf = j & 1;
    if (ovl && j >= 2) GW_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_free[buf], 0));
    gw::ContractBatch bt{};
    std::vector<int> active;
    std::vector<ProbPlan> plans(L.pp.size());
    for (int i = 0; i < (int)L.pp.size(); ++i) {
      ProbPlan& q = plans[i];
      q = L.pp[i];
      if (buf) {
        q.off_m = q.off_m2;
        q.off_w = q.off_w2;
        q.off_img = q.off_img2;
      }
      const int c0 = j * q.cc;
      if (c0 >= q.p->ncol) continue;
      gw_status s = band_to_real(ctx, L, q.p->geom->g, (const double2*)q.p->coef_c, q.p->nband, q.p->col_band, c0,
                                 q.p->ncol, q.cc, ws, ws + L.off_psic);
      if (s != GW_OK) return s;
      {
        gw::StageScope sc(ctx, gw::kStageWeights);
        for (int iw = 0; iw < nomega; ++iw)
          GW_HIP(ctx, gw::launch_weights(q.p->e_v, 0, q.p->nv, q.nvs, q.p->e_col, q.p->n_col, c0, q.p->ncol, q.cc,
                                         omega[iw], delta, L.nparts,
                                         (double*)(ws + q.off_w) + (size_t)iw * L.nparts * q.npair, ctx->stream));
      }
      s = pair_block(ctx, L, q, ws);
      if (s != GW_OK) return s;
      if (L.images) {
        gw::StageScope sc(ctx, gw::kStageContract);
        GW_HIP(ctx, gw::launch_split_ab(ws + q.off_m, (const double*)(ws + q.off_w), q.npair, q.p->geom->g.ngp,
                                        ws + q.off_img, ctx->stream));
      }
      active.push_back(i);
    }
    if (ovl) {
      GW_HIP(ctx, hipEventRecord(ctx->ev_ready[buf], ctx->stream));
      GW_HIP(ctx, hipStreamWaitEvent(cs, ctx->ev_ready[buf], 0));
    }
    // largest dielectric spheres first
    std::stable_sort(active.begin(), active.end(), [&](int a, int b) {
      return L.pp[a].p->geom->g.ngp > L.pp[b].p->geom->g.ngp;
    });
    bt.nprob = (int)active.size();
    long long item = 0;
    for (int k = 0; k < bt.nprob; ++k) {
      const ProbPlan& q = plans[active[k]];
      bt.item0[k] = item;
      bt.p[k] = gw::ContractProb{ws + q.off_m, (const double*)(ws + q.off_w), (double2*)(ws + q.off_acc), q.npair,
                                 q.p->geom->g.ngp, q.ksplit, q.ntl};
      if (L.images) {
        bt.p[k].aimg = ws + q.off_img;
        bt.p[k].bimg = ws + q.off_img + (size_t)q.npair / 16 * q.p->geom->g.ngp * 8 * 16;
      }
      item += (long long)items_per_job(q) * nomega * L.nparts;
    }
    bt.item0[bt.nprob] = item;
    int* counter = (int*)(ws + L.off_counter);
    GW_HIP(ctx, gw::launch_zero(counter, 256, cs));
    const int grid = (int)std::min<long long>(item, 256LL * 8);
    {
      gw::StageScope sc(ctx, gw::kStageContract, cs);
      GW_HIP(ctx, gw::launch_contract_batch(L.images ? 3 : L.mode, bt, counter, grid, !ovl, cs));
    }
    if (ovl) GW_HIP(ctx, hipEventRecord(ctx->ev_free[buf], cs));
    return GW_OK;
  };
  gw_status cst = GW_OK;
  for (int j = 0; j < nchunk && cst == GW_OK; ++j) cst = chunk(j);
  if (ovl) {   // join the side stream, also after an error
    GW_HIP(ctx, hipEventRecord(ctx->ev_join, cs));
    GW_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
  }
  if (cst != GW_OK) return cst;
  for (size_t i = 0; i < L.pp.size(); ++i) {
    const ProbPlan& q = L.pp[i];
    const Geom& g = q.p->geom->g;
    char* o = out;
    for (int iw = 0; iw < nomega; ++iw) {
      const double2* accA = (const double2*)(ws + q.off_acc + q.acc_one * ((size_t)iw * L.nparts));
      const double2* accB = L.nparts == 2 ? accA + q.acc_one / sizeof(double2) : nullptr;
      gw::StageScope sc(ctx, gw::kStageFinalize);
      GW_HIP(ctx, gw::launch_finalize(accA, accB, q.ksplit, g.ng, g.ngp, (double2*)o, ksum && (i > 0 || acc_out),
                                      ctx->stream));
      o += (size_t)g.ng * g.ng * sizeof(double2);
    }
    if (!ksum) out = o;
  }
  return GW_OK;
}

gw_status enqueue_build_all(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                            double delta, gw_precision prec, char* ws, size_t ws_bytes, char* out, bool ksum = false) {
  for (int b0 = 0; b0 < nprob; b0 += gw::kMaxBatch) {
    const int nb = std::min(gw::kMaxBatch, nprob - b0);
    gw_status s = enqueue_build(ctx, probs + b0, nb, nomega, omega, delta, prec, ws, ws_bytes, out, ksum, b0 > 0);
    if (s != GW_OK) return s;
    if (!ksum)
      for (int i = b0; i < b0 + nb; ++i) out += (size_t)nomega * probs[i].geom->g.ng * probs[i].geom->g.ng * 16;
  }
  return GW_OK;
}

// Coefficient gradients of one conduction chunk (float64; M of the chunk in the
// workspace): mbar = sum_w [conj(w) chi0bar m + w chi0bar^H m], its transpose through the
// finish stage into the Q buffer, then the column gradients of the chunk (added into gcc
// through col_band) and, with want_v, the chunk's share of ubar_v.
gw_status coef_grad_chunk(gw_ctx* ctx, const Layout& L, const ProbPlan& q, const Geom& g, const double* omega,
                          int nomega, double delta, const double2* gbar, int c0, char* ws, double2* gcc, bool want_v) {
  const gw_chi0_problem& p = *q.p;
  const size_t npts = (size_t)g.nd * g.nd * g.nd;
  double* w = (double*)(ws + q.off_w);
  GW_HIP(ctx, gw::launch_fill_c128(ws + L.off_mbar, (size_t)q.npair * g.ngp, ctx->stream));
  for (int iw = 0; iw < nomega; ++iw) {
    GW_HIP(ctx, gw::launch_weights(p.e_v, 0, p.nv, q.nvs, p.e_col, p.n_col, c0, p.ncol, q.cc, omega[iw], delta,
                                   L.nparts, w, ctx->stream));
    const double2* gb = gbar + (size_t)iw * g.ng * g.ng;
    // mbar += diag(conj w) M chi0bar^T  (rows: pairs, columns: G)
    GW_HIP(ctx, gw::launch_weight_rows(ws + q.off_m, q.npair, g.ngp, w, L.nparts, true, ws + L.off_atmp, ctx->stream));
    GW_HIP(ctx, gw::launch_zgemm_op(q.npair, g.ng, g.ng, double2{1.0, 0.0}, (const double2*)(ws + L.off_atmp), g.ngp,
                                    gw::kOpN, gb, g.ng, gw::kOpT, double2{1.0, 0.0}, (double2*)(ws + L.off_mbar), g.ngp,
                                    ctx->stream));
    // mbar += diag(w) M conj(chi0bar)
    GW_HIP(ctx, gw::launch_weight_rows(ws + q.off_m, q.npair, g.ngp, w, L.nparts, false, ws + L.off_atmp, ctx->stream));
    GW_HIP(ctx, gw::launch_zgemm_op(q.npair, g.ng, g.ng, double2{1.0, 0.0}, (const double2*)(ws + L.off_atmp), g.ngp,
                                    gw::kOpN, gb, g.ng, gw::kOpConj, double2{1.0, 0.0}, (double2*)(ws + L.off_mbar),
                                    g.ngp, ctx->stream));
  }
  GW_HIP(ctx, gw::launch_qbar(g, ws + L.off_mbar, q.npair, ws + L.off_q, ctx->stream));
  if (gcc) {
    GW_HIP(ctx, gw::launch_ubar(g, ws + L.off_q, ws + q.off_psiv, q.nvs, q.cc, true, ws + L.off_ubarc, ctx->stream));
    const int nvalid = std::min(q.cc, p.ncol - c0);
    for (int s0 = 0; s0 < nvalid; s0 += kBandBatch) {
      const int ns = std::min(kBandBatch, nvalid - s0);
      GW_HIP(ctx, gw::launch_band_from_real(g, ws + L.off_ubarc + (size_t)s0 * npts * sizeof(double2), ns,
                                            ws + L.off_scr, ws + L.off_cbar + (size_t)s0 * g.npw * sizeof(double2),
                                            ctx->stream));
    }
    GW_HIP(ctx, gw::launch_scatter_cols(ws + L.off_cbar, nvalid, p.col_band, c0, g.npw, p.nband, gcc, ctx->stream));
  }
  if (want_v)
    GW_HIP(ctx, gw::launch_ubar(g, ws + L.off_q, ws + L.off_psic, q.nvs, q.cc, false, ws + L.off_ubarv, ctx->stream));
  return GW_OK;
}

std::string graph_key(const gw_chi0_problem* probs, int nprob, int nomega, const double* omega, double delta,
                      gw_precision prec, const void* ws, size_t ws_bytes, const void* out, bool ksum) {
  std::string k;
  auto add = [&](const void* p, size_t n) { k.append((const char*)p, n); };
  add(&ksum, sizeof ksum);
  add(&nprob, sizeof nprob);
  add(probs, sizeof(gw_chi0_problem) * nprob);
  add(&nomega, sizeof nomega);
  add(omega, sizeof(double) * nomega);
  add(&delta, sizeof delta);
  add(&prec, sizeof prec);
  add(&ws, sizeof ws);
  add(&ws_bytes, sizeof ws_bytes);
  add(&out, sizeof out);
  for (int i = 0; i < nprob; ++i) add(&probs[i].geom->id, sizeof probs[i].geom->id);
  return k;
}

}  // namespace

extern "C" {

gw_status gw_chi0_workspace_size(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega,
                                 gw_precision prec, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!probs || nprob < 1 || nomega < 1 || !bytes) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return gw::fail(ctx, GW_EINVAL, "bad precision");
  size_t mx = 0;
  for (int i = 0; i < nprob; ++i) {
    gw_status s = check_problem(ctx, probs[i]);
    if (s != GW_OK) return s;
  }
  for (int b0 = 0; b0 < nprob; b0 += gw::kMaxBatch) {
    const int nb = std::min(gw::kMaxBatch, nprob - b0);
    // static and dynamic layouts split the contraction differently (one job, or two
    // parts per frequency), so either can be the larger
    for (const bool dyn : {false, true}) {
      const Layout f = make_layout(ctx, probs + b0, nb, nomega, dyn, prec, false);
      const Layout b = make_layout(ctx, probs + b0, nb, nomega, dyn, prec, true);
      mx = std::max({mx, f.total, b.total});
    }
  }
  *bytes = mx;
  return GW_OK;
}

}  // extern "C"

namespace {
gw_status build_entry(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                      double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0, bool ksum) {
  if (!ctx) return GW_EINVAL;
  gw_status s = check_common(ctx, probs, nprob, nomega, omega, delta, prec);
  if (s != GW_OK) return s;
  if (!chi0 || !workspace) return gw::fail(ctx, GW_EINVAL, "NULL workspace or output");
  if (ksum)
    for (int i = 1; i < nprob; ++i)
      if (probs[i].geom->g.ng != probs[0].geom->g.ng)
        return gw::fail(ctx, GW_EINVAL, "a k-point sum needs the same dielectric-sphere size in every problem");
  DeviceScope dev(ctx->device);
  if (!ctx->graph) {
    s = check_values(ctx, probs, nprob);
    if (s != GW_OK) return s;
    return enqueue_build_all(ctx, probs, nprob, nomega, omega, delta, prec, (char*)workspace, ws_bytes, (char*)chi0,
                             ksum);
  }
  // graph mode: replay the captured launch sequence of an identical call
  if (!ctx->stream) return gw::fail(ctx, GW_EINVAL, "graph mode needs a context on a non-null stream");
  const std::string key = graph_key(probs, nprob, nomega, omega, delta, prec, workspace, ws_bytes, chi0, ksum);
  for (auto& ge : ctx->graphs)
    if (ge.key == key) {
      GW_HIP(ctx, hipGraphLaunch(ge.exec, ctx->stream));
      return GW_OK;
    }
  s = check_values(ctx, probs, nprob);   // values are checked when a call is captured, not on replays
  if (s != GW_OK) return s;
  const bool timing = ctx->timing;
  ctx->timing = false;   // no event nodes in a captured graph
  GW_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  s = enqueue_build_all(ctx, probs, nprob, nomega, omega, delta, prec, (char*)workspace, ws_bytes, (char*)chi0, ksum);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  ctx->timing = timing;
  if (s != GW_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return gw::fail(ctx, GW_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return gw::fail(ctx, GW_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  std::vector<unsigned long long> ids;
  for (int i = 0; i < nprob; ++i) ids.push_back(probs[i].geom->id);
  ctx->graphs.push_back(gw_ctx::GraphEntry{key, graph, exec, ids});
  GW_HIP(ctx, hipGraphLaunch(exec, ctx->stream));
  return GW_OK;
}
}  // namespace

extern "C" {

gw_status gw_chi0_build(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                        double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0) {
  return build_entry(ctx, probs, nprob, nomega, omega, delta, prec, workspace, ws_bytes, chi0, false);
}

gw_status gw_chi0_build_ksum(gw_ctx* ctx, const gw_chi0_problem* probs, int nk, int nomega, const double* omega,
                             double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0) {
  return build_entry(ctx, probs, nk, nomega, omega, delta, prec, workspace, ws_bytes, chi0, true);
}

gw_status gw_ctx_set_graph(gw_ctx* ctx, int enable) {
  if (!ctx) return GW_EINVAL;
  ctx->graph = enable != 0;
  if (!ctx->graph) {
    for (auto& ge : ctx->graphs) {
      (void)hipGraphExecDestroy(ge.exec);
      (void)hipGraphDestroy(ge.graph);
    }
    ctx->graphs.clear();
  }
  return GW_OK;
}

}  // extern "C"

namespace {
// ksum: the problems are the k-points of one chi0 (gw_chi0_build_ksum), so every problem
// reads the same grad_chi0 block
gw_status backward_entry(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                         double delta, gw_precision prec, void* workspace, size_t ws_bytes, const void* grad_chi0,
                         double* grad_e_v, double* grad_e_col, double* grad_n_col, void* grad_coef_v,
                         void* grad_coef_c, bool ksum) {
  if (!ctx) return GW_EINVAL;
  if (ksum)
    for (int i = 1; i < nprob; ++i)
      if (probs && probs[i].geom && probs[0].geom && probs[i].geom->g.ng != probs[0].geom->g.ng)
        return gw::fail(ctx, GW_EINVAL, "a k-point sum needs the same dielectric-sphere size in every problem");
  gw_status st = check_common(ctx, probs, nprob, nomega, omega, delta, prec);
  if (st != GW_OK) return st;
  if (!grad_chi0 || !workspace) return gw::fail(ctx, GW_EINVAL, "NULL workspace or gradient");
  const bool want_coef = grad_coef_v || grad_coef_c;
  if (want_coef && prec != GW_FP64)
    return gw::fail(ctx, GW_EUNSUPPORTED, "coefficient gradients are computed in the float64 mode only");
  if (want_coef)
    for (int i = 0; i < nprob; ++i)
      if (probs && probs[i].geom && !gw::pair_instance(probs[i].geom->g.nd, probs[i].geom->g.K))
        return gw::fail(ctx, GW_EUNSUPPORTED,
                        "coefficient gradients need a compiled pair-transform instance for N = " +
                            std::to_string(probs[i].geom->g.nd) + ", K = " + std::to_string(probs[i].geom->g.K));
  DeviceScope dev(ctx->device);
  st = check_values(ctx, probs, nprob);
  if (st != GW_OK) return st;
  char* ws = (char*)workspace;
  const char* gin = (const char*)grad_chi0;
  size_t off_ev = 0, off_ec = 0, off_cv = 0, off_cc = 0;
  for (int ip = 0; ip < nprob; ++ip) {
    const gw_chi0_problem& p = probs[ip];
    const Geom& g = p.geom->g;
    const Layout L = make_layout(ctx, &p, 1, nomega, delta > 0.0, prec, true);
    if (L.total > ws_bytes) return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(L.total));
    const ProbPlan& q = L.pp[0];
    double* gev = grad_e_v ? grad_e_v + off_ev : nullptr;
    double* gec = grad_e_col ? grad_e_col + off_ec : nullptr;
    double* gn = grad_n_col ? grad_n_col + off_ec : nullptr;
    gw::StageScope sc(ctx, gw::kStageBackward);
    if (gev) GW_HIP(ctx, gw::launch_fill_f64(gev, p.nv, 0.0, ctx->stream));
    const size_t npts = (size_t)g.nd * g.nd * g.nd;
    double2* gcv = grad_coef_v ? (double2*)grad_coef_v + off_cv : nullptr;
    double2* gcc = grad_coef_c ? (double2*)grad_coef_c + off_cc : nullptr;
    if (gcc) GW_HIP(ctx, gw::launch_fill_c128(gcc, (size_t)p.nband * g.npw, ctx->stream));
    if (gcv) GW_HIP(ctx, gw::launch_fill_c128(ws + L.off_ubarv, (size_t)q.nvs * npts, ctx->stream));
    gw_status s = band_to_real(ctx, L, g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, q.nvs, ws, ws + q.off_psiv);
    if (s != GW_OK) return s;
    double* dx = (double*)(ws + L.off_dx);
    double* dn = (double*)(ws + L.off_dn);
    double2* part = (double2*)(ws + L.off_part);
    for (int c0 = 0; c0 < p.ncol; c0 += q.cc) {
      s = band_to_real(ctx, L, g, (const double2*)p.coef_c, p.nband, p.col_band, c0, p.ncol, q.cc, ws, ws + L.off_psic);
      if (s != GW_OK) return s;
      s = pair_block(ctx, L, q, ws);
      if (s != GW_OK) return s;
      GW_HIP(ctx, gw::launch_fill_f64(dx, q.npair, 0.0, ctx->stream));
      GW_HIP(ctx, gw::launch_fill_f64(dn, q.npair, 0.0, ctx->stream));
      if (L.mode == 2)
        GW_HIP(ctx, gw::launch_split_m(ws + q.off_m, q.npair, g.ng, g.ngp, ws + L.off_msplit, ctx->stream));
      for (int iw = 0; iw < nomega; ++iw) {
        const double2* gb = (const double2*)gin + (size_t)iw * g.ng * g.ng;
        hipError_t e =
            L.fp64        ? gw::launch_adjoint<double>(ws + q.off_m, q.npair, g.ng, g.ngp, gb, part, ctx->stream)
            : L.mode == 2 ? gw::launch_adjoint_bf16x3(ws + q.off_m, ws + L.off_msplit, q.npair, g.ng, g.ngp, gb,
                                                      ws + L.off_gsplit, part, ctx->stream)
                          : gw::launch_adjoint<float>(ws + q.off_m, q.npair, g.ng, g.ngp, gb, part, ctx->stream);
        GW_HIP(ctx, e);
        GW_HIP(ctx, gw::launch_adjoint_pairs(part, g.ngp / gw::adjoint_tile(L.mode), p.e_v, p.nv, q.nvs, p.e_col,
                                             p.n_col, c0, p.ncol, q.cc, omega[iw], delta, dx, dn, ctx->stream));
      }
      GW_HIP(ctx, gw::launch_adjoint_reduce(dx, dn, p.nv, q.cc, c0, p.ncol, gev, gec, gn, ctx->stream));
      if (want_coef) {
        s = coef_grad_chunk(ctx, L, q, g, omega, nomega, delta, (const double2*)gin, c0, ws, gcc, gcv != nullptr);
        if (s != GW_OK) return s;
      }
    }
    if (gcv) {
      // the valence gradients, from ubar_v summed over every chunk
      for (int s0 = 0; s0 < p.nv; s0 += kBandBatch) {
        const int ns = std::min(kBandBatch, p.nv - s0);
        GW_HIP(ctx, gw::launch_band_from_real(g, ws + L.off_ubarv + (size_t)s0 * npts * sizeof(double2), ns,
                                              ws + L.off_scr, gcv + (size_t)s0 * g.npw, ctx->stream));
      }
    }
    if (!ksum) gin += (size_t)nomega * g.ng * g.ng * sizeof(double2);
    off_ev += p.nv;
    off_ec += p.ncol;
    off_cv += (size_t)p.nv * g.npw;
    off_cc += (size_t)p.nband * g.npw;
  }
  return GW_OK;
}
}  // namespace

extern "C" {

gw_status gw_chi0_backward(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                           double delta, gw_precision prec, void* workspace, size_t ws_bytes, const void* grad_chi0,
                           double* grad_e_v, double* grad_e_col, double* grad_n_col, void* grad_coef_v,
                           void* grad_coef_c) {
  return backward_entry(ctx, probs, nprob, nomega, omega, delta, prec, workspace, ws_bytes, grad_chi0, grad_e_v,
                        grad_e_col, grad_n_col, grad_coef_v, grad_coef_c, false);
}

gw_status gw_chi0_backward_ksum(gw_ctx* ctx, const gw_chi0_problem* probs, int nk, int nomega, const double* omega,
                                double delta, gw_precision prec, void* workspace, size_t ws_bytes,
                                const void* grad_chi0, double* grad_e_v, double* grad_e_col, double* grad_n_col,
                                void* grad_coef_v, void* grad_coef_c) {
  return backward_entry(ctx, probs, nk, nomega, omega, delta, prec, workspace, ws_bytes, grad_chi0, grad_e_v,
                        grad_e_col, grad_n_col, grad_coef_v, grad_coef_c, true);
}

gw_status gw_pair_density_workspace_size(gw_ctx* ctx, const gw_chi0_problem* prob, int nvs, int ncs,
                                         gw_precision prec, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !bytes || nvs < 1 || ncs < 1) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  gw_status s = check_problem(ctx, *prob);
  if (s != GW_OK) return s;
  gw_chi0_problem sub = *prob;
  sub.nv = nvs;
  sub.ncol = ncs;
  *bytes = make_layout(ctx, &sub, 1, 1, false, prec, false).total;
  return GW_OK;
}

gw_status gw_pair_density(gw_ctx* ctx, const gw_chi0_problem* prob, int v0, int nvs, int c0, int ncs,
                          gw_precision prec, void* workspace, size_t ws_bytes, void* m_out) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !workspace || !m_out) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  gw_status s = check_problem(ctx, *prob);
  if (s != GW_OK) return s;
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return gw::fail(ctx, GW_EINVAL, "bad precision");
  if (nvs < 1 || ncs < 1 || v0 < 0 || c0 < 0 || v0 + nvs > prob->nv || c0 + ncs > prob->ncol)
    return gw::fail(ctx, GW_EINVAL, "pair block out of range");
  const Geom& g = prob->geom->g;
  gw_chi0_problem sub = *prob;
  sub.nv = nvs;
  sub.ncol = ncs;
  const Layout L = make_layout(ctx, &sub, 1, 1, false, prec, false);
  const ProbPlan& q = L.pp[0];
  if (q.cc < (int)round_up(ncs, 8)) return gw::fail(ctx, GW_EINVAL, "pair block too large for one pass");
  if (L.total > ws_bytes) return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(L.total));
  DeviceScope dev(ctx->device);
  s = check_values(ctx, prob, 1);
  if (s != GW_OK) return s;
  char* ws = (char*)workspace;
  s = band_to_real(ctx, L, g, (const double2*)prob->coef_v, prob->nv, nullptr, v0, v0 + nvs, q.nvs, ws, ws + q.off_psiv);
  if (s != GW_OK) return s;
  s = band_to_real(ctx, L, g, (const double2*)prob->coef_c, prob->nband, prob->col_band, c0, c0 + ncs, q.cc, ws,
                   ws + L.off_psic);
  if (s != GW_OK) return s;
  s = pair_block(ctx, L, q, ws);
  if (s != GW_OK) return s;
  GW_HIP(ctx, gw::launch_copy_m(ws + q.off_m, nvs, ncs, q.cc, g.ng, g.ngp, L.fp64, (double2*)m_out, ctx->stream));
  return GW_OK;
}

namespace {
// workspace of gw_sigma_coh_static: the float64 pair-transform layout of the states x one
// chunk of columns, A^T (padded), Z of one chunk and the reduction partials
struct CohLayout {
  Layout L;
  size_t off_a = 0, off_z = 0, off_part = 0, total = 0;
  int nblk = 0;
};
constexpr int kCohBlocks = 1024;

gw_status check_coh(gw_ctx* ctx, const gw_chi0_problem* p) {
  if (!p || !p->geom) return gw::fail(ctx, GW_EINVAL, "NULL problem or geometry");
  if (p->nv < 1 || p->nv > gw::coh_max_states())
    return gw::fail(ctx, GW_EINVAL, "1 .. " + std::to_string(gw::coh_max_states()) + " states");
  if (p->ncol < 1 || p->nband < 1 || !p->coef_v || !p->coef_c) return gw::fail(ctx, GW_EINVAL, "bad columns");
  if (!p->col_band && p->ncol > p->nband) return gw::fail(ctx, GW_EINVAL, "ncol > nband without col_band");
  return GW_OK;
}

CohLayout coh_layout(gw_ctx* ctx, const gw_chi0_problem& p) {
  CohLayout c;
  c.L = make_layout(ctx, &p, 1, 1, false, GW_FP64, false);
  const Geom& g = p.geom->g;
  const ProbPlan& q = c.L.pp[0];
  size_t o = c.L.total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  c.off_a = take((size_t)g.ngp * g.ngp * sizeof(double2));
  c.off_z = take((size_t)q.npair * g.ngp * sizeof(double2));
  c.nblk = kCohBlocks;
  c.off_part = take((size_t)c.nblk * p.nv * p.nv * sizeof(double2));
  c.total = o;
  return c;
}
}  // namespace

gw_status gw_sigma_coh_workspace_size(gw_ctx* ctx, const gw_chi0_problem* prob, size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!bytes) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  gw_status s = check_coh(ctx, prob);
  if (s != GW_OK) return s;
  *bytes = coh_layout(ctx, *prob).total;
  return GW_OK;
}

gw_status gw_sigma_coh_static(gw_ctx* ctx, const gw_chi0_problem* prob, const double* vcoul, const void* eps_inv,
                              void* workspace, size_t ws_bytes, void* sigma) {
  if (!ctx) return GW_EINVAL;
  gw_status s = check_coh(ctx, prob);
  if (s != GW_OK) return s;
  if (!vcoul || !eps_inv || !workspace || !sigma) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  const gw_chi0_problem& p = *prob;
  const CohLayout c = coh_layout(ctx, p);
  if (c.total > ws_bytes) return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(c.total));
  const Layout& L = c.L;
  const ProbPlan& q = L.pp[0];
  const Geom& g = p.geom->g;
  DeviceScope dev(ctx->device);
  s = check_values(ctx, prob, 1);
  if (s != GW_OK) return s;
  char* ws = (char*)workspace;
  GW_HIP(ctx, gw::launch_fill_c128(sigma, (size_t)p.nv * p.nv, ctx->stream));
  GW_HIP(ctx, gw::launch_coh_kernel(eps_inv, vcoul, g.ng, g.ngp, ws + c.off_a, ctx->stream));
  s = band_to_real(ctx, L, g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, q.nvs, ws, ws + q.off_psiv);
  if (s != GW_OK) return s;
  for (int c0 = 0; c0 < p.ncol; c0 += q.cc) {
    s = band_to_real(ctx, L, g, (const double2*)p.coef_c, p.nband, p.col_band, c0, p.ncol, q.cc, ws, ws + L.off_psic);
    if (s != GW_OK) return s;
    s = pair_block(ctx, L, q, ws);
    if (s != GW_OK) return s;
    // Z = conj(M) A^T over the padded sphere (zero rows and columns beyond ng)
    GW_HIP(ctx, gw::launch_zgemm_op(q.npair, g.ngp, g.ngp, double2{1.0, 0.0}, (const double2*)(ws + q.off_m), g.ngp,
                                    gw::kOpConj, (const double2*)(ws + c.off_a), g.ngp, gw::kOpN, double2{0.0, 0.0},
                                    (double2*)(ws + c.off_z), g.ngp, ctx->stream));
    const int nvalid = std::min(q.cc, p.ncol - c0);
    GW_HIP(ctx, gw::launch_coh_reduce(ws + q.off_m, ws + c.off_z, p.nv, q.cc, g.ngp, nvalid, p.n_col, c0, c.nblk,
                                      ws + c.off_part, sigma, ctx->stream));
  }
  return GW_OK;
}

namespace {
// workspace of gw_sigma_coh_gpp: per problem the float64 pair-transform layout of the states x
// one chunk of columns and the (B, wt) tiles (two ngp^2 complex arrays), the largest over the
// problems; then the tile partials of every (state block, state block, energy block) pass
struct GppCohLayout {
  size_t region = 0, off_part = 0, part_pass = 0, total = 0;
  int nsb = 0, neb = 0, ngp_max = 0;
};

GppCohLayout gpp_coh_layout(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, int nenergy) {
  GppCohLayout c;
  for (int i = 0; i < nq; ++i) {
    const Layout L = make_layout(ctx, probs + i, 1, 1, false, GW_FP64, false);
    const Geom& g = probs[i].geom->g;
    const size_t r = round_up(L.total, 256) + 2 * round_up((size_t)g.ngp * g.ngp * sizeof(double2), 256);
    c.region = std::max(c.region, r);
    c.ngp_max = std::max(c.ngp_max, g.ngp);
    c.part_pass = std::max(c.part_pass, gw::gpp_coh_part_bytes(g.ngp));
  }
  const int bs = gw::gpp_coh_states_per_block(), be = gw::gpp_coh_energies_per_pass();
  c.nsb = (probs[0].nv + bs - 1) / bs;
  c.neb = (nenergy + be - 1) / be;
  c.off_part = c.region;
  c.total = c.off_part + (size_t)c.nsb * c.nsb * c.neb * c.part_pass;
  return c;
}

gw_status check_gpp_coh(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, int nenergy, const double* energies,
                        double delta) {
  if (!probs || nq < 1) return gw::fail(ctx, GW_EINVAL, "no problems");
  for (int i = 0; i < nq; ++i) {
    gw_status s = check_coh(ctx, probs + i);
    if (s != GW_OK) return s;
    if (!probs[i].e_col) return gw::fail(ctx, GW_EINVAL, "the plasmon-pole form needs the column energies e_col");
    if (probs[i].nv != probs[0].nv) return gw::fail(ctx, GW_EINVAL, "every problem needs the same states");
    if (probs[i].geom->g.ngp % gw::gpp_coh_tile() != 0) return gw::fail(ctx, GW_EINVAL, "sphere padding");
  }
  if (nenergy < 1 || !energies) return gw::fail(ctx, GW_EINVAL, "nenergy must be >= 1");
  for (int j = 0; j < nenergy; ++j)
    if (!std::isfinite(energies[j])) return gw::fail(ctx, GW_EINVAL, "non-finite energy");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return gw::fail(ctx, GW_EINVAL, "delta must be finite and >= 0");
  return GW_OK;
}
}  // namespace

gw_status gw_sigma_coh_gpp_workspace_size(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, int nenergy,
                                          size_t* bytes) {
  if (!ctx) return GW_EINVAL;
  if (!bytes) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  const double e0 = 0.0;
  std::vector<double> zero(std::max(1, nenergy), e0);
  gw_status s = check_gpp_coh(ctx, probs, nq, nenergy, zero.data(), 0.0);
  if (s != GW_OK) return s;
  *bytes = gpp_coh_layout(ctx, probs, nq, nenergy).total;
  return GW_OK;
}

gw_status gw_sigma_coh_gpp(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, const double* const* vcoul,
                           const void* const* modes, int nenergy, const double* energies, double delta,
                           void* workspace, size_t ws_bytes, void* sigma) {
  if (!ctx) return GW_EINVAL;
  gw_status s = check_gpp_coh(ctx, probs, nq, nenergy, energies, delta);
  if (s != GW_OK) return s;
  if (!vcoul || !modes || !workspace || !sigma) return gw::fail(ctx, GW_EINVAL, "NULL argument");
  for (int i = 0; i < nq; ++i)
    if (!vcoul[i] || !modes[i]) return gw::fail(ctx, GW_EINVAL, "NULL Coulomb factors or plasmon-pole modes");
  const GppCohLayout c = gpp_coh_layout(ctx, probs, nq, nenergy);
  if (c.total > ws_bytes) return gw::fail(ctx, GW_EINVAL, "workspace too small: need " + std::to_string(c.total));
  DeviceScope dev(ctx->device);
  s = check_values(ctx, probs, nq);
  if (s != GW_OK) return s;
  char* ws = (char*)workspace;
  const int ns = probs[0].nv;
  const int be = gw::gpp_coh_energies_per_pass();
  GW_HIP(ctx, gw::launch_fill_c128(sigma, (size_t)nenergy * ns * ns, ctx->stream));
  GW_HIP(ctx, gw::launch_fill_c128(ws + c.off_part, (c.total - c.off_part) / sizeof(double2), ctx->stream));
  auto pass_part = [&](int sa, int sb, int eb) {
    return ws + c.off_part + ((size_t)(sa * c.nsb + sb) * c.neb + eb) * c.part_pass;
  };
  for (int iq = 0; iq < nq; ++iq) {
    const gw_chi0_problem& p = probs[iq];
    const Layout L = make_layout(ctx, &p, 1, 1, false, GW_FP64, false);
    const ProbPlan& q = L.pp[0];
    const Geom& g = p.geom->g;
    char* bw = ws + round_up(L.total, 256);
    char* wt = bw + round_up((size_t)g.ngp * g.ngp * sizeof(double2), 256);
    GW_HIP(ctx, gw::launch_gpp_coh_prep(modes[iq], vcoul[iq], g.ng, g.ngp, bw, wt, ctx->stream));
    s = band_to_real(ctx, L, g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, q.nvs, ws, ws + q.off_psiv);
    if (s != GW_OK) return s;
    for (int c0 = 0; c0 < p.ncol; c0 += q.cc) {
      s = band_to_real(ctx, L, g, (const double2*)p.coef_c, p.nband, p.col_band, c0, p.ncol, q.cc, ws,
                       ws + L.off_psic);
      if (s != GW_OK) return s;
      s = pair_block(ctx, L, q, ws);
      if (s != GW_OK) return s;
      const int nvalid = std::min(q.cc, p.ncol - c0);
      for (int sa = 0; sa < c.nsb; ++sa)
        for (int sb = 0; sb < c.nsb; ++sb)
          for (int eb = 0; eb < c.neb; ++eb)
            GW_HIP(ctx, gw::launch_gpp_coh(bw, wt, g.ngp, ws + q.off_m, q.cc, ns, sa, sb, nvalid, p.e_col, p.n_col,
                                           c0, energies + eb * be, std::min(be, nenergy - eb * be), delta,
                                           pass_part(sa, sb, eb), ctx->stream));
    }
  }
  for (int sa = 0; sa < c.nsb; ++sa)
    for (int sb = 0; sb < c.nsb; ++sb)
      for (int eb = 0; eb < c.neb; ++eb)
        GW_HIP(ctx, gw::launch_gpp_coh_sum(pass_part(sa, sb, eb), c.ngp_max, std::min(be, nenergy - eb * be), ns, sa,
                                           sb, eb * be, sigma, ctx->stream));
  return GW_OK;
}

// Launch-shape tuner: times the candidates of the tunable launches on the first chunk
// of each problem shape and keeps the fastest in the context.
gw_status gw_tune(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, gw_precision prec,
                  void* workspace, size_t ws_bytes) {
  if (!ctx) return GW_EINVAL;
  std::vector<double> om(std::max(1, nomega), 0.0);
  gw_status s = check_common(ctx, probs, nprob, std::max(1, nomega), om.data(), 0.0, prec);
  if (s != GW_OK) return s;
  if (!workspace) return gw::fail(ctx, GW_EINVAL, "NULL workspace");
  if (ctx->graph) return gw::fail(ctx, GW_EINVAL, "disable graph mode while tuning");
  DeviceScope dev(ctx->device);
  char* ws = (char*)workspace;
  hipEvent_t a, b;
  GW_HIP(ctx, hipEventCreate(&a));
  GW_HIP(ctx, hipEventCreate(&b));
  auto timed = [&](auto&& fn, float* ms) -> gw_status {
    GW_HIP(ctx, hipEventRecord(a, ctx->stream));
    gw_status r = fn();
    if (r != GW_OK) return r;
    GW_HIP(ctx, hipEventRecord(b, ctx->stream));
    GW_HIP(ctx, hipEventSynchronize(b));
    GW_HIP(ctx, hipEventElapsedTime(ms, a, b));
    return GW_OK;
  };
  const bool timing = ctx->timing;
  ctx->timing = false;
  gw_status result = GW_OK;
  for (int ip = 0; ip < nprob && result == GW_OK; ++ip) {
    const gw_chi0_problem& p = probs[ip];
    const std::string key = shape_key(p.geom->g, p.nv, p.ncol, prec);
    int best_minb = 0, best_ks = 0;
    float best = 1e30f;
    // pair kernel: 256 threads with one or two resident workgroups per CU, or the 512-thread split-line form
    Layout L = make_layout(ctx, &p, 1, std::max(1, nomega), false, prec, false);
    if (L.total > ws_bytes) {
      result = gw::fail(ctx, GW_EINVAL, "workspace too small for tuning");
      break;
    }
    ProbPlan q = L.pp[0];
    GW_HIP(ctx, gw::launch_weights(p.e_v, 0, p.nv, q.nvs, p.e_col, p.n_col, 0, p.ncol, q.cc, 0.0, 0.0, 1,
                                   (double*)(ws + q.off_w), ctx->stream));
    result = band_to_real(ctx, L, p.geom->g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, q.nvs, ws, ws + q.off_psiv);
    if (result == GW_OK)
      result = band_to_real(ctx, L, p.geom->g, (const double2*)p.coef_c, p.nband, p.col_band, 0, p.ncol, q.cc, ws,
                            ws + L.off_psic);
    for (int minb = 1; minb <= gw::kPairVariants && result == GW_OK; ++minb) {
      q.minb = minb;
      float t0 = 0, t1 = 0;
      result = timed([&] { return pair_block(ctx, L, q, ws); }, &t0);   // warm-up
      if (result == GW_OK) result = timed([&] { return pair_block(ctx, L, q, ws); }, &t1);
      if (result == GW_OK && t1 < best) {
        best = t1;
        best_minb = minb;
      }
    }
    // contraction: pair-range splits
    best = 1e30f;
    for (int ks : {1, 2, 4, 8, 16, 32}) {
      if (result != GW_OK) break;
      Layout Lk = make_layout(ctx, &p, 1, std::max(1, nomega), false, prec, false, ks);
      if (Lk.total > ws_bytes) continue;
      const ProbPlan& qk = Lk.pp[0];
      if (qk.ksplit != ks) continue;
      result = band_to_real(ctx, Lk, p.geom->g, (const double2*)p.coef_v, p.nv, nullptr, 0, p.nv, qk.nvs, ws,
                            ws + qk.off_psiv);
      if (result != GW_OK) break;
      result = band_to_real(ctx, Lk, p.geom->g, (const double2*)p.coef_c, p.nband, p.col_band, 0, p.ncol, qk.cc, ws,
                            ws + Lk.off_psic);
      if (result != GW_OK) break;
      GW_HIP(ctx, gw::launch_weights(p.e_v, 0, p.nv, qk.nvs, p.e_col, p.n_col, 0, p.ncol, qk.cc, 0.0, 0.0, 1,
                                     (double*)(ws + qk.off_w), ctx->stream));
      result = pair_block(ctx, Lk, qk, ws);
      if (result != GW_OK) break;
      gw::ContractBatch bt{};
      bt.nprob = 1;
      bt.item0[0] = 0;
      bt.item0[1] = items_per_job(qk);
      bt.p[0] = gw::ContractProb{ws + qk.off_m, (const double*)(ws + qk.off_w), (double2*)(ws + qk.off_acc), qk.npair,
                                 p.geom->g.ngp, qk.ksplit, qk.ntl};
      int* counter = (int*)(ws + Lk.off_counter);
      const int grid = (int)std::min<long long>(bt.item0[1], 256LL * 8);
      float t = 0;
      for (int rep = 0; rep < 2 && result == GW_OK; ++rep) {
        result = timed(
            [&]() -> gw_status {
              GW_HIP(ctx, gw::launch_zero(ws + qk.off_acc, qk.acc_one, ctx->stream));
              GW_HIP(ctx, gw::launch_zero(counter, 256, ctx->stream));
              GW_HIP(ctx, gw::launch_contract_batch(Lk.mode, bt, counter, grid, true, ctx->stream));
              return GW_OK;
            },
            &t);
      }
      if (result == GW_OK && t < best) {
        best = t;
        best_ks = ks;
      }
    }
    if (result == GW_OK && best_minb && best_ks) ctx->tune[key] = std::make_pair(best_minb, best_ks);
  }
  ctx->timing = timing;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return result;
}

gw_status gw_tune_set(gw_ctx* ctx, const gw_chi0_problem* prob, gw_precision prec, int pair_variant, int ksplit) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !prob->geom) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  if (prec != GW_FP64 && prec != GW_FP32 && prec != GW_BF16X3) return gw::fail(ctx, GW_EINVAL, "bad precision");
  if (pair_variant < 0 || pair_variant > gw::kPairVariants || ksplit < 0 || ksplit > 32)
    return gw::fail(ctx, GW_EINVAL, "pair-kernel form or split count out of range");
  const std::string key = shape_key(prob->geom->g, prob->nv, prob->ncol, prec);
  if (pair_variant == 0 && ksplit == 0)
    ctx->tune.erase(key);
  else
    ctx->tune[key] = std::make_pair(pair_variant, ksplit);
  return GW_OK;
}

gw_status gw_tune_get(gw_ctx* ctx, const gw_chi0_problem* prob, gw_precision prec, int* pair_variant, int* ksplit) {
  if (!ctx) return GW_EINVAL;
  if (!prob || !prob->geom || !pair_variant || !ksplit) return gw::fail(ctx, GW_EINVAL, "bad arguments");
  auto it = ctx->tune.find(shape_key(prob->geom->g, prob->nv, prob->ncol, prec));
  *pair_variant = it == ctx->tune.end() ? 0 : it->second.first;
  *ksplit = it == ctx->tune.end() ? 0 : it->second.second;
  return GW_OK;
}

}  // extern "C"
