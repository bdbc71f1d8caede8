// Gradients with respect to the wavefunction coefficients (float64): the adjoint of the
// path coefficients -> real-space bands -> pair densities of Eq. (chi0).
//
// With m_p = F(conj(u_v) u_c), F x (G) = (1/N) sum_r x(r) e^{iG.r}, and u_n = B c_n,
// B c (r) = sum_g c(g) e^{ig.r}, a real loss with chi0bar = dL/dRe chi0 + i dL/dIm chi0
// gives (same convention for every gradient):
//   mbar_p = sum_w [conj(w_p) chi0bar m_p + w_p chi0bar^H m_p]           (two GEMMs)
//   h_p    = F^H mbar_p,   h_p(r) = (1/N) sum_G mbar_p(G) e^{-iG.r}
//   ubar_c = sum_v h_vc u_v,   ubar_v = sum_c conj(h_vc) u_c
//   cbar_n = B^H ubar_n,   cbar_n(g) = sum_r ubar_n(r) e^{-ig.r}
// h_p is never stored: it is formed one x1 plane at a time, in the workgroup that
// accumulates the sum over partner bands for one band and one plane.  Each step is the
// transpose of a forward step, with the conjugate twiddles:
//   k_qbar      transpose of the pair finish stage (sphere scatter, x1 transform, 1/N)
//   k_ubar      transposes of the x2 and x3 stages of the pair kernel, times the partner
//               band, summed over the partners (conduction gradient: over the valence
//               bands; valence gradient: over the columns of the chunk, added up over chunks)
//   k_bandT_*   transpose of the band transform (x1, then x2 and x3, sphere gather)
// Every inverse line transform of k_qbar and k_ubar uses the radix split of the forward
// kernels, conjugated: conj(sum_n conj(t_n) e^{+2 pi i n x / N}) = sum_n t_n e^{-2 pi i n x / N}.
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace gw {

namespace {

__device__ __forceinline__ double2 conjd(double2 a) { return double2{a.x, -a.y}; }

// a[p][G] = s_p m[p][G], s_p = w_p or conj(w_p) (w_p = w[p] + i w[np + p] when nparts == 2)
__global__ void k_weight_rows(const double2* __restrict__ m, int npair, int ngp, const double* __restrict__ w,
                              int nparts, int conj_w, double2* __restrict__ a) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)npair * ngp) return;
  const int p = (int)(e / ngp);
  double2 s{w[p], nparts == 2 ? w[(size_t)npair + p] : 0.0};
  if (conj_w) s.y = -s.y;
  a[e] = cmul(s, m[e]);
}

// qbar[pair][p1][l] = scale sum_{n1} e^{-2 pi i n1 x1 / N} mbar[pair][G(n1, l)]  (x1 = b + S a,
// p1 = b R + a), the transpose of the finish stage; one workgroup per pair.
template <int ND, int R, int K>
__global__ __launch_bounds__(256) void k_qbar(const double2* __restrict__ mbar, const int32_t* __restrict__ chi_map,
                                              int ngp, double scale, const double2* __restrict__ twk,
                                              double2* __restrict__ qbar) {
  constexpr int S = ND / R;
  constexpr int RCH = (K - 1) / 2;
  const size_t pair = blockIdx.x;
  const double2* src = mbar + pair * ngp;
  double2* dst = qbar + pair * ND * (K * K);
  for (int l = threadIdx.x; l < K * K; l += blockDim.x) {
    double2 t[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int ig = chi_map[j * K * K + l];
      t[j] = ig >= 0 ? conjd(src[ig]) : double2{0.0, 0.0};
    }
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      double2 y[R];
#pragma unroll
      for (int r = 0; r < R; ++r) y[r] = double2{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < K; ++j) cmac(y[((j - RCH) % R + R) % R], twk[b * K + j], t[j]);
      dft<R>(y);
#pragma unroll
      for (int a = 0; a < R; ++a)
        dst[(size_t)(b * R + a) * (K * K) + l] = double2{y[a].x * scale, -y[a].y * scale};
    }
  }
}

template <int ND> constexpr int ubar_threads() { return ND <= 72 ? 256 : 512; }
// workgroups per plane: the rows p2 of a plane are split between them so that a thread
// keeps one (row, chunk) accumulator of R complex values at the largest grids
template <int ND> constexpr int ubar_split() { return ND <= 96 ? 1 : 2; }

// One workgroup per (x1 plane, row part, own band).  For every partner band: h of the pair on this
// plane from qbar (x2 transform into LDS, then x3 transform per (row, chunk) task), times
// the partner's plane, accumulated in registers; the plane of ubar is written (COND) or
// added (valence, accumulated over conduction chunks) at the end.
//   COND:  own = column c < ncs (pairs v * ncs + c, v < nvs), ubar_c += h_vc u_v
//   !COND: own = valence slot v < nvs (pairs v * ncs + c, c < ncs), ubar_v += conj(h_vc) u_c
template <int ND, int R, int K, bool COND>
__global__ __launch_bounds__(ubar_threads<ND>()) void k_ubar(const double2* __restrict__ qbar,
                                                             const double2* __restrict__ partner, int nvs, int ncs,
                                                             const double2* __restrict__ twk,
                                                             double2* __restrict__ ubar) {
  constexpr int NT = ubar_threads<ND>();
  constexpr int RS = ubar_split<ND>();
  constexpr int S = ND / R;
  constexpr int S2 = ND / kRows;
  constexpr int S2P = S2 / RS;                   // row groups b2 of this part
  constexpr int NROW = ND / RS;                  // rows p2 of this part
  constexpr int RCH = (K - 1) / 2;
  constexpr int NTASK = NROW * S;                // (row p2, x3 chunk b)
  constexpr int TPT = (NTASK + NT - 1) / NT;     // tasks per thread
  constexpr size_t NPL = (size_t)ND * ND;
  static_assert(S2 % RS == 0, "row groups split evenly");
  __shared__ double2 s_q[K * K];
  __shared__ double2 s_t[NROW * K];              // [p2 - row0][n3]
  const int x1 = blockIdx.x % ND;
  const int part = (blockIdx.x / ND) % RS;
  const int own = blockIdx.x / (ND * RS);
  const int b2_0 = part * S2P;
  const int row0 = b2_0 * kRows;
  const int p1 = (x1 % S) * R + x1 / S;
  const int tid = threadIdx.x;
  const int npart = COND ? nvs : ncs;
  double2 acc[TPT][R];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
#pragma unroll
    for (int a = 0; a < R; ++a) acc[k][a] = double2{0.0, 0.0};
#pragma unroll 1
  for (int q = 0; q < npart; ++q) {
    const size_t pair = COND ? (size_t)q * ncs + own : (size_t)own * ncs + q;
    const double2* src = qbar + (pair * ND + p1) * (K * K);
    __syncthreads();   // the previous partner's s_q / s_t are consumed
    for (int l = tid; l < K * K; l += NT) s_q[l] = conjd(src[l]);
    __syncthreads();
    // x2 transform: T[p2 = 8 b2 + a][n3] = sum_{n2} e^{-2 pi i n2 x2 / N} qbar[n2][n3], x2 = b2 + S2 a
    for (int task = tid; task < K * S2P; task += NT) {
      const int j3 = task % K, bl = task / K, b2 = b2_0 + bl;
      double2 y[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) y[r] = double2{0.0, 0.0};
#pragma unroll
      for (int j = 0; j < K; ++j) cmac(y[((j - RCH) % kRows + kRows) % kRows], twk[b2 * K + j], s_q[j * K + j3]);
      dft<kRows>(y);
#pragma unroll
      for (int a = 0; a < kRows; ++a) s_t[(bl * kRows + a) * K + j3] = y[a];   // still conjugated
    }
    __syncthreads();
    // x3 transform per (p2, b): h[p2][b R + a], then times the partner's plane
    const double2* up = partner + ((size_t)q * ND + x1) * NPL;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int task = tid + NT * k;
      if (task < NTASK) {
        const int pl = task / S, b = task % S;
        double2 y[R];
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = double2{0.0, 0.0};
        // s_t already holds conj(T), the inner conjugation of the identity
#pragma unroll
        for (int j = 0; j < K; ++j) cmac(y[((j - RCH) % R + R) % R], twk[b * K + j], s_t[pl * K + j]);
        dft<R>(y);
        const double2* u = up + (size_t)(row0 + pl) * ND + b * R;
#pragma unroll
        for (int a = 0; a < R; ++a) {
          const double2 h = conjd(y[a]);
          const double2 v = u[a];
          acc[k][a] = COND ? cadd(acc[k][a], cmul(h, v)) : cadd(acc[k][a], cmul(conjd(h), v));
        }
      }
    }
  }
  double2* out = ubar + ((size_t)own * ND + x1) * NPL;
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int task = tid + NT * k;
    if (task < NTASK) {
      const int pl = task / S, b = task % S;
      double2* o = out + (size_t)(row0 + pl) * ND + b * R;
#pragma unroll
      for (int a = 0; a < R; ++a) {
        if (COND)
          o[a] = acc[k][a];
        else
          o[a] = cadd(o[a], acc[k][a]);
      }
    }
  }
}

constexpr int kJB = 8;   // outputs per thread of the transposed band passes

// transpose of the x1 pass: tB[slot][j1][p23] = sum_{x1} e^{-2 pi i n1 x1 / N} ubar[slot][x1][p23]
__global__ __launch_bounds__(256) void k_bandT_c(const double2* __restrict__ ubar, int rw, int nd,
                                                 const double2* __restrict__ tw, double2* __restrict__ tB) {
  __shared__ double2 s_tw[128];
  for (int i = threadIdx.x; i < nd; i += blockDim.x) s_tw[i] = conjd(tw[i]);
  __syncthreads();
  const int W = 2 * rw + 1;
  const int nblk = (W + kJB - 1) / kJB;
  const size_t plane = (size_t)nd * nd;
  const int slot = blockIdx.y;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nblk * (long long)plane) return;
  const int p23 = (int)(t % (long long)plane);
  const int jb = (int)(t / (long long)plane);
  const double2* src = ubar + (size_t)slot * nd * plane + p23;
  double2 acc[kJB];
  int idx[kJB], step[kJB];
#pragma unroll
  for (int k = 0; k < kJB; ++k) {
    acc[k] = double2{0.0, 0.0};
    step[k] = wrap(jb * kJB + k - rw, nd);   // n1 mod N; x1 advances the twiddle index by n1
    idx[k] = 0;
  }
  for (int x1 = 0; x1 < nd; ++x1) {
    const double2 v = src[(size_t)x1 * plane];
#pragma unroll
    for (int k = 0; k < kJB; ++k) {
      cmac(acc[k], v, s_tw[idx[k]]);
      idx[k] += step[k];
      if (idx[k] >= nd) idx[k] -= nd;
    }
  }
  double2* dst = tB + (size_t)slot * W * plane + p23;
#pragma unroll
  for (int k = 0; k < kJB; ++k)
    if (jb * kJB + k < W) dst[(size_t)(jb * kJB + k) * plane] = acc[k];
}

// transposes of the x2 and x3 passes for one (slot, j1) slab, then the sphere gather:
// cbar[slot][ig] for ig = wf_map[j1][j2][j3] >= 0
__global__ __launch_bounds__(256) void k_bandT_ab(const double2* __restrict__ tB, int rw, int nd, int S2, int R3,
                                                  const int32_t* __restrict__ wf_map, int npw,
                                                  const double2* __restrict__ tw, double2* __restrict__ cbar) {
  extern __shared__ unsigned char s_raw[];
  double2* s_tw = (double2*)s_raw;   // conj twiddles, nd
  double2* s_t = s_tw + 128;         // [j2][p3], W x nd
  const int W = 2 * rw + 1;
  const int nblk = (W + kJB - 1) / kJB;
  const int j1 = blockIdx.x;
  const int slot = blockIdx.y;
  for (int i = threadIdx.x; i < nd; i += blockDim.x) s_tw[i] = conjd(tw[i]);
  __syncthreads();
  const double2* slab = tB + ((size_t)slot * W + j1) * nd * nd;
  // x2: s_t[j2][p3] = sum_{x2} e^{-2 pi i n2 x2 / N} slab[p2(x2)][p3],  p2 = 8 b2 + a2, x2 = b2 + S2 a2
  for (int task = threadIdx.x; task < nd * nblk; task += blockDim.x) {
    const int p3 = task % nd, jb = task / nd;
    double2 acc[kJB];
#pragma unroll
    for (int k = 0; k < kJB; ++k) acc[k] = double2{0.0, 0.0};
    for (int p2 = 0; p2 < nd; ++p2) {
      const int x2 = p2 / kRows + S2 * (p2 % kRows);
      const double2 v = slab[(size_t)p2 * nd + p3];
#pragma unroll
      for (int k = 0; k < kJB; ++k) cmac(acc[k], v, s_tw[wrap((jb * kJB + k - rw) * x2, nd)]);
    }
#pragma unroll
    for (int k = 0; k < kJB; ++k)
      if (jb * kJB + k < W) s_t[(size_t)(jb * kJB + k) * nd + p3] = acc[k];
  }
  __syncthreads();
  // x3: cbar(j1, j2, j3) = sum_{x3} e^{-2 pi i n3 x3 / N} s_t[j2][p3(x3)],  p3 = b R3 + a, x3 = b + S3 a
  const int S3 = nd / R3;
  for (int task = threadIdx.x; task < W * nblk; task += blockDim.x) {
    const int j2 = task % W, jb = task / W;
    double2 acc[kJB];
#pragma unroll
    for (int k = 0; k < kJB; ++k) acc[k] = double2{0.0, 0.0};
    for (int p3 = 0; p3 < nd; ++p3) {
      const int x3 = p3 / R3 + S3 * (p3 % R3);
      const double2 v = s_t[(size_t)j2 * nd + p3];
#pragma unroll
      for (int k = 0; k < kJB; ++k) cmac(acc[k], v, s_tw[wrap((jb * kJB + k - rw) * x3, nd)]);
    }
#pragma unroll
    for (int k = 0; k < kJB; ++k) {
      const int j3 = jb * kJB + k;
      if (j3 < W) {
        const int ig = wf_map[((size_t)j1 * W + j2) * W + j3];
        if (ig >= 0) cbar[(size_t)slot * npw + ig] = acc[k];
      }
    }
  }
}

// grad[row(c)][g] += cbar[c][g] for the valid columns c < ncol of a chunk, row(c) =
// col_band[c0 + c] (or c0 + c); one thread per g walks the columns in order.
__global__ void k_scatter_cols(const double2* __restrict__ cbar, int ncol, const int32_t* __restrict__ col_band,
                               int c0, int npw, int nband, double2* __restrict__ grad) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  for (int c = 0; c < ncol; ++c) {
    const int row = col_band ? col_band[c0 + c] : c0 + c;
    if (row < 0 || row >= nband) continue;   // an out-of-range column row is never written
    double2* d = grad + (size_t)row * npw + g;
    *d = cadd(*d, cbar[(size_t)c * npw + g]);
  }
}

__global__ void k_fill_c128(double2* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = double2{0.0, 0.0};
}

template <int ND, int R, int K>
hipError_t run_qbar(const Geom& g, const void* mbar, int npair, void* qbar, hipStream_t st) {
  k_qbar<ND, R, K><<<npair, 256, 0, st>>>((const double2*)mbar, g.d_chi_map, g.ngp, 1.0 / ((double)ND * ND * ND),
                                          g.d_twk64, (double2*)qbar);
  return hipGetLastError();
}

template <int ND, int R, int K>
hipError_t run_ubar(const Geom& g, const void* qbar, const void* partner, int nvs, int ncs, bool cond, int nown,
                    void* ubar, hipStream_t st) {
  constexpr int NT = ubar_threads<ND>();
  const dim3 grid((unsigned)(ND * ubar_split<ND>() * nown));
  if (cond)
    k_ubar<ND, R, K, true><<<grid, NT, 0, st>>>((const double2*)qbar, (const double2*)partner, nvs, ncs, g.d_twk64,
                                                (double2*)ubar);
  else
    k_ubar<ND, R, K, false><<<grid, NT, 0, st>>>((const double2*)qbar, (const double2*)partner, nvs, ncs, g.d_twk64,
                                                 (double2*)ubar);
  return hipGetLastError();
}

hipError_t allow_bandT_lds() {
  static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bandT_ab),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}

}  // namespace

hipError_t launch_weight_rows(const void* m, int npair, int ngp, const double* w, int nparts, bool conj_w, void* a,
                              hipStream_t st) {
  const size_t n = (size_t)npair * ngp;
  k_weight_rows<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const double2*)m, npair, ngp, w, nparts, conj_w ? 1 : 0,
                                                             (double2*)a);
  return hipGetLastError();
}

hipError_t launch_qbar(const Geom& g, const void* mbar, int npair, void* qbar, hipStream_t st) {
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_qbar<nd_, r_, k_>(g, mbar, npair, qbar, st);
  GW_PAIR_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_ubar(const Geom& g, const void* qbar, const void* partner, int nvs, int ncs, bool cond, void* ubar,
                       hipStream_t st) {
  const int nown = cond ? ncs : nvs;
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_ubar<nd_, r_, k_>(g, qbar, partner, nvs, ncs, cond, nown, ubar, st);
  GW_PAIR_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_band_from_real(const Geom& g, const void* ubar, int nslot, void* tB, void* cbar, hipStream_t st) {
  const int nd = g.nd, W = g.W;
  if (nd > 128 || nd % kRows != 0) return hipErrorInvalidValue;
  const size_t lds = (size_t)(128 + W * nd) * sizeof(double2);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const hipError_t ea = allow_bandT_lds();
  if (ea != hipSuccess) return ea;
  const int nblk = (W + kJB - 1) / kJB;
  const long long n = (long long)nblk * nd * nd;
  k_bandT_c<<<dim3((unsigned)((n + 255) / 256), nslot), 256, 0, st>>>((const double2*)ubar, g.rw, nd, g.d_tw64,
                                                                       (double2*)tB);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_bandT_ab<<<dim3(W, nslot), 256, lds, st>>>((const double2*)tB, g.rw, nd, nd / kRows, g.line.R, g.d_wf_map,
                                                g.npw, g.d_tw64, (double2*)cbar);
  return hipGetLastError();
}

hipError_t launch_scatter_cols(const void* cbar, int ncol, const int32_t* col_band, int c0, int npw, int nband,
                               void* grad, hipStream_t st) {
  k_scatter_cols<<<(npw + 255) / 256, 256, 0, st>>>((const double2*)cbar, ncol, col_band, c0, npw, nband,
                                                    (double2*)grad);
  return hipGetLastError();
}

hipError_t launch_fill_c128(void* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  k_fill_c128<<<(unsigned)blocks, 256, 0, st>>>((double2*)p, n);
  return hipGetLastError();
}

}  // namespace gw
