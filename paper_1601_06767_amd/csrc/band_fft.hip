// Band -> real space: u_n(r) = sum_G c_n(G) exp(iG.r) on the N^3 grid, the
// wavefunctions whose products form the matrix element of Eq. (chi0).
//
// The coefficients live on a sphere of half-width rw (W = 2 rw + 1 frequencies per
// axis), so each axis is transformed from its W nonzero frequencies only.  One line
// transform u[x] = sum_{|n| <= rw} t[n] w^{n x} (w = exp(2 pi i / N)) is split as
// x = b + S a (a < R, b < S, N = R S):
//   Y_b[r]     = sum_{n = r mod R} t[n] w^{n b}        (W multiply-adds per b)
//   u[b + S a] = sum_r exp(2 pi i r a / R) Y_b[r]      (one R-point DFT per b)
// i.e. S (W + R log R) operations per line instead of N W for the direct sum.
//
//   k_band_ab (one workgroup per band and n1): the x3 lines of the n1 slab,
//     t3[j2][p3] in LDS, then the x2 lines -> tB[j1][p2][p3];
//   k_band_c: the x1 lines -> u[x1][p2][p3].
// x2 and x3 are stored permuted (p = b R + a for x = b + S a) so that the pair
// kernel reads contiguous rows and contiguous radix-R groups.
#include "common.h"
#include "internal.h"

namespace gw {

namespace {

__device__ __forceinline__ int slot_band(const int32_t* band_idx, int band0, int nvalid, int nrows, int slot) {
  int idx = band0 + slot;
  if (idx >= nvalid) idx = nvalid - 1;
  const int band = band_idx ? band_idx[idx] : idx;
  return band < 0 ? 0 : (band >= nrows ? nrows - 1 : band);   // never read outside the coefficient rows
}

// Y_b[r] of one line for NB chunk indices b0 + k * bstep (k < NB), then the R-point DFTs:
// y[k][a] = u[b_k + S a].  load(n) returns t[n] for |n| <= rw.  The frequencies are
// visited in blocks of R starting at a multiple of R, so that n mod R is the (static)
// position within the block.
template <typename T, int R, int NB, typename Load>
__device__ __forceinline__ void line_split(int rw, int nd, int b0, int bstep, const cx<T>* s_tw, Load load,
                                           cx<T> (&y)[NB][R]) {
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r) y[k][r] = cx<T>{T(0), T(0)};
  const int nlo = -((rw + R - 1) / R) * R;
  int idx[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) idx[k] = wrap(nlo * (b0 + k * bstep), nd);
  for (int n0 = nlo; n0 <= rw; n0 += R) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = n0 + r;
      if (n >= -rw && n <= rw) {
        const cx<T> v = load(n);
#pragma unroll
        for (int k = 0; k < NB; ++k) cmac(y[k][r], v, s_tw[idx[k]]);
      }
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        idx[k] += b0 + k * bstep;
        if (idx[k] >= nd) idx[k] -= nd;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) dft<R>(y[k]);
}

constexpr int kMaxNd = 128;
// Threads of a k_band_ab workgroup.  Its LDS (the x3 slab) allows two or three workgroups per
// CU, so larger workgroups keep more waves in flight for the latency-bound gathers and line
// sums: per 576-band call, 128^3 takes 13.5 ms with 1024 threads, 14.2 with 576 and 18.6 with
// 256; 96^3 3.0 / 3.2 / 3.1 ms and 72^3 (float64) 1.74 / 1.92 / 2.04 ms with 576 / 1024 / 256.
constexpr int kBandAbThreads = 1024;   // the launch bound
inline int band_ab_threads(int nd) { return nd >= 128 ? 1024 : 576; }

// One workgroup per (band slot, j1).  R3 = the x3 line split (g.line.R), the x2 split is
// fixed at kRows (x2 = b2 + S2 a2, the row groups of the pair kernel).
template <typename T, int R3>
__global__ __launch_bounds__(kBandAbThreads) void k_band_ab(const double2* __restrict__ coef, int npw,
                                                 const int32_t* __restrict__ band_idx, int band0, int nvalid, int nrows,
                                                 const int32_t* __restrict__ wf_map, int rw, int nd,
                                                 const cx<T>* __restrict__ tw, cx<T>* __restrict__ tB) {
  extern __shared__ unsigned char s_raw[];
  cx<T>* s_tw = (cx<T>*)s_raw;                 // nd twiddles
  cx<T>* s_t3 = s_tw + kMaxNd;                 // [j2][p3], W x nd
  const int W = 2 * rw + 1;
  const int j1 = blockIdx.x;
  const int slot = blockIdx.y;
  for (int i = threadIdx.x; i < nd; i += blockDim.x) s_tw[i] = tw[i];
  const int band = slot_band(band_idx, band0, nvalid, nrows, slot);
  const double2* c = coef + (size_t)band * npw;
  __syncthreads();
  // x3 lines of the slab: line j2, chunk b3 -> p3 = b3 R3 + a
  const int S3 = nd / R3;
  for (int task = threadIdx.x; task < W * S3; task += blockDim.x) {
    const int j2 = task / S3, b3 = task % S3;
    const int32_t* map = wf_map + ((size_t)j1 * W + j2) * W + rw;   // index by n3
    cx<T> y[1][R3];
    line_split<T, R3, 1>(rw, nd, b3, 0, s_tw,
                         [&](int n) {
                           const int ig = map[n];
                           if (ig < 0) return cx<T>{T(0), T(0)};
                           const double2 v = c[ig];
                           return cx<T>{T(v.x), T(v.y)};
                         },
                         y);
    cx<T>* dst = s_t3 + (size_t)j2 * nd + b3 * R3;
#pragma unroll
    for (int a = 0; a < R3; ++a) dst[a] = y[0][a];
  }
  __syncthreads();
  // x2 lines: column p3, chunk b2 -> rows p2 = b2 kRows + a2
  const int S2 = nd / kRows;
  cx<T>* out = tB + ((size_t)slot * W + j1) * nd * nd;
  for (int task = threadIdx.x; task < nd * S2; task += blockDim.x) {
    const int p3 = task % nd, b2 = task / nd;
    cx<T> y[1][kRows];
    line_split<T, kRows, 1>(rw, nd, b2, 0, s_tw, [&](int n) { return s_t3[(size_t)(n + rw) * nd + p3]; }, y);
#pragma unroll
    for (int a = 0; a < kRows; ++a) out[((size_t)b2 * kRows + a) * nd + p3] = y[0][a];
  }
}

// x1 lines: one (p2, p3) column and NB chunk indices b1 = b + k S / NB per thread;
// x1 = b1 + S a1 with R = 8, planes stored in natural x1 order.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_band_c(const cx<T>* __restrict__ tB, int rw, int nd,
                                                const cx<T>* __restrict__ tw, cx<T>* __restrict__ psi) {
  constexpr int R = 8;
  __shared__ cx<T> s_tw[kMaxNd];
  for (int i = threadIdx.x; i < nd; i += blockDim.x) s_tw[i] = tw[i];
  __syncthreads();
  const int W = 2 * rw + 1;
  const int S = nd / R;
  const int slot = blockIdx.y;
  const size_t plane = (size_t)nd * nd;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int)((S / NB) * plane)) return;
  const int p23 = t % (int)plane;
  const int b = t / (int)plane;
  const cx<T>* src = tB + (size_t)slot * W * plane + p23 + (size_t)rw * plane;   // index by n1
  cx<T> y[NB][R];
  line_split<T, R, NB>(rw, nd, b, S / NB, s_tw, [&](int n) { return src[(ptrdiff_t)n * (ptrdiff_t)plane]; }, y);
  cx<T>* dst = psi + (size_t)slot * nd * plane + p23;
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int a = 0; a < R; ++a) dst[(size_t)(b + k * (S / NB) + S * a) * plane] = y[k][a];
}

template <typename T, int NB>
void launch_c(const Geom& g, const cx<T>* tB, const cx<T>* tw, cx<T>* psi, int nslot, hipStream_t st) {
  const int S = g.nd / 8;
  const int n = (S / NB) * g.nd * g.nd;
  k_band_c<T, NB><<<dim3((n + 255) / 256, nslot), 256, 0, st>>>(tB, g.rw, g.nd, tw, psi);
}

}  // namespace

size_t band_scratch_bytes(const Geom& g, int nslot, bool fp64) {
  const size_t e = fp64 ? 16 : 8;
  return (size_t)nslot * g.W * g.nd * g.nd * e;
}

namespace {
size_t band_lds_bytes(const Geom& g, bool fp64) {
  return (size_t)(kMaxNd + g.W * g.nd) * (fp64 ? 16 : 8);
}

// the x3 slab of the 96^3 and 128^3 grids needs more than the default dynamic-LDS limit
template <typename T, int R3>
hipError_t allow_lds() {
  static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_band_ab<T, R3>),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}
}  // namespace

template <typename T>
hipError_t launch_band_to_real(const Geom& g, const double2* coef, int nrows, const int32_t* band_idx, int band0, int nvalid,
                               int nslot, void* tB, void* psi, hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_tw64 : (const cx<T>*)g.d_tw32;
  const int nd = g.nd, W = g.W;
  if (nd > kMaxNd || nd % kRows != 0) return hipErrorInvalidValue;
  const size_t lds = band_lds_bytes(g, std::is_same<T, double>::value);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const dim3 grid(W, nslot);
  const hipError_t ea = g.line.R == 8 ? allow_lds<T, 8>() : allow_lds<T, 16>();
  if (ea != hipSuccess) return ea;
  if (g.line.R == 8)
    k_band_ab<T, 8><<<grid, band_ab_threads(nd), lds, st>>>(coef, g.npw, band_idx, band0, nvalid, nrows, g.d_wf_map, g.rw, nd, tw,
                                             (cx<T>*)tB);
  else if (g.line.R == 16)
    k_band_ab<T, 16><<<grid, band_ab_threads(nd), lds, st>>>(coef, g.npw, band_idx, band0, nvalid, nrows, g.d_wf_map, g.rw, nd, tw,
                                              (cx<T>*)tB);
  else
    return hipErrorInvalidValue;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int S = nd / 8;
  if (S % 3 == 0)
    launch_c<T, 3>(g, (const cx<T>*)tB, tw, (cx<T>*)psi, nslot, st);
  else if (S % 2 == 0)
    launch_c<T, 2>(g, (const cx<T>*)tB, tw, (cx<T>*)psi, nslot, st);
  else
    launch_c<T, 1>(g, (const cx<T>*)tB, tw, (cx<T>*)psi, nslot, st);
  return hipGetLastError();
}

template hipError_t launch_band_to_real<double>(const Geom&, const double2*, int, const int32_t*, int, int, int, void*,
                                                void*, hipStream_t);
template hipError_t launch_band_to_real<float>(const Geom&, const double2*, int, const int32_t*, int, int, int, void*,
                                               void*, hipStream_t);

}  // namespace gw
