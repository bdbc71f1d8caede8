// Band -> real space: u_n(r) = sum_G c_n(G) exp(iG.r) on the N^3 grid, the
// wavefunctions whose products form the matrix element of Eq. (chi0).
//
// The coefficients live on a sphere of half-width rw, so the transform is done as
// three separable passes that only visit nonzero inputs (direct sums over at most
// W = 2 rw + 1 frequencies per axis; this stage costs O(bands), not O(pairs)):
//   pass A  tA[j1][j2][p3] = sum_n3 c(n1, n2, n3) e^{2 pi i n3 x3 / N}
//   pass B  tB[j1][p2][p3] = sum_n2 tA[j1][j2][p3]  e^{2 pi i n2 x2 / N}
//   pass C  u [x1][p2][p3] = sum_n1 tB[j1][p2][p3]  e^{2 pi i n1 x1 / N}
// x2 and x3 are stored permuted (p = b R + a for x = b + S a) so that the pair
// kernel reads contiguous rows and contiguous radix-R groups.
#include "common.h"
#include "internal.h"

namespace gw {

namespace {

template <typename T>
__device__ __forceinline__ void load_table(cx<T>* s_tw, const cx<T>* tw, int nd) {
  for (int i = threadIdx.x; i < nd; i += blockDim.x) s_tw[i] = tw[i];
  __syncthreads();
}

__device__ __forceinline__ int slot_band(const int32_t* band_idx, int band0, int nvalid, int nrows, int slot) {
  int idx = band0 + slot;
  if (idx >= nvalid) idx = nvalid - 1;
  const int band = band_idx ? band_idx[idx] : idx;
  return band < 0 ? 0 : (band >= nrows ? nrows - 1 : band);   // never read outside the coefficient rows
}

template <typename T>
__global__ __launch_bounds__(256) void k_band_a(const double2* __restrict__ coef, int npw,
                                                const int32_t* __restrict__ band_idx, int band0, int nvalid, int nrows,
                                                const int32_t* __restrict__ wf_map, int rw, int nd, int R, int S,
                                                const cx<T>* __restrict__ tw, cx<T>* __restrict__ tA) {
  __shared__ cx<T> s_tw[128];
  load_table<T>(s_tw, tw, nd);
  const int W = 2 * rw + 1;
  const int slot = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * W * nd) return;
  const int band = slot_band(band_idx, band0, nvalid, nrows, slot);
  const int p3 = t % nd;
  const int j12 = t / nd;
  const int x3 = p3 / R + S * (p3 % R);
  const double2* c = coef + (size_t)band * npw;
  const int32_t* map = wf_map + (size_t)j12 * W;
  int idx = wrap(-rw * x3, nd);
  cx<T> acc{T(0), T(0)};
  for (int j3 = 0; j3 < W; ++j3) {
    const int ig = map[j3];
    if (ig >= 0) {
      const double2 cv = c[ig];
      cmac(acc, cx<T>{T(cv.x), T(cv.y)}, s_tw[idx]);
    }
    idx += x3;
    if (idx >= nd) idx -= nd;
  }
  tA[((size_t)slot * W * W + j12) * nd + p3] = acc;
}

// 8 outputs per thread: the rows a2 = 0..7 of x2-group b2 (x2 = b2 + S2 a2).
template <typename T>
__global__ __launch_bounds__(256) void k_band_b(const cx<T>* __restrict__ tA, int rw, int nd,
                                                const cx<T>* __restrict__ tw, cx<T>* __restrict__ tB) {
  __shared__ cx<T> s_tw[128];
  load_table<T>(s_tw, tw, nd);
  const int W = 2 * rw + 1;
  const int S2 = nd / kRows;
  const int slot = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W * S2 * nd) return;
  const int p3 = t % nd;
  const int b2 = (t / nd) % S2;
  const int j1 = t / (nd * S2);
  int idx[kRows], step[kRows];
  cx<T> acc[kRows];
#pragma unroll
  for (int a = 0; a < kRows; ++a) {
    const int x2 = b2 + S2 * a;
    step[a] = x2;
    idx[a] = wrap(-rw * x2, nd);
    acc[a] = cx<T>{T(0), T(0)};
  }
  const cx<T>* src = tA + ((size_t)slot * W + j1) * W * nd + p3;
  for (int j2 = 0; j2 < W; ++j2) {
    const cx<T> v = src[(size_t)j2 * nd];
#pragma unroll
    for (int a = 0; a < kRows; ++a) {
      cmac(acc[a], v, s_tw[idx[a]]);
      idx[a] += step[a];
      if (idx[a] >= nd) idx[a] -= nd;
    }
  }
  cx<T>* dst = tB + (((size_t)slot * W + j1) * nd + (size_t)b2 * kRows) * nd + p3;
#pragma unroll
  for (int a = 0; a < kRows; ++a) dst[(size_t)a * nd] = acc[a];
}

// 8 consecutive x1 planes per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_band_c(const cx<T>* __restrict__ tB, int rw, int nd,
                                                const cx<T>* __restrict__ tw, cx<T>* __restrict__ psi) {
  __shared__ cx<T> s_tw[128];
  load_table<T>(s_tw, tw, nd);
  const int W = 2 * rw + 1;
  const int nb1 = nd / 8;
  const int slot = blockIdx.y;
  const size_t plane = (size_t)nd * nd;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int)(nb1 * plane)) return;
  const int p23 = t % (int)plane;
  const int x1b = t / (int)plane;
  int idx[8];
  cx<T> acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    idx[i] = wrap(-rw * (8 * x1b + i), nd);
    acc[i] = cx<T>{T(0), T(0)};
  }
  const cx<T>* src = tB + (size_t)slot * W * plane + p23;
  for (int j1 = 0; j1 < W; ++j1) {
    const cx<T> v = src[(size_t)j1 * plane];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      cmac(acc[i], v, s_tw[idx[i]]);
      idx[i] += 8 * x1b + i;
      if (idx[i] >= nd) idx[i] -= nd;
    }
  }
  cx<T>* dst = psi + ((size_t)slot * nd + 8 * x1b) * plane + p23;
#pragma unroll
  for (int i = 0; i < 8; ++i) dst[(size_t)i * plane] = acc[i];
}

}  // namespace

size_t band_scratch_bytes(const Geom& g, int nslot, bool fp64) {
  const size_t e = fp64 ? 16 : 8;
  return (size_t)nslot * ((size_t)g.W * g.W * g.nd + (size_t)g.W * g.nd * g.nd) * e;
}

template <typename T>
hipError_t launch_band_to_real(const Geom& g, const double2* coef, int nrows, const int32_t* band_idx, int band0, int nvalid,
                               int nslot, void* tA, void* tB, void* psi, hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_tw64 : (const cx<T>*)g.d_tw32;
  const int nd = g.nd, W = g.W;
  const dim3 blk(256);
  {
    const int n = W * W * nd;
    k_band_a<T><<<dim3((n + 255) / 256, nslot), blk, 0, st>>>(coef, g.npw, band_idx, band0, nvalid, nrows, g.d_wf_map, g.rw,
                                                              nd, g.line.R, g.line.S, tw, (cx<T>*)tA);
  }
  {
    const int n = W * (nd / kRows) * nd;
    k_band_b<T><<<dim3((n + 255) / 256, nslot), blk, 0, st>>>((const cx<T>*)tA, g.rw, nd, tw, (cx<T>*)tB);
  }
  {
    const int n = (nd / 8) * nd * nd;
    k_band_c<T><<<dim3((n + 255) / 256, nslot), blk, 0, st>>>((const cx<T>*)tB, g.rw, nd, tw, (cx<T>*)psi);
  }
  return hipGetLastError();
}

template hipError_t launch_band_to_real<double>(const Geom&, const double2*, int, const int32_t*, int, int, int, void*,
                                                void*, void*, hipStream_t);
template hipError_t launch_band_to_real<float>(const Geom&, const double2*, int, const int32_t*, int, int, int, void*,
                                               void*, void*, hipStream_t);

}  // namespace gw
