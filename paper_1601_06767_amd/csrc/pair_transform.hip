// Pair transform: the matrix element of Eq. (chi0),
//   M_vc(G) = (1/N) sum_r conj(u_v(r)) u_c(r) exp(iG.r),   G in the dielectric sphere,
// formed as the product of two real-space bands followed by a forward transform
// that only produces the K = 2 rchi + 1 frequencies per axis the sphere needs.
//
// k_pair_planes (one x1 plane, 4 x 8 pairs per workgroup):
//   stage 1, per lane one (pair, x2 row): the product along x3 and a pruned x3
//     transform, x3 = b + S a:  X[n] = sum_b e^{2 pi i n b/N} DFT_R(x[b + S a])[n mod R],
//     n in [-rchi, rchi] -> Z[pair][row][n3] in LDS;
//   stage 2, per lane (pair, n3): the same split along x2 over the 8 rows of each
//     x2 group (x2 = b2 + S2 a2), accumulated over the S2 groups in registers;
//   output Q[pair][p1][n2][n3] for this plane (p1 = plane stored permuted).
// k_pair_finish (one pair per workgroup): pruned x1 transform of Q, the 1/N, and the
//   gather of the K^3 box onto the sphere order: M[pair][G] (zero padded to ngp).
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace gw {

namespace {

constexpr int kTV = 4;              // valence bands per workgroup (one per wave)
constexpr int kTC = 64 / kRows;     // conduction columns per workgroup (8)
constexpr int kLdsMax = 163840;

template <typename T, int ND, int K, bool STAGE>
struct PlaneLds {
  static constexpr int rowp = ND + 1;   // padded row: the 8 rows read together fall on distinct banks
  static constexpr size_t psic = STAGE ? (size_t)kTC * kRows * rowp * sizeof(cx<T>) : 0;
  static constexpr size_t z = (size_t)kTV * kTC * kRows * K * sizeof(cx<T>);
  static constexpr size_t total = psic + z;
};

template <typename T, int ND, int K>
constexpr bool stage_fits() {
  return PlaneLds<T, ND, K, true>::total <= (size_t)kLdsMax;
}

template <typename T, int ND, int R, int K, bool STAGE>
__global__ __launch_bounds__(256) void k_pair_planes(const cx<T>* __restrict__ psi_v, const cx<T>* __restrict__ psi_c,
                                                     int nvs, int ncs, const cx<T>* __restrict__ tw,
                                                     cx<T>* __restrict__ q) {
  using V = cx<T>;
  constexpr int S = ND / R;
  constexpr int S2 = ND / kRows;
  constexpr int RCH = (K - 1) / 2;
  constexpr int NPAIR = kTV * kTC;
  constexpr int NITEM = NPAIR * K;
  constexpr int IPL = (NITEM + 255) / 256;
  constexpr size_t NPL = (size_t)ND * ND;
  using L = PlaneLds<T, ND, K, STAGE>;
  extern __shared__ __align__(16) unsigned char smem[];
  V* s_psic = reinterpret_cast<V*>(smem);
  V* s_z = reinterpret_cast<V*>(smem + L::psic);

  const int nbc = ncs / kTC;
  const int nbv = nvs / kTV;
  const int pb = blockIdx.x % (nbc * nbv);
  const int x1 = blockIdx.x / (nbc * nbv);
  const int c0 = (pb % nbc) * kTC;
  const int v0 = (pb / nbc) * kTV;

  const int tid = threadIdx.x;
  const int wv = tid >> 6;            // valence band of this wave
  const int lane = tid & 63;
  const int cl = lane / kRows;        // conduction column of this lane
  const int a2 = lane % kRows;        // row within the x2 group

  V qacc[IPL][K];
#pragma unroll
  for (int r = 0; r < IPL; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) qacc[r][j] = V{T(0), T(0)};

  const V* pv_plane = psi_v + ((size_t)(v0 + wv) * ND + x1) * NPL;
  const V* pc_plane = psi_c + ((size_t)(c0 + cl) * ND + x1) * NPL;

  for (int b2 = 0; b2 < S2; ++b2) {
    if constexpr (STAGE) {
      __syncthreads();
      // stage the 8 rows of group b2 for the 8 columns: contiguous kRows*ND per column
      constexpr int per_col = kRows * ND;
      for (int i = tid; i < kTC * per_col; i += 256) {
        const int c = i / per_col, o = i % per_col;
        s_psic[(c * kRows + o / ND) * L::rowp + o % ND] =
            psi_c[((size_t)(c0 + c) * ND + x1) * NPL + (size_t)b2 * per_col + o];
      }
      __syncthreads();
    } else {
      __syncthreads();
    }
    // ---------------- stage 1: one row per lane
    {
      const V* rv = pv_plane + (size_t)(b2 * kRows + a2) * ND;
      const V* rc = STAGE ? s_psic + (cl * kRows + a2) * L::rowp : pc_plane + (size_t)(b2 * kRows + a2) * ND;
      V acc[K];
#pragma unroll
      for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll
      for (int b = 0; b < S; ++b) {
        V x[R];
#pragma unroll
        for (int a = 0; a < R; ++a) x[a] = cmulc(rv[b * R + a], rc[b * R + a]);
        dft<R>(x);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int n = j - RCH;
          const V t = tw[((n * b) % ND + ND) % ND];
          cmac(acc[j], t, x[((n % R) + R) % R]);
        }
      }
      V* z = s_z + ((wv * kTC + cl) * kRows + a2) * K;
#pragma unroll
      for (int j = 0; j < K; ++j) z[j] = acc[j];
    }
    __syncthreads();
    // ---------------- stage 2: one (pair, n3) line per item, 8-point split along x2
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const int it = tid + 256 * r;
      if (it < NITEM) {
        const int pair = it / K, j3 = it % K;
        V y[kRows];
#pragma unroll
        for (int a = 0; a < kRows; ++a) y[a] = s_z[(pair * kRows + a) * K + j3];
        dft<kRows>(y);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int n = j - RCH;
          const V t = tw[((n * b2) % ND + ND) % ND];
          cmac(qacc[r][j], t, y[((n % kRows) + kRows) % kRows]);
        }
      }
    }
  }
  // ---------------- write this plane's Q[pair][p1][n2][n3]
  const int p1 = (x1 % S) * R + x1 / S;
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const int it = tid + 256 * r;
    if (it < NITEM) {
      const int pair = it / K, j3 = it % K;
      const int pv = pair / kTC, pc = pair % kTC;
      const size_t pg = (size_t)(v0 + pv) * ncs + (c0 + pc);
      V* dst = q + (pg * ND + p1) * (K * K) + j3;
#pragma unroll
      for (int j = 0; j < K; ++j) dst[j * K] = qacc[r][j];
    }
  }
}

template <typename T, int ND, int R, int K>
__global__ __launch_bounds__(256) void k_pair_finish(const cx<T>* __restrict__ q, const int32_t* __restrict__ chi_map,
                                                     int ng, int ngp, T scale, const cx<T>* __restrict__ tw,
                                                     cx<T>* __restrict__ m) {
  using V = cx<T>;
  constexpr int S = ND / R;
  constexpr int RCH = (K - 1) / 2;
  const size_t pair = blockIdx.x;
  const V* src = q + pair * ND * (K * K);
  V* dst = m + pair * ngp;
  for (int l = threadIdx.x; l < K * K; l += blockDim.x) {
    V acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
    // not unrolled: the loads of all S groups would otherwise be hoisted and spill
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      V x[R];
#pragma unroll
      for (int a = 0; a < R; ++a) x[a] = src[(size_t)(b * R + a) * (K * K) + l];
      dft<R>(x);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int n = j - RCH;
        const V t = tw[((n * b) % ND + ND) % ND];
        cmac(acc[j], t, x[((n % R) + R) % R]);
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int ig = chi_map[j * K * K + l];
      if (ig >= 0) dst[ig] = V{acc[j].x * scale, acc[j].y * scale};
    }
  }
  for (int i = ng + threadIdx.x; i < ngp; i += blockDim.x) dst[i] = V{T(0), T(0)};
}

template <typename T, int ND, int R, int K>
hipError_t run_planes(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q,
                      hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_tw64 : (const cx<T>*)g.d_tw32;
  const int nblk = ND * (nvs / kTV) * (ncs / kTC);
  if constexpr (stage_fits<T, ND, K>()) {
    using L = PlaneLds<T, ND, K, true>;
    auto kern = k_pair_planes<T, ND, R, K, true>;
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::total);
    kern<<<nblk, 256, L::total, st>>>((const cx<T>*)psi_v, (const cx<T>*)psi_c, nvs, ncs, tw, (cx<T>*)q);
  } else {
    using L = PlaneLds<T, ND, K, false>;
    static_assert(L::total <= (size_t)kLdsMax, "pair kernel LDS");
    auto kern = k_pair_planes<T, ND, R, K, false>;
    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L::total);
    kern<<<nblk, 256, L::total, st>>>((const cx<T>*)psi_v, (const cx<T>*)psi_c, nvs, ncs, tw, (cx<T>*)q);
  }
  return hipGetLastError();
}

template <typename T, int ND, int R, int K>
hipError_t run_finish(const Geom& g, const void* q, int npair, void* m, hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_tw64 : (const cx<T>*)g.d_tw32;
  const T scale = T(1.0 / ((double)ND * ND * ND));
  k_pair_finish<T, ND, R, K><<<npair, 256, 0, st>>>((const cx<T>*)q, g.d_chi_map, g.ng, g.ngp, scale, tw,
                                                    (cx<T>*)m);
  return hipGetLastError();
}

// (ND, R, K) instances: the grids and dielectric-sphere widths the kernels are built for.
#define GW_PAIR_CASES(X) \
  X(24, 8, 5)            \
  X(24, 8, 7)            \
  X(24, 8, 9)            \
  X(24, 8, 11)           \
  X(72, 8, 9)            \
  X(72, 8, 11)           \
  X(72, 8, 13)           \
  X(72, 8, 15)           \
  X(72, 8, 17)           \
  X(72, 8, 19)           \
  X(96, 16, 17)          \
  X(96, 16, 19)          \
  X(96, 16, 21)          \
  X(128, 16, 23)         \
  X(128, 16, 25)         \
  X(128, 16, 27)

}  // namespace

bool pair_supported(int nd, int K) {
#define X(nd_, r_, k_) \
  if (nd == nd_ && K == k_) return true;
  GW_PAIR_CASES(X)
#undef X
  return false;
}

template <typename T>
hipError_t launch_pair_planes(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q,
                              hipStream_t st) {
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_planes<T, nd_, r_, k_>(g, psi_v, psi_c, nvs, ncs, q, st);
  GW_PAIR_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pair_finish(const Geom& g, const void* q, int npair, void* m, hipStream_t st) {
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_finish<T, nd_, r_, k_>(g, q, npair, m, st);
  GW_PAIR_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

template hipError_t launch_pair_planes<double>(const Geom&, const void*, const void*, int, int, void*, hipStream_t);
template hipError_t launch_pair_planes<float>(const Geom&, const void*, const void*, int, int, void*, hipStream_t);
template hipError_t launch_pair_finish<double>(const Geom&, const void*, int, void*, hipStream_t);
template hipError_t launch_pair_finish<float>(const Geom&, const void*, int, void*, hipStream_t);

}  // namespace gw
