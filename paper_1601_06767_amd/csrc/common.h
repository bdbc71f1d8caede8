// Device helpers shared by the gwchi0 kernels: complex arithmetic on HIP vector
// types, unit roots exp(+2 pi i m / R) as compile-time constants, and short
// unrolled DFTs of the sizes the pruned transforms are built from.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gw {

template <typename T> struct cx_t;
template <> struct cx_t<double> { using type = double2; };
template <> struct cx_t<float> { using type = float2; };
template <typename T> using cx = typename cx_t<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
  return V{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// acc += a * b
template <typename V> __device__ __forceinline__ void cmac(V& acc, V a, V b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// bfloat16 as the upper half of a float: float -> bf16 bits rounded to nearest even
// (v_cvt_pk_bf16_f32 on gfx950), and back
__device__ __forceinline__ unsigned short bf16_rne(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// ---------------------------------------------------------------- unit roots
// cos and sin of k pi / 16 for k = 0..4 (first octant), correctly rounded decimals.
constexpr double kOctC[5] = {1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                             0.70710678118654752440};
constexpr double kOctS[5] = {0.0, 0.19509032201612826785, 0.38268343236508977173, 0.55557023301960222474,
                             0.70710678118654752440};

// exp(+2 pi i m / 32), exact symmetries of the first octant.
constexpr double root32_c(int m) {
  m = ((m % 32) + 32) % 32;
  const int q = m / 8, r = m % 8;
  const double c = r <= 4 ? kOctC[r] : kOctS[8 - r];
  const double s = r <= 4 ? kOctS[r] : kOctC[8 - r];
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}
constexpr double root32_s(int m) {
  m = ((m % 32) + 32) % 32;
  const int q = m / 8, r = m % 8;
  const double c = r <= 4 ? kOctC[r] : kOctS[8 - r];
  const double s = r <= 4 ? kOctS[r] : kOctC[8 - r];
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}

// x * exp(+2 pi i m / R) with R | 32, trivial roots folded at compile time.
template <int R, int M, typename V> __device__ __forceinline__ V rot(V x) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return x;
  } else if constexpr (4 * m == R) {
    return V{-x.y, x.x};
  } else if constexpr (2 * m == R) {
    return V{-x.x, -x.y};
  } else if constexpr (4 * m == 3 * R) {
    return V{x.y, -x.x};
  } else {
    using T = decltype(x.x);
    constexpr double c = root32_c(m * (32 / R));
    constexpr double s = root32_s(m * (32 / R));
    return V{T(c) * x.x - T(s) * x.y, T(s) * x.x + T(c) * x.y};
  }
}

// In-place R-point DFT y[k] = sum_a x[a] exp(+2 pi i k a / R), R a power of two <= 32.
// Radix-2 decimation in time: bit-reversed reordering, then log2 R butterfly stages.
template <int R> constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// One butterfly (u, t) -> (u + w t, u - w t), w = exp(+2 pi i M / L).  Where w is not a power of
// i, the larger of its two components g is factored out: w t = g (y + i z) with y, z formed by one
// FMA each from the ratio of the smaller to the larger component (at most 1 in size), and then
// u +- g (y + i z) takes four FMAs: six operations where the rotation followed by the sum and
// difference takes eight.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int L, int M, typename V> __device__ __forceinline__ void bfly2(V& u, V& t) {
  constexpr int m = ((M % L) + L) % L;
  if constexpr (m == 0 || 4 * m == L || 2 * m == L || 4 * m == 3 * L) {
    const V r = rot<L, M>(t);
    const V a = u;
    u = cadd(a, r);
    t = csub(a, r);
  } else {
    using T = decltype(t.x);
    constexpr double c = root32_c(m * (32 / L));
    constexpr double s = root32_s(m * (32 / L));
    constexpr bool cbig = (c < 0 ? -c : c) >= (s < 0 ? -s : s);
    constexpr T g = T(cbig ? c : s);
    constexpr T q = T(cbig ? s / c : c / s);
    T y, z;
    if constexpr (cbig) {   // w t = c ((tr - q ti) + i (ti + q tr)), q = s / c
      y = fma_t(-q, t.y, t.x);
      z = fma_t(q, t.x, t.y);
    } else {                // w t = s ((q tr - ti) + i (tr + q ti)), q = c / s
      y = fma_t(q, t.x, -t.y);
      z = fma_t(q, t.y, t.x);
    }
    const V a = u;
    u = V{fma_t(g, y, a.x), fma_t(g, z, a.y)};
    t = V{fma_t(-g, y, a.x), fma_t(-g, z, a.y)};
  }
}

template <int R, int L, int I, int J, typename V> __device__ __forceinline__ void bfly(V* x) {
  if constexpr (I < R) {
    if constexpr (J < L / 2) {
      bfly2<L, J>(x[I + J], x[I + J + L / 2]);
      bfly<R, L, I, J + 1>(x);
    } else {
      bfly<R, L, I + L, 0>(x);
    }
  }
}

template <int R, int L, typename V> __device__ __forceinline__ void stages(V* x) {
  if constexpr (L <= R) {
    bfly<R, L, 0, 0>(x);
    stages<R, 2 * L>(x);
  }
}

template <int R, int I, typename V> __device__ __forceinline__ void bitrev_swap(V* x) {
  if constexpr (I < R) {
    constexpr int j = bitrev<R>(I);
    if constexpr (j > I) {
      V t = x[I];
      x[I] = x[j];
      x[j] = t;
    }
    bitrev_swap<R, I + 1>(x);
  }
}

template <int R, typename V> __device__ __forceinline__ void dft(V* x) {
  static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32, "radix");
  if constexpr (R > 1) {
    bitrev_swap<R, 0>(x);
    stages<R, 2>(x);
  }
}

// ---------------------------------------------------------------- direct-load pipelines
// s_waitcnt with vmcnt = n (0..63) and no wait on the other counters
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier for LDS data only: this wave's LDS operations complete (lgkmcnt 0), then
// all waves meet; the empty asm statements keep the compiler from moving memory accesses
// across it.  Unlike __syncthreads (whose fence also covers the LDS writes of direct loads,
// hence waits for every one in flight) it leaves the direct loads of later steps in flight;
// the wait for a step's own direct loads is explicit (wait_vm).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));   // lgkmcnt(0); vmcnt, expcnt not waited
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wrap n into [0, m).
__host__ __device__ __forceinline__ int wrap(int n, int m) {
  int r = n % m;
  return r < 0 ? r + m : r;
}

}  // namespace gw
