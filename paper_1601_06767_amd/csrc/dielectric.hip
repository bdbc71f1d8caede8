// Dielectric matrix eps = I - diag(v) chi0 and its inverse in float64 (the RPA relation
// stated before Eq. (chi0); Table 3's eps_inf = 1/[eps^-1]_00).
//
// Inversion: in-place Gauss-Jordan elimination with partial (row) pivoting, blocked by
// panels of kNb columns.  Within a panel every pivot step updates only the panel
// columns (all rows); the panel then holds the panel columns T[:, J] of the
// accumulated elimination transform, and the remaining columns are brought up to
// date with one rank-kNb update A[:, rest] += (T[:, J] - I[:, J]) A_old[J, rest] on
// float64 MFMA.  The column interchanges implied by the row pivots are undone at the
// end.  A zero or non-finite pivot raises a device flag read by gw_eps_inv_status.
//
// zgemm: C = alpha op(A) op(B) + beta C for complex128 row-major matrices, op = identity
// or conjugate transpose, on MFMA f64 16x16x4 with 64 x 64 tiles.
#include "common.h"
#include "internal.h"

namespace gw {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void k_form_eps(const double* __restrict__ v, const double2* __restrict__ chi, int n,
                           double2* __restrict__ eps) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  const double2 c = chi[e];
  const double vi = v[i];
  eps[e] = double2{(i == j ? 1.0 : 0.0) - vi * c.x, -vi * c.y};
}

__global__ void k_flag_clear(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

// Pivot of column j (rows j..n-1, largest |.|, lowest index on ties), full-row swap,
// and a copy of the pivot row's panel part.
__global__ __launch_bounds__(1024) void k_pivot(double2* __restrict__ a, int n, int j, int j0, int nbp,
                                                int* __restrict__ piv, double2* __restrict__ prow,
                                                int* __restrict__ flag) {
  __shared__ double s_v[1024];
  __shared__ int s_i[1024];
  const int t = threadIdx.x;
  double best = -1.0;
  int bi = n;
  for (int i = j + t; i < n; i += blockDim.x) {
    const double2 x = a[(size_t)i * n + j];
    const double m = x.x * x.x + x.y * x.y;
    if (m > best || (m == best && i < bi)) {
      best = m;
      bi = i;
    }
  }
  s_v[t] = best;
  s_i[t] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      const double m = s_v[t + s];
      const int i = s_i[t + s];
      if (m > s_v[t] || (m == s_v[t] && i < s_i[t])) {
        s_v[t] = m;
        s_i[t] = i;
      }
    }
    __syncthreads();
  }
  const int p = s_i[0];
  const double pm = s_v[0];
  if (t == 0) {
    piv[j] = p;
    if (!(pm > 0.0) || !isfinite(pm)) *flag = 1;
  }
  if (p != j && p < n) {
    for (int c = t; c < n; c += blockDim.x) {
      const double2 x = a[(size_t)j * n + c];
      a[(size_t)j * n + c] = a[(size_t)p * n + c];
      a[(size_t)p * n + c] = x;
    }
  }
  __syncthreads();
  for (int c = t; c < nbp; c += blockDim.x) prow[c] = a[(size_t)j * n + j0 + c];
}

// Elimination of pivot j restricted to the panel columns [j0, j0 + nbp): four rows per
// workgroup, one panel column per thread.
__global__ __launch_bounds__(256) void k_eliminate(double2* __restrict__ a, int n, int j, int j0, int nbp,
                                                   const double2* __restrict__ prow) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  const int jc = j - j0;
  double2 f{0.0, 0.0};
  if (i < n) f = a[(size_t)i * n + j];
  __syncthreads();
  if (i >= n || c >= nbp) return;
  const double2 p = prow[jc];
  const double den = p.x * p.x + p.y * p.y;
  const double2 pinv{p.x / den, -p.y / den};
  double2* dst = a + (size_t)i * n + j0 + c;
  if (i == j) {
    *dst = c == jc ? pinv : cmul(prow[c], pinv);
  } else {
    const double2 fp = cmul(f, pinv);
    if (c == jc) {
      *dst = double2{-fp.x, -fp.y};
    } else {
      const double2 r = cmul(fp, prow[c]);
      const double2 x = *dst;
      *dst = double2{x.x - r.x, x.y - r.y};
    }
  }
}

// Operands of the panel's rank-nbp update: bp = T[:, J] - I[:, J] (n x kNb, zero padded),
// tmp = A[J, :] with the panel columns zeroed (kNb x n).
__global__ void k_panel_operands(const double2* __restrict__ a, int n, int j0, int nbp, int nb,
                                 double2* __restrict__ bp, double2* __restrict__ tmp) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (size_t)n * nb) {
    const int i = (int)(e / nb), c = (int)(e % nb);
    double2 x{0.0, 0.0};
    if (c < nbp) {
      x = a[(size_t)i * n + j0 + c];
      if (i == j0 + c) x.x -= 1.0;
    }
    bp[e] = x;
  }
  if (e < (size_t)nb * n) {
    const int c = (int)(e / n), col = (int)(e % n);
    double2 x{0.0, 0.0};
    if (c < nbp && (col < j0 || col >= j0 + nbp)) x = a[(size_t)(j0 + c) * n + col];
    tmp[e] = x;
  }
}

__global__ void k_col_perm(const int* __restrict__ piv, int n, int* __restrict__ idx) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int c = 0; c < n; ++c) idx[c] = c;
  for (int j = n - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j && p >= 0 && p < n) {
      const int t = idx[j];
      idx[j] = idx[p];
      idx[p] = t;
    }
  }
}

__global__ void k_gather_cols(const double2* __restrict__ src, const int* __restrict__ idx, int n,
                              double2* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const size_t i = e / n;
  const int c = (int)(e % n);
  dst[e] = src[i * n + idx[c]];
}

// ---------------------------------------------------------------- zgemm
constexpr int ZT = 64, ZK = 16;

// element (r, k) of op(X) for X row-major with leading dimension ld
__device__ __forceinline__ double2 opget(const double2* x, int ld, int r, int k, bool ct) {
  if (!ct) return x[(size_t)r * ld + k];
  const double2 v = x[(size_t)k * ld + r];
  return double2{v.x, -v.y};
}

__global__ __launch_bounds__(256) void k_zgemm(int m, int n, int kd, double2 alpha, const double2* __restrict__ A,
                                               int lda, bool cta, const double2* __restrict__ B, int ldb, bool ctb,
                                               double2 beta, double2* __restrict__ C, int ldc) {
  __shared__ double2 sA[ZK][ZT + 1];   // sA[k][row]
  __shared__ double2 sB[ZK][ZT + 1];   // sB[k][col]
  const int tiles_n = (n + ZT - 1) / ZT;
  const int r0 = (blockIdx.x / tiles_n) * ZT, c0 = (blockIdx.x % tiles_n) * ZT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  f64x4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = f64x4{0, 0, 0, 0};
      cim[i][j] = f64x4{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < kd; k0 += ZK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (ZK * ZT) / 256; ++r) {
      const int e = tid + 256 * r;
      // A tile: rows r0 + (e % ZT), k = k0 + e / ZT
      {
        const int kk = e / ZT, rr = e % ZT;
        double2 x{0.0, 0.0};
        if (r0 + rr < m && k0 + kk < kd) x = opget(A, lda, r0 + rr, k0 + kk, cta);
        sA[kk][rr] = x;
      }
      {
        const int kk = e / ZT, cc = e % ZT;
        double2 x{0.0, 0.0};
        if (c0 + cc < n && k0 + kk < kd) x = ctb ? opget(B, ldb, k0 + kk, c0 + cc, true)
                                                 : B[(size_t)(k0 + kk) * ldb + c0 + cc];
        sB[kk][cc] = x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < ZK / 4; ++s) {
      const int k = 4 * s + lk;
      double2 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[k][32 * wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[k][32 * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = mfma64(a[i].x, b[j].x, cre[i][j]);
          cre[i][j] = mfma64(-a[i].y, b[j].y, cre[i][j]);
          cim[i][j] = mfma64(a[i].x, b[j].y, cim[i][j]);
          cim[i][j] = mfma64(a[i].y, b[j].x, cim[i][j]);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 32 * wr + 16 * i + lk + 4 * r;   // f64 MFMA output rows: lane/16 + 4 r
        const int col = c0 + 32 * wc + 16 * j + li;
        if (row < m && col < n) {
          const double2 ab{cre[i][j][r], cim[i][j][r]};
          double2 out = cmul(alpha, ab);
          double2* p = C + (size_t)row * ldc + col;
          if (beta.x != 0.0 || beta.y != 0.0) {
            const double2 o = cmul(beta, *p);
            out.x += o.x;
            out.y += o.y;
          }
          *p = out;
        }
      }
}

}  // namespace

hipError_t launch_zgemm(int m, int n, int k, double2 alpha, const double2* A, int lda, bool cta, const double2* B,
                        int ldb, bool ctb, double2 beta, double2* C, int ldc, hipStream_t st) {
  const int tiles = ((m + ZT - 1) / ZT) * ((n + ZT - 1) / ZT);
  k_zgemm<<<tiles, 256, 0, st>>>(m, n, k, alpha, A, lda, cta, B, ldb, ctb, beta, C, ldc);
  return hipGetLastError();
}

size_t eps_inv_workspace(int n) {
  const size_t nb = kNb;
  return (size_t)n * n * sizeof(double2) + 2 * (size_t)n * nb * sizeof(double2) + nb * sizeof(double2) +
         2 * (size_t)n * sizeof(int) + 1024;
}

hipError_t launch_eps_inv(int n, const double* v, const double2* chi, double2* out, void* ws, int* flag,
                          hipStream_t st) {
  char* w = (char*)ws;
  double2* a = (double2*)w;   // working matrix
  w += (size_t)n * n * sizeof(double2);
  double2* bp = (double2*)w;
  w += (size_t)n * kNb * sizeof(double2);
  double2* tmp = (double2*)w;
  w += (size_t)n * kNb * sizeof(double2);
  double2* prow = (double2*)w;
  w += kNb * sizeof(double2);
  int* piv = (int*)w;
  w += (size_t)n * sizeof(int);
  int* idx = (int*)w;
  const size_t nn = (size_t)n * n;
  const unsigned gnn = (unsigned)((nn + 255) / 256);
  k_form_eps<<<gnn, 256, 0, st>>>(v, chi, n, a);
  for (int j0 = 0; j0 < n; j0 += kNb) {
    const int nbp = n - j0 < kNb ? n - j0 : kNb;
    for (int j = j0; j < j0 + nbp; ++j) {
      k_pivot<<<1, 1024, 0, st>>>(a, n, j, j0, nbp, piv, prow, flag);
      k_eliminate<<<(n + 3) / 4, 256, 0, st>>>(a, n, j, j0, nbp, prow);
    }
    if (nbp == n) break;   // a single panel: no other columns to update
    const size_t nops = (size_t)n * kNb;
    k_panel_operands<<<(unsigned)((nops + 255) / 256), 256, 0, st>>>(a, n, j0, nbp, kNb, bp, tmp);
    hipError_t e = launch_zgemm(n, n, kNb, double2{1.0, 0.0}, bp, kNb, false, tmp, n, false, double2{1.0, 0.0}, a,
                                n, st);
    if (e != hipSuccess) return e;
  }
  k_col_perm<<<1, 64, 0, st>>>(piv, n, idx);
  k_gather_cols<<<gnn, 256, 0, st>>>(a, idx, n, out);
  return hipGetLastError();
}

// chibar = V Z^H Zbar Z^H  (V = diag v): t = Z^H Zbar, out = t Z^H, then rows scaled by v.
__global__ void k_scale_rows(double2* __restrict__ x, const double* __restrict__ v, int n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const double s = v[e / n];
  x[e] = double2{x[e].x * s, x[e].y * s};
}

size_t eps_inv_backward_workspace(int n) { return (size_t)n * n * sizeof(double2) + 256; }

hipError_t launch_eps_inv_backward(int n, const double* v, const double2* z, const double2* zbar, double2* out,
                                   void* ws, hipStream_t st) {
  double2* t = (double2*)ws;
  hipError_t e = launch_zgemm(n, n, n, double2{1.0, 0.0}, z, n, true, zbar, n, false, double2{0.0, 0.0}, t, n, st);
  if (e != hipSuccess) return e;
  e = launch_zgemm(n, n, n, double2{1.0, 0.0}, t, n, false, z, n, true, double2{0.0, 0.0}, out, n, st);
  if (e != hipSuccess) return e;
  const size_t nn = (size_t)n * n;
  k_scale_rows<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(out, v, n);
  return hipGetLastError();
}

hipError_t launch_flag_clear(int* flag, hipStream_t st) {
  k_flag_clear<<<1, 64, 0, st>>>(flag);
  return hipGetLastError();
}

}  // namespace gw
