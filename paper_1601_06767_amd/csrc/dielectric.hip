// Dielectric matrix eps = I - diag(v) chi0 and its inverse in float64 (the RPA relation
// stated before Eq. (chi0); Table 3's eps_inf = 1/[eps^-1]_00).
//
// Inversion: in-place Gauss-Jordan elimination with partial (row) pivoting, blocked by
// panels of kNb columns.  The panel columns (all rows) are copied to a buffer and each
// pivot step is one launch that reads the panel from one buffer and writes the updated
// panel (rows j and p interchanged, pivot row scaled, column j eliminated) to the other;
// the same launch leaves one pivot candidate per workgroup for the next column, so that
// the next step finds its pivot by reducing those candidates.  After the panel, its row
// interchanges are applied to the other columns, the panel holds the columns T[:, J] of
// the accumulated elimination transform, and the remaining columns are brought up to
// date with one rank-kNb update A[:, rest] += (T[:, J] - I[:, J]) A_old[J, rest] on
// float64 MFMA.  The column interchanges implied by the row pivots are undone at the
// end.  A zero or non-finite pivot raises a device flag read by gw_eps_inv_status.
//
// zgemm: C = alpha op(A) op(B) + beta C for complex128 row-major matrices, op = identity
// or conjugate transpose, on MFMA f64 16x16x4 with 64 x 64 tiles.
#include <mutex>

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

constexpr int kStepRows = 4;   // rows per workgroup of the panel kernels (one kNb-wide row per wave)

// candidate (|x|^2, row) of one workgroup's rows i >= i0 in panel column col (row index
// n and -1 when none qualifies); the larger value wins, the lower row on ties
__device__ __forceinline__ void step_candidate(const double2* __restrict__ p, int n, int i0, int col, double* cm,
                                               int* ci) {
  __shared__ double s_m[kStepRows];
  __shared__ int s_i[kStepRows];
  const int r = threadIdx.x >> 6;
  const int i = blockIdx.x * kStepRows + r;
  if ((threadIdx.x & 63) == 0) {
    double m = -1.0;
    if (i < n && i >= i0) {
      const double2 x = p[(size_t)i * kNb + col];
      m = x.x * x.x + x.y * x.y;
    }
    s_m[r] = m;
    s_i[r] = (i < n && i >= i0) ? i : n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double best = -1.0;
    int bi = n;
    for (int k = 0; k < kStepRows; ++k)
      if (s_i[k] < n && (s_m[k] > best || (s_m[k] == best && s_i[k] < bi))) {
        best = s_m[k];
        bi = s_i[k];
      }
    cm[blockIdx.x] = best;
    ci[blockIdx.x] = bi;
  }
}

// Panel columns [j0, j0 + nbp) of a into p (n x kNb, zero padded) and the pivot
// candidates of its first column.
__global__ __launch_bounds__(256) void k_panel_load(const double2* __restrict__ a, int n, int j0, int nbp,
                                                    double2* __restrict__ p, double* __restrict__ cm,
                                                    int* __restrict__ ci) {
  const int i = blockIdx.x * kStepRows + (threadIdx.x >> 6);
  const int c = threadIdx.x & 63;
  if (i < n) p[(size_t)i * kNb + c] = c < nbp ? a[(size_t)i * n + j0 + c] : double2{0.0, 0.0};
  __syncthreads();
  step_candidate(p, n, j0, 0, cm, ci);
}

// One pivot step j = j0 + jc on the panel: pivot p from the candidates, then
// row j <- row p / d, row p <- row j (old) eliminated, every other row eliminated,
// column jc <- the corresponding column of the transform.  Reads pin, writes pout.
__global__ __launch_bounds__(256) void k_gj_step(const double2* __restrict__ pin, double2* __restrict__ pout, int n,
                                                 int j0, int jc, int nbp, const double* __restrict__ cm_in,
                                                 const int* __restrict__ ci_in, int ncand, double* __restrict__ cm_out,
                                                 int* __restrict__ ci_out, int* __restrict__ piv,
                                                 int* __restrict__ flag) {
  __shared__ double s_m[256];
  __shared__ int s_i[256];
  __shared__ double2 s_prow[kNb], s_rowj[kNb];
  const int t = threadIdx.x;
  const int j = j0 + jc;
  double best = -1.0;
  int bi = n;
  for (int k = t; k < ncand; k += blockDim.x) {
    const double m = cm_in[k];
    const int i = ci_in[k];
    if (i < n && (m > best || (m == best && i < bi))) {
      best = m;
      bi = i;
    }
  }
  s_m[t] = best;
  s_i[t] = bi;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double m = s_m[t + h];
      const int i = s_i[t + h];
      if (i < n && (m > s_m[t] || (m == s_m[t] && i < s_i[t]))) {
        s_m[t] = m;
        s_i[t] = i;
      }
    }
    __syncthreads();
  }
  const double pm = s_m[0];
  const int p = s_i[0] < n ? s_i[0] : j;   // no finite candidate: keep row j, the flag reports it
  if (blockIdx.x == 0 && t == 0) {
    piv[j] = p;
    if (!(pm > 0.0) || !isfinite(pm)) *flag = 1;
  }
  if (t < kNb) {
    s_prow[t] = pin[(size_t)p * kNb + t];
    s_rowj[t] = pin[(size_t)j * kNb + t];
  }
  __syncthreads();
  const double2 d = s_prow[jc];
  const double den = d.x * d.x + d.y * d.y;
  const double2 dinv = den > 0.0 ? double2{d.x / den, -d.y / den} : double2{0.0, 0.0};
  const int i = blockIdx.x * kStepRows + (t >> 6);
  const int c = t & 63;
  if (i < n) {
    double2 out;
    if (i == j) {
      out = c == jc ? dinv : cmul(s_prow[c], dinv);
    } else {
      const double2 x = i == p ? s_rowj[c] : pin[(size_t)i * kNb + c];
      const double2 f = i == p ? s_rowj[jc] : pin[(size_t)i * kNb + jc];
      const double2 fp = cmul(f, dinv);
      if (c == jc) {
        out = double2{-fp.x, -fp.y};
      } else {
        const double2 r = cmul(fp, s_prow[c]);
        out = double2{x.x - r.x, x.y - r.y};
      }
    }
    pout[(size_t)i * kNb + c] = out;
  }
  if (jc + 1 < nbp) {
    __syncthreads();
    step_candidate(pout, n, j + 1, jc + 1, cm_out, ci_out);
  }
}

// The panel's row interchanges, in order, on the columns outside the panel.
__global__ void k_row_swaps(double2* __restrict__ a, int n, int j0, int nbp, const int* __restrict__ piv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || (c >= j0 && c < j0 + nbp)) return;
  for (int j = j0; j < j0 + nbp; ++j) {
    const int p = piv[j];
    if (p != j && p >= 0 && p < n) {
      const double2 x = a[(size_t)j * n + c];
      a[(size_t)j * n + c] = a[(size_t)p * n + c];
      a[(size_t)p * n + c] = x;
    }
  }
}

// The finished panel T[:, J] back into a, and the operands of the rank-nbp update:
// bp = T[:, J] - I[:, J] (in place in the panel buffer, n x kNb), tmp = A[J, :] with the
// panel columns zeroed (kNb x n).
__global__ void k_panel_operands(double2* __restrict__ a, int n, int j0, int nbp, double2* __restrict__ bp,
                                 double2* __restrict__ tmp) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (size_t)n * kNb) {
    const int i = (int)(e / kNb), c = (int)(e % kNb);
    double2 x{0.0, 0.0};
    if (c < nbp) {
      x = bp[e];
      a[(size_t)i * n + j0 + c] = x;
      if (i == j0 + c) x.x -= 1.0;
    }
    bp[e] = x;
  }
  if (e < (size_t)kNb * n) {
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

// element (r, k) of op(X) for X row-major with leading dimension ld; op: kOpN, kOpC
// (conjugate transpose), kOpT (transpose), kOpConj (conjugate)
__device__ __forceinline__ double2 opget(const double2* x, int ld, int r, int k, int op) {
  const bool tr = op == kOpC || op == kOpT;
  const double2 v = tr ? x[(size_t)k * ld + r] : x[(size_t)r * ld + k];
  return (op == kOpC || op == kOpConj) ? double2{v.x, -v.y} : v;
}

__global__ __launch_bounds__(256) void k_zgemm(int m, int n, int kd, double2 alpha, const double2* __restrict__ A,
                                               int lda, int opa, const double2* __restrict__ B, int ldb, int opb,
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
      // consecutive threads walk the operand's contiguous index: k for A stored by rows (N,
      // conj) and for B stored transposed (T, C), the row / column index otherwise
      {
        const bool along_k = opa == kOpN || opa == kOpConj;
        const int kk = along_k ? e % ZK : e / ZT, rr = along_k ? e / ZK : e % ZT;
        double2 x{0.0, 0.0};
        if (r0 + rr < m && k0 + kk < kd) x = opget(A, lda, r0 + rr, k0 + kk, opa);
        sA[kk][rr] = x;
      }
      {
        const bool along_k = opb == kOpT || opb == kOpC;
        const int kk = along_k ? e % ZK : e / ZT, cc = along_k ? e / ZK : e % ZT;
        double2 x{0.0, 0.0};
        if (c0 + cc < n && k0 + kk < kd) x = opget(B, ldb, k0 + kk, c0 + cc, opb);
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


// ---------------------------------------------------------------- static inverse by block sweeps
// For a static chi0 (Hermitian, negative semidefinite) and v > 0, eps~ = I - V^1/2 chi0 V^1/2 is
// Hermitian positive definite and eps^-1 = V^1/2 eps~^-1 V^-1/2.  The sweep operator on a block K
// of 64 indices, D = A_KK:
//   A_ij -= A_iK D^-1 A_Kj (i, j outside K),  A_iK <- A_iK D^-1,  A_Kj <- D^-1 A_Kj,  A_KK <- -D^-1;
// sweeping every block in turn leaves -A^-1.  The part not yet swept is a Schur complement of
// eps~, positive definite, so D needs no pivoting: D = L L^H, and the update is the Hermitian
// rank-64 product A -= C C^H with C = A_.K L^-H, on the lower 64 x 64 tiles only (the float64
// MFMA contraction tile).  Only the lower triangle is stored.  Half the arithmetic of the
// pivoted Gauss-Jordan path and four launches per block of 64 instead of about 68.
constexpr int kSw = 64;

// lower triangle a[i][j] = delta_ij - sqrt(v_i) chi_ij sqrt(v_j) (i >= j), identity in the padding
__global__ void k_sweep_form(const double* __restrict__ v, const double2* __restrict__ chi, int n, int ldp,
                             double2* __restrict__ a, int* __restrict__ flag) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ldp * ldp) return;
  const int i = (int)(e / ldp), j = (int)(e % ldp);
  if (j > i) return;
  double2 x{i == j ? 1.0 : 0.0, 0.0};
  if (i < n && j < n) {
    const double vi = v[i], vj = v[j];
    double s = 0.0;   // a v <= 0 is reported; the entry is then left at the identity's
    if (!(vi > 0.0) || !(vj > 0.0))
      atomicOr(flag, 1);
    else
      s = sqrt(vi) * sqrt(vj);
    const double2 c = chi[(size_t)i * n + j];
    x.x -= s * c.x;
    x.y -= s * c.y;
  }
  a[e] = x;
}

// one workgroup: D = A_KK (lower) = L L^H in LDS, X = L^-1, then linvT[l][k] = X[k][l] and
// dinv = X^H X = D^-1 (full 64 x 64).  A pivot that is not positive sets the flag.
// One barrier per step: step j of the factorisation subtracts the outer product of column j
// divided by its pivot d_j from the trailing triangle, and scales column j - 1 by 1/sqrt(d_{j-1})
// (no one reads that column in step j); step j of the inversion (rows of L X = I from the top)
// subtracts L[i][j] / L[j][j] times row j from the rows below and scales row j - 1 likewise.
// Threads cover the (row, column) ranges on a fixed 16 x 16 grid (no integer division), and
// D^-1 is formed in 4 x 4 blocks per thread.  (Measured at NG 8000: 176 us per block with three
// barriers per factorisation step, divisions in the index arithmetic and the inverse by one
// thread per column; the 125 blocks were 22 of the 75 ms of the inverse.)
__global__ __launch_bounds__(256) void k_sweep_diag(const double2* __restrict__ a, int ldp, int k0,
                                                    double2* __restrict__ linvT, double2* __restrict__ dinv,
                                                    int* __restrict__ flag) {
  __shared__ double2 L[kSw][kSw + 1];
  __shared__ double2 X[kSw][kSw + 1];
  __shared__ double dv[kSw];   // pivots d_j, then 1 / L[j][j]
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  for (int e = tid; e < kSw * kSw; e += 256) {
    const int r = e / kSw, c = e % kSw;
    L[r][c] = c <= r ? a[(size_t)(k0 + r) * ldp + k0 + c] : double2{0.0, 0.0};
    X[r][c] = double2{r == c ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  // factorisation: L[i][k] -= L[i][j] conj(L[k][j]) / d_j for j < k <= i
  for (int j = 0; j <= kSw; ++j) {
    if (j < kSw) {
      double d = L[j][j].x;
      if (!(d > 0.0) || !isfinite(d)) {
        if (tid == 0) atomicOr(flag, 1);
        d = 1.0;
      }
      if (tid == 0) dv[j] = d;
      const double rd = 1.0 / d;
      for (int i = j + 1 + ty; i < kSw; i += 16) {
        const double2 x = L[i][j];
        const double2 xs{x.x * rd, x.y * rd};
        for (int k = j + 1 + tx; k <= i; k += 16) {
          const double2 y = L[k][j];
          L[i][k].x -= xs.x * y.x + xs.y * y.y;
          L[i][k].y -= xs.y * y.x - xs.x * y.y;
        }
      }
    }
    if (j > 0) {   // column j - 1 is final: scale it, its diagonal becomes sqrt(d)
      const int c = j - 1;
      const double sq = sqrt(dv[c]);
      const double inv = 1.0 / sq;
      for (int i = c + 1 + tid; i < kSw; i += 256) L[i][c] = double2{L[i][c].x * inv, L[i][c].y * inv};
      if (tid == 0) L[c][c] = double2{sq, 0.0};
    }
    __syncthreads();
  }
  if (tid < kSw) dv[tid] = 1.0 / L[tid][tid].x;
  __syncthreads();
  // inversion: L X = I by rows; row j of X is final (unscaled) once step j starts
  for (int j = 0; j <= kSw; ++j) {
    if (j < kSw) {
      const double rj = dv[j];
      for (int i = j + 1 + ty; i < kSw; i += 16) {
        const double2 l = L[i][j];
        const double2 f{l.x * rj, l.y * rj};
        for (int c = tx; c <= j; c += 16) {
          const double2 x = X[j][c];
          X[i][c].x -= f.x * x.x - f.y * x.y;
          X[i][c].y -= f.x * x.y + f.y * x.x;
        }
      }
    }
    if (j > 0) {
      const int r = j - 1;
      const double rr = dv[r];
      for (int c = tid; c <= r; c += 256) X[r][c] = double2{X[r][c].x * rr, X[r][c].y * rr};
    }
    __syncthreads();
  }
  for (int e = tid; e < kSw * kSw; e += 256) {
    const int r = e / kSw, c = e % kSw;
    linvT[(size_t)c * kSw + r] = X[r][c];
  }
  // dinv[r][c] = sum_k conj(X[k][r]) X[k][c] over the 4 x 4 block (4 ty.., 4 tx..); X is lower
  // triangular, so the terms with k below max(r, c) vanish and the sum starts at the block's
  // larger first index
  const int r0 = 4 * ty, c0 = 4 * tx;
  double2 s[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) s[p][q] = double2{0.0, 0.0};
  for (int k = r0 > c0 ? r0 : c0; k < kSw; ++k) {
    double2 xr[4], xc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      xr[p] = X[k][r0 + p];
      xc[p] = X[k][c0 + p];
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        s[p][q].x += xr[p].x * xc[q].x + xr[p].y * xc[q].y;
        s[p][q].y += xr[p].x * xc[q].y - xr[p].y * xc[q].x;
      }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) dinv[(size_t)(r0 + p) * kSw + c0 + q] = s[p][q];
}

// 64 rows i per workgroup: x_i = A_iK from the lower storage, C_i = x_i L^-H into ct[k][i] (zero for
// i in K, whose tiles the write pass replaces), P_i = x_i D^-1 into pp[i][k]
__global__ __launch_bounds__(256) void k_sweep_panel(const double2* __restrict__ a, int ldp, int k0,
                                                     const double2* __restrict__ linvT,
                                                     const double2* __restrict__ dinv, double2* __restrict__ ct,
                                                     double2* __restrict__ pp) {
  __shared__ double2 xs[4][kSw];
  __shared__ double2 cs[kSw][kSw + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i0 = blockIdx.x * kSw;
  for (int rr = 0; rr < kSw / 4; ++rr) {
    const int r = rr * 4 + wave;
    const int i = i0 + r;
    const bool inK = i >= k0 && i < k0 + kSw;
    double2 x{0.0, 0.0};
    if (!inK) {
      if (i > k0) {
        x = a[(size_t)i * ldp + k0 + lane];
      } else {
        const double2 y = a[(size_t)(k0 + lane) * ldp + i];
        x = double2{y.x, -y.y};
      }
    }
    xs[wave][lane] = x;
    __syncthreads();
    double2 c{0.0, 0.0}, q{0.0, 0.0};
    for (int l = 0; l < kSw; ++l) {
      const double2 xv = xs[wave][l];
      const double2 li = linvT[(size_t)l * kSw + lane];   // L^-1[lane][l]
      const double2 d = dinv[(size_t)l * kSw + lane];
      c.x += xv.x * li.x + xv.y * li.y;   // x conj(li)
      c.y += xv.y * li.x - xv.x * li.y;
      q.x += xv.x * d.x - xv.y * d.y;
      q.y += xv.x * d.y + xv.y * d.x;
    }
    cs[r][lane] = c;
    pp[(size_t)i * kSw + lane] = q;
    __syncthreads();
  }
  for (int kk = 0; kk < kSw / 4; ++kk) {
    const int k = kk * 4 + wave;
    ct[(size_t)k * ldp + i0 + lane] = cs[lane][k];
  }
}

// the swept block's new entries in the lower storage: A_iK = P_i (i > K), A_Ki = conj(P_i)
// (i < K), A_KK = -D^-1
__global__ void k_sweep_write(double2* __restrict__ a, int ldp, int k0, const double2* __restrict__ pp,
                              const double2* __restrict__ dinv) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ldp * kSw) return;
  const int i = (int)(e / kSw), k = (int)(e % kSw);
  if (i >= k0 && i < k0 + kSw) {
    const int r = i - k0;
    if (k <= r) {
      const double2 d = dinv[(size_t)r * kSw + k];
      a[(size_t)i * ldp + k0 + k] = double2{-d.x, -d.y};
    }
  } else if (i > k0) {
    a[(size_t)i * ldp + k0 + k] = pp[e];
  } else {
    const double2 p = pp[e];
    a[(size_t)(k0 + k) * ldp + i] = double2{p.x, -p.y};
  }
}

// eps^-1[i][j] = sqrt(v_i) (-A)_ij / sqrt(v_j) for i, j < n, A Hermitian from its lower triangle
__global__ void k_sweep_out(const double* __restrict__ v, const double2* __restrict__ a, int n, int ldp,
                            double2* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  double2 x = i >= j ? a[(size_t)i * ldp + j] : a[(size_t)j * ldp + i];
  if (i < j) x.y = -x.y;
  const double s = -sqrt(v[i]) / sqrt(v[j]);
  out[e] = double2{s * x.x, s * x.y};
}

__global__ void k_fill_f64_neg(double* __restrict__ w, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = -1.0;
}

}  // namespace

hipError_t launch_zgemm_op(int m, int n, int k, double2 alpha, const double2* A, int lda, int opa, const double2* B,
                           int ldb, int opb, double2 beta, double2* C, int ldc, hipStream_t st) {
  if (m < 1 || n < 1 || k < 1 || opa < kOpN || opa > kOpConj || opb < kOpN || opb > kOpConj) return hipErrorInvalidValue;
  const int tiles = ((m + ZT - 1) / ZT) * ((n + ZT - 1) / ZT);
  k_zgemm<<<tiles, 256, 0, st>>>(m, n, k, alpha, A, lda, opa, B, ldb, opb, beta, C, ldc);
  return hipGetLastError();
}

hipError_t launch_zgemm(int m, int n, int k, double2 alpha, const double2* A, int lda, bool cta, const double2* B,
                        int ldb, bool ctb, double2 beta, double2* C, int ldc, hipStream_t st) {
  return launch_zgemm_op(m, n, k, alpha, A, lda, cta ? kOpC : kOpN, B, ldb, ctb ? kOpC : kOpN, beta, C, ldc, st);
}

constexpr size_t sweep_bytes(int n) {
  return (size_t)((n + kSw - 1) / kSw * kSw) * ((n + kSw - 1) / kSw * kSw) * sizeof(double2) +
         2 * (size_t)kSw * ((n + kSw - 1) / kSw * kSw) * sizeof(double2) + 2 * (size_t)kSw * kSw * sizeof(double2) +
         kSw * sizeof(double) + 4096;
}

constexpr size_t gj_bytes(int n) {
  return (size_t)n * n * sizeof(double2) + 2 * (size_t)n * kNb * sizeof(double2) + 2 * (size_t)n * sizeof(int) +
         2 * (size_t)((n + kStepRows - 1) / kStepRows) * (sizeof(double) + sizeof(int)) + 1024;
}
// either route of the inverse (pivoted Gauss-Jordan, or the sweeps of the static form)
constexpr size_t eps_inv_bytes(int n) { return gj_bytes(n) > sweep_bytes(n) ? gj_bytes(n) : sweep_bytes(n); }

size_t eps_inv_workspace(int n) { return eps_inv_bytes(n); }

// ---------------------------------------------------------------- inverse without allocation
// Scratch of gw_eps_inv_noalloc: one file-scope device array, one copy per GPU, held until the
// process ends.  Host code never uses the array's name for its memory: the device address is
// looked up once per device (noalloc_scratch_init, called with the device current when a
// context is created there) and kept in noalloc_ptr.
constexpr size_t kNoAllocBytes = eps_inv_bytes(kNoAllocMaxNg);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_noalloc_ptr[device] = ptr;
  return e;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

size_t noalloc_scratch_bytes() { return kNoAllocBytes; }

hipError_t launch_eps_inv(int n, const double* v, const double2* chi, double2* out, void* ws, int* flag,
                          hipStream_t st) {
  const int ncand = (n + kStepRows - 1) / kStepRows;
  char* w = (char*)ws;
  double2* a = (double2*)w;   // working matrix
  w += (size_t)n * n * sizeof(double2);
  double2* pb[2];              // panel buffers (n x kNb); afterwards the update operands
  pb[0] = (double2*)w;
  w += (size_t)n * kNb * sizeof(double2);
  pb[1] = (double2*)w;
  w += (size_t)n * kNb * sizeof(double2);
  int* piv = (int*)w;
  w += (size_t)n * sizeof(int);
  int* idx = (int*)w;
  w += (size_t)n * sizeof(int);
  double* cm[2];
  int* ci[2];
  cm[0] = (double*)w;
  w += ncand * sizeof(double);
  cm[1] = (double*)w;
  w += ncand * sizeof(double);
  ci[0] = (int*)w;
  w += ncand * sizeof(int);
  ci[1] = (int*)w;
  const size_t nn = (size_t)n * n;
  const unsigned gnn = (unsigned)((nn + 255) / 256);
  k_form_eps<<<gnn, 256, 0, st>>>(v, chi, n, a);
  for (int j0 = 0; j0 < n; j0 += kNb) {
    const int nbp = n - j0 < kNb ? n - j0 : kNb;
    k_panel_load<<<ncand, 256, 0, st>>>(a, n, j0, nbp, pb[0], cm[0], ci[0]);
    for (int jc = 0; jc < nbp; ++jc)
      k_gj_step<<<ncand, 256, 0, st>>>(pb[jc & 1], pb[(jc + 1) & 1], n, j0, jc, nbp, cm[jc & 1], ci[jc & 1], ncand,
                                       cm[(jc + 1) & 1], ci[(jc + 1) & 1], piv, flag);
    double2* fin = pb[nbp & 1];
    double2* other = pb[(nbp + 1) & 1];
    if (nbp < n) k_row_swaps<<<(n + 255) / 256, 256, 0, st>>>(a, n, j0, nbp, piv);
    const size_t nops = (size_t)n * kNb;
    k_panel_operands<<<(unsigned)((nops + 255) / 256), 256, 0, st>>>(a, n, j0, nbp, fin, other);
    if (nbp == n) break;   // a single panel: no other columns to update
    hipError_t e = launch_zgemm(n, n, kNb, double2{1.0, 0.0}, fin, kNb, false, other, n, false, double2{1.0, 0.0},
                                a, n, st);
    if (e != hipSuccess) return e;
  }
  k_col_perm<<<1, 64, 0, st>>>(piv, n, idx);
  k_gather_cols<<<gnn, 256, 0, st>>>(a, idx, n, out);
  return hipGetLastError();
}

hipError_t launch_eps_inv_sweep(int n, const double* v, const double2* chi, double2* out, void* ws, int* flag,
                                hipStream_t st) {
  const int ldp = (n + kSw - 1) / kSw * kSw;
  char* w = (char*)ws;
  double2* a = (double2*)w;
  w += (size_t)ldp * ldp * sizeof(double2);
  double2* ct = (double2*)w;
  w += (size_t)kSw * ldp * sizeof(double2);
  double2* pp = (double2*)w;
  w += (size_t)kSw * ldp * sizeof(double2);
  double2* linvT = (double2*)w;
  w += (size_t)kSw * kSw * sizeof(double2);
  double2* dinv = (double2*)w;
  w += (size_t)kSw * kSw * sizeof(double2);
  double* wneg = (double*)w;
  w += kSw * sizeof(double);
  int* counter = (int*)(((uintptr_t)w + 255) / 256 * 256);
  const size_t nn = (size_t)ldp * ldp;
  k_sweep_form<<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(v, chi, n, ldp, a, flag);
  k_fill_f64_neg<<<1, kSw, 0, st>>>(wneg, kSw);
  const int nt = ldp / kSw;
  ContractBatch bt{};
  bt.nprob = 1;
  bt.item0[0] = 0;
  bt.item0[1] = (long long)nt * (nt + 1) / 2;
  bt.p[0] = ContractProb{ct, wneg, a, kSw, ldp, 1, nt * (nt + 1) / 2};
  const int grid = (int)std::min<long long>(bt.item0[1], 256LL * 8);
  for (int k0 = 0; k0 < ldp; k0 += kSw) {
    k_sweep_diag<<<1, 256, 0, st>>>(a, ldp, k0, linvT, dinv, flag);
    k_sweep_panel<<<nt, 256, 0, st>>>(a, ldp, k0, linvT, dinv, ct, pp);
    if (nt > 1) {
      hipError_t e = launch_zero(counter, 256, st);
      if (e != hipSuccess) return e;
      e = launch_contract_batch(0, bt, counter, grid, true, st);
      if (e != hipSuccess) return e;
    }
    k_sweep_write<<<(unsigned)(((size_t)ldp * kSw + 255) / 256), 256, 0, st>>>(a, ldp, k0, pp, dinv);
  }
  k_sweep_out<<<(unsigned)(((size_t)n * n + 255) / 256), 256, 0, st>>>(v, a, n, ldp, out);
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
