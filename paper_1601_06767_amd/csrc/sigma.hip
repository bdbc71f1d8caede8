// Static limit of the COH self-energy of Eq. (sigmach), summed with the same column form
// (bands and energy-window representatives with their weights) as Eq. (energyintegration):
//   S[n][n'] = 1/2 sum_c w_c sum_{G G'} M_{n c}(G) A_{G G'} conj(M_{n' c}(G')),
//   A = [eps^-1 - I] diag(v).
// The pair densities of a chunk come from the pair kernels; then Z = conj(M) A^T (one
// float64 MFMA GEMM) and S += X Z^T over the flattened (column, G) index with X = w_c M (split
// into blocks whose partial sums are added in a fixed order).
#include "common.h"
#include "internal.h"

namespace gw {

namespace {

// at[h][g] = A[g][h] = (eps_inv[g][h] - delta_gh) v[h] for g, h < ng (A transposed, so that
// Z = conj(M) A^T reads it row by row); zero in the padding up to ngp
__global__ void k_coh_kernel(const double2* __restrict__ eps_inv, const double* __restrict__ v, int ng, int ngp,
                             double2* __restrict__ a) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ngp * ngp) return;
  const int h = (int)(e / ngp), g = (int)(e % ngp);
  double2 x{0.0, 0.0};
  if (g < ng && h < ng) {
    x = eps_inv[(size_t)g * ng + h];
    if (g == h) x.x -= 1.0;
    x.x *= v[h];
    x.y *= v[h];
  }
  a[e] = x;
}

constexpr int kCohTile = 32;     // k-values per LDS tile
constexpr int kCohMaxStates = 32;

// part[blk][n][n'] = sum over the block's k-range of w_c M[n][k] Z[n'][k], k = c ngp + G,
// rows of length cc ngp (pairs v-major), columns c >= nvalid weigh 0.
__global__ __launch_bounds__(256) void k_coh_reduce(const double2* __restrict__ m, const double2* __restrict__ z,
                                                    int ns, int cc, int ngp, int nvalid,
                                                    const double* __restrict__ n_col, int c0, long long kper,
                                                    double2* __restrict__ part) {
  __shared__ double2 sx[kCohMaxStates][kCohTile];
  __shared__ double2 sz[kCohMaxStates][kCohTile];
  const long long klen = (long long)cc * ngp;
  const long long k0 = (long long)blockIdx.x * kper;
  const long long k1 = k0 + kper < klen ? k0 + kper : klen;
  const int tid = threadIdx.x;
  const int nout = ns * ns;
  double2 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = double2{0.0, 0.0};
  for (long long kt = k0; kt < k1; kt += kCohTile) {
    __syncthreads();
    for (int e = tid; e < ns * kCohTile; e += 256) {
      const int n = e / kCohTile, j = e % kCohTile;
      const long long k = kt + j;
      double2 x{0.0, 0.0}, y{0.0, 0.0};
      if (k < k1) {
        const int c = (int)(k / ngp);
        const double w = c < nvalid ? (n_col ? n_col[c0 + c] : 1.0) : 0.0;
        x = m[(size_t)n * klen + k];
        x.x *= w;
        x.y *= w;
        y = z[(size_t)n * klen + k];
      }
      sx[n][j] = x;
      sz[n][j] = y;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = tid + 256 * r;
      if (o < nout) {
        const int n = o / ns, np = o % ns;
#pragma unroll 8
        for (int j = 0; j < kCohTile; ++j) cmac(acc[r], sx[n][j], sz[np][j]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int o = tid + 256 * r;
    if (o < nout) part[(size_t)blockIdx.x * nout + o] = acc[r];
  }
}

// s[o] += 1/2 sum_blk part[blk][o], blocks in order
__global__ void k_coh_sum(const double2* __restrict__ part, int nblk, int nout, double2* __restrict__ s) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double2 t{0.0, 0.0};
  for (int b = 0; b < nblk; ++b) t = cadd(t, part[(size_t)b * nout + o]);
  s[o] = cadd(s[o], double2{0.5 * t.x, 0.5 * t.y});
}

}  // namespace

int coh_max_states() { return kCohMaxStates; }

hipError_t launch_coh_kernel(const void* eps_inv, const double* v, int ng, int ngp, void* a, hipStream_t st) {
  const size_t n = (size_t)ngp * ngp;
  k_coh_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((const double2*)eps_inv, v, ng, ngp, (double2*)a);
  return hipGetLastError();
}

hipError_t launch_coh_reduce(const void* m, const void* z, int ns, int cc, int ngp, int nvalid, const double* n_col,
                             int c0, int nblk, void* part, void* s, hipStream_t st) {
  if (ns < 1 || ns > kCohMaxStates || nblk < 1) return hipErrorInvalidValue;
  const long long klen = (long long)cc * ngp;
  long long kper = (klen + nblk - 1) / nblk;
  kper = (kper + kCohTile - 1) / kCohTile * kCohTile;
  const int nb = (int)((klen + kper - 1) / kper);
  k_coh_reduce<<<nb, 256, 0, st>>>((const double2*)m, (const double2*)z, ns, cc, ngp, nvalid, n_col, c0, kper,
                                   (double2*)part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nout = ns * ns;
  k_coh_sum<<<(nout + 255) / 256, 256, 0, st>>>((const double2*)part, nb, nout, (double2*)s);
  return hipGetLastError();
}

}  // namespace gw
