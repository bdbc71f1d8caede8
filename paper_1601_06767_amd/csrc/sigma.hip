// The COH self-energy of Eq. (sigmach), static limit and plasmon-pole form.
//
// Static limit, summed with the same column form
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

// ---------------------------------------------------------------- plasmon-pole COH
// Eq. (sigmach) with the plasmon-pole eps^-1 (each element a single pole of weight Omega^2 at
// wt), after the E' integral:
//   S_j[n][n'] = 1/2 sum_c w_c sum_{G G'} M_{n c}(G) A_{GG'}(x_jc) conj(M_{n' c}(G')),
//   A_{GG'}(x) = B_{GG'} / (x - wt_{GG'}),  B = Omega^2 v(G') / wt,  x_jc = E_j - E_c + i delta.
// k_gpp_coh_prep forms (B, wt) once per call; k_coh_gpp keeps a 64 x 64 tile of them in
// registers (each lane one column G' and 16 rows) and streams the columns c of a chunk and the
// energies E_j past it: W[n][G'] = sum_{G in the wave's 16 rows} M_n(G) A_GG' (M_n(G) read as an
// LDS broadcast), then each lane (n, n') adds sum_{G'} W[n][G'] conj(M_n'(G')) over the tile's
// columns to its own accumulator.  Partial sums per (tile, wave) are reduced in a fixed order.
constexpr int kGpT = 64;      // G rows and G' columns of a tile
constexpr int kGpRW = 16;     // rows per wave
constexpr int kGpS = 8;       // states per block
constexpr int kGpE = 8;       // energies per pass

struct GppEnergies {
  double e[kGpE];
};

// principal square root (non-negative real part; the sign of the imaginary part follows the
// argument's, signed zeros included)
__device__ __forceinline__ double2 csqrt_principal(double2 z) {
  const double r = hypot(z.x, z.y);
  const double re = sqrt(0.5 * (r + z.x));
  const double im = copysign(sqrt(0.5 * (r - z.x)), z.y);
  return double2{re, im};
}

// (B, wt) for G, G' < ngp (rows G); elements without a pole (wt^2 not finite), with Omega^2 = 0,
// or in the padding: B = 0, wt = 1, so that their term vanishes for every x
__global__ void k_gpp_coh_prep(const double2* __restrict__ om2, const double2* __restrict__ wt2,
                               const double* __restrict__ v, int ng, int ngp, double2* __restrict__ bb,
                               double2* __restrict__ ww) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ngp * ngp) return;
  const int g = (int)(e / ngp), h = (int)(e % ngp);
  double2 b{0.0, 0.0}, w{1.0, 0.0};
  if (g < ng && h < ng) {
    const size_t i = (size_t)g * ng + h;
    const double2 o = om2[i], t = wt2[i];
    if (isfinite(t.x) && isfinite(t.y) && (o.x != 0.0 || o.y != 0.0)) {
      w = csqrt_principal(t);
      // B = o v(h) / w
      const double d = w.x * w.x + w.y * w.y;
      const double vr = v[h] / d;
      b = double2{(o.x * w.x + o.y * w.y) * vr, (o.y * w.x - o.x * w.y) * vr};
    }
  }
  bb[e] = b;
  ww[e] = w;
}

// part[((tile * 4 + wave) * kGpE + j) * 64 + lane] += sum over the chunk's columns for lane's
// (n, n') = (lane / 8, lane % 8) of state blocks (sa, sb); states >= ns count as zero.
__global__ __launch_bounds__(256) void k_coh_gpp(const double2* __restrict__ bb, const double2* __restrict__ ww,
                                                 int ngp, int ntile1, const double2* __restrict__ m, int cc, int ns,
                                                 int sa, int sb, int nvalid, const double* __restrict__ e_col,
                                                 const double* __restrict__ n_col, int c0, GppEnergies en, int ne,
                                                 double delta, double2* __restrict__ part) {
  __shared__ double2 s_mr[kGpS][kGpT];          // M_n(G), the tile's rows, state block sa
  __shared__ double2 s_mc[kGpS][kGpT];          // M_n'(G'), the tile's columns, state block sb
  __shared__ double2 s_w[4][kGpS][kGpT];        // W of each wave
  const int tile = blockIdx.x;
  const int t0 = tile / ntile1, t1 = tile % ntile1;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int col = t1 * kGpT + lane;
  const int row0 = t0 * kGpT + wave * kGpRW;
  double2 bq[kGpRW], wq[kGpRW];
#pragma unroll
  for (int r = 0; r < kGpRW; ++r) {
    bq[r] = bb[(size_t)(row0 + r) * ngp + col];
    wq[r] = ww[(size_t)(row0 + r) * ngp + col];
  }
  const int pn = lane / kGpS, pm = lane % kGpS;   // this lane's (n, n')
  double2 acc[kGpE];
#pragma unroll
  for (int j = 0; j < kGpE; ++j) acc[j] = double2{0.0, 0.0};
  const size_t klen = (size_t)cc * ngp;
  for (int c = 0; c < nvalid; ++c) {
    __syncthreads();   // the previous column's stage is no longer read
    for (int e = tid; e < 2 * kGpS * kGpT; e += 256) {
      const int which = e / (kGpS * kGpT), n = (e / kGpT) % kGpS, k = e % kGpT;
      const int st = (which ? sb : sa) * kGpS + n;
      const int g = (which ? t1 : t0) * kGpT + k;
      const double2 x = st < ns ? m[(size_t)st * klen + (size_t)c * ngp + g] : double2{0.0, 0.0};
      if (which)
        s_mc[n][k] = x;
      else
        s_mr[n][k] = x;
    }
    __syncthreads();
    const double wc = n_col ? n_col[c0 + c] : 1.0;
    const double ec = e_col[c0 + c];
#pragma unroll 1
    for (int j = 0; j < ne; ++j) {
      const double xr = en.e[j] - ec;
      double2 w[kGpS];
#pragma unroll
      for (int n = 0; n < kGpS; ++n) w[n] = double2{0.0, 0.0};
#pragma unroll
      for (int r = 0; r < kGpRW; ++r) {
        const double dr = xr - wq[r].x, di = delta - wq[r].y;
        const double inv = 1.0 / (dr * dr + di * di);
        const double2 a{(bq[r].x * dr + bq[r].y * di) * inv, (bq[r].y * dr - bq[r].x * di) * inv};
#pragma unroll
        for (int n = 0; n < kGpS; ++n) cmac(w[n], s_mr[n][wave * kGpRW + r], a);
      }
#pragma unroll
      for (int n = 0; n < kGpS; ++n) s_w[wave][n][lane] = w[n];
      __syncthreads();
      double2 t{0.0, 0.0};
#pragma unroll 8
      for (int k = 0; k < kGpT; ++k) {
        const double2 y = s_mc[pm][k];
        cmac(t, s_w[wave][pn][k], double2{y.x, -y.y});
      }
      // acc_j += w_c t (j is uniform: select the accumulator without dynamic indexing)
#pragma unroll
      for (int q = 0; q < kGpE; ++q)
        if (q == j) {
          acc[q].x = fma(wc, t.x, acc[q].x);
          acc[q].y = fma(wc, t.y, acc[q].y);
        }
      __syncthreads();   // every lane has read s_w before the next energy rewrites it
    }
  }
  double2* dst = part + ((size_t)(tile * 4 + wave) * kGpE) * 64 + lane;
#pragma unroll
  for (int j = 0; j < kGpE; ++j) dst[(size_t)j * 64] = cadd(dst[(size_t)j * 64], acc[j]);
}

// out[j][n][n'] += 1/2 sum over tiles and waves of part (fixed order: each thread a fixed
// strided subset, then a fixed tree), one workgroup per (j, n, n') of the pass
__global__ __launch_bounds__(256) void k_coh_gpp_sum(const double2* __restrict__ part, int nslot, int ne, int ns,
                                                     int sa, int sb, int e0, double2* __restrict__ out) {
  __shared__ double2 red[256];
  const int o = blockIdx.x;   // j * 64 + lane
  const int j = o / 64, lane = o % 64;
  const int n = sa * kGpS + lane / kGpS, np = sb * kGpS + lane % kGpS;
  double2 t{0.0, 0.0};
  for (int sl = threadIdx.x; sl < nslot; sl += 256) t = cadd(t, part[((size_t)sl * kGpE + j) * 64 + lane]);
  red[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && j < ne && n < ns && np < ns) {
    double2* d = out + ((size_t)(e0 + j) * ns + n) * ns + np;
    *d = cadd(*d, double2{0.5 * red[0].x, 0.5 * red[0].y});
  }
}

}  // namespace

int coh_max_states() { return kCohMaxStates; }

int gpp_coh_tile() { return kGpT; }
int gpp_coh_states_per_block() { return kGpS; }
int gpp_coh_energies_per_pass() { return kGpE; }
size_t gpp_coh_part_bytes(int ngp) {
  const size_t nt = (size_t)(ngp / kGpT) * (ngp / kGpT);
  return nt * 4 * kGpE * 64 * sizeof(double2);
}

hipError_t launch_gpp_coh_prep(const void* modes, const double* v, int ng, int ngp, void* b, void* w, hipStream_t st) {
  const size_t n = (size_t)ngp * ngp;
  const double2* om2 = (const double2*)modes;
  k_gpp_coh_prep<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(om2, om2 + (size_t)ng * ng, v, ng, ngp,
                                                               (double2*)b, (double2*)w);
  return hipGetLastError();
}

hipError_t launch_gpp_coh(const void* b, const void* w, int ngp, const void* m, int cc, int ns, int sa, int sb,
                          int nvalid, const double* e_col, const double* n_col, int c0, const double* energies, int ne,
                          double delta, void* part, hipStream_t st) {
  if (ngp % kGpT != 0 || ne < 1 || ne > kGpE) return hipErrorInvalidValue;
  GppEnergies en{};
  for (int j = 0; j < ne; ++j) en.e[j] = energies[j];
  const int nt1 = ngp / kGpT;
  k_coh_gpp<<<nt1 * nt1, 256, 0, st>>>((const double2*)b, (const double2*)w, ngp, nt1, (const double2*)m, cc, ns, sa,
                                       sb, nvalid, e_col, n_col, c0, en, ne, delta, (double2*)part);
  return hipGetLastError();
}

hipError_t launch_gpp_coh_sum(const void* part, int ngp, int ne, int ns, int sa, int sb, int e0, void* out,
                              hipStream_t st) {
  const int nt1 = ngp / kGpT;
  k_coh_gpp_sum<<<kGpE * 64, 256, 0, st>>>((const double2*)part, nt1 * nt1 * 4, ne, ns, sa, sb, e0, (double2*)out);
  return hipGetLastError();
}

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
