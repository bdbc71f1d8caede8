// Weights and the dense contraction of Eq. (chi0):
//   chi0_GG' += sum_p w_p M_p(G) conj(M_p(G')),
//   w_p = n_c * 1/2 [1/(E_v - E_c - w + i delta) + 1/(E_v - E_c + w + i delta)]   (float64).
// A complex weight splits into two real ones, chi0 = H_a + i H_b with
// H_x = sum_p x_p M_p M_p^H Hermitian, so every job is a Hermitian rank-k update with
// real per-pair weights, computed for the lower tiles only and mirrored at the end.
//
// One work item = one lower tile (G, G') of one job (q-point, frequency, part), 64 x 64 in
// float64 and 128 x 128 otherwise, over one of ksplit ranges of pairs; each item owns a
// float64 partial sum (no atomics, fixed summation order).  The next stage of pairs is
// loaded (straight into LDS in float64 / float32, into registers in split-bf16) while the
// current one runs on MFMA.  A persistent grid pulls the items from a counter, ordered so
// that the problems with the largest dielectric spheres come first.
//
// MFMA forms: f64 / f32 16x16x4 with Re += a.re b.re + a.im b.im and
// Im += a.im b.re - a.re b.im (b = w M(G')), and split-bf16 x3 (see below).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace gw {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Output row of accumulator register r in lane group lk = lane / 16 (column = lane % 16);
// the f64 and f32 16x16x4 instructions differ here.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = f64x4;
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  using acc = f32x4;
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

__global__ void k_weights(const double* __restrict__ e_v, int v0, int nv_valid, int nvs,
                          const double* __restrict__ e_col, const double* __restrict__ n_col, int c0, int nc_valid,
                          int ncs, double omega, double delta, int nparts, double* __restrict__ w) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = nvs * ncs;
  if (p >= np) return;
  const int v = v0 + p / ncs;
  const int c = c0 + p % ncs;
  double wr = 0.0, wi = 0.0;
  if (v < nv_valid && c < nc_valid) {
    const double n = n_col ? n_col[c] : 1.0;
    const double x = e_v[v] - e_col[c];
    if (delta == 0.0 && omega == 0.0) {
      wr = 0.5 * n * (1.0 / x + 1.0 / x);
    } else {
      // 1/(x - w + i d) + 1/(x + w + i d), each as conj(z)/|z|^2
      const double a = x - omega, b = x + omega;
      const double da = a * a + delta * delta, db = b * b + delta * delta;
      wr = 0.5 * n * (a / da + b / db);
      wi = 0.5 * n * (-delta / da - delta / db);
    }
  }
  w[p] = wr;
  if (nparts == 2) w[np + p] = wi;
}

// Values the band sum cannot use set bits of *flag (NULL arrays are not read): 1 a non-finite band or column energy,
// 2 a negative or non-finite column multiplicity, 4 a column row outside [0, nband).
__global__ void k_check_columns(const double* __restrict__ e_v, int nv, const double* __restrict__ e_col,
                                const double* __restrict__ n_col, const int32_t* __restrict__ col_band, int ncol,
                                int nband, int* __restrict__ flag) {
  int bad = 0;
  const int n = nv > ncol ? nv : ncol;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i < nv && e_v && !isfinite(e_v[i])) bad |= 1;
    if (i < ncol) {
      if (e_col && !isfinite(e_col[i])) bad |= 1;
      if (n_col && !(n_col[i] >= 0.0 && isfinite(n_col[i]))) bad |= 2;
      if (col_band && (col_band[i] < 0 || col_band[i] >= nband)) bad |= 4;
    }
  }
  if (bad) atomicOr(flag, bad);
}

__device__ __forceinline__ void tile_coords(int t, int* ti, int* tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *ti = i;
  *tj = t - i * (i + 1) / 2;
}

// The same lower triangle in 8 x 8 super-blocks of tiles (super-blocks in the order above,
// tiles column by column inside the off-diagonal ones): a run of consecutive indices covers few distinct tile rows
// and columns, so the workgroups of one XCD that take such a run share most operand rows in
// their L2.
__device__ __forceinline__ void tile_coords_blocked(int t, int nt, int* ti, int* tj) {
  constexpr int S = 8;
  const int ns = (nt + S - 1) / S;
  for (int bi = 0; bi < ns; ++bi) {
    const int r0 = bi * S, nr = min(S, nt - r0);
    for (int bj = 0; bj <= bi; ++bj) {
      const int c0 = bj * S, nc = min(S, nt - c0);
      // tiles (i, j), j <= i, of this super-block
      const int cnt = bi == bj ? nr * (nr + 1) / 2 : nr * nc;
      if (t < cnt) {
        if (bi == bj) {
          int i = 0;
          while ((i + 1) * (i + 2) / 2 <= t) ++i;
          *ti = r0 + i;
          *tj = c0 + t - i * (i + 1) / 2;
        } else {   // column by column: a run of 32 covers 8 tile rows (A, 128 B per row and
                   // stage) and 4 tile columns (B, 192 B per row and stage)
          *ti = r0 + t % nr;
          *tj = c0 + t / nr;
        }
        return;
      }
      t -= cnt;
    }
  }
  *ti = *tj = 0;   // not reached for t < nt (nt + 1) / 2
}

// Tile geometry: TILE x TILE outputs per workgroup of NW waves on a WR x WC grid, each
// wave owning (16 MI) x (16 NJ) outputs as MI x NJ MFMA blocks.
template <int TILE> struct TileGeo;
template <> struct TileGeo<64> {
  static constexpr int NW = 4, WR = 2, WC = 2, MI = 2, NJ = 2;
};
template <> struct TileGeo<128> {
  static constexpr int NW = 8, WR = 2, WC = 4, MI = 4, NJ = 2;
};

// float64 partial sum of one item; rows of block (i, j) start at r0 + 16 i, columns at c0 + 16 j
template <int MI, int NJ, typename A4>
__device__ __forceinline__ void store_tile(double2* out, int ngp, int r0, int c0, const A4 (&cre)[MI][NJ],
                                           const A4 (&cim)[MI][NJ], int li, int lk, bool f64_rows) {
  // eight results at a time: their loads first, so that they are in flight together (the
  // compiler cannot tell that the stores do not alias the later loads)
  constexpr int NB = 8;
  static_assert((NJ * 4) % NB == 0, "batches of whole result rows");
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int b = 0; b < NJ * 4; b += NB) {
      double2 o[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int j = (b + q) / 4, r = (b + q) % 4;
        const int row = r0 + 16 * i + (f64_rows ? lk + 4 * r : 4 * lk + r);
        o[q] = out[(size_t)row * ngp + c0 + 16 * j + li];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int j = (b + q) / 4, r = (b + q) % 4;
        const int row = r0 + 16 * i + (f64_rows ? lk + 4 * r : 4 * lk + r);
        out[(size_t)row * ngp + c0 + 16 * j + li] =
            double2{o[q].x + (double)cre[i][j][r], o[q].y + (double)cim[i][j][r]};
      }
    }
}

constexpr int KC = 16;   // pairs per LDS stage

// Length of each of the ksplit pair ranges: a multiple of the 16-pair stage, so that only
// a range's last stage can be partial and every stage starts on a multiple of 16.
__device__ __forceinline__ int range_len(int nk, int ksplit) {
  const int per = (nk + ksplit - 1) / ksplit;
  return (per + 15) / 16 * 16;
}

// ---------------------------------------------------------------- f64 / f32 MFMA tile
// A stage is KD pairs.  Its rows of M (1 KB per tile row in both precisions) go straight
// into LDS by 16-byte direct loads (global_load_lds_dwordx4, one wave instruction per row),
// into two buffers that are separate arrays, with the stage loop unrolled by two: the
// compiler then sees that the reads of one buffer cannot alias the loads in flight into the
// other and does not wait for them, and the staging holds no registers.  Two 8-pair
// buffers take the LDS of one 16-pair stage, so three float64 workgroups still share a CU.
// The weights scale the A fragments in registers; rows past the range load the range's last
// row and get weight 0.
constexpr int KD = 8;   // pairs per stage of the direct-load tile
template <typename T, int TILE>
__device__ void tile_mfma(const cx<T>* __restrict__ m, const double* __restrict__ w, int nk, int ngp, int ksplit,
                          double2* __restrict__ acc, int t, int ks) {
  using V = cx<T>;
  using A4 = typename Mfma<T>::acc;
  using G = TileGeo<TILE>;
  constexpr int NW = G::NW;
  constexpr int MI = G::MI, NJ = G::NJ;
  static_assert(TILE * sizeof(V) == 1024, "a tile row is one wave instruction of 64 x 16 bytes");
  constexpr int RPW = 2 * KD / NW;   // rows (A then B) per wave per stage
  static_assert(RPW * NW == 2 * KD, "the 2 KD rows of a stage must split evenly over the waves");
  __shared__ __align__(16) V sA0[KD][TILE];
  __shared__ __align__(16) V sB0[KD][TILE];
  __shared__ __align__(16) V sA1[KD][TILE];
  __shared__ __align__(16) V sB1[KD][TILE];
  int ti, tj;
  tile_coords(t, &ti, &tj);
  const int g0 = ti * TILE, h0 = tj * TILE;
  const int per = range_len(nk, ksplit);
  const int k0 = ks * per;
  const int k1 = min(nk, k0 + per);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wr = wave / G::WC, wc = wave % G::WC;
  const int li = lane & 15, lk = lane >> 4;

  A4 cre[MI][NJ], cim[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      cre[i][j] = A4{0, 0, 0, 0};
      cim[i][j] = A4{0, 0, 0, 0};
    }
  // row q = NW i + wave of a stage (wave-uniform): A rows are q < KD, B rows the rest
  auto issue = [&](int kk, V (*dA)[TILE], V (*dB)[TILE]) {
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int q = NW * i + wave;
      const bool isb = q >= KD;
      const int k = isb ? q - KD : q;
      const int row = min(kk + k, k1 - 1);
      const char* src = (const char*)(m + (size_t)row * ngp + (isb ? h0 : g0)) + 16 * lane;
      V* dst = isb ? &dB[k][0] : &dA[k][0];
      __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  double wn[KD / 4];
  auto load_w = [&](int kk) {
#pragma unroll
    for (int s = 0; s < KD / 4; ++s) {
      const int k = kk + 4 * s + lk;
      wn[s] = k < k1 ? w[k] : 0.0;
    }
  };
  auto stage = [&](int kk, V (*cA)[TILE], V (*cB)[TILE], V (*nA)[TILE], V (*nB)[TILE]) {
    // this wave's loads of the stage have landed; the barrier makes everyone's visible and
    // ends every wave's reads of the buffer that the next issue overwrites
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    double wcur[KD / 4];
#pragma unroll
    for (int s = 0; s < KD / 4; ++s) wcur[s] = wn[s];
    if (kk + KD < k1) {
      issue(kk + KD, nA, nB);
      load_w(kk + KD);
    }
#pragma unroll
    for (int s = 0; s < KD / 4; ++s) {
      const int k = 4 * s + lk;
      const T ws = T(wcur[s]);
      V a[MI], b[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const V x = cA[k][16 * MI * wr + 16 * i + li];
        a[i] = V{x.x * ws, x.y * ws};
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = cB[k][16 * NJ * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          cre[i][j] = Mfma<T>::run(a[i].x, b[j].x, cre[i][j]);
          cre[i][j] = Mfma<T>::run(a[i].y, b[j].y, cre[i][j]);
          cim[i][j] = Mfma<T>::run(a[i].y, b[j].x, cim[i][j]);
          cim[i][j] = Mfma<T>::run(-a[i].x, b[j].y, cim[i][j]);
        }
    }
  };
  if (k0 < k1) {
    issue(k0, sA0, sB0);
    load_w(k0);
  }
  for (int kk = k0; kk < k1; kk += 2 * KD) {
    stage(kk, sA0, sB0, sA1, sB1);
    if (kk + KD < k1) stage(kk + KD, sA1, sB1, sA0, sB0);
  }
  store_tile<MI, NJ>(acc + (size_t)ks * ngp * ngp, ngp, g0 + 16 * MI * wr, h0 + 16 * NJ * wc, cre, cim, li, lk,
                     std::is_same<T, double>::value);
}

// ---------------------------------------------------------------- split-bf16 x3 tile
// Each float32 operand x = hi + lo (hi = bf16(x), lo = bf16(x - hi), round to nearest
// even); products use hi*hi + hi*lo + lo*hi on MFMA 16x16x32 bf16 with float32
// accumulation.  The complex Hermitian update is two real products over a doubled
// inner index k' = [re of 16 pairs | im of 16 pairs]:
//   Re C = [ar | ai] [br | bi]^T,   Im C = [ar | ai] [-bi | br]^T,   b = w M(G'),
// so both products share the A fragments; the B rows carry a negated copy of bi.
// MFMA 16x16x32 bf16 operands: lane l holds row l % 16, inner indices 8 (l / 16) + 0..7;
// result rows 4 (l / 16) + r, column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));


constexpr int BK = 16;          // pairs per MFMA step
static_assert(BK == KC && KC == 16, "pair ranges are aligned to 16-pair stages");
// bf16 per LDS row: [re | im] of the 16 pairs, then -im (B rows only), then padding so
// that 8 rows read together hit distinct banks
constexpr int BROW = 56;

template <int TILE>
__device__ void tile_bf16x3(const void* __restrict__ mv, const double* __restrict__ w, int nk, int ngp, int ksplit,
                            double2* __restrict__ acc, int t, int ks) {
  using G = TileGeo<TILE>;
  constexpr int MI = G::MI, NJ = G::NJ;
  const float2* m = (const float2*)mv;
  // [A|B][hi|lo][row][k']
  __shared__ __align__(16) unsigned short s[2][2][TILE][BROW];
  int ti, tj;
  tile_coords(t, &ti, &tj);
  const int g0 = ti * TILE, h0 = tj * TILE;
  const int per = range_len(nk, ksplit);
  const int k0 = ks * per;
  const int k1 = min(nk, k0 + per);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave / G::WC, wc = wave % G::WC;
  const int li = lane & 15, lg = lane >> 4;
  // staging role: operand (A or B), row, half of the 16 pairs
  const int op = __builtin_amdgcn_readfirstlane(tid / (2 * TILE));   // 0: A rows (G), 1: B rows (G'); wave-uniform
  const int srow = tid % TILE;
  const int shalf = (tid / TILE) % 2;        // pairs [8 shalf, 8 shalf + 8)
  const int gcol = (op ? h0 : g0) + srow;

  f32x4 cre[MI][NJ], cim[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      cre[i][j] = f32x4{0, 0, 0, 0};
      cim[i][j] = f32x4{0, 0, 0, 0};
    }
  float2 pf[8];
  auto fetch = [&](int kk) {
    const int kb = kk + 8 * shalf;
    if (kk + BK <= k1) {   // every stage but the last of a range: no masks
      double wk[8];
      if (op) {
        // kb is a multiple of 8 (stage-aligned ranges), so 16-byte loads of the weights
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const double2 w2 = *(const double2*)(w + kb + e);
          wk[e] = w2.x;
          wk[e + 1] = w2.y;
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float2 x = m[(size_t)(kb + e) * ngp + gcol];
        if (op) {
          const float sw = (float)wk[e];
          x.x *= sw;
          x.y *= sw;
        }
        pf[e] = x;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = kb + e;
      float2 x{0.f, 0.f};
      if (k < k1) {
        x = m[(size_t)k * ngp + gcol];
        if (op) {
          const float sw = (float)w[k];
          x.x *= sw;
          x.y *= sw;
        }
      }
      pf[e] = x;
    }
  };
  if (k0 < k1) fetch(k0);
  // the imaginary product's right operand [-bi | br]: lanes of groups 0, 1 read the
  // negated copy of bi, those of groups 2, 3 read br
  const int boff = lg < 2 ? 32 + 8 * lg : 8 * (lg - 2);
  for (int kk = k0; kk < k1; kk += BK) {
    __syncthreads();
    {
      u16x8 rh, rl, ih, il;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const unsigned short a = bf16_rne(pf[e].x), b = bf16_rne(pf[e].y);
        rh[e] = a;
        ih[e] = b;
        rl[e] = bf16_rne(pf[e].x - bf16_val(a));
        il[e] = bf16_rne(pf[e].y - bf16_val(b));
      }
      *(u16x8*)&s[op][0][srow][8 * shalf] = rh;
      *(u16x8*)&s[op][0][srow][16 + 8 * shalf] = ih;
      *(u16x8*)&s[op][1][srow][8 * shalf] = rl;
      *(u16x8*)&s[op][1][srow][16 + 8 * shalf] = il;
      if (op == 1) {
        // bf16 negation flips the sign bit, so -hi and -lo split -bi exactly
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 sign = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
        *(u32x4*)&s[1][0][srow][32 + 8 * shalf] = __builtin_bit_cast(u32x4, ih) ^ sign;
        *(u32x4*)&s[1][1][srow][32 + 8 * shalf] = __builtin_bit_cast(u32x4, il) ^ sign;
      }
    }
    __syncthreads();
    if (kk + BK < k1) fetch(kk + BK);
    bf16x8 xh[MI], xl[MI], bh[NJ], bl[NJ], ch[NJ], cl[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int r = 16 * MI * wr + 16 * i + li;
      xh[i] = *(const bf16x8*)&s[0][0][r][8 * lg];
      xl[i] = *(const bf16x8*)&s[0][1][r][8 * lg];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = 16 * NJ * wc + 16 * j + li;
      bh[j] = *(const bf16x8*)&s[1][0][r][8 * lg];
      bl[j] = *(const bf16x8*)&s[1][1][r][8 * lg];
      ch[j] = *(const bf16x8*)&s[1][0][r][boff];
      cl[j] = *(const bf16x8*)&s[1][1][r][boff];
    }
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], bh[j], cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], bl[j], cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], bh[j], cre[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], ch[j], cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], cl[j], cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], ch[j], cim[i][j], 0, 0, 0);
      }
  }
  store_tile<MI, NJ>(acc + (size_t)ks * ngp * ngp, ngp, g0 + 16 * MI * wr, h0 + 16 * NJ * wc, cre, cim, li, lg, false);
}

// ---------------------------------------------------------------- split-bf16 x3 from row images
// Static jobs (one real weight per pair): the chunk's pair densities are split once per chunk
// into bf16 row images (k_split_ab): per block of 16 pairs kb and row G,
//   A[kb][G] = [hi re(16) | hi im(16) | lo re(16) | lo im(16)] of M      (8 units of 16 bytes)
//   B[kb][G] = [hi br | hi bi | hi -bi | lo br | lo bi | lo -bi] of b = w M  (12 units)
// and the tile stages both straight into LDS by 16-byte direct loads (global_load_lds_dwordx4),
// as the split-bf16 adjoint does: no staging registers, no conversion and one barrier per
// 16-pair stage.  LDS units of a stage: the 128 A rows of 8 (unit c of row r
// at 8 r + (c ^ (r & 7))), then the 128 B rows of 12 (unit p at UA + 12 r + (p ^ 2 ((r >> 2) & 1)));
// the XORs spread the 16 rows x 4 units of a fragment read over the bank groups.
constexpr int IMT = 128;                       // tile
constexpr int IUA = IMT * 8, IUB = IMT * 12;   // A and B units of a stage
constexpr int IUS = IUA + IUB;
// 8 waves (each 64 x 32 outputs), one workgroup per CU, and loads two stages ahead through
// three LDS buffers: the stage barrier orders LDS only (lds_barrier) and each stage waits for
// its own direct loads, so the next stages' loads stay in flight across it.  Every stage
// issues (past the range end: its last stage again, into a buffer not read), so the wait count
// is one constant.  Measured per chunk against four waves of 64 x 64 outputs, two workgroups
// per CU and two buffers: 19.5 against 20.1 ms at NG 8000 (32k pairs), 1.69 against 1.98 ms
// at NG 2000.
constexpr int INT = 512;
constexpr int IUPL = IUS / INT;                // units per lane per stage
static_assert(IUPL * INT == IUS && IUA % 64 == 0, "stage units must split into whole wave instructions");

__device__ void tile_bf16x3_img(const uint4* __restrict__ aimg, const uint4* __restrict__ bimg, int nk, int ngp,
                                 int ksplit, double2* __restrict__ acc, int t, int ks, uint4* sa, uint4* sb,
                                 uint4* sc) {
  constexpr int MI = 4, NJ = 2;
  int ti, tj;
  tile_coords_blocked(t, ngp / IMT, &ti, &tj);
  const int g0 = ti * IMT, h0 = tj * IMT;
  const int per = range_len(nk, ksplit);
  const int kb0 = ks * per / 16;
  const int kb1 = min(nk, ks * per + per) / 16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 2, wc = wave & 3;
  const int li = lane & 15, lg = lane >> 4;
  unsigned off[IUPL];
#pragma unroll
  for (int i = 0; i < IUPL; ++i) {
    const int ub = 8 * i + wave;
    const int u = 64 * ub + lane;
    if (ub * 64 < IUA) {
      const int r = u / 8, c = (u % 8) ^ (r & 7);
      off[i] = (unsigned)((g0 + r) * 8 + c);
    } else {
      const int u2 = u - IUA, r = u2 / 12, pc = (u2 % 12) ^ (2 * ((r >> 2) & 1));
      off[i] = (unsigned)((h0 + r) * 12 + pc);
    }
  }
  auto issue = [&](int kb, uint4* buf) {
    const uint4* ab = aimg + (size_t)kb * ngp * 8;
    const uint4* bbase = bimg + (size_t)kb * ngp * 12;
#pragma unroll
    for (int i = 0; i < IUPL; ++i) {
      const int ub = 8 * i + wave;
      const uint4* src = (ub * 64 < IUA ? ab : bbase) + off[i];
      __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)&buf[64 * ub], 16,
                                       0, 0);
    }
  };
  f32x4 cre[MI][NJ], cim[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      cre[i][j] = f32x4{0, 0, 0, 0};
      cim[i][j] = f32x4{0, 0, 0, 0};
    }
  const int pre = lg;
  const int pim = lg < 2 ? 4 + lg : lg - 2;
  auto stage = [&](int kb, const uint4* cur, uint4* next) {
    wait_vm<IUPL>();
    lds_barrier();
    issue(min(kb + 2, kb1 - 1), next);
    const uint4* sm = cur;
    const uint4* sg = cur + IUA;
    bf16x8 xh[MI], xl[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const int r = 16 * MI * wr + 16 * i + li;
      xh[i] = __builtin_bit_cast(bf16x8, sm[8 * r + (lg ^ (r & 7))]);
      xl[i] = __builtin_bit_cast(bf16x8, sm[8 * r + ((4 + lg) ^ (r & 7))]);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = 16 * NJ * wc + 16 * j + li;
      const int sw = 2 * ((r >> 2) & 1);
      const bf16x8 reh = __builtin_bit_cast(bf16x8, sg[12 * r + (pre ^ sw)]);
      const bf16x8 rel = __builtin_bit_cast(bf16x8, sg[12 * r + ((6 + pre) ^ sw)]);
      const bf16x8 imh = __builtin_bit_cast(bf16x8, sg[12 * r + (pim ^ sw)]);
      const bf16x8 iml = __builtin_bit_cast(bf16x8, sg[12 * r + ((6 + pim) ^ sw)]);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], reh, cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], rel, cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], reh, cre[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], imh, cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], iml, cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], imh, cim[i][j], 0, 0, 0);
      }
    }
  };
  // The diagonal G = G' sums w |M(G)|^2 terms of one sign, so float32 accumulation there errs
  // in proportion to the number of pairs (one 32k-pair range: 7.6e-6 of max |chi| against
  // 1.5e-7 off the diagonal); diagonal tiles add their sum into the float64 output every
  // kFlush stages (1056 pairs) and start again from zero.  Segments are whole multiples of
  // three stages, so that each starts on buffer sa; the loop runs whole triples and the
  // remainder after it (with the second and third stages conditional, the compiler's wait
  // tracking would merge paths on which another buffer's loads are the newest and wait for
  // every load before the LDS reads).
  constexpr int kFlush = 66;
  double2* out = acc + (size_t)ks * ngp * ngp;
  const int seg = ti == tj ? kFlush : (kb1 - kb0 + 2) / 3 * 3;
  if (kb0 < kb1) {
    issue(kb0, sa);
    issue(min(kb0 + 1, kb1 - 1), sb);
  }
  int s0 = kb0;
  do {
    const int s1 = min(kb1, s0 + seg);
    int kb = s0;
    for (; kb + 3 <= s1; kb += 3) {
      stage(kb, sa, sc);
      stage(kb + 1, sb, sa);
      stage(kb + 2, sc, sb);
    }
    if (kb < s1) stage(kb, sa, sc);
    if (kb + 1 < s1) stage(kb + 1, sb, sa);
    store_tile<MI, NJ>(out, ngp, g0 + 16 * MI * wr, h0 + 16 * NJ * wc, cre, cim, li, lg, false);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        cre[i][j] = f32x4{0, 0, 0, 0};
        cim[i][j] = f32x4{0, 0, 0, 0};
      }
    s0 = s1;
  } while (s0 < kb1);
  wait_vm<0>();   // no direct load may still be writing LDS when the next item starts
}

// Static schedule over the batch's items (no item counter).  Workgroups are dealt to the 8 XCDs
// round robin (workgroup b to XCD b mod 8), so each pass over a grid's worth of items gives
// XCD x the contiguous run of items [x grid / 8, (x + 1) grid / 8): with the blocked tile
// order, one compact group of tiles per L2.  The grid is a multiple of 8.  The barrier at the
// top of each item ends every wave's reads of the buffers before the next item's first loads.
__global__ __launch_bounds__(INT, 1) void k_contract_img(ContractBatch bt) {
  __shared__ __align__(16) uint4 sa[IUS];
  __shared__ __align__(16) uint4 sb[IUS];
  __shared__ __align__(16) uint4 sc[IUS];
  const long long n = bt.item0[bt.nprob];
  const int per_xcd = gridDim.x / 8;
  const int slot = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  for (long long base = 0; base + slot < n; base += gridDim.x) {
    const long long item = base + slot;
    __syncthreads();
    int b = 0;
    while (b + 1 < bt.nprob && item >= bt.item0[b + 1]) ++b;
    const ContractProb& p = bt.p[b];
    const long long local = item - bt.item0[b];
    const int per_job = p.ntl * p.ksplit;
    const int job = (int)(local / per_job);
    const int rem = (int)(local % per_job);
    double2* acc = p.acc + (size_t)job * p.ksplit * p.ngp * p.ngp;
    tile_bf16x3_img((const uint4*)p.aimg, (const uint4*)p.bimg, p.nk, p.ngp, p.ksplit, acc, rem % p.ntl,
                    rem / p.ntl, sa, sb, sc);
  }
}

// Row images of one chunk: one thread per (G, half h of a 16-pair block) packs whole 16-byte units
// (8 pairs) of the row: A units h, 2 + h, 4 + h, 6 + h and B units h, 2 + h, 4 + h, 6 + h, 8 + h,
// 10 + h.  Loads of M run along G (two lanes per G, the halves 8 rows apart); the two lanes of a G
// together write its whole A and B rows.
__global__ __launch_bounds__(256) void k_split_ab(const float2* __restrict__ m, const double* __restrict__ w, int ngp,
                                                  uint4* __restrict__ aimg, uint4* __restrict__ bimg) {
  const int kb = blockIdx.y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int g = t >> 1, h = t & 1;
  if (g >= ngp) return;
  u16x8 ahr, ahi, alr, ali, bhr, bhi, blr, bli;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 16 * kb + 8 * h + e;
    const float2 x = m[(size_t)k * ngp + g];
    const float sw = (float)w[k];
    const float yr = x.x * sw, yi = x.y * sw;
    const unsigned short a0 = bf16_rne(x.x), a1 = bf16_rne(x.y);
    ahr[e] = a0;
    ahi[e] = a1;
    alr[e] = bf16_rne(x.x - bf16_val(a0));
    ali[e] = bf16_rne(x.y - bf16_val(a1));
    const unsigned short b0 = bf16_rne(yr), b1 = bf16_rne(yi);
    bhr[e] = b0;
    bhi[e] = b1;
    blr[e] = bf16_rne(yr - bf16_val(b0));
    bli[e] = bf16_rne(yi - bf16_val(b1));
  }
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 sign = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};   // bf16 negation: -hi, -lo split -bi
  uint4* ad = aimg + ((size_t)kb * ngp + g) * 8;
  ad[h] = __builtin_bit_cast(uint4, ahr);
  ad[2 + h] = __builtin_bit_cast(uint4, ahi);
  ad[4 + h] = __builtin_bit_cast(uint4, alr);
  ad[6 + h] = __builtin_bit_cast(uint4, ali);
  uint4* bd = bimg + ((size_t)kb * ngp + g) * 12;
  bd[h] = __builtin_bit_cast(uint4, bhr);
  bd[2 + h] = __builtin_bit_cast(uint4, bhi);
  bd[4 + h] = __builtin_bit_cast(uint4, __builtin_bit_cast(u32x4, bhi) ^ sign);
  bd[6 + h] = __builtin_bit_cast(uint4, blr);
  bd[8 + h] = __builtin_bit_cast(uint4, bli);
  bd[10 + h] = __builtin_bit_cast(uint4, __builtin_bit_cast(u32x4, bli) ^ sign);
}

// ---------------------------------------------------------------- kernels
template <int MODE, int TILE>   // MODE 0 f64, 1 f32, 2 bf16x3 (register-staged)
__device__ __forceinline__ void run_item(const ContractProb& p, const double* w, double2* acc, int t, int ks) {
  if constexpr (MODE == 0)
    tile_mfma<double, TILE>((const double2*)p.m, w, p.nk, p.ngp, p.ksplit, acc, t, ks);
  else if constexpr (MODE == 1)
    tile_mfma<float, TILE>((const float2*)p.m, w, p.nk, p.ngp, p.ksplit, acc, t, ks);
  else
    tile_bf16x3<TILE>(p.m, w, p.nk, p.ngp, p.ksplit, acc, t, ks);
}

// Persistent grid over all items of a batch; items of problem b occupy
// [item0[b], item0[b+1]) and decode as (job, split, tile), job = w_index * nparts + part,
// tile fastest: pair-range major (all tiles of range 0, then range 1, ...), so that the
// workgroups in flight read the same few thousand rows of M, which stay in cache.  MINW = waves per SIMD the registers must
// allow: 4 holds two 512-thread split-bf16 workgroups per CU (128 registers), used when
// the contraction has the CUs to itself; 1 leaves registers for the pair kernels that run
// beside it on the other stream.
template <int MODE, int TILE, int MINW = 1>
__global__ __launch_bounds__(64 * TileGeo<TILE>::NW, MINW) void k_contract_batch(ContractBatch bt,
                                                                                 int* __restrict__ counter) {
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const long long item = s_item;
    if (item >= bt.item0[bt.nprob]) break;
    int b = 0;
    while (b + 1 < bt.nprob && item >= bt.item0[b + 1]) ++b;
    const ContractProb& p = bt.p[b];
    const long long local = item - bt.item0[b];
    const int per_job = p.ntl * p.ksplit;
    const int job = (int)(local / per_job);
    const int rem = (int)(local % per_job);
    const double* w = p.w + (size_t)job * p.nk;
    double2* acc = p.acc + (size_t)job * p.ksplit * p.ngp * p.ngp;
    run_item<MODE, TILE>(p, w, acc, rem % p.ntl, rem / p.ntl);
  }
}

__global__ void k_finalize(const double2* __restrict__ accA, const double2* __restrict__ accB, int ksplit, int ng,
                           int ngp, int accumulate, double2* __restrict__ chi) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)ng * ng) return;
  const int g = (int)(e / ng), h = (int)(e % ng);
  const bool lower = g >= h;
  const size_t src = lower ? (size_t)g * ngp + h : (size_t)h * ngp + g;
  double2 a{0.0, 0.0}, b{0.0, 0.0};
  for (int k = 0; k < ksplit; ++k) {
    const double2 x = accA[(size_t)k * ngp * ngp + src];
    a.x += x.x;
    a.y += x.y;
    if (accB) {
      const double2 y = accB[(size_t)k * ngp * ngp + src];
      b.x += y.x;
      b.y += y.y;
    }
  }
  if (!lower) {
    a.y = -a.y;
    b.y = -b.y;
  } else if (g == h) {
    // H_a and H_b are Hermitian: their diagonals are real (rounding leaves a residue)
    a.y = 0.0;
    b.y = 0.0;
  }
  const double2 r{a.x - b.y, a.y + b.x};
  if (accumulate) {
    const double2 o = chi[e];
    chi[e] = double2{o.x + r.x, o.y + r.y};
  } else {
    chi[e] = r;
  }
}

__global__ void k_zero(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = uint4{0, 0, 0, 0};
}

// out[(v * ncs + c) * ng + g] = m[(v * ncs_pad + c) * ngp + g] for v < nvs, c < ncs
template <typename T>
__global__ void k_copy_m(const cx<T>* __restrict__ m, int nvs, int ncs, int ncs_pad, int ng, int ngp,
                         double2* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nvs * ncs * ng) return;
  const size_t p = e / ng, g = e % ng;
  const size_t v = p / ncs, c = p % ncs;
  const cx<T> x = m[(v * ncs_pad + c) * ngp + g];
  out[e] = double2{(double)x.x, (double)x.y};
}

}  // namespace

hipError_t launch_weights(const double* e_v, int v0, int nv_valid, int nvs, const double* e_col, const double* n_col,
                          int c0, int nc_valid, int ncs, double omega, double delta, int nparts, double* w,
                          hipStream_t st) {
  const int np = nvs * ncs;
  k_weights<<<(np + 255) / 256, 256, 0, st>>>(e_v, v0, nv_valid, nvs, e_col, n_col, c0, nc_valid, ncs, omega, delta,
                                               nparts, w);
  return hipGetLastError();
}

hipError_t launch_check_columns(const double* e_v, int nv, const double* e_col, const double* n_col,
                                const int32_t* col_band, int ncol, int nband, int* flag, hipStream_t st) {
  const int n = nv > ncol ? nv : ncol;
  const int blocks = n < 256 * 64 ? (n + 255) / 256 : 64;
  k_check_columns<<<blocks, 256, 0, st>>>(e_v, nv, e_col, n_col, col_band, ncol, nband, flag);
  return hipGetLastError();
}

int contract_tile(int mode) { return mode == 0 ? 64 : 128; }

size_t split_image_bytes(int npair, int ngp) { return (size_t)npair * ngp * 20; }

hipError_t launch_split_ab(const void* m, const double* w, int npair, int ngp, void* img, hipStream_t st) {
  if (npair % 16 != 0 || ngp % 128 != 0) return hipErrorInvalidValue;
  uint4* a = (uint4*)img;
  uint4* b = a + (size_t)npair / 16 * ngp * 8;
  k_split_ab<<<dim3(ngp / 128, npair / 16), 256, 0, st>>>((const float2*)m, w, ngp, a, b);
  return hipGetLastError();
}

// Tiles per mode (contract_tile): 64 in float64, 128 in float32 and split-bf16 x3; only
// these forms are built.
hipError_t launch_contract_batch(int mode, const ContractBatch& bt, int* counter, int grid, bool alone,
                                 hipStream_t st) {
  for (int b = 0; b < bt.nprob; ++b)
    if (bt.p[b].ngp % contract_tile(mode) != 0) return hipErrorInvalidValue;
  if (mode == 3) {
    for (int b = 0; b < bt.nprob; ++b)
      if (!bt.p[b].aimg || !bt.p[b].bimg || bt.p[b].nk % 16 != 0) return hipErrorInvalidValue;
    (void)counter;
    long long items = bt.item0[bt.nprob];
    const int g1 = (int)std::min<long long>((items + 7) / 8 * 8, 256LL);
    k_contract_img<<<std::max(g1, 8), INT, 0, st>>>(bt);
  } else if (mode == 0)
    k_contract_batch<0, 64><<<grid, 64 * TileGeo<64>::NW, 0, st>>>(bt, counter);
  else if (mode == 1)
    k_contract_batch<1, 128><<<grid, 64 * TileGeo<128>::NW, 0, st>>>(bt, counter);
  else if (alone)
    k_contract_batch<2, 128, 4><<<grid, 64 * TileGeo<128>::NW, 0, st>>>(bt, counter);
  else
    k_contract_batch<2, 128><<<grid, 64 * TileGeo<128>::NW, 0, st>>>(bt, counter);
  return hipGetLastError();
}

hipError_t launch_finalize(const double2* accA, const double2* accB, int ksplit, int ng, int ngp, double2* chi,
                           bool accumulate, hipStream_t st) {
  const size_t n = (size_t)ng * ng;
  k_finalize<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(accA, accB, ksplit, ng, ngp, accumulate ? 1 : 0, chi);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n16 + 255) / 256, 65536);
  k_zero<<<nb, 256, 0, st>>>((uint4*)p, n16);
  return hipGetLastError();
}

hipError_t launch_copy_m(const void* m, int nvs, int ncs, int ncs_pad, int ng, int ngp, bool fp64, double2* out,
                         hipStream_t st) {
  const size_t n = (size_t)nvs * ncs * ng;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (fp64)
    k_copy_m<double><<<nb, 256, 0, st>>>((const double2*)m, nvs, ncs, ncs_pad, ng, ngp, out);
  else
    k_copy_m<float><<<nb, 256, 0, st>>>((const float2*)m, nvs, ncs, ncs_pad, ng, ngp, out);
  return hipGetLastError();
}

}  // namespace gw
