// Adjoint of the band sum of Eq. (chi0) with respect to the band energies, the
// column (window) energies and the column multiplicities.
//
// For a real loss L with chibar(w) = dL/dRe chi0(w) + i dL/dIm chi0(w):
//   s_p(w)  = m_p^H chibar(w) m_p                  (wbar of pair p, complex)
//   dL/dx_p = sum_w Re(conj(s_p) dw_p/dx),  dL/dn_p = sum_w Re(conj(s_p) dw_p/dn),  x = E_v - E_c
//   dL/dE_v = sum_c dL/dx_vc,  dL/dE_c = -sum_v dL/dx_vc,  dL/dn_c = sum_v dL/dn_vc.
// The pair densities m_p are recomputed chunk by chunk (never stored for all pairs).
// k_adjoint: Y = M chibar^T on MFMA (64 pairs x 64 G per workgroup, inner G'), fused
// with the row dot sum_G conj(M[p][G]) Y[p][G] over the tile's 64 G; the per-tile
// partial sums are reduced in float64 in fixed order by k_adjoint_pairs.
// k_adjoint_bf16x3: the same product for the split-bf16 mode on bf16 MFMA, 128 x 128 tiles.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace gw {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct AMfma;
template <> struct AMfma<double> {
  using acc = f64x4;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct AMfma<float> {
  using acc = f32x4;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// Tile order.  The 32 CUs of one XCD share its L2, and workgroup b runs on XCD b mod 8, so XCD
// x takes the contiguous run of tiles [x n / 8, (x + 1) n / 8) of a blocked order: bands of 8
// pair tiles, cut into blocks of 4 chibar tiles, each block pair-tile-fastest.  The 32 tiles an
// XCD holds at once then share 4 M and 8 chibar row slices of a stage, where the row-major
// order (the tiles of one pair tile spread over all XCDs) had each XCD read about 32 chibar
// slices per stage, all of chibar once per pair tile (split-BF16x3 at NG 8000, 32k pairs: L2
// misses 225 -> 62 GB, 41.1 -> 35.9 ms per launch).  The grid is rounded up to a multiple of
// 8; the workgroups past the last tile return at once.
__device__ __forceinline__ void adj_tile(int t, int npt, int ntg, int* pt, int* tg) {
  constexpr int BP = 8, BG = 4;
  const int band = t / (BP * ntg);
  const int nr = min(BP, npt - band * BP);   // pair tiles in this band
  const int local = t - band * BP * ntg;
  const int cb = local / (nr * BG);
  const int w = local - cb * nr * BG;
  *pt = band * BP + w % nr;
  *tg = cb * BG + w / nr;
}

constexpr int AT = 64, AK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_adjoint(const cx<T>* __restrict__ m, int npair, int ng, int ngp,
                                                 const double2* __restrict__ gbar, double2* __restrict__ part) {
  using V = cx<T>;
  using A4 = typename AMfma<T>::acc;
  __shared__ V sA[AK][AT + 1];   // M[p0 + i][G' = k]
  __shared__ V sB[AK][AT + 1];   // chibar[G0 + j][G' = k]
  __shared__ double2 sred[2][AT];
  const int ntg = ngp / AT;
  const int npt = (npair + AT - 1) / AT;
  const int t = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
  if (t >= npt * ntg) return;
  int pt, tg;
  adj_tile(t, npt, ntg, &pt, &tg);
  const int p0 = pt * AT;
  const int q0 = tg * AT;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;
  A4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = A4{0, 0, 0, 0};
      cim[i][j] = A4{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < ng; k0 += AK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < (AK * AT) / 256; ++r) {
      const int e = tid + 256 * r;
      const int row = e / AK, kk = e % AK;   // consecutive threads: consecutive G' of one row
      V a{T(0), T(0)}, b{T(0), T(0)};
      if (k0 + kk < ng) {
        if (p0 + row < npair) a = m[(size_t)(p0 + row) * ngp + k0 + kk];
        if (q0 + row < ng) {
          const double2 x = gbar[(size_t)(q0 + row) * ng + k0 + kk];
          b = V{T(x.x), T(x.y)};
        }
      }
      sA[kk][row] = a;
      sB[kk][row] = b;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < AK / 4; ++s) {
      const int k = 4 * s + lk;
      V a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[k][32 * wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[k][32 * wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = AMfma<T>::run(a[i].x, b[j].x, cre[i][j]);
          cre[i][j] = AMfma<T>::run(-a[i].y, b[j].y, cre[i][j]);
          cim[i][j] = AMfma<T>::run(a[i].x, b[j].y, cim[i][j]);
          cim[i][j] = AMfma<T>::run(a[i].y, b[j].x, cim[i][j]);
        }
    }
  }
  // epilogue: per pair row, sum over this tile's G of conj(M[p][G]) Y[p][G]
  double2 rs[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[i][r] = double2{0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = 32 * wr + 16 * i + AMfma<T>::row(lk, r);
        const int gc = q0 + 32 * wc + 16 * j + li;
        if (p0 + pr < npair && gc < ng) {
          const V mv = m[(size_t)(p0 + pr) * ngp + gc];
          const double yr = (double)cre[i][j][r], yi = (double)cim[i][j][r];
          rs[i][r].x += (double)mv.x * yr + (double)mv.y * yi;
          rs[i][r].y += (double)mv.x * yi - (double)mv.y * yr;
        }
      }
  // reduce over the 16 lanes li that share a row (xor shuffles within the 16-lane group)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) {
        rs[i][r].x += __shfl_xor(rs[i][r].x, o, 64);
        rs[i][r].y += __shfl_xor(rs[i][r].y, o, 64);
      }
  if (li == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) sred[wc][32 * wr + 16 * i + AMfma<T>::row(lk, r)] = rs[i][r];
  }
  __syncthreads();
  if (tid < AT && p0 + tid < npair) {
    const double2 a = sred[0][tid], b = sred[1][tid];
    part[(size_t)(p0 + tid) * ntg + tg] = double2{a.x + b.x, a.y + b.y};
  }
}

// ---------------------------------------------------------------- split-bf16 x3 form
// M (float) and chibar (rounded to float) are each split into hi = bf16(x) and
// lo = bf16(x - hi); products hi*hi + hi*lo + lo*hi on MFMA 16x16x32 bf16 with float32
// accumulation.  Over the doubled inner index k' = [re of 16 G' | im of 16 G']:
//   Re Y = [mr | mi] [br | -bi]^T,   Im Y = [mr | mi] [bi | br]^T,   b = chibar[G][G'],
// so both products share the M fragments; the chibar rows in LDS hold [br | bi | -bi].
// 128 pairs x 128 G per workgroup, 8 waves on a 2 x 4 grid, each 64 pairs x 32 G.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BT = 128;     // pairs and G per tile
constexpr int BKS = 16;     // G' per stage
constexpr int BMI = 4, BNJ = 2;

// chibar split once per call into the LDS image of its rows: for row G and block kb of 16 G',
// 96 bf16 = hi [re | im | -im] then lo [re | im | -im] (zero beyond ng), so that the tiles
// stage chibar with plain 16-byte copies instead of converting it once per pair tile.
constexpr int GSPLIT = 96;   // bf16 per (row, 16-G' block)
__global__ void k_split_gbar(const double2* __restrict__ gbar, int ng, int nkb, unsigned short* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // (row, block, G' in block)
  if (e >= (size_t)ng * nkb * 16) return;
  const int i = (int)(e % 16);
  const size_t rb = e / 16;   // row * nkb + kb
  const int kb = (int)(rb % nkb), row = (int)(rb / nkb);
  const int col = kb * 16 + i;
  float re = 0.f, im = 0.f;
  if (col < ng) {
    const double2 x = gbar[(size_t)row * ng + col];
    re = (float)x.x;
    im = (float)x.y;
  }
  const unsigned short rh = bf16_rne(re), ih = bf16_rne(im);
  const unsigned short rl = bf16_rne(re - bf16_val(rh)), il = bf16_rne(im - bf16_val(ih));
  unsigned short* o = out + rb * GSPLIT;
  o[i] = rh;
  o[16 + i] = ih;
  o[32 + i] = ih ^ 0x8000;
  o[48 + i] = rl;
  o[64 + i] = il;
  o[80 + i] = il ^ 0x8000;
}

// The pair densities split the same way, once per chunk: for pair row p and block kb of 16 G',
// 64 bf16 = hi [re | im] then lo [re | im] (zero beyond ng).
constexpr int MSPLIT = 64;   // bf16 per (pair row, 16-G' block)
__global__ void k_split_m(const float2* __restrict__ m, int npair, int ng, int ngp, int nkb,
                          unsigned short* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // (row, block, G' in block)
  if (e >= (size_t)npair * nkb * 16) return;
  const int i = (int)(e % 16);
  const size_t rb = e / 16;
  const int kb = (int)(rb % nkb), row = (int)(rb / nkb);
  const int col = kb * 16 + i;
  float re = 0.f, im = 0.f;
  if (col < ng) {
    const float2 x = m[(size_t)row * ngp + col];
    re = x.x;
    im = x.y;
  }
  const unsigned short rh = bf16_rne(re), ih = bf16_rne(im);
  unsigned short* o = out + rb * MSPLIT;
  o[i] = rh;
  o[16 + i] = ih;
  o[32 + i] = bf16_rne(re - bf16_val(rh));
  o[48 + i] = bf16_rne(im - bf16_val(ih));
}

// Both operands are staged straight from their split images into LDS by 16-byte direct loads
// (one wave instruction fills 64 consecutive 16-byte LDS units), two stages ahead, into three
// buffers, so the staging takes no registers and no LDS store pass.  The buffers are separate
// arrays and the stage loop runs whole triples of stages (the remainder after it), so that the
// compiler sees that a stage's LDS reads cannot alias the direct loads in flight into the other
// buffers and does not wait for them; the stage barrier orders LDS only (lds_barrier), so the loads of the next stage stay in
// flight across it, and each stage waits for its own loads explicitly.  LDS units of one stage: the 128 M rows
// of 8 pieces (piece c of row r at unit 8 r + (c ^ (r & 7))), then the 128 chibar rows of 12
// (piece p of row r at UM + 12 r + (p ^ 2 ((r >> 2) & 1))); the XORs give every MFMA fragment
// read of 16 rows x 4 pieces four accesses per bank group, the minimum.  Rows past npair or
// ng load the last valid row: they only feed products that the epilogue drops.
// One workgroup per CU.  Measured with register staging (the former form), per 32k-pair
// launch at NG 2000: 5.4 ms converting chibar in every tile, 4.2 ms with it pre-split;
// capped at 128 registers for a second workgroup it spilled (9.4 ms); stages of 32 G' were
// no faster (5.6 ms).
constexpr int UM = BT * 8, UG = BT * 12, UST = UM + UG;   // 16-byte LDS units per stage
constexpr int UPL = UST / 512;                            // units per lane per stage
static_assert(UPL * 512 == UST && UM % 64 == 0, "stage units must split into whole wave instructions");
__global__ __launch_bounds__(512) void k_adjoint_bf16x3(const float2* __restrict__ m, int npair, int ng, int ngp,
                                                           const uint4* __restrict__ msplit,
                                                           const uint4* __restrict__ gsplit,
                                                           double2* __restrict__ part) {
  __shared__ __align__(16) uint4 sa[UST];
  __shared__ __align__(16) uint4 sb[UST];
  __shared__ __align__(16) uint4 sc[UST];
  __shared__ double2 sred[4][BT];
  const int ntg = ngp / BT;
  const int npt = (npair + BT - 1) / BT;
  const int ntile = npt * ntg;
  const int t = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
  if (t >= ntile) return;
  int pt, tg;
  adj_tile(t, npt, ntg, &pt, &tg);
  const int p0 = pt * BT;
  const int q0 = tg * BT;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave / 4, wc = wave % 4;
  const int li = lane & 15, lg = lane >> 4;
  const int nkb = (ng + BKS - 1) / BKS;

  // this lane's source of unit 64 (8 i + wave) + lane, for every stage (block kb adds
  // 8 kb or 12 kb pieces; the block of 64 units, and so the operand, is wave-uniform)
  const uint4* src[UPL];
#pragma unroll
  for (int i = 0; i < UPL; ++i) {
    const int ub = 8 * i + wave;
    const int u = 64 * ub + lane;
    if (ub * 64 < UM) {
      const int r = u / 8, c = (u % 8) ^ (r & 7);
      src[i] = msplit + (size_t)min(p0 + r, npair - 1) * nkb * 8 + c;
    } else {
      const int u2 = u - UM, r = u2 / 12, pc = (u2 % 12) ^ (2 * ((r >> 2) & 1));
      src[i] = gsplit + (size_t)min(q0 + r, ng - 1) * nkb * 12 + pc;
    }
  }
  auto issue = [&](int kb, uint4* buf) {
#pragma unroll
    for (int i = 0; i < UPL; ++i) {
      const int ub = 8 * i + wave;
      const int step = ub * 64 < UM ? 8 : 12;
      __builtin_amdgcn_global_load_lds((const void*)(src[i] + (size_t)kb * step),
                                       (__attribute__((address_space(3))) void*)&buf[64 * ub], 16, 0, 0);
    }
  };

  f32x4 cre[BMI][BNJ], cim[BMI][BNJ];
#pragma unroll
  for (int i = 0; i < BMI; ++i)
#pragma unroll
    for (int j = 0; j < BNJ; ++j) {
      cre[i][j] = f32x4{0, 0, 0, 0};
      cim[i][j] = f32x4{0, 0, 0, 0};
    }
  // chibar pieces of the two products: Re takes [br | -bi] (0, 1, 4, 5), Im [bi | br] (2, 3, 0, 1)
  const int pre = lg < 2 ? lg : 2 + lg;
  const int pim = lg < 2 ? 2 + lg : lg - 2;
  auto stage = [&](int kb, const uint4* cur, uint4* next) {
    // this wave's direct loads of stage kb have landed (only stage kb + 1's, issued after them,
    // may still be in flight); the barrier makes everyone's visible and ends every wave's reads
    // of the buffer that the next issue overwrites (stage kb - 1's).  Every stage issues (past
    // the end: the last stage again, into a buffer not read), so the wait count is a constant.
    wait_vm<UPL>();
    lds_barrier();
    issue(min(kb + 2, nkb - 1), next);
    const uint4* sm = cur;
    const uint4* sg = cur + UM;
    bf16x8 xh[BMI], xl[BMI], reh[BNJ], rel[BNJ], imh[BNJ], iml[BNJ];
#pragma unroll
    for (int i = 0; i < BMI; ++i) {
      const int r = 16 * BMI * wr + 16 * i + li;
      xh[i] = __builtin_bit_cast(bf16x8, sm[8 * r + (lg ^ (r & 7))]);
      xl[i] = __builtin_bit_cast(bf16x8, sm[8 * r + ((4 + lg) ^ (r & 7))]);
    }
#pragma unroll
    for (int j = 0; j < BNJ; ++j) {
      const int r = 16 * BNJ * wc + 16 * j + li;
      const int sw = 2 * ((r >> 2) & 1);
      reh[j] = __builtin_bit_cast(bf16x8, sg[12 * r + (pre ^ sw)]);
      rel[j] = __builtin_bit_cast(bf16x8, sg[12 * r + ((6 + pre) ^ sw)]);
      imh[j] = __builtin_bit_cast(bf16x8, sg[12 * r + (pim ^ sw)]);
      iml[j] = __builtin_bit_cast(bf16x8, sg[12 * r + ((6 + pim) ^ sw)]);
    }
#pragma unroll
    for (int i = 0; i < BMI; ++i)
#pragma unroll
      for (int j = 0; j < BNJ; ++j) {
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], reh[j], cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], rel[j], cre[i][j], 0, 0, 0);
        cre[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], reh[j], cre[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], imh[j], cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[i], iml[j], cim[i][j], 0, 0, 0);
        cim[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[i], imh[j], cim[i][j], 0, 0, 0);
      }
  };
  issue(0, sa);
  issue(min(1, nkb - 1), sb);
  // Whole triples in the loop and the remainder after it: with the second and third stages
  // conditional, the compiler's wait tracking would merge paths on which another buffer's loads
  // are the newest and wait for every load before the LDS reads.
  int kb = 0;
  for (; kb + 3 <= nkb; kb += 3) {
    stage(kb, sa, sc);
    stage(kb + 1, sb, sa);
    stage(kb + 2, sc, sb);
  }
  if (kb < nkb) stage(kb, sa, sc);
  if (kb + 1 < nkb) stage(kb + 1, sb, sa);
  wait_vm<0>();   // no direct load may still be writing LDS when the epilogue's barrier passes
  // epilogue: per pair row, sum over this tile's G of conj(M[p][G]) Y[p][G]; result rows of
  // the bf16 16x16x32 MFMA are 4 (lane / 16) + r, columns lane % 16
  // (one block row i at a time, to keep few registers live beside the accumulators)
#pragma unroll
  for (int i = 0; i < BMI; ++i) {
    double2 rs[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rs[r] = double2{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < BNJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = 16 * BMI * wr + 16 * i + 4 * lg + r;
        const int gc = q0 + 16 * BNJ * wc + 16 * j + li;
        if (p0 + pr < npair && gc < ng) {
          const float2 mv = m[(size_t)(p0 + pr) * ngp + gc];
          const double yr = (double)cre[i][j][r], yi = (double)cim[i][j][r];
          rs[r].x += (double)mv.x * yr + (double)mv.y * yi;
          rs[r].y += (double)mv.x * yi - (double)mv.y * yr;
        }
      }
    // sum over the 16 lanes li of a row (xor shuffles within the 16-lane group)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) {
        rs[r].x += __shfl_xor(rs[r].x, o, 64);
        rs[r].y += __shfl_xor(rs[r].y, o, 64);
      }
    if (li == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) sred[wc][16 * BMI * wr + 16 * i + 4 * lg + r] = rs[r];
    }
  }
  __syncthreads();
  if (tid < BT && p0 + tid < npair) {
    double2 a = sred[0][tid];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
      a.x += sred[c][tid].x;
      a.y += sred[c][tid].y;
    }
    part[(size_t)(p0 + tid) * ntg + tg] = a;
  }
}

// Per pair: s = sum over G tiles (fixed order), then dL/dx and dL/dn accumulated over w.
__global__ void k_adjoint_pairs(const double2* __restrict__ part, int ntg, const double* __restrict__ e_v, int nv,
                                int nvs, const double* __restrict__ e_col, const double* __restrict__ n_col, int c0,
                                int ncol, int cc, double omega, double delta, double* __restrict__ dx,
                                double* __restrict__ dn) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nvs * cc) return;
  const int v = p / cc, c = c0 + p % cc;
  double2 s{0.0, 0.0};
  for (int t = 0; t < ntg; ++t) {
    const double2 x = part[(size_t)p * ntg + t];
    s.x += x.x;
    s.y += x.y;
  }
  if (v >= nv || c >= ncol) return;
  const double n = n_col ? n_col[c] : 1.0;
  const double x = e_v[v] - e_col[c];
  const double a = x - omega, b = x + omega;
  const double da = a * a + delta * delta, db = b * b + delta * delta;
  // 1/(a + i d) = (a - i d)/da;  (a + i d)^-2 = (a^2 - d^2 - 2 i a d)/da^2
  const double2 ia{a / da, -delta / da}, ib{b / db, -delta / db};
  const double2 ia2{(a * a - delta * delta) / (da * da), -2.0 * a * delta / (da * da)};
  const double2 ib2{(b * b - delta * delta) / (db * db), -2.0 * b * delta / (db * db)};
  const double2 dwdx{-0.5 * n * (ia2.x + ib2.x), -0.5 * n * (ia2.y + ib2.y)};
  const double2 dwdn{0.5 * (ia.x + ib.x), 0.5 * (ia.y + ib.y)};
  // Re(conj(s) z) = s.x z.x + s.y z.y
  dx[p] += s.x * dwdx.x + s.y * dwdx.y;
  dn[p] += s.x * dwdn.x + s.y * dwdn.y;
}

// Deterministic reductions of one chunk: each valence band adds the sum over the chunk's
// columns; each column (present in exactly one chunk) gets the sum over valence bands.
__global__ void k_adjoint_reduce(const double* __restrict__ dx, const double* __restrict__ dn, int nv, int cc,
                                 int c0, int ncol, double* __restrict__ g_ev, double* __restrict__ g_ec,
                                 double* __restrict__ g_n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nv && g_ev) {
    double acc = 0.0;
    for (int c = 0; c < cc && c0 + c < ncol; ++c) acc += dx[(size_t)t * cc + c];
    g_ev[t] += acc;
  }
  if (t < cc && c0 + t < ncol) {
    double ax = 0.0, an = 0.0;
    for (int v = 0; v < nv; ++v) {
      ax += dx[(size_t)v * cc + t];
      an += dn[(size_t)v * cc + t];
    }
    if (g_ec) g_ec[c0 + t] = -ax;
    if (g_n) g_n[c0 + t] = an;
  }
}

__global__ void k_fill_f64(double* __restrict__ p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  k_fill_f64<<<nb, 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

size_t adjoint_partial_bytes(int npair, int ngp) { return (size_t)npair * (ngp / AT) * sizeof(double2); }

int adjoint_tile(int mode) { return mode == 2 ? BT : AT; }

size_t gbar_split_bytes(int ng) { return (size_t)ng * ((ng + BKS - 1) / BKS) * GSPLIT * sizeof(unsigned short); }

size_t m_split_bytes(int npair, int ng) {
  return (size_t)npair * ((ng + BKS - 1) / BKS) * MSPLIT * sizeof(unsigned short);
}

hipError_t launch_split_m(const void* m, int npair, int ng, int ngp, void* msplit, hipStream_t st) {
  const int nkb = (ng + BKS - 1) / BKS;
  const size_t ne = (size_t)npair * nkb * 16;
  k_split_m<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>((const float2*)m, npair, ng, ngp, nkb,
                                                         (unsigned short*)msplit);
  return hipGetLastError();
}

hipError_t launch_adjoint_bf16x3(const void* m, const void* msplit, int npair, int ng, int ngp, const double2* gbar,
                                 void* gsplit, double2* part, hipStream_t st) {
  if (ngp % BT != 0) return hipErrorInvalidValue;
  const int nkb = (ng + BKS - 1) / BKS;
  const size_t ne = (size_t)ng * nkb * 16;
  k_split_gbar<<<(unsigned)((ne + 255) / 256), 256, 0, st>>>(gbar, ng, nkb, (unsigned short*)gsplit);
  const int ntg = ngp / BT;
  const int nb = ((npair + BT - 1) / BT) * ntg;
  k_adjoint_bf16x3<<<(nb + 7) / 8 * 8, 512, 0, st>>>((const float2*)m, npair, ng, ngp, (const uint4*)msplit, (const uint4*)gsplit,
                                       part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint(const void* m, int npair, int ng, int ngp, const double2* gbar, double2* part,
                          hipStream_t st) {
  const int ntg = ngp / AT;
  const int nb = ((npair + AT - 1) / AT) * ntg;
  k_adjoint<T><<<(nb + 7) / 8 * 8, 256, 0, st>>>((const cx<T>*)m, npair, ng, ngp, gbar, part);
  return hipGetLastError();
}
template hipError_t launch_adjoint<double>(const void*, int, int, int, const double2*, double2*, hipStream_t);
template hipError_t launch_adjoint<float>(const void*, int, int, int, const double2*, double2*, hipStream_t);

hipError_t launch_adjoint_pairs(const double2* part, int ntg, const double* e_v, int nv, int nvs, const double* e_col,
                                const double* n_col, int c0, int ncol, int cc, double omega, double delta, double* dx,
                                double* dn, hipStream_t st) {
  const int np = nvs * cc;
  k_adjoint_pairs<<<(np + 255) / 256, 256, 0, st>>>(part, ntg, e_v, nv, nvs, e_col, n_col, c0, ncol, cc, omega, delta,
                                                     dx, dn);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const double* dx, const double* dn, int nv, int cc, int c0, int ncol, double* g_ev,
                                 double* g_ec, double* g_n, hipStream_t st) {
  const int n = nv > cc ? nv : cc;
  k_adjoint_reduce<<<(n + 255) / 256, 256, 0, st>>>(dx, dn, nv, cc, c0, ncol, g_ev, g_ec, g_n);
  return hipGetLastError();
}

}  // namespace gw
