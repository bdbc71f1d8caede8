// Pair transform: the matrix element of Eq. (chi0),
//   M_vc(G) = (1/N) sum_r conj(u_v(r)) u_c(r) exp(iG.r),   G in the dielectric sphere,
// formed as the product of two real-space bands followed by a forward transform
// that only produces the K = 2 rchi + 1 frequencies per axis the sphere needs.
//
// k_pair_planes (one x1 plane, 4 x 8 pairs per workgroup):
//   stage 1, per lane one (pair, x2 row): the product along x3 and a pruned x3
//     transform, x3 = b + S a:  X[n] = sum_b e^{2 pi i n b/N} DFT_R(x[b + S a])[n mod R],
//     n in [-rchi, rchi] -> Z[pair][row][n3] in LDS.  The conduction and valence rows
//     arrive one radix-R chunk (one b) at a time through a double buffer in LDS, the
//     next chunk in flight while the current one is used;
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

// LDS of one workgroup: double buffers with the radix-R chunk (one b of the x3 split) of
// the 64 conduction rows and the 32 valence rows in flight, and Z of the current x2 group.
template <typename T, int R, int K>
struct PlaneLds {
  static constexpr int rp = R + 1;   // padded chunk row: the 8 rows read together fall on distinct banks
  static constexpr size_t chunk = (size_t)kTC * kRows * rp;
  static constexpr size_t vchunk = (size_t)kTV * kRows * rp;
  static constexpr size_t bytes = (2 * chunk + 2 * vchunk + (size_t)kTV * kTC * kRows * K) * sizeof(cx<T>);
};

// Two resident workgroups per CU when the per-lane state (Q of IPL items, the stage-1
// accumulators and one radix-R chunk) fits half the register file; one otherwise.
template <typename T, int R, int K>
constexpr int planes_min_blocks() {
  constexpr int ipl = (kTV * kTC * K + 255) / 256;
  constexpr int words = (ipl * K + K + R) * (int)(2 * sizeof(T) / 4);
  return words + 24 <= 256 ? 2 : 1;
}

template <typename T, int ND, int R, int K, int MINB>
__global__ __launch_bounds__(256, MINB) void k_pair_planes(const cx<T>* __restrict__ psi_v,
                                                        const cx<T>* __restrict__ psi_c, int nvs, int ncs,
                                                        const cx<T>* __restrict__ twk, cx<T>* __restrict__ q) {
  using V = cx<T>;
  using L = PlaneLds<T, R, K>;
  constexpr int S = ND / R;
  constexpr int S2 = ND / kRows;
  constexpr int NSTEP = S2 * S;
  constexpr int RCH = (K - 1) / 2;
  constexpr int NPAIR = kTV * kTC;
  constexpr int NITEM = NPAIR * K;
  constexpr int IPL = (NITEM + 255) / 256;
  constexpr int CH = kTC * kRows * R;          // conduction chunk elements
  constexpr int CV = kTV * kRows * R;          // valence chunk elements
  constexpr int PER = (CH + CV) / 256;         // chunk elements per thread
  constexpr size_t NPL = (size_t)ND * ND;
  __shared__ V s_c[2 * L::chunk];
  __shared__ V s_v[2 * L::vchunk];
  __shared__ V s_z[NPAIR * kRows * K];

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

  // chunk staging: element e of step s (x2 group s / S, x3 group b = s % S); conduction
  // rows first, then valence rows.  Whether element i is a conduction or a valence one
  // changes only at multiples of 64 (wave-uniform), so a step's source is a wave-uniform
  // base plus this lane's fixed byte offset, and its LDS slot is fixed.
  static_assert(CH % 64 == 0, "element kinds change at wave boundaries");
  const int wave = __builtin_amdgcn_readfirstlane(wv);
  const V* pc_base = psi_c + ((size_t)c0 * ND + x1) * NPL;
  const V* pv_base = psi_v + ((size_t)v0 * ND + x1) * NPL;
  unsigned voff[PER];   // bytes from the row set's base at g2 = 0, b = 0
  int slot[PER];        // element of s_c / s_v in buffer 0
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + 256 * i;
    const int e2 = e < CH ? e : e - CH;
    const int row = e2 / R, a = e2 % R;
    voff[i] = (unsigned)(((size_t)(row / kRows) * ND * NPL + (size_t)(row % kRows) * ND + a) * sizeof(V));
    slot[i] = row * L::rp + a;
  }
  V pf[PER];
  auto fetch = [&](int st) {
    const int g2 = st / S, b = st % S;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const bool isc = wave * 64 + 256 * i < CH;
      const char* sb = (const char*)(isc ? pc_base : pv_base) + ((size_t)g2 * kRows * ND + (size_t)b * R) * sizeof(V);
      pf[i] = *(const V*)(sb + voff[i]);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (wave * 64 + 256 * i < CH)
        s_c[buf * L::chunk + slot[i]] = pf[i];
      else
        s_v[buf * L::vchunk + slot[i]] = pf[i];
    }
  };

  V qacc[IPL][K];
#pragma unroll
  for (int r = 0; r < IPL; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) qacc[r][j] = V{T(0), T(0)};

  fetch(0);
  stash(0);
  __syncthreads();

  for (int b2 = 0; b2 < S2; ++b2) {
    // ---------------- stage 1: one (pair, x2 row) line per lane
    V acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      const int st = b2 * S + b;
      if (st + 1 < NSTEP) fetch(st + 1);
      const V* rc = s_c + (st & 1) * L::chunk + (cl * kRows + a2) * L::rp;
      const V* rv = s_v + (st & 1) * L::vchunk + (wv * kRows + a2) * L::rp;
      V x[R];
#pragma unroll
      for (int a = 0; a < R; ++a) x[a] = cmulc(rv[a], rc[a]);
      dft<R>(x);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int n = j - RCH;
        const V t = twk[b * K + j];
        cmac(acc[j], t, x[((n % R) + R) % R]);
      }
      if (st + 1 < NSTEP) stash((st + 1) & 1);
      __syncthreads();
    }
    V* z = s_z + ((wv * kTC + cl) * kRows + a2) * K;
#pragma unroll
    for (int j = 0; j < K; ++j) z[j] = acc[j];
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
          const V t = twk[b2 * K + j];
          cmac(qacc[r][j], t, y[((n % kRows) + kRows) % kRows]);
        }
      }
    }
    // s_z is rewritten only after the S barriers of the next group's stage 1
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

// Split-line variant, TV valence bands x 8 conduction columns per workgroup, 128 TV
// threads: waves [0, TV) and [TV, 2 TV) take the first and second half of each line's
// x3 chunks (b < SL and b >= SL), so every lane carries half the stage-1 work and at most
// one stage-2 item; the two partial Z halves are added in LDS.  It halves the per-lane
// register state of the 256-thread kernel (no spills in float64); TV = 2 also halves the
// LDS, so that two workgroups share a CU.
//
// From K = 17 on a workgroup has more stage-2 items (8 TV K) than threads (128 TV); the
// lean form (LEAN) keeps one item per lane in registers and the accumulators of the
// remaining items in LDS, and stages the chunks through one LDS buffer instead of two
// (one more barrier per step), so that registers and LDS both fit two workgroups per CU.
template <typename T, int R, int K, int TV, bool LEAN = false>
struct SplitLds {
  static constexpr int rp = R + 1;
  static constexpr int nbuf = LEAN ? 1 : 2;
  static constexpr int nitem = TV * kTC * K;
  static constexpr int nover = LEAN && nitem > 128 * TV ? nitem - 128 * TV : 0;   // items kept in LDS
  static constexpr size_t chunk = (size_t)kTC * kRows * rp;   // one radix-R chunk of the 64 conduction rows
  static constexpr size_t vchunk = (size_t)TV * kRows * rp;   // and of the 8 TV valence rows
  static constexpr size_t bytes =
      (nbuf * 2 * (chunk + vchunk) + (size_t)TV * kTC * kRows * K + (size_t)nover * K) * sizeof(cx<T>);
};

template <typename T, int R, int K, int TV = kTV>
constexpr bool split_fits() {
  return SplitLds<T, R, K, TV>::bytes <= 160 * 1024;
}

// The lean form is built where it has items beyond one per lane (at most one more per
// lane) and two workgroups share the LDS.
template <typename T, int R, int K>
constexpr bool lean_fits() {
  using L = SplitLds<T, R, K, 2, true>;
  return L::nover > 0 && L::nover <= 256 && 2 * L::bytes <= 160 * 1024;
}

// Direct-load form of the split-line kernel.  The chunk rows go from global memory straight
// into LDS by 16-byte direct loads (global_load_lds_dwordx4, one wave instruction per block of
// 8 rows of one kind and half), NBUF - 1 steps ahead of their use, into NBUF separate LDS
// arrays (separate objects, so that the compiler does not wait for the loads in flight into
// one buffer before reading another).  No registers hold the staged chunks and no LDS stores
// are issued for them.  A chunk row is R x sizeof(V) = 128 bytes, eight 16-byte units; a
// block keeps them unit-major (unit u of row r in slot 8 u + r), so that the 8 lanes that
// read unit u of the block's 8 rows read 128 contiguous bytes, and the second block of each
// pair starts 1152 bytes after the first, so that the two blocks read by one 16-lane group
// fall on different banks.
template <typename T, int R, int K, int TV, int NBUF>
struct DlLds {
  static constexpr int UR = R * (int)sizeof(cx<T>) / 16;   // 16-byte units per chunk row
  static constexpr int nblk = 2 * (kTC + TV);               // 8-row blocks of one step
  static constexpr int units = nblk / 2 * 136;              // block pairs of 64 + 64 + 8 units
  static constexpr size_t bytes = NBUF * (size_t)units * 16 + (size_t)TV * kTC * kRows * K * sizeof(cx<T>) +
                                  (size_t)32 * K * sizeof(cx<T>);   // twiddles of up to 32 chunk rows
};

template <typename T, int R, int K, int TV, int NBUF>
constexpr bool dl_fits() {
  using L = DlLds<T, R, K, TV, NBUF>;
  return L::UR == 8 && L::nblk % (2 * TV) == 0 && L::bytes <= 160 * 1024;
}

// buffers of the four-valence direct-load form: as many as fit (three or four), none if
// fewer than three fit
template <typename T, int R, int K>
constexpr int dl4_nbuf() {
  return dl_fits<T, R, K, 4, 4>() ? 4 : dl_fits<T, R, K, 4, 3>() ? 3 : 0;
}

// first unit of block qb of a step buffer
__device__ __forceinline__ int dl_block(int qb) { return (qb >> 1) * 136 + (qb & 1) * 72; }

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Threads of a finish workgroup: the K^2 lines of the pair in one pass (measured in float32 at
// 128^3 K 25: 640 threads 4.90 ms per 32k pairs, 512: 5.51, 320: 5.57, 256 (three passes, the
// last 44% full): 5.89, 128: 7.9; at 72^3 K 15, 256 threads (one pass) and 640 take the same
// time).  In float64 above 512 lines, two passes: one pass would hold three waves per SIMD to
// 168 registers and spill.
template <typename T, int K>
constexpr int kFinishThreads =
    sizeof(T) == 8 && K * K > 512 ? ((K * K + 1) / 2 + 63) / 64 * 64 : (K * K + 63) / 64 * 64;


// Automatic form (measured per 32k-pair launch on one MI355X).  float64: the lean
// two-valence kernel where it is built (72^3 K 17: 19.9 against 34.3 ms for the plain
// two-valence form; K 19: 21.2 against 36.5 ms), else the two-valence split-line kernel
// wherever it fits (72^3 K 15: 17.7 against 31.5 ms; 96^3 K 19: 68 against 101 ms; 128^3
// K 25: 176 against 402 ms), since it halves the per-lane state that otherwise costs the
// 256-thread kernel its second resident workgroup or spills.  float32: on radix-8 grids
// the lean kernel where it is built (72^3 K 17: 10.7 against 12.9 ms for the 256-thread
// one; K 19: 12.1 against 13.6 ms), else the 256-thread kernel up to K = 21 (72^3 K 15:
// 8.7 ms; 96^3 K 17: 21.7 against 23.7 for the direct-load form and 26.4 for the lean one;
// K 19: 23.0 against 24.8, both with two workgroups per CU, 42.4 with one), and from K = 23 on
// the four-valence direct-load kernel where its rows are 128 bytes (128^3 K 23: 59.5 against
// 70.7 for the four-valence split-line kernel and 74.4 for the 256-thread one; K 25: 62.0
// against 74.7 and 123), else the four-valence split-line kernel.
template <typename T, int R, int K>
constexpr int auto_variant() {
  if constexpr (std::is_same<T, double>::value) {
    if constexpr (lean_fits<T, R, K>()) return 5;
    if constexpr (split_fits<T, R, K, 2>()) return 4;
  } else {
    if constexpr (R <= 8 && lean_fits<T, R, K>()) return 5;
    if constexpr (K >= 23 && dl4_nbuf<T, R, K>() > 0) return 6;
    if constexpr (K >= 23 && split_fits<T, R, K, 4>()) return 3;
  }
  return planes_min_blocks<T, R, K>();
}

// Two register sets for the staged rows (PF2, loads two steps ahead of their use) where that
// was measured faster per 32k-pair launch: the 128^3 grid (float64 two-valence K 25: 78.6
// against 88.1 ms per 16k pairs; float32 four-valence K 25: 62.1 against 74.0 ms).  On 72^3 it
// gains nothing (float64 K 15: 17.3 against 17.4 ms) or loses (float32 four-valence K 15: 12.6
// against 9.0 ms), and on 96^3 float64 it spills (91 against 68 ms).
template <int ND>
constexpr bool kSplitPf2 = ND == 128;

template <typename T, int ND, int R, int K, int TV, bool LEAN = false, bool PF2 = false>
__global__ __launch_bounds__(128 * TV, LEAN ? 2 : 1) void k_pair_planes_split(const cx<T>* __restrict__ psi_v,
                                                                         const cx<T>* __restrict__ psi_c, int nvs,
                                                                         int ncs, const cx<T>* __restrict__ twk,
                                                                         cx<T>* __restrict__ q) {
  using V = cx<T>;
  using L = SplitLds<T, R, K, TV, LEAN>;
  constexpr int NT = 128 * TV;           // threads
  constexpr int S = ND / R;
  constexpr int SL = (S + 1) / 2;        // chunks of the first half
  constexpr int SH = S - SL;             // chunks of the second half
  constexpr int S2 = ND / kRows;
  constexpr int NSTEP = S2 * SL;
  constexpr int RCH = (K - 1) / 2;
  constexpr int NPAIR = TV * kTC;
  constexpr int NITEM = NPAIR * K;
  constexpr int NOV = L::nover;          // items whose accumulators live in LDS (lanes 0..NOV-1)
  constexpr int IPL = LEAN ? 1 : (NITEM + NT - 1) / NT;   // items in registers per lane
  static_assert(!LEAN || (NOV > 0 && NOV <= NT), "lean form: at most one item per lane beyond the first");
  constexpr int CH = kTC * kRows * R;    // conduction elements of one chunk
  constexpr int CV = TV * kRows * R;     // valence elements of one chunk
  constexpr int PER = 2 * (CH + CV) / NT;
  static_assert(PER * NT == 2 * (CH + CV), "chunk elements must divide evenly");
  constexpr size_t NPL = (size_t)ND * ND;
  __shared__ V s_c[L::nbuf * 2 * L::chunk];   // [buffer][half][row][rp]
  __shared__ V s_v[L::nbuf * 2 * L::vchunk];
  __shared__ V s_z[NPAIR * kRows * K];
  __shared__ V s_q[NOV > 0 ? NOV * K : 1];    // [item - NT][j]

  const int nbc = ncs / kTC;
  const int nbv = nvs / TV;
  const int pb = blockIdx.x % (nbc * nbv);
  const int x1 = blockIdx.x / (nbc * nbv);
  const int c0 = (pb % nbc) * kTC;
  const int v0 = (pb / nbc) * TV;

  const int tid = threadIdx.x;
  // wave-uniform: the chunk index b and its twiddles then live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wv = wave % TV;           // valence band of this wave
  const int hf = wave / TV;           // half of the x3 chunks
  const int lane = tid & 63;
  const int cl = lane / kRows;
  const int a2 = lane % kRows;

  // element e of a step: half h = e / (CH + CV), then conduction rows, then valence rows.
  // The kind of element i (half, conduction or valence) changes only at multiples of 64,
  // so it is wave-uniform: a step's source is a wave-uniform base plus this lane's fixed
  // byte offset (no per-step index arithmetic), and its LDS slot is fixed too.
  static_assert(CH % 64 == 0 && CV % 64 == 0 && NT % 64 == 0, "element kinds change at wave boundaries");
  const V* pc_base = psi_c + ((size_t)c0 * ND + x1) * NPL;
  const V* pv_base = psi_v + ((size_t)v0 * ND + x1) * NPL;
  unsigned voff[PER];   // bytes from the row set's base at g2 = 0, b = 0
  int slot[PER];        // element of s_c / s_v in buffer 0
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + NT * i;
    const int h = e / (CH + CV), e1 = e % (CH + CV);
    const int e2 = e1 < CH ? e1 : e1 - CH;
    const int row = e2 / R, a = e2 % R;
    voff[i] = (unsigned)(((size_t)(row / kRows) * ND * NPL + (size_t)(row % kRows) * ND + a) * sizeof(V));
    slot[i] = h * (e1 < CH ? (int)L::chunk : (int)L::vchunk) + row * L::rp + a;
  }
  auto fetch = [&](int st, V (&pf)[PER]) {
    const int g2 = st / SL, t = st % SL;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ew = wave * 64 + NT * i;   // the wave's first element
      const int h = ew / (CH + CV);
      const bool isc = ew % (CH + CV) < CH;
      const int b = h ? SL + t : t;
      V x{T(0), T(0)};
      if (b < S) {
        const char* sb = (const char*)(isc ? pc_base : pv_base) + ((size_t)g2 * kRows * ND + (size_t)b * R) * sizeof(V);
        x = *(const V*)(sb + voff[i]);
      }
      pf[i] = x;
    }
  };
  auto stash = [&](int buf, const V (&pf)[PER]) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ew = wave * 64 + NT * i;
      if (ew % (CH + CV) < CH)
        s_c[buf * 2 * L::chunk + slot[i]] = pf[i];
      else
        s_v[buf * 2 * L::vchunk + slot[i]] = pf[i];
    }
  };

  V qacc[IPL][K];
#pragma unroll
  for (int r = 0; r < IPL; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) qacc[r][j] = V{T(0), T(0)};
  if (NOV > 0 && tid < NOV) {
#pragma unroll
    for (int j = 0; j < K; ++j) s_q[tid * K + j] = V{T(0), T(0)};
  }

  // stage 1 of one chunk step: products, R-point DFT and the twiddled sum into acc
  auto step1 = [&](int st, int t, V (&acc)[K]) {
    const int b = hf ? SL + t : t;
    const int buf = LEAN ? 0 : (st & 1);
    if (hf == 0 || t < SH) {
      const V* rc = s_c + (buf * 2 + hf) * L::chunk + (cl * kRows + a2) * L::rp;
      const V* rv = s_v + (buf * 2 + hf) * L::vchunk + (wv * kRows + a2) * L::rp;
      V x[R];
#pragma unroll
      for (int a = 0; a < R; ++a) x[a] = cmulc(rv[a], rc[a]);
      dft<R>(x);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int n = j - RCH;
        const V tv = twk[b * K + j];
        cmac(acc[j], tv, x[((n % R) + R) % R]);
      }
    }
  };
  // end of an x2 group: the two halves' Z added in LDS, then stage 2 of the group
  auto group_end = [&](int b2, const V (&acc)[K]) {
    V* z = s_z + ((wv * kTC + cl) * kRows + a2) * K;
    if (hf == 1) {
#pragma unroll
      for (int j = 0; j < K; ++j) z[j] = acc[j];
    }
    __syncthreads();
    if (hf == 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) z[j] = cadd(z[j], acc[j]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const int it = tid + NT * r;
      if (it < NITEM) {
        const int pair = it / K, j3 = it % K;
        V y[kRows];
#pragma unroll
        for (int a = 0; a < kRows; ++a) y[a] = s_z[(pair * kRows + a) * K + j3];
        dft<kRows>(y);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int n = j - RCH;
          const V tv = twk[b2 * K + j];
          cmac(qacc[r][j], tv, y[((n % kRows) + kRows) % kRows]);
        }
      }
    }
    if (NOV > 0 && tid < NOV) {
      // the items beyond one per lane, accumulated in LDS by the first NOV lanes
      const int it = NT + tid;
      const int pair = it / K, j3 = it % K;
      V y[kRows];
#pragma unroll
      for (int a = 0; a < kRows; ++a) y[a] = s_z[(pair * kRows + a) * K + j3];
      dft<kRows>(y);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int n = j - RCH;
        const V tv = twk[b2 * K + j];
        V acc = s_q[tid * K + j];
        cmac(acc, tv, y[((n % kRows) + kRows) % kRows]);
        s_q[tid * K + j] = acc;
      }
    }
    // s_z is rewritten only after the SL barriers of the next group's stage 1
  };

  if constexpr (LEAN || !PF2) {
    // one register set: the rows of the next step are loaded at the start of a step and
    // stored to LDS at its end (lean form: one LDS buffer, so after a barrier)
    V pf[PER];
    fetch(0, pf);
    stash(0, pf);
    __syncthreads();
    for (int b2 = 0; b2 < S2; ++b2) {
      V acc[K];
#pragma unroll
      for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll 1
      for (int t = 0; t < SL; ++t) {
        const int st = b2 * SL + t;
        if (st + 1 < NSTEP) fetch(st + 1, pf);
        step1(st, t, acc);
        if (LEAN) {
          if (st + 1 < NSTEP) {
            __syncthreads();
            stash(0, pf);
          }
        } else if (st + 1 < NSTEP) {
          stash((st + 1) & 1, pf);
        }
        __syncthreads();
      }
      group_end(b2, acc);
    }
  } else {
    // Two LDS buffers and two register sets: the rows of step s travel in set s mod 2, loaded
    // two steps ahead of their use and stored to LDS one step ahead, so that each load has a
    // whole step to arrive.  Steps are unrolled over one x2 group (and the groups in pairs, so
    // that every set index is a constant); the loads past the last step repeat it, unused.
    V pf[2][PER];
    fetch(0, pf[0]);
    stash(0, pf[0]);
    fetch(min(1, NSTEP - 1), pf[1]);
    __syncthreads();
    auto group = [&](int b2, auto par) {
      constexpr int P = decltype(par)::value;   // parity of the group's first step
      V acc[K];
#pragma unroll
      for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
      // one step whose rows are in set Q
      auto one = [&](int t, auto set) {
        constexpr int Q = decltype(set)::value;
        const int st = b2 * SL + t;
        fetch(min(st + 2, NSTEP - 1), pf[Q]);
        step1(st, t, acc);
        stash((st + 1) & 1, pf[Q ^ 1]);
        __syncthreads();
      };
      // steps in pairs, the loop kept rolled so that no step's loads are hoisted into another
      int t = 0;
#pragma unroll 1
      for (; t + 2 <= SL; t += 2) {
        one(t, std::integral_constant<int, P>{});
        one(t + 1, std::integral_constant<int, P ^ 1>{});
      }
      if constexpr (SL & 1) one(t, std::integral_constant<int, P>{});
      group_end(b2, acc);
    };
    for (int b2 = 0; b2 < S2; b2 += 2) {
      group(b2, std::integral_constant<int, 0>{});
      if (b2 + 1 < S2) group(b2 + 1, std::integral_constant<int, SL & 1>{});
    }
  }
  const int p1 = (x1 % S) * R + x1 / S;
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const int it = tid + NT * r;
    if (it < NITEM) {
      const int pair = it / K, j3 = it % K;
      const int pv = pair / kTC, pc = pair % kTC;
      const size_t pg = (size_t)(v0 + pv) * ncs + (c0 + pc);
      V* dst = q + (pg * ND + p1) * (K * K) + j3;
#pragma unroll
      for (int j = 0; j < K; ++j) dst[j * K] = qacc[r][j];
    }
  }
  if (NOV > 0 && tid < NOV) {
    const int it = NT + tid;
    const int pair = it / K, j3 = it % K;
    const int pv = pair / kTC, pc = pair % kTC;
    const size_t pg = (size_t)(v0 + pv) * ncs + (c0 + pc);
    V* dst = q + (pg * ND + p1) * (K * K) + j3;
#pragma unroll
    for (int j = 0; j < K; ++j) dst[j * K] = s_q[tid * K + j];
  }
}

template <typename T, int ND, int R, int K, int TV, int NBUF>
__global__ __launch_bounds__(128 * TV, 1) void k_pair_planes_dl(const cx<T>* __restrict__ psi_v,
                                                                const cx<T>* __restrict__ psi_c, int nvs, int ncs,
                                                                const cx<T>* __restrict__ twk,
                                                                cx<T>* __restrict__ q) {
  using V = cx<T>;
  using L = DlLds<T, R, K, TV, NBUF>;
  constexpr int NT = 128 * TV;
  constexpr int NW = NT / 64;
  constexpr int S = ND / R;
  constexpr int SL = (S + 1) / 2;
  constexpr int SH = S - SL;
  constexpr int S2 = ND / kRows;
  constexpr int NSTEP = S2 * SL;
  constexpr int RCH = (K - 1) / 2;
  constexpr int NPAIR = TV * kTC;
  constexpr int NITEM = NPAIR * K;
  constexpr int IPL = (NITEM + NT - 1) / NT;
  constexpr int UR = L::UR;
  constexpr int EPU = 16 / (int)sizeof(V);       // elements per unit
  constexpr int IPW = L::nblk / NW;              // load instructions per wave and step
  static_assert(NBUF >= 2 && NBUF <= 4 && IPW * (NBUF - 2) < 64, "load pipeline");
  constexpr size_t NPL = (size_t)ND * ND;
  __shared__ __align__(16) uint4 sb0[L::units];
  __shared__ __align__(16) uint4 sb1[L::units];
  __shared__ __align__(16) uint4 sb2[NBUF > 2 ? L::units : 1];
  __shared__ __align__(16) uint4 sb3[NBUF > 3 ? L::units : 1];
  __shared__ V s_z[NPAIR * kRows * K];
  constexpr int NTW = (S > S2 ? S : S2) * K;
  __shared__ V s_tw[NTW];   // twiddles of both stages, read as LDS broadcasts (scalar loads of
                            // every unrolled step's twiddles would not fit the scalar registers)

  const int nbc = ncs / kTC;
  const int nbv = nvs / TV;
  const int pb = blockIdx.x % (nbc * nbv);
  const int x1 = blockIdx.x / (nbc * nbv);
  const int c0 = (pb % nbc) * kTC;
  const int v0 = (pb / nbc) * TV;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wv = wave % TV;
  const int hf = wave / TV;
  const int lane = tid & 63;
  const int cl = lane / kRows;
  const int a2 = lane % kRows;

  // Load block qb = NW i + wave of a step: conduction blocks h kTC + column, then valence
  // blocks 2 kTC + h TV + band; lane l loads unit l / 8 of x2 row l % 8.
  const char* pc_base = (const char*)(psi_c + ((size_t)c0 * ND + x1) * NPL);
  const char* pv_base = (const char*)(psi_v + ((size_t)v0 * ND + x1) * NPL);
  unsigned loff[IPW];
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    const int qb = NW * i + wave;
    const bool isc = qb < 2 * kTC;
    const int band = isc ? qb % kTC : (qb - 2 * kTC) % TV;
    loff[i] = (unsigned)(((size_t)band * ND * NPL + (size_t)(lane % 8) * ND) * sizeof(V) + 16 * (lane / 8));
  }
  auto issue = [&](int st, uint4* buf) {
    const int g2 = st / SL, t = st % SL;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int qb = NW * i + wave;
      const bool isc = qb < 2 * kTC;
      const int h = isc ? qb / kTC : (qb - 2 * kTC) / TV;
      const int b = min(h ? SL + t : t, S - 1);   // a missing last chunk of the second half: any valid row
      const char* src = (isc ? pc_base : pv_base) + ((size_t)g2 * kRows * ND + (size_t)b * R) * sizeof(V) + loff[i];
      __builtin_amdgcn_global_load_lds((const void*)src,
                                       (__attribute__((address_space(3))) void*)&buf[dl_block(qb)], 16, 0, 0);
    }
  };

  for (int e = tid; e < NTW; e += NT) s_tw[e] = twk[e];   // visible after the first step's barrier
  V qacc[IPL][K];
#pragma unroll
  for (int r = 0; r < IPL; ++r)
#pragma unroll
    for (int j = 0; j < K; ++j) qacc[r][j] = V{T(0), T(0)};
  V acc[K];

  // this lane's rows: conduction (half hf, column cl, x2 row a2), valence (half hf, band wv);
  // unit u is 8 u further
  const int cbase = dl_block(hf * kTC + cl) + a2;
  const int vbase = dl_block(2 * kTC + hf * TV + wv) + a2;

  // Every step issues the loads of step st + NBUF - 1 (past the end: the last step's rows
  // again, into a buffer that is not read), so that exactly (NBUF - 2) IPW loads of this
  // wave are issued after step st's: the wait count is one constant, and the step has no
  // branches (across which the compiler would sink every step's arithmetic into the last).
  auto step = [&](int st, const uint4* cur, uint4* nxt) {
    wait_vm<(NBUF - 2) * IPW>();
    lds_barrier();   // everyone's loads of this step landed; everyone is done with step st - 1
    issue(min(st + NBUF - 1, NSTEP - 1), nxt);
    const int t = st % SL;
    // the second half has one chunk fewer for odd S: that step computes on the clamped rows
    // with zero twiddles
    const bool live = hf == 0 || t < SH;
    const int b = hf ? min(SL + t, S - 1) : t;
    {
      V x[R];
#pragma unroll
      for (int u = 0; u < UR; ++u) {
        const uint4 cu = cur[cbase + 8 * u];
        const uint4 vu = cur[vbase + 8 * u];
        V cv[EPU], vv[EPU];
        __builtin_memcpy(cv, &cu, 16);
        __builtin_memcpy(vv, &vu, 16);
#pragma unroll
        for (int e = 0; e < EPU; ++e) x[u * EPU + e] = cmulc(vv[e], cv[e]);
      }
      dft<R>(x);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int n = j - RCH;
        const V tw = s_tw[b * K + j];
        const V tv = live ? tw : V{T(0), T(0)};
        cmac(acc[j], tv, x[((n % R) + R) % R]);
      }
    }
  };
  // end of x2 group b2: the two halves' Z into LDS, then stage 2
  auto group_end = [&](int b2) {
    V* z = s_z + ((wv * kTC + cl) * kRows + a2) * K;
    if (hf == 1) {
#pragma unroll
      for (int j = 0; j < K; ++j) z[j] = acc[j];
    }
    lds_barrier();
    if (hf == 0) {
#pragma unroll
      for (int j = 0; j < K; ++j) z[j] = cadd(z[j], acc[j]);
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const int it = tid + NT * r;
      if (it < NITEM) {
        const int pair = it / K, j3 = it % K;
        V y[kRows];
#pragma unroll
        for (int a = 0; a < kRows; ++a) y[a] = s_z[(pair * kRows + a) * K + j3];
        dft<kRows>(y);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const int n = j - RCH;
          const V tv = s_tw[b2 * K + j];
          cmac(qacc[r][j], tv, y[((n % kRows) + kRows) % kRows]);
        }
      }
    }
    // s_z is rewritten only after the barriers of the next group's steps
  };

  // groups are unrolled GU at a time, so that every step's buffer is a fixed array
  constexpr int GU = NBUF / gcd_c(SL, NBUF);
  uint4* const bufs[4] = {sb0, sb1, sb2, sb3};
#pragma unroll
  for (int k = 0; k < NBUF - 1; ++k)
    if (k < NSTEP) issue(k, bufs[k]);
  for (int b20 = 0; b20 < S2; b20 += GU) {
#pragma unroll
    for (int gg = 0; gg < GU; ++gg) {
      const int b2 = b20 + gg;
      if (b2 < S2) {
#pragma unroll
        for (int j = 0; j < K; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll
        for (int t = 0; t < SL; ++t) {
          const int k = (gg * SL + t) % NBUF;
          step(b2 * SL + t, bufs[k], bufs[(k + NBUF - 1) % NBUF]);
        }
        group_end(b2);
      }
    }
  }
  wait_vm<0>();   // no direct load may still be writing this workgroup's LDS when it ends

  const int p1 = (x1 % S) * R + x1 / S;
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const int it = tid + NT * r;
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

// Generic form, for grids and dielectric spheres without a compiled instance: the two-valence
// split-line kernel with the grid N = R S and the output count K taken at run time, K <= KMAX.
// The per-lane state is sized for KMAX and indexed by the output frequency n + (KMAX - 1) / 2,
// |n| <= (K - 1) / 2 active, so every register index stays a compile-time constant (only the
// twiddle table and Z are indexed at run time, in memory).  It is slower than the instances
// (unused outputs still hold registers) and serves any grid the band transform splits.
template <typename T, int R, int KMAX>
__global__ __launch_bounds__(256, 1) void k_pair_planes_gen(const cx<T>* __restrict__ psi_v,
                                                            const cx<T>* __restrict__ psi_c, int nvs, int ncs,
                                                            int nd, int K, const cx<T>* __restrict__ twk,
                                                            cx<T>* __restrict__ q) {
  using V = cx<T>;
  constexpr int TV = 2;
  constexpr int NT = 128 * TV;
  using L = SplitLds<T, R, KMAX, TV, false>;
  constexpr int RMAX = (KMAX - 1) / 2;
  constexpr int NPAIR = TV * kTC;
  constexpr int IPL = (NPAIR * KMAX + NT - 1) / NT;
  constexpr int CH = kTC * kRows * R;
  constexpr int CV = TV * kRows * R;
  constexpr int PER = 2 * (CH + CV) / NT;
  static_assert(PER * NT == 2 * (CH + CV), "chunk elements must divide evenly");
  const int S = nd / R;
  const int SL = (S + 1) / 2;
  const int SH = S - SL;
  const int S2 = nd / kRows;
  const int NSTEP = S2 * SL;
  const int RCH = (K - 1) / 2;
  const int NITEM = NPAIR * K;
  const size_t NPL = (size_t)nd * nd;
  __shared__ V s_c[2 * 2 * L::chunk];   // [buffer][half][row][rp]
  __shared__ V s_v[2 * 2 * L::vchunk];
  __shared__ V s_z[NPAIR * kRows * KMAX];

  const int nbc = ncs / kTC;
  const int nbv = nvs / TV;
  const int pb = blockIdx.x % (nbc * nbv);
  const int x1 = blockIdx.x / (nbc * nbv);
  const int c0 = (pb % nbc) * kTC;
  const int v0 = (pb / nbc) * TV;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wv = wave % TV;
  const int hf = wave / TV;
  const int lane = tid & 63;
  const int cl = lane / kRows;
  const int a2 = lane % kRows;

  const V* pc_base = psi_c + ((size_t)c0 * nd + x1) * NPL;
  const V* pv_base = psi_v + ((size_t)v0 * nd + x1) * NPL;
  unsigned voff[PER];
  int slot[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + NT * i;
    const int h = e / (CH + CV), e1 = e % (CH + CV);
    const int e2 = e1 < CH ? e1 : e1 - CH;
    const int row = e2 / R, a = e2 % R;
    voff[i] = (unsigned)(((size_t)(row / kRows) * nd * NPL + (size_t)(row % kRows) * nd + a) * sizeof(V));
    slot[i] = h * (e1 < CH ? (int)L::chunk : (int)L::vchunk) + row * L::rp + a;
  }
  V pf[PER];
  auto fetch = [&](int st) {
    const int g2 = st / SL, t = st % SL;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ew = wave * 64 + NT * i;
      const int h = ew / (CH + CV);
      const bool isc = ew % (CH + CV) < CH;
      const int b = h ? SL + t : t;
      V x{T(0), T(0)};
      if (b < S) {
        const char* sb = (const char*)(isc ? pc_base : pv_base) + ((size_t)g2 * kRows * nd + (size_t)b * R) * sizeof(V);
        x = *(const V*)(sb + voff[i]);
      }
      pf[i] = x;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int ew = wave * 64 + NT * i;
      if (ew % (CH + CV) < CH)
        s_c[buf * 2 * L::chunk + slot[i]] = pf[i];
      else
        s_v[buf * 2 * L::vchunk + slot[i]] = pf[i];
    }
  };

  V qacc[IPL][KMAX];
#pragma unroll
  for (int r = 0; r < IPL; ++r)
#pragma unroll
    for (int j = 0; j < KMAX; ++j) qacc[r][j] = V{T(0), T(0)};

  fetch(0);
  stash(0);
  __syncthreads();

  for (int b2 = 0; b2 < S2; ++b2) {
    V acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll 1
    for (int t = 0; t < SL; ++t) {
      const int st = b2 * SL + t;
      if (st + 1 < NSTEP) fetch(st + 1);
      const int b = hf ? SL + t : t;
      const int buf = st & 1;
      if (hf == 0 || t < SH) {
        const V* rc = s_c + (buf * 2 + hf) * L::chunk + (cl * kRows + a2) * L::rp;
        const V* rv = s_v + (buf * 2 + hf) * L::vchunk + (wv * kRows + a2) * L::rp;
        V x[R];
#pragma unroll
        for (int a = 0; a < R; ++a) x[a] = cmulc(rv[a], rc[a]);
        dft<R>(x);
#pragma unroll
        for (int n = -RMAX; n <= RMAX; ++n)
          if (n >= -RCH && n <= RCH) cmac(acc[n + RMAX], twk[b * K + n + RCH], x[((n % R) + R) % R]);
      }
      if (st + 1 < NSTEP) stash((st + 1) & 1);
      __syncthreads();
    }
    V* z = s_z + ((wv * kTC + cl) * kRows + a2) * K;
    if (hf == 1) {
#pragma unroll
      for (int n = -RMAX; n <= RMAX; ++n)
        if (n >= -RCH && n <= RCH) z[n + RCH] = acc[n + RMAX];
    }
    __syncthreads();
    if (hf == 0) {
#pragma unroll
      for (int n = -RMAX; n <= RMAX; ++n)
        if (n >= -RCH && n <= RCH) z[n + RCH] = cadd(z[n + RCH], acc[n + RMAX]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < IPL; ++r) {
      const int it = tid + NT * r;
      if (it < NITEM) {
        const int pair = it / K, j3 = it % K;
        V y[kRows];
#pragma unroll
        for (int a = 0; a < kRows; ++a) y[a] = s_z[(pair * kRows + a) * K + j3];
        dft<kRows>(y);
#pragma unroll
        for (int n = -RMAX; n <= RMAX; ++n)
          if (n >= -RCH && n <= RCH)
            cmac(qacc[r][n + RMAX], twk[b2 * K + n + RCH], y[((n % kRows) + kRows) % kRows]);
      }
    }
    // s_z is rewritten only after the SL barriers of the next group's stage 1
  }
  const int p1 = (x1 % S) * R + x1 / S;
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const int it = tid + NT * r;
    if (it < NITEM) {
      const int pair = it / K, j3 = it % K;
      const int pv = pair / kTC, pc = pair % kTC;
      const size_t pg = (size_t)(v0 + pv) * ncs + (c0 + pc);
      V* dst = q + (pg * nd + p1) * ((size_t)K * K) + j3;
#pragma unroll
      for (int n = -RMAX; n <= RMAX; ++n)
        if (n >= -RCH && n <= RCH) dst[(size_t)(n + RCH) * K] = qacc[r][n + RMAX];
    }
  }
}

// Generic finish (runtime N and K <= KMAX, outputs indexed by frequency as above).
template <typename T, int R, int KMAX>
__global__ __launch_bounds__(256) void k_pair_finish_gen(const cx<T>* __restrict__ q,
                                                         const int32_t* __restrict__ chi_map, int ng, int ngp,
                                                         int nd, int K, T scale, const cx<T>* __restrict__ twk,
                                                         cx<T>* __restrict__ m) {
  using V = cx<T>;
  constexpr int RMAX = (KMAX - 1) / 2;
  const int S = nd / R;
  const int RCH = (K - 1) / 2;
  const int KK = K * K;
  const size_t pair = blockIdx.x;
  const V* src = q + pair * nd * (size_t)KK;
  V* dst = m + pair * ngp;
  for (int l = threadIdx.x; l < KK; l += blockDim.x) {
    V acc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) acc[j] = V{T(0), T(0)};
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      V x[R];
#pragma unroll
      for (int a = 0; a < R; ++a) x[a] = src[(size_t)(b * R + a) * KK + l];
      dft<R>(x);
#pragma unroll
      for (int n = -RMAX; n <= RMAX; ++n)
        if (n >= -RCH && n <= RCH) cmac(acc[n + RMAX], twk[b * K + n + RCH], x[((n % R) + R) % R]);
    }
#pragma unroll
    for (int n = -RMAX; n <= RMAX; ++n) {
      if (n >= -RCH && n <= RCH) {
        const int ig = chi_map[(n + RCH) * KK + l];
        if (ig >= 0) dst[ig] = V{acc[n + RMAX].x * scale, acc[n + RMAX].y * scale};
      }
    }
  }
  for (int i = ng + threadIdx.x; i < ngp; i += blockDim.x) dst[i] = V{T(0), T(0)};
}

template <typename T, int ND, int R, int K>
__global__ __launch_bounds__((kFinishThreads<T, K>)) void k_pair_finish(const cx<T>* __restrict__ q, const int32_t* __restrict__ chi_map,
                                                     int ng, int ngp, T scale, const cx<T>* __restrict__ twk,
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
    // the R planes of chunk b + 1 are loaded while chunk b is transformed; the loop stays
    // rolled (unrolled, the loads of all S chunks would be hoisted and spill)
    V nx[R];
#pragma unroll
    for (int a = 0; a < R; ++a) nx[a] = src[(size_t)a * (K * K) + l];
#pragma unroll 1
    for (int b = 0; b < S; ++b) {
      V x[R];
#pragma unroll
      for (int a = 0; a < R; ++a) x[a] = nx[a];
      if (b + 1 < S) {
#pragma unroll
        for (int a = 0; a < R; ++a) nx[a] = src[(size_t)((b + 1) * R + a) * (K * K) + l];
      }
      dft<R>(x);
#pragma unroll
      for (int j = 0; j < K; ++j) cmac(acc[j], twk[b * K + j], x[((j - RCH) % R + R) % R]);
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
hipError_t run_planes(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q, int minb,
                      hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_twk64 : (const cx<T>*)g.d_twk32;
  const cx<T>* pv = (const cx<T>*)psi_v;
  const cx<T>* pc = (const cx<T>*)psi_c;
  // variant: 1 / 2 = 256-thread kernel with one / two resident workgroups per CU,
  // 3 / 4 = split-line kernel with 4 / 2 valence bands per workgroup, 5 = lean split-line
  // kernel with 2 valence bands, 6 / 7 = direct-load split-line kernel with 4 valence bands
  // and four (or three) buffers / 2 valence bands and two buffers, 0 = automatic
  int variant = minb;
  if (variant == 0) variant = auto_variant<T, R, K>();
  if constexpr (dl4_nbuf<T, R, K>() > 0) {
    if (variant == 6) {
      const int nblk = ND * (nvs / 4) * (ncs / kTC);
      k_pair_planes_dl<T, ND, R, K, 4, dl4_nbuf<T, R, K>()><<<nblk, 512, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
      return hipGetLastError();
    }
  }
  if constexpr (dl_fits<T, R, K, 2, 2>()) {
    if (variant == 7) {
      const int nblk = ND * (nvs / 2) * (ncs / kTC);
      k_pair_planes_dl<T, ND, R, K, 2, 2><<<nblk, 256, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
      return hipGetLastError();
    }
  }
  if constexpr (lean_fits<T, R, K>()) {
    if (variant == 5) {
      const int nblk = ND * (nvs / 2) * (ncs / kTC);
      k_pair_planes_split<T, ND, R, K, 2, true><<<nblk, 256, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
      return hipGetLastError();
    }
  }
  if constexpr (split_fits<T, R, K, 4>()) {
    if (variant == 3) {
      const int nblk = ND * (nvs / 4) * (ncs / kTC);
      k_pair_planes_split<T, ND, R, K, 4, false, kSplitPf2<ND>><<<nblk, 512, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
      return hipGetLastError();
    }
  }
  if constexpr (split_fits<T, R, K, 2>()) {
    if (variant == 4) {
      const int nblk = ND * (nvs / 2) * (ncs / kTC);
      k_pair_planes_split<T, ND, R, K, 2, false, kSplitPf2<ND>><<<nblk, 256, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
      return hipGetLastError();
    }
  }
  const int nblk = ND * (nvs / kTV) * (ncs / kTC);
  if (variant == 2)
    k_pair_planes<T, ND, R, K, 2><<<nblk, 256, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
  else
    k_pair_planes<T, ND, R, K, 1><<<nblk, 256, 0, st>>>(pv, pc, nvs, ncs, tw, (cx<T>*)q);
  return hipGetLastError();
}

template <typename T, int ND, int R, int K>
hipError_t run_finish(const Geom& g, const void* q, int npair, void* m, hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_twk64 : (const cx<T>*)g.d_twk32;
  const T scale = T(1.0 / ((double)ND * ND * ND));
  k_pair_finish<T, ND, R, K><<<npair, kFinishThreads<T, K>, 0, st>>>((const cx<T>*)q, g.d_chi_map, g.ng, g.ngp, scale, tw,
                                                    (cx<T>*)m);
  return hipGetLastError();
}

// (ND, R, K) instances: the grids and dielectric-sphere widths the kernels are built for.

}  // namespace

bool pair_instance(int nd, int K) {
#define X(nd_, r_, k_) \
  if (nd == nd_ && K == k_) return true;
  GW_PAIR_CASES(X)
#undef X
  return false;
}

bool pair_supported(int nd, int K) {
  LineSplit ls;
  return pair_instance(nd, K) || (K >= 1 && K <= kPairGenKMax && K % 2 == 1 && line_split(nd, &ls));
}

int pair_radix(int nd, int K) {
#define X(nd_, r_, k_) \
  if (nd == nd_ && K == k_) return r_;
  GW_PAIR_CASES(X)
#undef X
  LineSplit ls;
  return line_split(nd, &ls) ? ls.R : 0;
}

namespace {
template <typename T, int R>
hipError_t run_planes_gen(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q,
                          hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_twk64 : (const cx<T>*)g.d_twk32;
  const int nblk = g.nd * (nvs / 2) * (ncs / kTC);
  if (g.K <= 15)
    k_pair_planes_gen<T, R, 15><<<nblk, 256, 0, st>>>((const cx<T>*)psi_v, (const cx<T>*)psi_c, nvs, ncs, g.nd, g.K,
                                                      tw, (cx<T>*)q);
  else
    k_pair_planes_gen<T, R, kPairGenKMax><<<nblk, 256, 0, st>>>((const cx<T>*)psi_v, (const cx<T>*)psi_c, nvs, ncs,
                                                                g.nd, g.K, tw, (cx<T>*)q);
  return hipGetLastError();
}

template <typename T, int R>
hipError_t run_finish_gen(const Geom& g, const void* q, int npair, void* m, hipStream_t st) {
  const cx<T>* tw = std::is_same<T, double>::value ? (const cx<T>*)g.d_twk64 : (const cx<T>*)g.d_twk32;
  const T scale = T(1.0 / ((double)g.nd * g.nd * g.nd));
  if (g.K <= 15)
    k_pair_finish_gen<T, R, 15><<<npair, 256, 0, st>>>((const cx<T>*)q, g.d_chi_map, g.ng, g.ngp, g.nd, g.K, scale,
                                                       tw, (cx<T>*)m);
  else
    k_pair_finish_gen<T, R, kPairGenKMax><<<npair, 256, 0, st>>>((const cx<T>*)q, g.d_chi_map, g.ng, g.ngp, g.nd,
                                                                 g.K, scale, tw, (cx<T>*)m);
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_pair_planes(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q, int minb,
                              hipStream_t st) {
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_planes<T, nd_, r_, k_>(g, psi_v, psi_c, nvs, ncs, q, minb, st);
  GW_PAIR_CASES(X)
#undef X
  // no compiled instance: the generic kernel (the geometry admitted only shapes it serves)
  if (g.K > kPairGenKMax || nvs % 2 != 0) return hipErrorInvalidValue;
  if (g.line.R == 8) return run_planes_gen<T, 8>(g, psi_v, psi_c, nvs, ncs, q, st);
  if (g.line.R == 16) return run_planes_gen<T, 16>(g, psi_v, psi_c, nvs, ncs, q, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pair_finish(const Geom& g, const void* q, int npair, void* m, hipStream_t st) {
#define X(nd_, r_, k_) \
  if (g.nd == nd_ && g.K == k_) return run_finish<T, nd_, r_, k_>(g, q, npair, m, st);
  GW_PAIR_CASES(X)
#undef X
  if (g.K > kPairGenKMax) return hipErrorInvalidValue;
  if (g.line.R == 8) return run_finish_gen<T, 8>(g, q, npair, m, st);
  if (g.line.R == 16) return run_finish_gen<T, 16>(g, q, npair, m, st);
  return hipErrorInvalidValue;
}

template hipError_t launch_pair_planes<double>(const Geom&, const void*, const void*, int, int, void*, int,
                                               hipStream_t);
template hipError_t launch_pair_planes<float>(const Geom&, const void*, const void*, int, int, void*, int,
                                              hipStream_t);
template hipError_t launch_pair_finish<double>(const Geom&, const void*, int, void*, hipStream_t);
template hipError_t launch_pair_finish<float>(const Geom&, const void*, int, void*, hipStream_t);

}  // namespace gw
