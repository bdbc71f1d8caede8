// Internal declarations of the gwchi0 library (host side of the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gwchi0.h"

namespace gw {
enum Stage { kStageBand = 0, kStagePlanes, kStageFinish, kStageWeights, kStageContract, kStageFinalize,
             kStageEpsInv, kStageBackward, kNumStages };
}

struct gw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // second stream of the forward build: the contraction of a conduction chunk runs there
  // while the pair transforms of the next chunk run on `stream` (events order the two)
  int overlap = 1;   // 0 off, 1 where it pays (split-BF16x3), 2 always
  hipStream_t side = nullptr;
  hipEvent_t ev_ready[2] = {}, ev_free[2] = {}, ev_join = nullptr;
  std::string err;
  int* d_pivot_flag = nullptr;   // set by the inversion kernels on a zero pivot
  int* d_check_flag = nullptr;   // set by the input check of the band-sum entry points
  int* h_check_flag = nullptr;   // pinned host copy of it
  // stage timers: events recorded around launches while timing is on
  bool timing = false;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  double stage_ms[gw::kNumStages] = {};
  long long stage_n[gw::kNumStages] = {};
  // launch shapes chosen by gw_tune, by problem shape: (pair-kernel residency, pair-range splits)
  std::map<std::string, std::pair<int, int>> tune;
  // graph mode: captured launch sequences of gw_chi0_build, by argument signature
  bool graph = false;
  struct GraphEntry {
    std::string key;
    hipGraph_t graph;
    hipGraphExec_t exec;
    std::vector<unsigned long long> geoms;   // ids of the geometries the captured launches read
  };
  std::vector<GraphEntry> graphs;
  // live geometries created on this context (a context destroyed first detaches them)
  std::vector<struct gw_geom*> geoms;
};

namespace gw {
inline gw_status fail(gw_ctx* ctx, gw_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}
}  // namespace gw

#define GW_HIP(ctx, expr)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return gw::fail((ctx), GW_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

namespace gw {
// Records an event pair around the launches in its scope when the context times stages.
struct StageScope {
  gw_ctx* ctx;
  gw_ctx::Mark m{};
  bool on;
  hipStream_t st;
  StageScope(gw_ctx* c, int stage) : StageScope(c, stage, c->stream) {}
  StageScope(gw_ctx* c, int stage, hipStream_t s) : ctx(c), on(c->timing), st(s) {
    if (on) {
      m.stage = stage;
      on = hipEventCreate(&m.a) == hipSuccess && hipEventCreate(&m.b) == hipSuccess &&
           hipEventRecord(m.a, st) == hipSuccess;
    }
  }
  ~StageScope() {
    if (on && hipEventRecord(m.b, st) == hipSuccess) ctx->marks.push_back(m);
  }
};
}  // namespace gw

namespace gw {

// Line decomposition of an N-point transform, x = b + S a  (a in [0,R), b in [0,S)),
// stored permuted at p = b R + a so that the R points of one b are contiguous.
struct LineSplit {
  int R, S;
};
bool line_split(int nd, LineSplit* out);
constexpr int kRows = 8;   // rows of one x2 group in the pair kernel (x2 = b2 + S2 a2, a2 < 8)

struct Geom {
  int nd = 0;          // grid points per axis
  int npw = 0, ng = 0;
  int rw = 0, W = 0;   // wavefunction sphere half-width, W = 2 rw + 1
  int rchi = 0, K = 0; // chi sphere half-width, K = 2 rchi + 1
  int ngp = 0;         // ng rounded up to the contraction tile
  LineSplit line{};    // split of the x3 (and x1) transforms
  int32_t* d_wf_map = nullptr;   // W^3 box -> wavefunction index or -1
  int32_t* d_chi_map = nullptr;  // K^3 box -> chi index or -1
  double2* d_tw64 = nullptr;     // exp(+2 pi i j / nd), j < nd
  float2* d_tw32 = nullptr;
  double2* d_twk64 = nullptr;    // [b][j] = exp(+2 pi i (j - rchi) b / nd), b < nd, j < K
  float2* d_twk32 = nullptr;
  bool has_q = false;            // cell and q given: the dielectric sphere's order was checked
  double q[3] = {0.0, 0.0, 0.0}; // reciprocal-lattice units
  double cell[9] = {};           // lattice vectors as rows (bohr)
};

}  // namespace gw

struct gw_geom {
  gw_ctx* ctx = nullptr;
  unsigned long long id = 0;   // unique per geometry in the process (graph-cache keys)
  gw::Geom g;
};

namespace gw {

// ---------------------------------------------------------------- launches
// Band -> real space: psi[slot][x1][p2][p3] for nslot bands.  Band of slot s:
// idx = band0 + s; if idx >= nvalid it is clamped to nvalid - 1; then
// band = band_idx ? band_idx[idx] : idx.  tB: band_scratch_bytes of scratch.
template <typename T>
hipError_t launch_band_to_real(const Geom& g, const double2* coef, int nrows, const int32_t* band_idx, int band0, int nvalid,
                               int nslot, void* tB, void* psi, hipStream_t st);
size_t band_scratch_bytes(const Geom& g, int nslot, bool fp64);

// Pair planes: Q[pair][p1][j2][j3] for pairs (v, c), v < nvs (multiple of 4), c < ncs (multiple of 8);
// pair = v * ncs + c.
// static COH self-energy (sigma.hip)
int coh_max_states();
hipError_t launch_coh_kernel(const void* eps_inv, const double* v, int ng, int ngp, void* at, hipStream_t st);
hipError_t launch_coh_reduce(const void* m, const void* z, int ns, int cc, int ngp, int nvalid, const double* n_col,
                             int c0, int nblk, void* part, void* s, hipStream_t st);
// plasmon-pole COH self-energy (sigma.hip): (B, wt) tiles, the tile kernel over a chunk of
// pair densities M[n][c][ngp], and the fixed-order sum of the tile partials into out[j][n][n']
int gpp_coh_tile();
int gpp_coh_states_per_block();
int gpp_coh_energies_per_pass();
size_t gpp_coh_part_bytes(int ngp);
hipError_t launch_gpp_coh_prep(const void* modes, const double* v, int ng, int ngp, void* b, void* w, hipStream_t st);
hipError_t launch_gpp_coh(const void* b, const void* w, int ngp, const void* m, int cc, int ns, int sa, int sb,
                          int nvalid, const double* e_col, const double* n_col, int c0, const double* energies, int ne,
                          double delta, void* part, hipStream_t st);
hipError_t launch_gpp_coh_sum(const void* part, int ngp, int ne, int ns, int sa, int sb, int e0, void* out,
                              hipStream_t st);
// plasmon-pole extension (gpp.hip)
hipError_t launch_gpp(const void* eps0, int ng, const double* kvec, const int32_t* gvec, const void* rho, int half,
                      const double* omega, int nomega, double eta, void* modes, void* out, hipStream_t st);
constexpr int kPairVariants = 7;   // forms of the pair kernel a tuned shape may name
// minb: 0 = automatic, 1 or 2 = 256-thread kernel with that many resident workgroups per CU,
// 3 / 4 = split-line kernel with 4 / 2 valence bands per workgroup, 5 = its lean form,
// 6 / 7 = its direct-load form with 4 / 2 valence bands (a form not built for the instance
// falls back to the 256-thread kernel).
template <typename T>
hipError_t launch_pair_planes(const Geom& g, const void* psi_v, const void* psi_c, int nvs, int ncs, void* q,
                              int minb, hipStream_t st);
// Pair finish: x1 transforms, 1/N, gather to the chi sphere: m[pair][ngp] (zero padded).
template <typename T>
hipError_t launch_pair_finish(const Geom& g, const void* q, int npair, void* m, hipStream_t st);
bool pair_instance(int nd, int K);    // a compiled (N, R, K) instance exists
bool pair_supported(int nd, int K);   // an instance, or the generic kernel (K <= kPairGenKMax, N split by line_split)
int pair_radix(int nd, int K);   // line radix R of the (nd, K) instance, else line_split's (0 if none); must equal Geom::line.R
constexpr int kPairGenKMax = 31;   // widest dielectric sphere (outputs per axis) of the generic pair kernel
// (grid N, line radix R, pruned outputs K) of the compiled pair-transform instances
#define GW_PAIR_CASES(X) \
  X(24, 8, 5)            \
  X(24, 8, 7)            \
  X(24, 8, 9)            \
  X(24, 8, 11)           \
  X(48, 8, 15)           \
  X(64, 16, 19)          \
  X(72, 8, 9)            \
  X(72, 8, 11)           \
  X(72, 8, 13)           \
  X(72, 8, 15)           \
  X(72, 8, 17)           \
  X(72, 8, 19)           \
  X(96, 16, 17)          \
  X(96, 16, 19)          \
  X(96, 16, 21)          \
  X(96, 16, 25)          \
  X(128, 16, 23)         \
  X(128, 16, 25)         \
  X(128, 16, 27)


// Weights of Eq. (chi0) per pair p = v * ncs + c (zero for padded pairs):
// part 0 = Re w, part 1 = Im w, w[part][p].
// w[p] = Re w_p; with nparts == 2 also w[np + p] = Im w_p.
hipError_t launch_weights(const double* e_v, int v0, int nv_valid, int nvs, const double* e_col, const double* n_col,
                          int c0, int nc_valid, int ncs, double omega, double delta, int nparts, double* w,
                          hipStream_t st);

// Contraction acc[ks][G][G'] (lower tiles) += sum_k m[k][G] w[k] conj(m[k][G']) (mode 0 f64,
// 1 f32, 2 bf16x3), batched: per problem, nomega * nparts jobs (job j uses w + j nk and
// acc + j ksplit ngp^2), each split into ntl lower tiles x ksplit pair ranges; one
// persistent launch pulls the items from *counter (zeroed beforehand).
struct ContractProb {
  const void* m;
  const double* w;
  double2* acc;
  int nk, ngp, ksplit, ntl;
  const void* aimg = nullptr;   // mode 3: the bf16 row images of M and w M (launch_split_ab)
  const void* bimg = nullptr;
};
constexpr int kMaxBatch = 16;
struct ContractBatch {
  int nprob;
  long long item0[kMaxBatch + 1];
  ContractProb p[kMaxBatch];
};
// alone: no other kernel shares the CUs (no chunk overlap): the split-bf16 form then holds
// two workgroups per CU.
hipError_t launch_contract_batch(int mode, const ContractBatch& bt, int* counter, int grid, bool alone,
                                 hipStream_t st);
// chi[G][G'] = sum_ks accA + i sum_ks accB (Hermitian parts mirrored), for G, G' < ng.
hipError_t launch_finalize(const double2* accA, const double2* accB, int ksplit, int ng, int ngp, double2* chi,
                           bool accumulate, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_copy_m(const void* m, int nvs, int ncs, int ncs_pad, int ng, int ngp, bool fp64, double2* out,
                         hipStream_t st);

constexpr int kTile = 128;  // the dielectric-sphere padding: a multiple of every contraction tile
int contract_tile(int mode);   // G x G' tile of the contraction in this mode (64 or 128)
// static split-bf16 x3: the chunk's M (float, npair x ngp) and w M split into bf16 row images
// per 16-pair block, A [npair/16][ngp][8 units] then B [npair/16][ngp][12 units] (16-byte units),
// which mode 3 of launch_contract_batch stages by direct loads
size_t split_image_bytes(int npair, int ngp);
hipError_t launch_split_ab(const void* m, const double* w, int npair, int ngp, void* img, hipStream_t st);

// ---------------------------------------------------------------- coefficient gradients (float64)
// a = diag(s) m over npair rows of ngp, s_p = w_p or conj(w_p) (w as launch_weights writes it)
hipError_t launch_weight_rows(const void* m, int npair, int ngp, const double* w, int nparts, bool conj_w, void* a,
                              hipStream_t st);
// qbar[pair][p1][K^2] from mbar[pair][ngp]: the transpose of the pair finish stage
hipError_t launch_qbar(const Geom& g, const void* mbar, int npair, void* qbar, hipStream_t st);
// cond: ubar[c][x1][p2][p3] = sum_v h_vc u_v over the nvs valence slots (written);
// else: ubar[v][...] += sum_c conj(h_vc) u_c over the ncs columns (added).  partner: the
// other set's real-space bands (float64, band layout), qbar: pairs v * ncs + c.
hipError_t launch_ubar(const Geom& g, const void* qbar, const void* partner, int nvs, int ncs, bool cond, void* ubar,
                       hipStream_t st);
// cbar[slot][npw] = the transpose of the band transform of ubar[slot] (tB: band scratch)
hipError_t launch_band_from_real(const Geom& g, const void* ubar, int nslot, void* tB, void* cbar, hipStream_t st);
// grad[row(c)] += cbar[c] for c < ncol, row(c) = col_band ? col_band[c0 + c] : c0 + c
hipError_t launch_scatter_cols(const void* cbar, int ncol, const int32_t* col_band, int c0, int npw, int nband,
                               void* grad, hipStream_t st);
hipError_t launch_fill_c128(void* p, size_t n, hipStream_t st);

// ---------------------------------------------------------------- dielectric
constexpr int kNb = 64;     // Gauss-Jordan panel width
hipError_t launch_zgemm(int m, int n, int k, double2 alpha, const double2* A, int lda, bool cta, const double2* B,
                        int ldb, bool ctb, double2 beta, double2* C, int ldc, hipStream_t st);
// the same with op(X) in {X, X^H, X^T, conj X}
enum { kOpN = 0, kOpC = 1, kOpT = 2, kOpConj = 3 };
hipError_t launch_zgemm_op(int m, int n, int k, double2 alpha, const double2* A, int lda, int opa, const double2* B,
                           int ldb, int opb, double2 beta, double2* C, int ldc, hipStream_t st);
size_t eps_inv_workspace(int n);
// allocation-free inverse: a static device scratch array for spheres up to kNoAllocMaxNg
constexpr int kNoAllocMaxNg = 2048;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch_init(int device);   // with the device current; once per device
void* noalloc_scratch(int device);             // its device address there (nullptr before init)
size_t noalloc_scratch_bytes();
hipError_t launch_eps_inv(int n, const double* v, const double2* chi, double2* out, void* ws, int* flag,
                          hipStream_t st);
// static chi0 (Hermitian, negative semidefinite) and v > 0: block sweeps of the positive
// definite I - V^1/2 chi0 V^1/2 (lower triangle of chi read); a pivot block that is not
// positive definite sets *flag.  Workspace: eps_inv_workspace(n) covers it.
hipError_t launch_eps_inv_sweep(int n, const double* v, const double2* chi, double2* out, void* ws, int* flag,
                                hipStream_t st);
size_t eps_inv_backward_workspace(int n);
hipError_t launch_eps_inv_backward(int n, const double* v, const double2* z, const double2* zbar, double2* out,
                                   void* ws, hipStream_t st);
hipError_t launch_flag_clear(int* flag, hipStream_t st);

// ---------------------------------------------------------------- adjoint
size_t adjoint_partial_bytes(int npair, int ngp);   // enough for every tile width
int adjoint_tile(int mode);                          // G per partial sum in this mode (64 or 128)
template <typename T>
hipError_t launch_adjoint(const void* m, int npair, int ng, int ngp, const double2* gbar, double2* part,
                          hipStream_t st);
// split-bf16 x3 form over float pair densities (ngp a multiple of 128): msplit holds the pair
// densities split into bf16 row images (m_split_bytes(npair, ng), written by launch_split_m once
// per chunk), gsplit is scratch of gbar_split_bytes(ng) for chibar split the same way
size_t gbar_split_bytes(int ng);
size_t m_split_bytes(int npair, int ng);
hipError_t launch_split_m(const void* m, int npair, int ng, int ngp, void* msplit, hipStream_t st);
hipError_t launch_adjoint_bf16x3(const void* m, const void* msplit, int npair, int ng, int ngp, const double2* gbar,
                                 void* gsplit, double2* part, hipStream_t st);
// ntg = ngp / adjoint_tile(mode) partial sums per pair
hipError_t launch_adjoint_pairs(const double2* part, int ntg, const double* e_v, int nv, int nvs, const double* e_col,
                                const double* n_col, int c0, int ncol, int cc, double omega, double delta, double* dx,
                                double* dn, hipStream_t st);
hipError_t launch_adjoint_reduce(const double* dx, const double* dn, int nv, int cc, int c0, int ncol, double* g_ev,
                                 double* g_ec, double* g_n, hipStream_t st);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_check_columns(const double* e_v, int nv, const double* e_col, const double* n_col,
                                const int32_t* col_band, int ncol, int nband, int* flag, hipStream_t st);

}  // namespace gw
