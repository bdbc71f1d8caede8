/*
 * gwchi0 -- RPA polarizability band sum on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libgwchi0.so.  It computes the independent-particle
 * polarizability of Gao, Xia, Gao & Zhang, "Towards Fully Converged GW
 * Calculations for Large Systems" (arXiv:1601.06767):
 *
 *   Eq. (chi0):  chi0_GG'(q,w) = 1/2 sum_{c,v} M_vc(G) M*_vc(G')
 *                  [1/(E_v - E_c - w + i delta) + 1/(E_v - E_c + w + i delta)]
 *   with the matrix element M_vc(G) = <v,k+q| exp(i(q+G).r) |c,k>, formed here as
 *   M_vc(G) = (1/N) sum_r conj(u_v(r)) u_c(r) exp(iG.r) on an N-point FFT grid,
 *
 * the grouped form of Eqs. (chi02) and (energyintegration) (each conduction
 * "column" carries an energy and a multiplicity, so an energy window's
 * representative state with weight g(E_i) dE_i is just another column), and the
 * RPA dielectric matrix eps = 1 - v chi0 with its inverse (the relation stated
 * before Eq. (chi0); Table 3 uses [eps^-1]_00).
 *
 * Conventions shared by every entry point
 *  - Energies and frequencies are in Hartree; all inputs are float64 / complex128
 *    (complex = two interleaved doubles, re then im).
 *  - "device" pointers are HIP device memory on the context's device, owned by the
 *    caller; "host" pointers are ordinary host memory, read before the call returns.
 *  - Work is enqueued on the context's stream; calls return after enqueue.  A kernel
 *    fault is reported as GW_EDEVICE by a later call or by the caller's sync.
 *  - Every function returns a gw_status; on failure the context keeps a message,
 *    readable with gw_last_error.  Nothing throws across the ABI.
 *  - One context per stream.  A context is not re-entrant: calls on one context must
 *    not overlap from several host threads.
 */
#ifndef GWCHI0_H
#define GWCHI0_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GW_OK = 0,
  GW_EINVAL = -1,        /* bad argument: shapes, ranges, aliasing, workspace too small */
  GW_ENOMEM = -2,        /* a library-internal allocation failed (set-up calls only; for tests,
                            GW_FAULT=alloc:N in the environment fails the N-th device allocation
                            of each gw_ctx_create / gw_geom_create call) */
  GW_EDEVICE = -3,       /* a HIP runtime call failed */
  GW_ESINGULAR = -4,     /* a pivot of the dielectric matrix was zero or non-finite */
  GW_EUNSUPPORTED = -5   /* a size or mode with no compiled kernel */
} gw_status;

/* Arithmetic of the pair transform and of the contraction.  The band energies,
 * the weights of Eq. (chi0), the final accumulation and eps^-1 are float64 in
 * every mode.
 *   GW_FP64   wavefunctions, pair transforms and contraction in float64.
 *   GW_FP32   wavefunctions and pair transforms in float32; contraction on float32
 *             MFMA, accumulated in float32 within a chunk of band pairs and in
 *             float64 across chunks.
 *   GW_BF16X3 as GW_FP32, but the contraction splits each float32 operand into a
 *             bfloat16 high and low part and sums hi*hi + hi*lo + lo*hi on bf16 MFMA
 *             with float32 accumulation. */
typedef enum { GW_FP64 = 0, GW_FP32 = 1, GW_BF16X3 = 2 } gw_precision;

typedef struct gw_ctx gw_ctx;
typedef struct gw_geom gw_geom;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out is set on success. */
gw_status gw_ctx_create(int device, void* hip_stream, gw_ctx** out);
gw_status gw_ctx_destroy(gw_ctx* ctx);
/* Message of the last failing call on ctx ("" if none).  With ctx == NULL: the
 * message of the last failing gw_ctx_create in this process. */
const char* gw_last_error(const gw_ctx* ctx);
/* Library version string, e.g. "gwchi0 0.1 gfx950". */
const char* gw_version(void);

/* Stage timers (diagnostics, not part of any result).  With enable != 0, later calls
 * record a HIP event pair on the context's stream around each group of launches and
 * accumulate the device time per stage:
 *   0 band -> real-space transforms   1 pair planes (product, x3 and x2 transforms)
 *   2 pair finish (x1 transform, sphere gather)   3 weights   4 contraction
 *   5 finalize (split sum, Hermitian mirror)   6 eps^-1   7 backward
 * gw_ctx_stage_times waits for the recorded events and copies 8 accumulated
 * milliseconds and launch-group counts; reset != 0 clears the accumulators. */
gw_status gw_ctx_set_timing(gw_ctx* ctx, int enable);
gw_status gw_ctx_stage_times(gw_ctx* ctx, double* ms, long long* counts, int reset);

/* Chunk overlap of gw_chi0_build: the contraction of a conduction chunk runs on a second
 * stream of the context while the band and pair transforms of the next chunk run on the
 * context's stream, with events between the two and a join before the call's last
 * launches, so the call stays ordered on the context's stream.
 *   mode 0  off;  1  where it pays (default): the split-BF16x3 mode of a dynamic build
 *   (several frequencies or delta > 0) with dielectric spheres of at most 2048 (padded)
 *   G-vectors, whose register-staged contraction then leaves room on each CU for a
 *   pair-transform workgroup (the static split-BF16x3 contraction fills the CU's LDS and
 *   runs alone);  2  in every mode.
 * The results do not depend on the mode (same arithmetic, same summation order).  With
 * timing on, the contraction's stage time is measured on the second stream and overlaps
 * the others.  GW_EINVAL for another mode. */
gw_status gw_ctx_set_overlap(gw_ctx* ctx, int mode);

/* ---------------------------------------------------------------- geometry */

/* Plane-wave geometry of one q-point (set-up; synchronises the stream).
 *   n_fft[3]   FFT grid N1, N2, N3 (host).  The kernels need N1 = N2 = N3, a multiple
 *              of 8 from 16 to 128; other grids give GW_EUNSUPPORTED.
 *   cell, q    host, or both NULL: the lattice vectors a1, a2, a3 as rows (9 doubles, bohr)
 *              and q in reciprocal-lattice units (3 doubles).  With them the dielectric
 *              sphere is checked to be the first ng G-vectors in the order
 *              (|q+G|^2, n1, n2, n3) -- the cutoff sphere of the dielectric matrix, ordered
 *              as the library's output rows -- with keys equal to a relative 1e-12 counted
 *              as ties and decided by the Miller indices, and with no G missing below the cut
 *              (GW_EINVAL otherwise, naming the entry).  The pair densities themselves do not
 *              use q: the caller supplies the valence states at k+q.  NULL skips the check
 *              (e.g. for the k-point sum's shifted spheres G + G0 of gw_chi0_build_ksum).
 *   npw, gvec_wf   wavefunction sphere: npw x 3 int32 Miller indices (host), the
 *              order in which coefficient rows are stored.
 *   ng, gvec_chi   dielectric sphere: ng x 3 int32 Miller indices (host), the row and
 *              column order of chi0 and eps^-1.
 * Checks: indices distinct modulo the grid, and the alias-free bound
 * 2 max|n_wf,i| + max|n_chi,i| < N_i per axis, which makes the grid evaluation of
 * M_vc(G) equal to the plane-wave convolution sum_G' conj(c_v(G'+G)) c_c(G')
 * (reading of Eq. (chi0)'s matrix element, whose exponent is printed without ".r").
 * Every grid that meets the bound gives the same chi0 up to rounding, so the smallest
 * supported one is the cheapest (the 72^3 workload's spheres, 2 x 18 + 7 = 43, are exact on
 * 48^3).  Tuned pair kernels are compiled for these (grid, K = 2 max|n_chi| + 1): 24^3 with
 * K 5, 7, 9, 11; 48^3 with 15; 64^3 with 19; 72^3 with 9 ... 19 (odd); 96^3 with 17, 19, 21,
 * 25; 128^3 with 23, 25, 27.  Any other grid and K <= 31 runs a generic pair kernel (run-time
 * N and K, slower); K > 31 gives GW_EUNSUPPORTED, and so do the coefficient gradients of
 * gw_chi0_backward on a shape without a compiled kernel.  The geometry keeps
 * its own device copies of the index tables.  Destroying a geometry also drops the graphs
 * that graph mode captured with it (gw_ctx_set_graph); a geometry may outlive its context
 * (it is then only destroyed). */
gw_status gw_geom_create(gw_ctx* ctx, const int n_fft[3], const double* cell, const double* q, int npw,
                         const int32_t* gvec_wf, int ng, const int32_t* gvec_chi, gw_geom** out);
gw_status gw_geom_destroy(gw_geom* geom);

/* The dielectric-sphere check of gw_geom_create on its own (host only, no context or GPU):
 * GW_OK if gvec_chi (ng x 3 int32, host) is the first ng G-vectors in the order
 * (|q+G|^2, n1, n2, n3) for the cell (9 doubles, rows = lattice vectors, bohr) and q
 * (3 doubles, reciprocal-lattice units); else GW_EINVAL with the reason copied into msg
 * (msg_len bytes including the terminating zero; msg may be NULL). */
gw_status gw_sphere_check(const double* cell, const double* q, int ng, const int32_t* gvec_chi, char* msg,
                          size_t msg_len);

/* ---------------------------------------------------------------- chi0 */

/* One q-point's band data (all arrays device memory, read-only).
 *   nv, coef_v, e_v       valence states at k+q: nv x npw complex128 row-major, energies nv.
 *   nband, coef_c         conduction states at k: nband x npw complex128 row-major.
 *   ncol, col_band        the columns summed over: column j uses coefficient row
 *                         col_band[j] (int32, NULL = identity, then ncol <= nband).
 *   e_col, n_col          column energy E_c (a band energy, or a window energy E_i) and
 *                         multiplicity (1 for a band, g(E_i) dE_i for a window);
 *                         n_col NULL = all 1.  Eq. (energyintegration) is then the
 *                         plain column sum.
 * Value checks: the entry points that take problems (gw_chi0_build, gw_chi0_build_ksum,
 * gw_chi0_backward, gw_chi0_backward_ksum, gw_pair_density, gw_sigma_coh_static,
 * gw_sigma_coh_gpp) run one small kernel over the device arrays and read its flag back
 * (a synchronisation of the stream): GW_EINVAL for a non-finite energy (e_v, e_col), a
 * negative or non-finite n_col, or a col_band entry outside [0, nband).  The check is
 * skipped while the context's stream is being captured into a HIP graph (no
 * synchronisation is allowed there) and on replays of graph mode (checked when captured);
 * the kernels then never read or write outside the coefficient rows (column rows are
 * clamped on reads and skipped on writes) and only the result is undefined.  A zero
 * denominator E_v - E_col with omega = delta = 0 gives non-finite output. */
typedef struct {
  const gw_geom* geom;
  int nv;
  const void* coef_v;
  const double* e_v;
  int nband;
  const void* coef_c;
  int ncol;
  const int32_t* col_band;
  const double* e_col;
  const double* n_col;
} gw_chi0_problem;

/* Workspace bytes gw_chi0_build / gw_chi0_backward need for these problems: the largest
 * of the forward and backward layouts, static or dynamic, for any number of frequencies
 * up to nomega.  In GW_FP64 the backward layout includes the coefficient-gradient buffers
 * (two pair-density blocks and the real-space gradients of one conduction chunk). */
gw_status gw_chi0_workspace_size(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega,
                                 gw_precision prec, size_t* bytes);

/* chi0 of Eq. (chi0) for nprob q-points (each with its own geometry and dielectric
 * sphere size) and nomega real frequencies.  Up to 16 q-points run together: after the
 * pair densities of one conduction chunk exist for all of them, a single persistent
 * launch contracts every (q-point, frequency, tile) item, largest spheres first.
 *   omega   host, nomega doubles (read before the call returns).  omega[i] == 0 with
 *           delta == 0 is the static case of Eq. (chi02): a Hermitian, negative
 *           semidefinite matrix.  With delta == 0 every chi0(omega) is Hermitian.
 *   delta   broadening, >= 0 (both terms carry +i delta, as printed).
 *   workspace, ws_bytes   device scratch of at least gw_chi0_workspace_size bytes.
 *   chi0    device output, complex128: for each problem p in order, nomega blocks of
 *           ng_p x ng_p row-major, [p][omega][G][G'].
 * GW_EINVAL: nprob < 1, nomega < 1, delta < 0, nv < 1, ncol < 1, NULL data pointers,
 * ncol > nband without col_band, workspace too small, and the value checks above. */
gw_status gw_chi0_build(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                        double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0);

/* The k-point sum of Eq. (chi0) for one q: chi0 = sum over the nk problems, one per k, all
 * with the same dielectric-sphere size; the output is one set of nomega ng x ng blocks
 * (gw_chi0_build's layout for a single problem), the problems added in order.  Problem k
 * holds the conduction columns and energies at k (coef_c, e_col) and the valence states at
 * k + q = k'' + G0 (gw_kq_map) with their energies E_{v,k''} (coef_v, e_v), in either form
 * (coefficients outside a state's own sphere are zero):
 *   relabelled   the valence row entry at Miller index g holds c_{v,k''}(g + G0), and the
 *                dielectric sphere is G as usual: one geometry, whose wavefunction sphere
 *                contains the spheres of every k and every k'' shifted by -G0, serves all k
 *                and the sphere's width (and so the pair kernel's work) is unchanged;
 *   shifted      the valence rows as stored at k'', and the problem's dielectric sphere entered
 *                as G + G0: <v,k+q| e^{i(q+G).r} |c,k> is the pair density of the two rows at
 *                G + G0 (a geometry per distinct G0, spheres up to one shell wider).
 * Arguments, workspace (gw_chi0_workspace_size over the nk problems), modes and errors as
 * for gw_chi0_build; GW_EINVAL if the sphere sizes differ. */
gw_status gw_chi0_build_ksum(gw_ctx* ctx, const gw_chi0_problem* probs, int nk, int nomega, const double* omega,
                             double delta, gw_precision prec, void* workspace, size_t ws_bytes, void* chi0);

/* Adjoint of gw_chi0_build for a real loss L (same problems, frequencies, precision and
 * workspace size as the forward call).
 *   grad_chi0   device complex128, the layout of gw_chi0_build's output, holding
 *               chibar = dL/dRe chi0 + i dL/dIm chi0.
 *   grad_e_v    device, sum over problems of nv doubles: dL/dE_v (nullable = skip).
 *   grad_e_col  device, sum over problems of ncol doubles: dL/dE_col, which for a window
 *               column is the derivative with respect to its energy E_i (nullable).
 *   grad_n_col  device, same length: dL/dn_col, the derivative with respect to the
 *               weight g(E_i) dE_i of Eq. (energyintegration) (nullable).
 *   grad_coef_v  device complex128, sum over problems of nv x npw: dL/dRe + i dL/dIm of
 *               coef_v (nullable = skip).  GW_FP64 only, and only for (grid, K) shapes with a
 *               compiled pair kernel (gw_geom_create; GW_EUNSUPPORTED otherwise).
 *   grad_coef_c  device complex128, sum over problems of nband x npw, per coefficient row
 *               of coef_c: the columns that use one row (col_band) add up; rows no column
 *               uses get zero (nullable = skip; GW_FP64 only).
 * With s_p = m_p^H chibar m_p (pair densities recomputed, never stored for all pairs):
 * dL/dE_v = sum_c Re(conj(s) dw/dx), dL/dE_c = -sum_v Re(conj(s) dw/dx),
 * dL/dn_c = sum_v Re(conj(s) dw/dn), summed over frequencies, x = E_v - E_c and w the
 * energy factor of Eq. (chi0).  The coefficient gradients go back through the matrix
 * element: mbar_p = sum_w [conj(w_p) chibar m_p + w_p chibar^H m_p], h_p = F^H mbar_p on
 * the grid (F the transform of Eq. (chi0) including 1/N), dL/du_c = sum_v h_vc u_v,
 * dL/du_v = sum_c conj(h_vc) u_c, then the transpose of the band transform.  Every
 * reduction is float64 in a fixed order.  The product chibar m_p runs in the precision's
 * arithmetic: float64, float32, or split-bf16 x3 with float32 accumulation (chibar rounded
 * to float32 first). */
gw_status gw_chi0_backward(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, const double* omega,
                           double delta, gw_precision prec, void* workspace, size_t ws_bytes, const void* grad_chi0,
                           double* grad_e_v, double* grad_e_col, double* grad_n_col, void* grad_coef_v,
                           void* grad_coef_c);

/* Adjoint of gw_chi0_build_ksum: as gw_chi0_backward, except that grad_chi0 is one set of
 * nomega ng x ng blocks (the layout of the k-summed output), read by every problem.  The
 * gradients are per problem (concatenated like gw_chi0_backward's): a problem's e_v and
 * coef_v rows are the states at k'' = k + q - G0, so the caller adds them into those. */
gw_status gw_chi0_backward_ksum(gw_ctx* ctx, const gw_chi0_problem* probs, int nk, int nomega, const double* omega,
                                double delta, gw_precision prec, void* workspace, size_t ws_bytes,
                                const void* grad_chi0, double* grad_e_v, double* grad_e_col, double* grad_n_col,
                                void* grad_coef_v, void* grad_coef_c);

/* Graph mode (enable != 0): gw_chi0_build captures its launch sequence into a HIP
 * graph the first time it sees a given argument signature (problem records, frequency
 * values, delta, precision, workspace and output pointers) and replays the graph on
 * later identical calls; the data behind the pointers may change between calls.
 * Needs a context on a non-null stream.  Disabling drops the cached graphs. */
gw_status gw_ctx_set_graph(gw_ctx* ctx, int enable);

/* Launch-shape tuner: on the first conduction chunk of each problem, times the five
 * forms of the pair kernel and the contraction with
 * 1..32 pair-range splits, and keeps the fastest per problem shape in the context.
 * Later gw_chi0_workspace_size / gw_chi0_build calls use the tuned shapes (query the
 * workspace size again after tuning).  Synchronises the stream; workspace as for
 * gw_chi0_build. */
gw_status gw_tune(gw_ctx* ctx, const gw_chi0_problem* probs, int nprob, int nomega, gw_precision prec,
                  void* workspace, size_t ws_bytes);
/* The tuned shapes for prob's problem shape: pair-kernel form (1, 2 = 256 threads with
 * one or two resident workgroups per CU, 3 / 4 = split-line form with 4 / 2 valence bands
 * per workgroup, 5 = lean split-line form with 2 valence bands, which keeps the stage-2
 * items beyond one per thread in LDS; it exists where the dielectric sphere spans 17 or 19
 * frequencies along x3 on the 72^3 grid, and in float32 also from 17 on the 96^3 grid and
 * from 23 on the 128^3 grid; elsewhere form 5 runs form 1; 6 / 7 = direct-load split-line form
 * with 4 valence bands and four step buffers / 2 valence bands and two step buffers, which
 * streams the band rows from memory straight into LDS; it exists where a radix-R chunk row is
 * 128 bytes (float32 on 64^3, 96^3 and 128^3 grids, float64 on radix-8 grids) and its LDS
 * fits, elsewhere it runs form 1) and the number of pair-range splits of the contraction;
 * both 0 if the shape was not tuned. */
gw_status gw_tune_get(gw_ctx* ctx, const gw_chi0_problem* prob, gw_precision prec, int* pair_variant, int* ksplit);
/* Sets the shapes for prob's problem shape, e.g. to restore what gw_tune_get reported in
 * an earlier process: pair_variant 0..7 (0 = automatic), ksplit 0..32 (0 = automatic);
 * both 0 forgets the shape.  GW_EINVAL outside those ranges. */
gw_status gw_tune_set(gw_ctx* ctx, const gw_chi0_problem* prob, gw_precision prec, int pair_variant, int ksplit);

/* Workspace bytes for gw_pair_density with an nvs x ncs block. */
gw_status gw_pair_density_workspace_size(gw_ctx* ctx, const gw_chi0_problem* prob, int nvs, int ncs,
                                         gw_precision prec, size_t* bytes);

/* Pair densities M_vc(G) of Eq. (chi0) for one problem and a block of pairs
 * v in [v0, v0+nvs), columns j in [c0, c0+ncs):
 *   m_out   device complex128, (nvs * ncs) x ng row-major, pair index (v - v0) * ncs + (j - c0).
 * Uses the same kernels as gw_chi0_build; nvs * ncs must fit one pass (GW_EINVAL otherwise,
 * about 32768 pairs). */
gw_status gw_pair_density(gw_ctx* ctx, const gw_chi0_problem* prob, int v0, int nvs, int c0, int ncs,
                          gw_precision prec, void* workspace, size_t ws_bytes, void* m_out);

/* ---------------------------------------------------------------- dielectric */

/* eps^-1 = (I - diag(v) chi0)^-1 for nbatch matrices, in float64 (RPA relation before
 * Eq. (chi0); Table 3's eps_inf = 1/[eps^-1]_00).
 *   hermitian 0: any chi0 (a dynamic one included): Gauss-Jordan elimination with partial
 *             pivoting.  1: a static chi0, Hermitian and negative semidefinite, with v > 0: then
 *             eps~ = I - V^1/2 chi0 V^1/2 is Hermitian positive definite, eps^-1 = V^1/2 eps~^-1
 *             V^-1/2, and eps~ is inverted by block sweeps (a Cholesky factor per 64 x 64 pivot
 *             block, no pivoting, half the arithmetic); only the lower triangle of chi0
 *             (i >= j) is read.  Other values: GW_EINVAL.
 *   vcoul     device, nbatch x ng doubles, v(q+G) including its normalisation.
 *   chi0      device complex128, nbatch x ng x ng row-major.
 *   eps_inv   device complex128 output, same shape; may not alias chi0.
 *   workspace device scratch of at least gw_eps_inv_workspace_size bytes (either route).
 * Runs on the stream.  GW_ESINGULAR is reported by gw_eps_inv_status after the stream has
 * run: a zero or non-finite pivot, or with hermitian = 1 a pivot block that is not positive
 * definite or a v <= 0 (the output is then undefined; a chi0 that is not negative
 * semidefinite needs hermitian = 0). */
gw_status gw_eps_inv_workspace_size(gw_ctx* ctx, int ng, int nbatch, size_t* bytes);
gw_status gw_eps_inv(gw_ctx* ctx, int ng, int nbatch, int hermitian, const double* vcoul, const void* chi0,
                     void* workspace, size_t ws_bytes, void* eps_inv);
/* gw_eps_inv for callers that cannot allocate (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same inverse and kernels, with the scratch in a static
 * device array of the library (about 68 MiB per GPU, set up when the first context is created
 * on a GPU and held until the process ends) instead of a workspace argument.  The caller passes
 * inputs, hermitian and outputs as for gw_eps_inv; the call allocates nothing.  ng <= 2048 (GW_EINVAL
 * beyond: use gw_eps_inv).  Every call on a GPU shares that GPU's array, so calls that overlap on
 * one GPU (other streams, contexts or host threads) race: serialise them.  Zero pivots are
 * reported by gw_eps_inv_status as for gw_eps_inv. */
gw_status gw_eps_inv_noalloc(gw_ctx* ctx, int ng, int nbatch, int hermitian, const double* vcoul, const void* chi0,
                             void* eps_inv);
/* Synchronises the stream; GW_ESINGULAR if the last gw_eps_inv met a zero pivot (or, with
 * hermitian = 1, a pivot block that is not positive definite). */
gw_status gw_eps_inv_status(gw_ctx* ctx);

/* Adjoint of gw_eps_inv for a real loss L: with Z = eps^-1 (the saved output) and
 * Zbar = dL/dRe Z + i dL/dIm Z (device, complex128, same shape), writes
 *   chi0bar = diag(v) Z^H Zbar Z^H
 * (device complex128, may not alias the inputs).  Workspace: gw_eps_inv_workspace_size. */
gw_status gw_eps_inv_backward(gw_ctx* ctx, int ng, int nbatch, const double* vcoul, const void* eps_inv,
                              const void* grad_eps_inv, void* workspace, size_t ws_bytes, void* grad_chi0);

/* ---------------------------------------------------------------- COH self-energy */

/* Static limit of the COH self-energy of Eq. (sigmach): with the energy denominator taken
 * as -E', the frequency integral of eps^r^-1 - eps^a^-1 gives half the static
 * eps^-1 - 1 (Kramers-Kronig), and for states n, n' (Gamma, q -> 0)
 *   <n|Sigma_COH|n'> = 1/2 sum_c w_c sum_{G G'} M_{n c}(G) [eps^-1 - I]_{G G'} v(G')
 *                      conj(M_{n' c}(G')),
 * M the matrix element of Eq. (chi0) between state n and band c.  The sum over "all bands"
 * runs over the problem's columns with the weights of Eq. (energyintegration), which the
 * paper applies to this sum as well: bands with w = 1 and window representatives with
 * w = g(E_i) dE_i (any valence, conduction and window columns the caller lists).
 *   prob      coef_v / nv: the states n (1 .. 32 rows); coef_c, nband, ncol, col_band,
 *             n_col (NULL = all 1): the columns.  Energies are not read in this limit.
 *   vcoul     device, ng doubles v(q+G);  eps_inv  device complex128 ng x ng (static,
 *             gw_eps_inv's output layout).
 *   sigma     device complex128 nv x nv, row-major [n][n'] (overwritten).
 * Float64 throughout.  Workspace: gw_sigma_coh_workspace_size.  GW_EINVAL for more than 32
 * states, NULL arguments or a small workspace. */
gw_status gw_sigma_coh_workspace_size(gw_ctx* ctx, const gw_chi0_problem* prob, size_t* bytes);
gw_status gw_sigma_coh_static(gw_ctx* ctx, const gw_chi0_problem* prob, const double* vcoul, const void* eps_inv,
                              void* workspace, size_t ws_bytes, void* sigma);

/* The COH self-energy of Eq. (sigmach) with the plasmon-pole model the paper uses for the
 * frequency dependence of eps^-1 (gw_gpp_eps_inv).  Each element of [eps^r]^-1 - [eps^a]^-1 on
 * E' > 0 is then -i pi (Omega^2 / wt) delta(E' - wt) (as the pole's broadening goes to zero),
 * and the E' integral leaves, for states n, n' and energies E_j,
 *   <n|Sigma_COH(E_j)|n'> = 1/2 sum_q sum_c w_c sum_{G G'} M_{n c}(G)
 *        Omega^2_GG' v(q+G') / (wt_GG' (E_j - E_c - wt_GG' + i delta)) conj(M_{n' c}(G')),
 * M the matrix element of Eq. (chi0) between state n and column c (a band with weight w = 1 at
 * its energy E_c, or a window representative with w = g(E_i) dE_i at E_i: the grouping of Eq.
 * (energyintegration), which the paper applies to this sum), wt the principal square root of
 * wt^2.  Elements without a pole (wt^2 = +inf, unscreened) or with Omega^2 = 0 add nothing.
 * With E_j - E_c -> 0 every term becomes 1/2 [eps^-1(0) - 1] v: the static form above.
 *   probs, nq   one problem per q of the sum (the sum over q of Eq. (sigmach)): coef_v / nv the
 *               states n at k (1 .. 32, the same count in every problem), coef_c, nband, ncol,
 *               col_band, e_col (required), n_col (NULL = all 1) the columns at k - q.  A column
 *               set at k - q = k'' + G0 is passed relabelled, as for gw_chi0_build_ksum.  The
 *               problems are added in order; a 1/N_q goes into v.
 *   vcoul       host array of nq device pointers: ng_q doubles v(q+G) each.
 *   modes       host array of nq device pointers: 2 ng_q^2 complex128 each, Omega^2 then wt^2,
 *               row-major (the modes output of gw_gpp_eps_inv).
 *   energies    host, nenergy >= 1 real energies E_j (Hartree);  delta >= 0.
 *   sigma       device complex128 nenergy x nv x nv, [j][n][n'] (overwritten).
 * Float64 throughout.  Workspace: gw_sigma_coh_gpp_workspace_size.  GW_EINVAL for more than 32
 * states, differing state counts, NULL arguments, non-finite energies, a small workspace or the
 * value checks of gw_chi0_problem. */
gw_status gw_sigma_coh_gpp_workspace_size(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, int nenergy,
                                          size_t* bytes);
gw_status gw_sigma_coh_gpp(gw_ctx* ctx, const gw_chi0_problem* probs, int nq, const double* const* vcoul,
                           const void* const* modes, int nenergy, const double* energies, double delta,
                           void* workspace, size_t ws_bytes, void* sigma);

/* ---------------------------------------------------------------- plasmon pole */

/* Generalized plasmon-pole extension of a static eps^-1 to real frequencies, the frequency
 * model of the paper's calculations (Hybertsen-Louie).  Hartree atomic units:
 *   Omega^2_GG' = 4 pi [(q+G).(q+G') / |q+G|^2] rho(G - G')        (= w_p^2 ... rho/rho(0))
 *   wt^2_GG'    = Omega^2_GG' / (delta_GG' - eps^-1_GG'(0))
 *   eps^-1_GG'(w) = delta_GG' + Omega^2_GG' / ((w + i eta)^2 - wt^2_GG')
 * An element with delta - eps^-1(0) = 0 exactly has no pole (wt^2 = +inf) and keeps its
 * static value at every w.
 *   gvec_chi  host, ng x 3 Miller indices of the dielectric sphere (gw_eps_inv's order).
 *   q, bvec   host: q in reciprocal-lattice units (3), reciprocal lattice vectors as rows
 *             (9, 1/bohr); |q + G| must not vanish.
 *   rho       device complex128 valence density rho(G) (electrons / bohr^3) on the Miller
 *             box |n_i| <= rho_half, index ((n1 + h) W + n2 + h) W + n3 + h, W = 2 h + 1;
 *             the box must cover every G - G' of the sphere (GW_EINVAL otherwise).
 *   eps_inv_static  device complex128 ng x ng.
 *   omega     host, nomega >= 0 real frequencies; eta >= 0 broadening.
 *   modes     device complex128 2 ng^2 or NULL: Omega^2 then wt^2, row-major.
 *   eps_inv_omega  device complex128 nomega x ng x ng.
 * Synchronises the stream.  Workspace: gw_gpp_workspace_size (device copies of the sphere
 * and the frequencies). */
gw_status gw_gpp_workspace_size(gw_ctx* ctx, int ng, int nomega, size_t* bytes);
gw_status gw_gpp_eps_inv(gw_ctx* ctx, int ng, const int32_t* gvec_chi, const double* q, const double* bvec,
                         int rho_half, const void* rho, const void* eps_inv_static, int nomega, const double* omega,
                         double eta, void* workspace, size_t ws_bytes, void* modes, void* eps_inv_omega);

/* ---------------------------------------------------------------- k-points */

/* k + q mapping of a k-point set (host arrays): for each k (fractional coordinates,
 * nk x 3), kq_index[k] = the first k'' of the set with k + q - k'' integral (each
 * coordinate within tol of an integer, 0 < tol < 0.5) and g0[3 k ..] = that integer vector
 * G0, so that k + q = k'' + G0.  GW_EINVAL if some k + q is not in the set modulo G. */
gw_status gw_kq_map(int nk, const double* kpts, const double* q, double tol, int32_t* kq_index, int32_t* g0);

/* ---------------------------------------------------------------- grouping */

/* Columns of Eq. (energyintegration) from a conduction spectrum (host arrays).
 *   e_band    nband band energies (any order).
 *   e0, de, nwin   windows [e0 + i de, e0 + (i+1) de), i < nwin, the last one closed
 *             at e0 + nwin de.  Bands with E <= e0 are explicit columns (index order,
 *             multiplicity 1).
 *   mode      0 = count (multiplicity = number of bands in the window),
 *             1 = dos (multiplicity = dos_a * sqrt(E_i - dos_v0) * de, the weight
 *             g(E_i) dE_i with g of the form printed after Eq. (chi02)).
 * Each non-empty window gives one column: the band nearest its midpoint E_i =
 * e0 + (i + 1/2) de (lower index on a tie), energy E_i.
 * Outputs (host, capacity >= nband + nwin): col_band, e_col, n_col; *ncol_out columns,
 * *n0_out explicit ones.  GW_EINVAL if a band lies above the last window. */
gw_status gw_group_windows(int nband, const double* e_band, double e0, double de, int nwin, int mode, double dos_a,
                           double dos_v0, int32_t* col_band, double* e_col, double* n_col, int* ncol_out,
                           int* n0_out);

/* Columns of Eq. (energyintegration) on an arbitrary energy grid: the uniform or
 * nonuniform grids and the higher-order rules the paper allows for the integral.
 *   edges     host, nwin + 1 strictly increasing energies; window i is
 *             [edges[i], edges[i+1]) (the last one closed), bands with E <= edges[0] = E0
 *             are explicit columns.
 *   rule      0 = midpoint: one node at the window centre;
 *             1 = two-point Gauss-Legendre: nodes centre -+ dE / (2 sqrt 3), weight dE / 2
 *             each (mode 1 only).
 *   mode      0 = count (the number of bands in the window, midpoint rule only),
 *             1 = dos (dos_a * sqrt(node - dos_v0) times the rule's weight).
 * Each window holding at least one band gives one column per node: the window's band
 * nearest the node (lower index on a tie), energy = the node.  Outputs (host, capacity
 * >= nband + 2 nwin) as for gw_group_windows.  GW_EINVAL for edges that do not increase,
 * a band above the last edge, an unknown rule or mode, or rule 1 with mode 0. */
gw_status gw_group_windows_edges(int nband, const double* e_band, int nwin, const double* edges, int mode, int rule,
                                 double dos_a, double dos_v0, int32_t* col_band, double* e_col, double* n_col,
                                 int* ncol_out, int* n0_out);

#ifdef __cplusplus
}
#endif
#endif /* GWCHI0_H */
