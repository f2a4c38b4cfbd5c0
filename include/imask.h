/*
 * imask.h - C ABI of libimask, the MI355X (gfx950) implementation of the
 * ImaSk hot path: stochastic multiresolution image-domain sketching for CT
 * (Perelli, Schönlieb, Ehrhardt, arXiv 2412.10249).
 *
 * Problem (Sec. 1, eq. (min_obj)):  min_x 1/2 |K x - b|^2 + R(x), K the 2-D
 * parallel-beam (or fan-beam) CT model.  ImaSk (Alg. 1) replaces K by a family of sketched
 * operators K_i = K S_i (eq. (CT_sketches)) with probabilities p_i and runs a
 * SAGA-type primal-dual iteration that applies one K_i and one K_i^T per step.
 *
 * Conventions (all functions):
 *   - The image domain is [-E,E]^2, E = imask_geometry.extent (1 by
 *     default).  A full-resolution image is N x N, row-major, float32; pixel
 *     (i,j) is row i (y), column j (x), centre (-E + (j+1/2)h, -E + (i+1/2)h),
 *     h = 2E/N.
 *   - Level l (l = log2 of the downsampling factor) has N_l = N >> l pixels
 *     per side; N must be divisible by 2^l.
 *   - Angle a of n_angles is a*pi/n_angles or the a-th listed angle; bin b
 *     of n_det has centre (b - (n_det-1)/2)*det_spacing + det_offset; the
 *     ray is x cos(theta) + y sin(theta) = s.  Sinograms are
 *     [n_angles][n_det] float32.
 *   - Every array argument is a DEVICE pointer owned by the caller, unless
 *     the comment says "host".  The library allocates no device memory and
 *     keeps no pointer after a call returns.
 *   - `stream` is a hipStream_t (NULL = default stream).  All device work is
 *     enqueued asynchronously on it; no call synchronises the device, so the
 *     calls can be captured into a HIP graph (set-up calls excepted: they
 *     say so).
 *   - Return value: IMASK_OK (0) or a negative error code.  Arguments are
 *     validated before anything is enqueued, so a failed call writes nothing.
 *     IMASK_EHIP reports a failed kernel launch (hipGetLastError).
 */
#ifndef IMASK_H
#define IMASK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IMASK_MAX_LEVELS 8   /* sketches per level set (r) */
#define IMASK_MAX_LOG2F 7    /* coarsest level: 2^7 downsampling (r = 8 levels 0..7) */
#define IMASK_MAX_TV_INNER 12
#define IMASK_MAX_BLOCKS 1024 /* measurement blocks (imask_levels.n_blocks) */

enum {
    IMASK_OK = 0,
    IMASK_EINVAL = -1,  /* bad size, pointer, level set or parameter */
    IMASK_ENOTSUP = -2, /* valid but unsupported combination */
    IMASK_EHIP = -3,    /* a HIP launch failed */
    IMASK_ESIZE = -4,   /* workspace too small */
    IMASK_ENONFINITE = -5 /* opt-in check: an iterate holds a NaN or infinity */
};

enum { IMASK_FULL_PAPER = 0, IMASK_FULL_UNBIASED = 1 };
enum { IMASK_REG_TIKHONOV = 0, IMASK_REG_SMOOTH_TV = 1, IMASK_REG_TV = 2 };
enum { IMASK_SCHEDULE_PARALLEL = 0, IMASK_SCHEDULE_SEQUENTIAL = 1 };
enum { IMASK_DRAW_COMMON = 0, IMASK_DRAW_INDEPENDENT = 1 };
enum {
    IMASK_RESTRICT = 0,     /* out (N_l^2)  = T_l in, 2^l x 2^l block mean (Sec. 4.1) */
    IMASK_PROLONG = 1,      /* out (N^2)    = T_l^* in, replication (Sec. 4.1) */
    IMASK_RESTRICT_ADJ = 2, /* out (N^2)    = T_l^T in = 4^{-l} T_l^* in (true adjoint of T_l) */
    IMASK_PROJECT = 3,      /* out (N^2)    = P_l in = T_l^* T_l in (S_i of Sec. 4.1) */
    IMASK_COMPENSATE = 4    /* out (N^2)    = S_r in = p_0^{-1}(in - sum_{k>0} p_k P_{l_k} in) */
};
enum { IMASK_BUDGET_ITERS = 0, IMASK_BUDGET_EPOCHS = 1 };

/* Acquisition geometry (Sec. 4.1: parallel beam, m = n_angles * n_det).
 * The image covers the square [-E, E]^2 (E = extent) with N x N pixels of
 * side 2E/N; bin b has centre s_b = (b - (n_det-1)/2) det_spacing + s0 and
 * angle a the ray set x cos(theta_a) + y sin(theta_a) = s_b.  Sinograms are
 * stored angle-major in the order of the angles.
 * angles: NULL selects theta_a = a*pi/n_angles; otherwise a HOST array of
 * n_angles finite angles in radians (any real values, any order, repeats
 * allowed).  imask_prepare copies it into the workspace, where the kernels
 * read it, and waits for its stream; later calls read the host array only to
 * size their launches, so they must pass the same values.  A listed angle
 * steps along rows when |cos| >= |sin| in FP64, else along columns; the
 * default angles step along rows iff 4a <= n_angles or 4a >= 3 n_angles.
 *
 * Fan beam (src_dist = D > 0; the divergent-beam case of the same line-
 * integral operator, Sec. 4.1, and a geometry of the outlook of Sec. 6):
 * view a puts the source at D (cos beta_a, sin beta_a), beta_a =
 * 2 pi a / n_angles or the a-th listed angle, and a flat detector through
 * -det_dist (cos beta_a, sin beta_a), perpendicular to the central ray; bin
 * b sits at t_b = (b - (n_det-1)/2) det_spacing + det_offset along
 * (-sin beta_a, cos beta_a) and its ray joins the source to that point.
 * Each ray steps along rows when the x component of its unit normal is at
 * least the y component in magnitude (FP64, computed once by
 * imask_prepare, which also tabulates every ray's line in the workspace and
 * waits for its stream).  det_spacing <= 0 selects the pixel size magnified
 * onto the detector, 2E/N (D + det_dist)/D.  Every entry point takes a fan
 * geometry; measurement blocks (imask_levels.n_blocks) are contiguous
 * ranges of views.
 *
 * Invalid (EINVAL): n outside 4..16384,
 * not a multiple of 4, or above 16 not a multiple of 16; n_angles or n_det
 * out of range; a non-finite spacing, offset, extent, listed angle, source
 * or detector distance; an extent outside [1e-100, 1e100]; a positive
 * spacing outside [1/64, 64] full-resolution pixels (fan beam: magnified
 * pixels); |det_offset| > 4E (fan beam: 4E (D + det_dist)/D); a source
 * distance outside (2E, 1e4 E] or a negative one; a detector distance
 * outside [0, 1e4 E]. */
typedef struct {
    int32_t n;            /* full-resolution image side N */
    int32_t n_angles;     /* 1 .. 65536 (fan beam: views) */
    int32_t n_det;        /* 1 .. 8192 */
    double det_spacing;   /* bin spacing; <= 0 selects the default above */
    double det_offset;    /* detector centre offset s0 */
    double extent;        /* half side E of the image square; <= 0 selects 1 */
    const double* angles; /* host, n_angles radians, or NULL (see above) */
    double src_dist;      /* fan beam: source distance D from the centre; 0 selects parallel beam */
    double det_dist;      /* fan beam: detector distance beyond the centre; ignored for parallel beam */
} imask_geometry;

/* Resolution set and sampling probabilities (Alg. 1 REQUIRE line; Sec. 4.1).
 * Sketch k uses level log2f[k]; log2f[0] must be 0 (the full-resolution
 * sketch) and the list strictly increasing; p[k] > 0 with sum 1 (1e-9).
 * full_mode selects the full-resolution sketch:
 *   IMASK_FULL_PAPER    K_0 = K S_r, S_r = p_0^{-1}(I - sum_{k>0} p_k P_k)
 *                       (the paper's construction; cost 1 epoch)
 *   IMASK_FULL_UNBIASED K_0 = p_0^{-1}(R_0 - sum_{k>0} p_k R_{l_k} T_{l_k}),
 *                       so that sum_k p_k K_k = R_0 exactly
 *                       (cost 1 + sum_{k>0} 2^{-l_k} epochs).
 * n_blocks = S > 1 combines the image sketches with measurement
 * sub-selection (the outlook of Sec. 6), read as Alg. 1 over the sketches
 * K_kb = S E_b K_k: the angles form S contiguous blocks, block b = angles
 * [floor(b n_angles / S), floor((b+1) n_angles / S)), E_b keeps its rows,
 * and each step draws b uniformly from the low 32 bits of the same
 * generator output whose high bits pick k (b = (lo32 * S) >> 32).  phi
 * then holds S copies of the r tables (block b's at b * sum_k N_{l_k}^2),
 * psi stays r sinograms (block b's rows of table k hold K_kb x), the dual
 * step still updates every row, and a step costs its sketch's cost times
 * its block's share of the angles.  Read by imask_step / imask_solve
 * (parallel schedule, full tables, common draws and the default angles or
 * fan-beam views, not listed ones; IMASK_ENOTSUP otherwise), imask_phi_floats and imask_block_draws; the
 * other calls apply the level sketches alone.  0 or 1: no blocks;
 * 2 .. min(n_angles, IMASK_MAX_BLOCKS), else IMASK_EINVAL. */
typedef struct {
    int32_t r;
    int32_t log2f[IMASK_MAX_LEVELS];
    double p[IMASK_MAX_LEVELS];
    int32_t full_mode;
    int32_t n_blocks;
} imask_levels;

/* Regulariser R, mu-strongly convex with mu = lambda (Sec. 2.2, Sec. 4.2):
 *   IMASK_REG_TIKHONOV  R = lambda/2 |x|^2, prox closed form
 *   IMASK_REG_SMOOTH_TV R = tv_weight * sum sqrt(|grad x|^2 + tv_eps^2)
 *                           + lambda/2 |x|^2, prox by tv_inner FISTA steps
 *                           (Sec. 4.5 evaluates the TV prox with FISTA)
 *   IMASK_REG_TV        the paper's prior of Sec. 4.5, tv_weight |grad x|_{1,2}
 *                       + chi_{x >= 0}, plus lambda/2 |x|^2 (which supplies
 *                       the strong convexity mu = lambda of the step rule);
 *                       prox by tv_inner iterations of the fast gradient
 *                       projection on the dual (Beck-Teboulle), warm-started at
 *                       the dual pair kept in imask_state.tvd; tv_eps unused.
 * Differences are forward, with zero difference past the last row/column. */
typedef struct {
    int32_t kind;
    double lambda;    /* > 0 */
    double tv_weight; /* >= 0 */
    double tv_eps;    /* > 0 */
    int32_t tv_inner; /* 1 .. IMASK_MAX_TV_INNER */
} imask_reg;

/* Step size sigma (Alg. 1) and the sketch-index generator: SplitMix64 in
 * counter form; stream seed = the stream_id-th output of the generator at
 * state `seed`; draw k uses the k-th output of the stream (top 32 bits)
 * against floor(2^32 * cumulative p).
 * schedule selects the iteration:
 *   IMASK_SCHEDULE_PARALLEL   Alg. 1: primal and dual steps both from
 *                             (x^k, y^k); theta is ignored
 *   IMASK_SCHEDULE_SEQUENTIAL the ImaSk-Seq variant of Sec. 5: the dual step
 *                             uses K_i xbar^k, the primal step K_i^T y^{k+1},
 *                             and xbar^{k+1} = x^{k+1} + theta (x^{k+1} - x^k);
 *                             0 <= theta <= 1, and imask_state.xbar is needed
 * draw_mode selects the sketch draws:
 *   IMASK_DRAW_COMMON      Alg. 1: one index per iteration for both steps
 *   IMASK_DRAW_INDEPENDENT the outlook of Sec. 6: the primal step (K_i^T,
 *                          phi) uses stream_id, the dual step (K_j, psi) an
 *                          independent index from stream dual_stream_id;
 *                          an iteration then costs (c(i) + c(j)) / 2 epochs.
 *                          Parallel schedule with full tables only
 *                          (IMASK_ENOTSUP otherwise)
 * check_finite (opt-in): nonzero makes imask_step / imask_solve test x and y
 * of this problem for NaN or infinity once, after its last step; the test
 * synchronises `stream` and the call then returns IMASK_ENONFINITE if one
 * is found (the steps have still been applied).  Zero: no test, no sync. */
typedef struct {
    double sigma;
    uint64_t seed;
    uint32_t stream_id;
    int32_t schedule;
    double theta;
    int32_t draw_mode;
    uint32_t dual_stream_id;
    int32_t check_finite;
    int32_t reserved; /* must be 0 */
} imask_params;

/* ImaSk state (Alg. 1): iterates, gradient tables and counters.
 *   x[2]   two N*N buffers (ping-pong): x[cur] is the current iterate
 *   y[2]   two n_angles*n_det buffers: y[cur] is the current dual iterate
 *   phi    image-space table K_k^T y: sketch 0 holds N*N floats, sketch k>0
 *          holds its coarse image N_{l_k}^2 (phi_k = T_{l_k}^T(...) is
 *          piecewise constant); concatenated in sketch order,
 *          imask_phi_floats() floats in total
 *   psi    sinogram-space table K_k x: r * n_angles*n_det floats
 *   work   workspace prepared by imask_prepare() for this geometry
 *   xbar   N*N extrapolated point (IMASK_SCHEDULE_SEQUENTIAL only, updated
 *          in place; start it equal to x, e.g. both zero); may be NULL for
 *          the parallel schedule
 *   tvd[2] two buffers of 2*N*N floats (IMASK_REG_TV only, ping-pong with
 *          cur like x): the TV dual pair, row differences then column
 *          differences; start tvd[cur] at zero; may be NULL otherwise
 *   ztab   NULL for the tables above.  Non-NULL selects the compact dual
 *          tables of Remark 1 (the iterate is kept instead of its
 *          projection): psi then holds only the running average
 *          sum_k p_k K_k x^{(k)} (n_angles*n_det floats) and ztab the
 *          restricted iterate at each sketch's last refresh (sketch 0 the
 *          N*N image, sketch k > 0 its N_{l_k}^2 block mean; the phi layout,
 *          imask_phi_floats() floats); start both at zero.  One projection of
 *          the difference per step gives psi_new - psi_k, so the cost is
 *          unchanged and the dual tables shrink from r*m to m + sum d_l
 *          floats.  Parallel schedule only (IMASK_ENOTSUP otherwise)
 *   k      iteration counter (index of the next draw)
 *   epochs equivalent full-resolution operator applications so far
 *   cur    0 or 1 */
typedef struct {
    float* x[2];
    float* y[2];
    float* phi;
    float* psi;
    void* work;
    uint64_t k;
    double epochs;
    int32_t cur;
    float* xbar;
    float* tvd[2];
    float* ztab;
} imask_state;

/* Bytes of device workspace needed for geometry g (host function). */
size_t imask_workspace_bytes(const imask_geometry* g);

/* Floats in the phi table for level set lv (host function): sum over the
 * sketches of N_{l_k}^2, times n_blocks when that is above 1. */
size_t imask_phi_floats(const imask_geometry* g, const imask_levels* lv);

/* Measurement blocks b_k of draws k = k0 .. k0+count-1 (host function; all 0
 * without blocks), the companions of the sketch indices of imask_draws. */
int imask_block_draws(const imask_params* prm, const imask_levels* lv, uint64_t k0, int32_t count,
                      int32_t* out_host);

/* Fills `work` (device, work_bytes >= imask_workspace_bytes(g)) with the
 * per-(level, angle) projector constants and zeroes its scratch.  Every
 * other call taking `work` requires a workspace prepared for the same
 * geometry; calls sharing one workspace must be ordered on one stream.
 * With listed angles it also copies them from the host and synchronises
 * `stream` before returning (set-up, not for graph capture). */
int imask_prepare(const imask_geometry* g, void* work, size_t work_bytes, void* stream);

/* sino = R_l T_l x_full  (x_full N*N; T_0 = I).  R_l is the ray-driven
 * Joseph projector on the level-l grid, i.e. the CT model discretised on the
 * coarse grid of Sec. 4.1 (eq. (CT_sketches), K_i = R_i T_i), with the same
 * detector at every level. */
int imask_project(const imask_geometry* g, int32_t log2f, const void* work,
                  const float* x_full, float* sino, void* stream);

/* x_full = T_l^T R_l^T sino = 4^{-l} T_l^* R_l^T sino, the exact transpose
 * of imask_project: the operator K_i^T of the primal step of Alg. 1 for a
 * coarse sketch (Sec. 4.1, eq. (CT_sketches); the true adjoint of T_l carries
 * the factor 4^{-l}).  Ray-driven: the weights come from the forward's own
 * fixed-point coordinate; each image row is accumulated by one wavefront, so
 * there are no atomics and the result is deterministic). */
int imask_backproject(const imask_geometry* g, int32_t log2f, const void* work,
                      const float* sino, float* x_full, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transpose of imask_backproject without a workspace argument.  x_full
 * receives what imask_backproject writes for the same arguments, bit for
 * bit (same kernels, same partial-image order).  Instead of a workspace the
 * call uses a static device array of IMASK_NOALLOC_SCRATCH_BYTES per GPU,
 * held until the process ends, for the projector constants (recomputed on
 * every call: 64 B per level and angle), the partial images (as many as a
 * workspace holds: P = max(16 N^2, min(64 N^2, 2^23)) floats) and the
 * coarse result (N^2 floats); the first call on a device looks up
 * the array's address there.  Every call on one GPU shares that array, so
 * calls that overlap on one GPU (several streams or host threads) race and
 * must be ordered by the caller; each call writes every byte it reads
 * before reading it, so the previous call's contents do not matter.
 * Allocates nothing (no hipMalloc, hipFree or allocating library call) and
 * does not synchronise.  Parallel beam with the default angles only
 * (IMASK_ENOTSUP for listed angles or a fan beam); IMASK_ESIZE when the
 * geometry needs more than the array: 4 (P + N^2 + 16 (lmax+1) n_angles)
 * bytes, so N <= 512 with up to 30720 angles; IMASK_EINVAL as for
 * imask_backproject. */
#define IMASK_NOALLOC_SCRATCH_BYTES (48u << 20)
int imask_backproject_noalloc(const imask_geometry* g, int32_t log2f, const float* sino, float* x_full,
                              void* stream);

/* Resampling operators of Sec. 4.1 on an N x N grid (see IMASK_RESTRICT ...).
 * lv is read only for IMASK_COMPENSATE (may be NULL otherwise). */
int imask_resample(int32_t n, int32_t log2f, int32_t mode, const imask_levels* lv,
                   const float* in, float* out, void* stream);

/* out = K_k in (adjoint == 0: in N*N, out sinogram) or K_k^T in (adjoint != 0:
 * in sinogram, out N*N) for sketch k of level set lv (eq. (CT_sketches)). */
int imask_sketch_apply(const imask_geometry* g, const imask_levels* lv, int32_t k,
                       int32_t adjoint, const void* work, const float* in, float* out,
                       void* stream);

/* Diagnostic (not on the hot path): average duration in ms over `reps`
 * back-to-back launches of one projector kernel at level log2f, exactly as
 * a step launches it, measured with HIP events recorded on `stream`;
 * synchronises on the second event.  IMASK_KERNEL_FORWARD: the Joseph
 * forward kernel on the level-l restriction of `in` (N*N; `out`, a
 * sinogram, receives one full projection first).  IMASK_KERNEL_TRANSPOSE:
 * the transpose kernel on sinogram `in` (its partial images stay in the
 * workspace; `out` is unused but must be non-null).
 * IMASK_KERNEL_TRANSPOSE_SUM: that kernel and the ordered sum of its
 * partial images into the level image (the coarse result in the
 * workspace; `out` unused but non-null), the pair a step launches. */
enum { IMASK_KERNEL_FORWARD = 0, IMASK_KERNEL_TRANSPOSE = 1, IMASK_KERNEL_TRANSPOSE_SUM = 2 };
int imask_time_kernel(const imask_geometry* g, int32_t which, int32_t log2f, const void* work, const float* in,
                      float* out, int32_t reps, void* stream, double* avg_ms);

/* Diagnostic (not on the hot path): n_steps steps of one problem, as
 * imask_step runs them in one call, with a HIP event recorded on `stream`
 * before the first step and after each one; synchronises and writes each
 * step's GPU time in ms to ms_out[0 .. n_steps-1] (host memory).  The times
 * are the GPU's own when the caller keeps the GPU behind the host (for
 * example with a long kernel enqueued first). */
int imask_step_timed(const imask_geometry* g, const imask_levels* lv, const imask_reg* reg, const imask_params* prm,
                     const float* b, imask_state* s, int32_t n_steps, float* ms_out, void* stream);

/* Step-size constants (setup, not the hot path; synchronises `stream`).
 * For ImaSk as the saddle-point method of Sec. 3 with A_i = p_i K_i,
 * mu_f* = 1 and mu_g = mu, writes to out_host[0..2] the normalised squared
 * norms of Sec. 3.4:
 *   L^2      = lmax(Kbar^T Kbar)/mu, Kbar = sum_i p_i K_i
 *   Lbar^2   = max(lmax(sum p_i^2 K_i^T K_i), lmax(sum p_i^2 K_i K_i^T))/mu
 *   Lbar_p^2 = max(lmax(sum p_i K_i^T K_i),   lmax(sum p_i K_i K_i^T))/mu
 * each by `iters` power iterations on the GPU sketch operators from a
 * random start drawn from `seed`.  `scratch`: device, at least
 * imask_constants_scratch_bytes(g) bytes; `work` as for imask_sketch_apply. */
size_t imask_constants_scratch_bytes(const imask_geometry* g);
int imask_step_constants(const imask_geometry* g, const imask_levels* lv, double mu, int32_t iters, uint64_t seed,
                         const void* work, void* scratch, double* out_host, void* stream);

/* Host: the comparison step size of Sec. 3.6 taken from Balamurugan & Bach,
 * sigma_B = 1 / (L^2 + 3 Lbar^2), from the constants of imask_step_constants.
 * Returns IMASK_EINVAL for non-positive constants or a NULL output. */
int imask_sigma_balamurugan(double L2, double Lbar2, double* sigma_out);

/* Host: the step size of Thm. 3 (eq. (opt:cond) and eq. (eta_opt)),
 * minimising the rate theta over c = cbar*i/(grid+1), rho = j/(grid+1),
 * i, j = 1..grid, cbar = 1/(1 + L^2 + Lbar_p^2); sigma = eta_opt/(1 - eta_opt).
 * pmin is the smallest sampling probability; theta_out (may be NULL)
 * receives the rate.  Returns IMASK_EINVAL for non-positive constants, pmin
 * outside (0, 1], grid < 2 or a NULL sigma_out. */
int imask_sigma_thm3(double L2, double Lbar2, double Lbarp2, double pmin, int32_t grid, double* sigma_out,
                     double* theta_out);

/* Host: the sketch indices i_k, k = k0 .. k0+count-1 (Alg. 1: one random level per iteration). */
int imask_draws(const imask_params* prm, const imask_levels* lv, uint64_t k0, int32_t count,
                int32_t* out_host);

/* Runs n_steps iterations of Alg. 1 on each of n_problems independent
 * problems (arrays of n_problems structs; b[q] is problem q's data, a
 * sinogram).  For each step: draw k, psi_new = K_k x^k, phi_new = K_k^T y^k
 * (both from the old iterates), xi/zeta from the old tables,
 * x^{k+1} = prox_{sigma/mu R}(x^k - sigma/mu xi),
 * y^{k+1} = (y^k + sigma zeta - sigma b)/(1 + sigma), then the tables are
 * refreshed, cur flips, k += 1 and epochs += the sketch's cost. */
int imask_step(int32_t n_problems, const imask_geometry* g, const imask_levels* lv,
               const imask_reg* reg, const imask_params* prm, const float* const* b,
               imask_state* s, int32_t n_steps, void* stream);

/* Runs Alg. 1 (the loop of imask_step) until every problem has done
 * `budget` more iterations (IMASK_BUDGET_ITERS) or accumulated `budget` more
 * epochs (IMASK_BUDGET_EPOCHS), the budget unit of the experiments of
 * Sec. 4.3 (one epoch = the cost of one full-resolution operator pair).
 * Returns after enqueueing; the epoch budget is evaluated on the host from
 * the draws, without synchronising.  Errors as for imask_step. */
int imask_solve(int32_t n_problems, const imask_geometry* g, const imask_levels* lv,
                const imask_reg* reg, const imask_params* prm, const float* const* b,
                imask_state* s, double budget, int32_t budget_kind, void* stream);

/* ---- Launch shapes (an autotuner's knobs; set-up calls) ----
 * The kernels of a level whose grid side is nl, in geometries of n_angles x
 * n_det, take these shapes instead of the defaults:
 *   bp_rows x bp_waves  the transpose's tile: image rows per wavefront and
 *                       wavefronts per workgroup (2x8, 4x4, 2x4 or 1x4; a
 *                       shape whose rows do not fit in the LDS falls back
 *                       to the default)
 *   bp_wg               the transpose's target workgroup count (64..16384;
 *                       angle groups are also bounded by the partial images
 *                       the workspace holds)
 *   fwd_lds_kb          the forward's band budget in KB (the level's
 *                       default or more, up to 156: never more bands than
 *                       the workspace is sized for)
 * Zero fields keep the defaults; t == NULL resets the entry.  Every shape
 * computes the same matrices; only the order of floating-point sums (band
 * partials, angle groups) changes.  The table is global to the process and
 * read at every launch: do not change it while another thread launches, or
 * between imask_batch_prepare and the batch's steps.  IMASK_EINVAL for an
 * unsupported shape or out-of-range sizes. */
typedef struct {
    int32_t bp_rows, bp_waves, bp_wg, fwd_lds_kb;
} imask_tiles;
int imask_set_tiles(int32_t nl, int32_t n_angles, int32_t n_det, const imask_tiles* t);
int imask_get_tiles(int32_t nl, int32_t n_angles, int32_t n_det, imask_tiles* out);

/* ---- Batched steps: many independent problems of mixed sizes advanced
 * together (Alg. 1 for each; the batching is a systems layer, not part of
 * the paper's method).  A batch buffer (device, caller-owned) holds, for
 * every problem and every (sketch, parity of the ping-pong buffers), the
 * launch records of one step: the kernels, grids and arguments that
 * imask_step would launch for it.  Each batched step then runs one plan
 * kernel (it draws every problem's sketch index on the device, from the
 * same SplitMix64 stream as the host draw), one persistent launch per kernel
 * variant over the work items of all problems, and one kernel that advances
 * the counters.  The launches of a step do not depend on the draws, so a
 * captured step (hipStreamBeginCapture / a torch CUDA graph) can be replayed
 * for every step.  Each problem computes exactly what imask_step computes
 * for it (same kernels, shapes and summation order: equal bit for bit).
 *
 * Supported problems: parallel beam (default or listed angles), the
 * parallel schedule with common draws, no measurement blocks, the standard
 * tables and the Tikhonov prior (IMASK_ENOTSUP otherwise).  At most 4096
 * problems; the problems must not share state, data or workspace buffers.
 */

/* Bytes of the batch buffer for these problems (0 if invalid). */
size_t imask_batch_bytes(int32_t n_problems, const imask_geometry* g, const imask_levels* lv);

/* Set-up (synchronises `stream`): validates the problems, fills the batch
 * buffer from their current states (s[q].k, cur, epochs and buffers) and
 * fixes each problem's budget: `budget` more iterations (IMASK_BUDGET_ITERS)
 * or epochs (IMASK_BUDGET_EPOCHS), evaluated from the host draws as
 * imask_solve does; a problem idles once its budget is met.  steps_out
 * (may be NULL) receives the number of batched steps after which every
 * problem has met its budget.  Errors: IMASK_EINVAL / IMASK_ENOTSUP as for
 * imask_step and above, IMASK_ESIZE for a buffer below imask_batch_bytes. */
int imask_batch_prepare(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, const imask_reg* reg,
                        const imask_params* prm, const float* const* b, const imask_state* s, double budget,
                        int32_t budget_kind, void* batch, size_t batch_bytes, int64_t* steps_out, void* stream);

/* Enqueues n_steps batched steps on `stream` (no synchronisation; the
 * problems' counters advance on the device, not in the host structs).
 * g and lv must be those given to imask_batch_prepare. */
int imask_batch_step(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, void* batch,
                     int32_t n_steps, void* stream);

/* The four parts of one batched step, for callers that run the two
 * independent halves of Alg. 1's step concurrently:
 *   IMASK_BATCH_PLAN       draws and work lists (first)
 *   IMASK_BATCH_FORWARD    restriction, forward projection, dual step
 *   IMASK_BATCH_TRANSPOSE  transposes, prolongation, primal step
 *   IMASK_BATCH_ADVANCE    the counters (last)
 * FORWARD and TRANSPOSE read the step's old iterates and write disjoint
 * buffers, so they may run on two streams between PLAN and ADVANCE (the
 * caller orders them with events).  imask_batch_step runs all four in
 * order on one stream. */
enum { IMASK_BATCH_PLAN = 0, IMASK_BATCH_FORWARD = 1, IMASK_BATCH_TRANSPOSE = 2, IMASK_BATCH_ADVANCE = 3 };
int imask_batch_step_part(int32_t n_problems, const imask_geometry* g, const imask_levels* lv, void* batch,
                          int32_t part, void* stream);

/* Copies the problems' counters (k, cur, epochs) from the batch buffer into
 * s[0..n_problems) (synchronises `stream`); lv as given to prepare. */
int imask_batch_state(int32_t n_problems, const imask_levels* lv, const void* batch, imask_state* s, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* IMASK_H */
