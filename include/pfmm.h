/*
 * pfmm.h -- C ABI of the MI355X periodic field evaluator.
 *
 * Evaluates, for sources s_j with densities q_j and targets t_i in a 2D
 * doubly periodic cell with lattice vectors e1, e2,
 *     u(t_i) = sum_j sum_{(m,n) in Z^2} G(t_i - s_j - m e1 - n e2) q_j
 * and its gradient (Sec. 1, eq. psum), for
 *     PFMM_LAPLACE  G = -(1/2pi) log r                  (Sec. 1; needs sum q = 0)
 *     PFMM_YUKAWA   G = (1/2pi) K0(beta r)              (Sec. 1, modified Helmholtz)
 *     PFMM_STOKES   G = -(1/4pi)(log r I - r r^T/r^2)   (Sec. 5.2, eq. stokeslet; needs sum f = 0)
 * by the paper's splitting (Sec. 1, Def. 1, eq. nearfarsplit): a direct sum
 * over the cell and its nearest images (3 x (2 m0 + 1) copies), plus the
 * explicit low-rank plane-wave factorisation of all farther images,
 * P = L D R, for the south/north rows (Thm. south_thm and its corollary;
 * Thm. south_thm_lap; Thm. south_thm_s) and the west/east columns (Thm.
 * west_thm, west_thm_lap, west_thm_s), applied right to left (Sec. 6); when
 * the aspect ratio is large the south/north factors are applied through
 * type-1/type-2 NUFFTs on Gauss-Legendre lines in y (Sec. 6.1, eqs.
 * fastanterp, fastinterp).
 *
 * Conventions
 *  - All coordinate, density and output pointers passed to pfmm_eval are
 *    DEVICE pointers (HIP global memory) unless a comment says "host".
 *    The caller owns every buffer; the plan owns only its small tables.
 *  - Arrays are structure-of-arrays, float64:
 *      src_xy [2][n_src]   (x then y), trg_xy [2][n_trg] (may equal src_xy)
 *      dens   [n_dens][n_src]        (Laplace, Yukawa)
 *             [n_dens][2][n_src]     (Stokes: force components f1, f2)
 *      out_pot  [n_dens][n_trg]      (Stokes: velocity [n_dens][2][n_trg])
 *      out_grad [n_dens][2][n_trg]   (d/dx, d/dy; Stokes: [n_dens][4][n_trg]
 *                                     = du1/dx, du1/dy, du2/dx, du2/dy)
 *  - Points may lie anywhere; they are wrapped into the cell (the sum is
 *    periodic). Outputs are in the caller's frame and are OVERWRITTEN.
 *  - Laplace and Stokes return the zero-cell-mean solution (the paper
 *    leaves the additive constant free, Sec. 4); densities must be
 *    neutral (sum_j q_j = 0, eq. chargeneutral; sum_j f_j = 0 for Stokes).
 *  - self_exclude = 1 means target i IS source i (n_trg == n_src and the
 *    same coordinates): the term (j = i, zero lattice vector) is left out.
 *    A target that coincides exactly with another source or source image
 *    is a singularity of the sum; such inputs are not supported.
 *  - Evaluation is asynchronous on the caller's HIP stream. Scratch memory
 *    comes from `workspace`, of at least pfmm_workspace_bytes() bytes,
 *    256-byte aligned. Device allocations: the plan's small table (a few
 *    KB): pfmm_plan_upload makes it, and the first pfmm_eval on a device
 *    calls pfmm_plan_upload itself (hipMalloc plus a synchronous copy) when
 *    the table is not there yet; and, for evaluations whose near part takes
 *    the FMM, its interaction-list tables (FP64 kernel samples per level and
 *    box-offset class: every Laplace and Yukawa level with at least 64
 *    boxes, the FP64-sampled Stokes levels; MB to at most 1 GiB, one set per
 *    plan): the first evaluation of a tree size allocates them and builds
 *    them on its stream, a later evaluation with another tree (see
 *    pfmm_fmm_tree) frees and rebuilds them. Other evaluations allocate
 *    nothing. A plan must not be evaluated on two streams at once
 *    with sizes that give different FMM trees.
 *  - n_src and n_trg (per cell in a batch) are at most PFMM_MAX_POINTS
 *    (point indices are 32-bit inside the kernels); larger sizes are
 *    PFMM_EINVAL, and pfmm_workspace_bytes* return 0 for them.
 *  - Return value 0 on success, a negative PFMM_E* code otherwise; on an
 *    argument error nothing is launched and outputs are untouched.
 */
#ifndef PFMM_H
#define PFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { PFMM_LAPLACE = 0, PFMM_YUKAWA = 1, PFMM_STOKES = 2 } pfmm_kernel;
typedef enum { PFMM_FP64 = 0, PFMM_MIXED = 1 } pfmm_precision;
typedef enum { PFMM_FAR_AUTO = 0, PFMM_FAR_DIRECT = 1, PFMM_FAR_NUFFT = 2 } pfmm_far_mode;

#define PFMM_MAX_POINTS ((int64_t)1 << 30)

enum {
  PFMM_OK = 0,
  PFMM_EINVAL = -1,          /* bad argument (NULL, negative size, ...)      */
  PFMM_EINVAL_LATTICE = -2,  /* e1, e2 not finite or linearly dependent      */
  PFMM_EINVAL_TOL = -3,      /* tol outside [1e-14, 1e-2]                    */
  PFMM_EWORKSPACE = -4,      /* workspace NULL, too small or misaligned      */
  PFMM_EHIP = -5,            /* a HIP runtime call failed                    */
  PFMM_ENOT_NEUTRAL = -6,    /* check_neutral set and densities not neutral  */
  PFMM_ENOMEM = -7           /* plan tables could not be allocated           */
};

typedef struct {
  double beta;        /* Yukawa parameter (> 0); ignored otherwise. Yukawa     */
                      /* near-field pairs farther apart than r_c, with         */
                      /* e^{-beta r_c} = eps / 30, are dropped (a truncation   */
                      /* of the same order as the far field's)                 */
  int precision;      /* pfmm_precision: FP64 everywhere, or MIXED (near-field  */
                      /* pair arithmetic in FP32 on coordinate differences     */
                      /* taken in FP64, short FP32 sums (over 16 sources or a  */
                      /* pair's images) combined with the FP64 densities in    */
                      /* FP64, log terms from FP32 log2 of r^2 products added  */
                      /* in FP64; FMM near part: kernel samples in FP32 on the */
                      /* two finest levels (every level for Yukawa), every     */
                      /* expansion and sum in FP64;                            */
                      /* the far field (coefficients, weights, plane waves at  */
                      /* the targets) in FP64)                                 */
  int far_mode;       /* pfmm_far_mode: AUTO uses the NUFFT when 2M+1 >= 256   */
  int m0;             /* near-region half width in e1 (Def. 1); 0 = automatic  */
  int n_dens;         /* number of density vectors evaluated together (>= 1)   */
  int self_exclude;   /* 1: target i is source i                               */
  int m_gl;           /* Gauss-Legendre lines for the NUFFT path; 0 = automatic*/
  int check_neutral;  /* 1: pfmm_eval syncs the stream and rejects non-neutral */
                      /*    Laplace/Stokes densities with PFMM_ENOT_NEUTRAL;   */
                      /*    the sync and host copy cannot run under stream     */
                      /*    capture, and pfmm_batch_create rejects such plans  */
  int profile;        /* 1: record HIP events around the near-field launches   */
                      /*    and the whole evaluation (see pfmm_plan_stage_times)*/
  int near_mode;      /* pfmm_near_mode: AUTO evaluates each pair of a         */
                      /* self-target plan once for both of its points (the     */
                      /* kernel is symmetric, Sec. 1 eq. psum); ONE_SIDED      */
                      /* always sums per target; MUTUAL needs self_exclude;    */
                      /* NONE leaves the near images out: the outputs are the  */
                      /* far part alone, the periodizing operator P applied to */
                      /* the densities (Sec. 1, eq. peropdef; Sec. 6). Batches */
                      /* reject NONE plans. FMM evaluates the near images by a */
                      /* fast multipole method on a tree of boxes in lattice   */
                      /* coordinates whose image boxes share the cell boxes'   */
                      /* expansions (the remark of Sec. 7): Chebyshev          */
                      /* interpolants of P x P points per box (P from tol and  */
                      /* the kernel, see pfmm_plan_info_t.fmm_order), direct   */
                      /* sums over neighbouring leaf boxes; O(N) work instead  */
                      /* of the direct sum's 3 (2 m0 + 1) N_S N_T. Doubly      */
                      /* periodic plans only; batches evaluate the near part  */
                      /* directly and reject FMM plans. AUTO takes the FMM for */
                      /* doubly periodic evaluations with N_S N_T >= 2^32      */
                      /* (its error is then that of the interpolation, kept   */
                      /* below tol / 10, instead of rounding alone)            */
  int periodic;       /* 2 (or 0): doubly periodic in e1 and e2 (operator P2). */
                      /* 1: singly periodic in e1 alone (operator P1, Sec. 3   */
                      /* eq. ksplitting1): images m e1 only, near part the     */
                      /* cell and its 2 neighbours, far part the west/east     */
                      /* columns (Thm. west_thm and its Laplace/Stokes forms   */
                      /* with one row). e2 then only sets the strip height:    */
                      /* points must lie within half of e2's extent across e1 */
                      /* of the line through the origin along e1 (outside it   */
                      /* the west/east rule is not accurate). Laplace and      */
                      /* Stokes sums are the symmetric limits over |m| <= M    */
                      /* (neutral densities); no additive constant is removed. */
                      /* Batches reject P1 plans; the NUFFT does not apply     */
  int ew_rule;        /* west/east quadrature in the canonical frame: 0 = the  */
                      /* Gauss-Legendre panel rule compressed by pivoted QR    */
                      /* node selection and least-squares weights (kept only   */
                      /* if it reproduces the panel rule to eps on a check     */
                      /* set), 1 = the panel rule as built                     */
} pfmm_opts;

typedef enum { PFMM_NEAR_AUTO = 0, PFMM_NEAR_ONE_SIDED = 1, PFMM_NEAR_MUTUAL = 2,
               PFMM_NEAR_NONE = 3, PFMM_NEAR_FMM = 4 } pfmm_near_mode;

/* Read-only description of a plan (host struct). */
typedef struct {
  int kernel, precision, far_mode_used, m0, n_dens, self_exclude;
  double d, xi, eta;          /* canonical lattice e1 = (d, 0), e2 = (xi, eta) */
  double rot_cos, rot_sin;    /* canonical = R * user, R = [[c, -s], [s, c]]   */
  double eps;                 /* internal truncation tolerance (tol / 10)      */
  int n_modes;                /* M: south/north modes m = -M..M (eq. mpk0s);
                                 0 for singly periodic plans (no rows)        */
  int n_quad;                 /* west/east quadrature nodes                    */
  int m_gl, nufft_nf, nufft_w;/* NUFFT lines, fine grid size, kernel width     */
  int n_images;               /* near images (2 m0 + 1) * 3                    */
  int n_log_groups;           /* mixed symmetric near field: image groups whose
                                 r^2 product shares one log2 (1, 3 or n_images) */
  int periodic;               /* 2: doubly periodic, 1: singly periodic in e1   */
  int ew_rotated;             /* 1: west/east waves along e2-perp (Appendix A)  */
  double ew_cos, ew_sin;      /* canonical -> west/east frame: x' = c x - s y,
                                 y' = s x + c y (identity when ew_rotated = 0)  */
  int fmm_order;              /* Chebyshev points per box dimension of the FMM
                                 near part (0: the plan never takes it)        */
  int fmm_symmetric;          /* 1: its leaves evaluate each pair of
                                 neighbouring boxes once for both (targets =
                                 sources; pfmm_tuning_t.fmm_leaves)             */
} pfmm_plan_info_t;

typedef struct pfmm_plan_s* pfmm_plan_t;

/* Build a plan (host only; no device work). e1, e2: host double[2], the
 * lattice vectors in the caller's frame (any basis of the lattice; it is
 * reduced and rotated so that e1 = (d, 0), |e2| <= d, |xi| <= d/2 as in
 * Sec. 1). tol: requested relative accuracy in [1e-14, 1e-2]. opts may be
 * NULL (FP64, AUTO far mode, n_dens 1). On success *out receives a plan
 * that pfmm_destroy releases. */
int pfmm_plan(int kernel, const double* e1, const double* e2, double tol,
              const pfmm_opts* opts, pfmm_plan_t* out);

/* Copy the plan's tables to the current HIP device (synchronous). Done
 * implicitly by the first pfmm_eval on a device; call it beforehand when
 * the first evaluation happens inside stream capture. */
int pfmm_plan_upload(pfmm_plan_t plan);

/* Host: fill *info. */
int pfmm_plan_get_info(pfmm_plan_t plan, pfmm_plan_info_t* info);

/* Host: copy the west/east quadrature rule (nodes lambda_k and weights
 * w_k, host arrays of plan->n_quad doubles each) used by Thm. west_thm /
 * west_thm_lap / west_thm_s. Either pointer may be NULL. */
int pfmm_plan_get_quadrature(pfmm_plan_t plan, double* nodes, double* weights);

/* Host: the image groups of the mixed symmetric near field (Def. 1 near
 * region, images ordered row by row: n = -1, 0, 1 outer, m = -m0..m0
 * inner): ends[g] is one past the last image of group g and e0[g] the
 * exponent its FP32 r^2 product starts at (2^e0), for g < n_log_groups
 * (pfmm_plan_get_info); host int arrays of at least n_log_groups entries.
 * Either pointer may be NULL. */
int pfmm_plan_get_log_groups(pfmm_plan_t plan, int* ends, int* e0);

/* Host: the NUFFT spreading kernel as the device evaluates it (Sec. 6.1):
 * the exponential of semicircle phi(z) = exp(beta_es (sqrt(1 - z^2) - 1))
 * at the w + 1 taps of a point, each tap t a polynomial
 * sum_k coef[t * 20 + k] u^k of degree *deg - 1 in u = 2f - 1, where f in
 * [0, 1) is the offset of the first tap (see the plan's nufft_w). coef: host
 * array of 17 * 20 doubles (unused entries zero); any pointer may be NULL. */
int pfmm_plan_get_spread_kernel(pfmm_plan_t plan, double* coef, int* deg, double* beta_es);

/* Profiling plans only (opts.profile = 1): wait for the events recorded by
 * every pfmm_eval since the last call, and return the summed GPU time of
 * the near-field kernel launches (*near_ms), of whole evaluations
 * (*total_ms) and the number of evaluations (*n_evals); then forget them.
 * Host pointers; any may be NULL. */
int pfmm_plan_stage_times(pfmm_plan_t plan, double* near_ms, double* total_ms, int* n_evals);

/* Profiling plans only: the same for the stages of the FMM near part of
 * every pfmm_eval that took it since the last call (events on the
 * evaluation's stream between the launches): stage_ms[0] upward pass
 * (equivalent densities of the leaves and of every coarser level),
 * [1] interaction lists whose kernel samples are FP64, [2] those sampled in
 * FP32 (mixed plans: the two finest levels), [3] downward pass (local fields
 * interpolated level to level), [4] leaves (local fields at the targets plus
 * the neighbouring leaves' direct sums). Host pointers; stage_ms holds 5
 * doubles; either may be NULL. */
int pfmm_plan_fmm_stage_times(pfmm_plan_t plan, double* stage_ms, int* n_evals);

/* Host: whether an evaluation with these sizes takes the FMM near part, and
 * its tree: out[0] = 1 if so (else 0 and the rest 0), out[1] = leaf level
 * L, out[2], out[3] = top boxes k1 x k2 (level l has (k1 2^l) x (k2 2^l)
 * boxes over the cell in lattice coordinates), out[4] = Chebyshev points per
 * box dimension. out: host int[5]. */
int pfmm_fmm_tree(pfmm_plan_t plan, int64_t n_src, int64_t n_trg, int* out);

/* Workspace size in bytes for pfmm_eval with these sizes. */
size_t pfmm_workspace_bytes(pfmm_plan_t plan, int64_t n_src, int64_t n_trg);

/* Evaluate potentials and gradients (see the conventions above). out_pot
 * or out_grad may be NULL to skip that output. hip_stream: hipStream_t
 * (NULL = default stream). n_src = 0 is allowed: the outputs are set to
 * zero (src_xy and dens may then be NULL). n_trg = 0 (or both outputs NULL)
 * returns PFMM_OK with nothing launched. */
int pfmm_eval(pfmm_plan_t plan, int64_t n_src, const double* src_xy, const double* dens,
              int64_t n_trg, const double* trg_xy, double* out_pot, double* out_grad,
              void* workspace, size_t workspace_bytes, void* hip_stream);

/* Allocation-free evaluation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc). Same arguments and results as pfmm_eval, without the
 * workspace: scratch memory is a fixed device array of
 * PFMM_STATIC_WORKSPACE_BYTES inside the library, one per device, held
 * until the process ends. Sizes whose pfmm_workspace_bytes() exceeds it
 * return PFMM_EWORKSPACE. The plan's table must already be on the current
 * device (call pfmm_plan_upload at set-up), else PFMM_EINVAL; plans with
 * check_neutral or profile set are PFMM_EINVAL too (those options copy to
 * the host or create events). Nothing is allocated and nothing
 * synchronises: an FMM near part uses the plan's interaction-list tables
 * when they were built for this tree size (by a pfmm_eval of the same
 * sizes), else samples the kernel for every level (same results to
 * rounding, slower). All calls on one device share that device's array and the
 * array keeps the last call's contents (every evaluation rewrites what it
 * reads), so calls that overlap in time on one device -- different streams,
 * or host threads -- race and give wrong results: order them on one
 * stream. */
#define PFMM_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int pfmm_eval_static(pfmm_plan_t plan, int64_t n_src, const double* src_xy, const double* dens,
                     int64_t n_trg, const double* trg_xy, double* out_pot, double* out_grad,
                     void* hip_stream);

/* Adjoint for targets == sources (plans with self_exclude = 1 and n_dens = 1,
 * any kernel). With pot = K q the potential at the sources and g = dL/dpot
 * (device, laid out like out_pot: [n_src], Stokes [2][n_src]) for a loss L,
 * writes
 *   out_dq  (like dens)  = dL/dq_j = sum_i g_i K(t_i, s_j) = u[g](x_j)
 *   out_dxy [2][n_src]   = dL/dx_j = g_j grad u[q](x_j) + q_j grad u[g](x_j)
 *                          (Stokes: summed over the two velocity components)
 * using the symmetry of the periodic kernel (Sec. 1, eq. psum). For Laplace
 * and Stokes, g is first projected onto neutral vectors (its mean is
 * removed), which is exact when L does not depend on the free constant of
 * the potential (e.g. the energy 1/2 q.pot); out_dq is not projected.
 * Workspace: at least pfmm_workspace_bytes_adjoint() bytes. A plan must not
 * be used by two host threads at once. Either output may be NULL. */
size_t pfmm_workspace_bytes_adjoint(pfmm_plan_t plan, int64_t n_src);
int pfmm_eval_adjoint(pfmm_plan_t plan, int64_t n_src, const double* src_xy,
                      const double* dens, const double* g_pot, double* out_dq,
                      double* out_dxy, void* workspace, size_t workspace_bytes,
                      void* hip_stream);

/* Pressure of the periodic Stokeslet sum (Stokes plans only): the
 * Stokeslet's pressure p = (1/2pi) r.f/r^2 (Sec. 5.2, eq. stokeslet; the
 * pressurelet of Thms. south_thm_stokes_pressure and west_thm_stokes_pressure)
 * summed over the same images as the velocity, with zero cell mean (doubly
 * periodic) or as the symmetric limit along e1 (singly periodic). Arguments
 * as for pfmm_eval with the Stokes plan's forces; out_pres [n_dens][n_trg]
 * (device) is overwritten. It is evaluated as -div of the periodic Laplace
 * gradient with the force components as charges (a Laplace plan of the same
 * lattice and options that every Stokes plan holds), so its cost is that of
 * one Laplace evaluation with 2 n_dens densities. Workspace: at least
 * pfmm_workspace_bytes_pressure() bytes. Other plans: PFMM_EINVAL. */
size_t pfmm_workspace_bytes_pressure(pfmm_plan_t plan, int64_t n_src, int64_t n_trg);
int pfmm_eval_pressure(pfmm_plan_t plan, int64_t n_src, const double* src_xy, const double* dens,
                       int64_t n_trg, const double* trg_xy, double* out_pres, void* workspace,
                       size_t workspace_bytes, void* hip_stream);

/* Batched evaluation of many independent cells. plans[c] (n_cells of them)
 * must share precision, n_dens and self_exclude, and be all scalar kernels
 * (Laplace/Yukawa, mixed freely) or all Stokes. src_off/trg_off (host
 * int64[n_cells + 1], starting at 0; trg_off ignored and may be NULL for
 * self_exclude plans) give each cell's range in concatenated device arrays:
 *   src_xy [2][S], dens [n_dens][S] (Stokes [n_dens][2][S]), trg_xy [2][T],
 *   out_pot [n_dens][T] (Stokes [n_dens][2][T]), out_grad [n_dens][2|4][T]
 * with S = src_off[n_cells], T = trg_off[n_cells]. The near fields of all
 * cells run in one persistent launch over (cell, target tile, source split)
 * tasks; each cell's far field follows (Sec. 6). Creation uploads the plans'
 * tables and a task table to the device; use_graph = 1 captures the whole
 * launch sequence into a hipGraph on the first pfmm_eval_batch call (and
 * again whenever a pointer argument changes) and replays it afterwards.
 * The plans must outlive the batch. Plans with check_neutral set are
 * rejected (PFMM_EINVAL). Changing the NUFFT grid of a plan held by a batch
 * (pfmm_plan_set_tuning, pfmm_autotune) changes that cell's workspace: the
 * next pfmm_batch_workspace_bytes or pfmm_eval_batch call rebuilds the
 * batch's layout and task table (host work, hipMalloc and a synchronous
 * copy; not under stream capture) and drops its graph, and pfmm_eval_batch
 * then returns PFMM_EWORKSPACE if the workspace passed is now too small:
 * read pfmm_batch_workspace_bytes again after retuning a plan. */
typedef struct pfmm_batch_s* pfmm_batch_t;
int pfmm_batch_create(int n_cells, const pfmm_plan_t* plans, const int64_t* src_off,
                      const int64_t* trg_off, int use_graph, pfmm_batch_t* out);
size_t pfmm_batch_workspace_bytes(pfmm_batch_t batch);
int pfmm_eval_batch(pfmm_batch_t batch, const double* src_xy, const double* dens,
                    const double* trg_xy, double* out_pot, double* out_grad,
                    void* workspace, size_t workspace_bytes, void* hip_stream);
void pfmm_batch_destroy(pfmm_batch_t batch);

/* Launch-shape tuning (host struct). The choices change only how the work
 * is split across the GPU and the NUFFT grid; the NUFFT kernel width is
 * chosen by the library for each grid so that the plan's tolerance holds. */
typedef struct {
  int64_t near_blocks;  /* near field: target number of blocks in flight (0 = default: 2048 for the
                           one-sided sum, 8192 for the symmetric one) */
  int nufft_grid;       /* NUFFT path: 0 = smallest power-of-two grid >= 2(2M+1) with width
                           ceil(log10(1/eps)) + 1; 1 = twice that grid, one point narrower */
  int fmm_level;        /* FMM near part: leaf level of the tree, 1..11 (its leaves are the
                           k1 x k2 top boxes split 4^level times); 0 = from a cost model of
                           neighbour pairs against interaction-list node pairs */
  int fmm_leaves;       /* FMM near part with targets = sources (self_exclude): 2 = symmetric
                           leaves, each pair of a leaf box and one of its four forward
                           neighbours (the row above, the box to the right) evaluated once
                           for the points of both boxes; 1 = one-sided, every box against
                           its 3 x 3 neighbours; 0 = symmetric except for mixed Stokes
                           (whose FP32 pair costs less than the extra terms). Same results
                           to rounding; symmetric leaves need 4 n_dens NOUT n doubles more
                           workspace */
} pfmm_tuning_t;

/* Host: read or set a plan's tuning. nufft_grid = 1 is rejected (PFMM_EINVAL)
 * when the doubled grid would exceed 2^20 points per line. Not while an evaluation with
 * this plan is being captured into a graph. */
int pfmm_plan_get_tuning(pfmm_plan_t plan, pfmm_tuning_t* tuning);
int pfmm_plan_set_tuning(pfmm_plan_t plan, const pfmm_tuning_t* tuning);

typedef struct {
  int n_tried;          /* configurations timed */
  double default_ms;    /* GPU time of one evaluation with the tuning in place before the call */
  double best_ms;       /* the same for the chosen tuning */
} pfmm_tune_report_t;

/* Autotuner: times candidate tunings (near_blocks, or for an FMM near part
 * the leaf levels next to the cost model's and, when the targets are the
 * sources, the other leaf form; for NUFFT plans both grids) on
 * the caller's inputs with HIP events, keeps the fastest in the
 * plan and leaves the result of an evaluation with it in out_pot/out_grad.
 * Arguments as for pfmm_eval; candidates that would need more than
 * workspace_bytes are skipped. Synchronises hip_stream; not for use under
 * stream capture. report (host) may be NULL. */
int pfmm_autotune(pfmm_plan_t plan, int64_t n_src, const double* src_xy, const double* dens, int64_t n_trg,
                  const double* trg_xy, double* out_pot, double* out_grad, void* workspace,
                  size_t workspace_bytes, void* hip_stream, pfmm_tune_report_t* report);

/* Batched autotuner: times task lengths (4096, 8192, 16384 sources) and
 * persistent grid sizes (2, 4, 8 blocks per compute unit) of a batch on the
 * caller's inputs, keeps the fastest and leaves its result in the outputs.
 * The batch's workspace size may change: read pfmm_batch_workspace_bytes
 * again afterwards (candidates larger than workspace_bytes are skipped, so
 * the chosen one fits the workspace passed here). */
int pfmm_batch_autotune(pfmm_batch_t batch, const double* src_xy, const double* dens, const double* trg_xy,
                        double* out_pot, double* out_grad, void* workspace, size_t workspace_bytes,
                        void* hip_stream, pfmm_tune_report_t* report);

void pfmm_destroy(pfmm_plan_t plan);
const char* pfmm_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* PFMM_H */
