/*
 * fmgsr.h -- C ABI of the MI355X (gfx950) FMG-FAS-SR solver for the 1D model
 * problem.
 *
 * Method: M. F. Adams, "A low memory, highly concurrent multigrid algorithm"
 * (arXiv:1207.6720).  One full-multigrid (FMG) cycle with the full
 * approximation scheme (FAS, Sec. 2.2, Eqs. 1-2, Fig. 1) and segmental
 * refinement (SR, Sec. 2.4 and Sec. 3, Fig. 3): the finest level is cut into
 * segments with buffer cells, smoothed segment by segment without ever being
 * stored, restricted with the tau-correction of Eq. 7, and rebuilt on the way
 * up by the full update of Eq. 5 with the fourth-order FMG interpolation and
 * compatible (Kaczmarz) relaxation (Sec. 3.1, Eq. 8, Fig. 5).
 *
 * Problem (Sec. 4): -u'' = f on [0,1], u(0) = g_left, u(1) = g_right, second
 * order cell-centred finite volumes on n cells (cell i centred at
 * (i + 1/2)/n).  Level l of L = `levels` grids has n >> (L-1-l) cells; the
 * coarsest has N0 = n >> (L-1) cells and is solved exactly.
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers to contiguous FP64 data owned by the
 *    caller; the library never frees them.  Host pointers are rejected.
 *  - Calls are asynchronous and ordered on `hip_stream` (a hipStream_t; NULL
 *    is the default stream): they validate, enqueue and return.  Results are
 *    ready when the stream is synchronised.  A device fault surfaces as
 *    FMGSR_EDEVICE from the next call or from the stream synchronisation.
 *  - Invalid arguments return FMGSR_EINVAL before anything is enqueued.
 *  - No C++ exception crosses the ABI.
 *  - Calls on different streams may run concurrently provided each has its
 *    own workspace (or lets the library allocate one).
 */
#ifndef FMGSR_H
#define FMGSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMGSR_OK = 0,
  FMGSR_EINVAL = -1,   /* argument out of range; nothing enqueued            */
  FMGSR_ENOMEM = -2,   /* workspace allocation failed or workspace too small */
  FMGSR_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed         */
  FMGSR_ENOTSUP = -4,  /* valid request this library does not implement     */
  FMGSR_ENONFINITE = -5 /* fmgsr_options.check_finite: NaN or Inf in the
                           input (nothing solved) or in the result          */
} fmgsr_status;

/* How tau (Eq. 7) enters the coarse right-hand side (Eq. 6).
 * SPLIT: with the average solution restriction and the full-weighting
 *   residual restriction, L_H(I^ u) = I(L_h u) holds identically, so the
 *   Laplacian part of tau is exactly zero and f^H = I f^h; only non-Laplacian
 *   operator parts would contribute.  Equal to LITERAL in exact arithmetic
 *   and free of its O(eps n^2 |u|) cancellation noise.
 * LITERAL: f^H = I(f^h - L_h u^h) + L_H(I^ u^h), evaluated as written (on SR
 *   levels per patch, from the patch's extended iterate, Fig. 3 step 4). */
enum { FMGSR_TAU_SPLIT = 0, FMGSR_TAU_LITERAL = 1 };

/* Operator kinds.
 * POISSON          -u'' = f (Sec. 4).
 * CUBIC_REACTION   -u'' + kappa(x) u^3 = f: the nonlinear problem FAS is made
 *                  for (Sec. 2.2, Eqs. 1-2); smoother = red-black nonlinear
 *                  Gauss-Seidel (one Newton step per point), coarse
 *                  coefficient = two-cell average, coarsest level = Newton
 *                  with exact tridiagonal steps.
 * LINEAR_REACTION  -u'' + c(x) u = f (kappa holds c >= 0); the operator of the
 *                  adjoint of the cubic problem.
 * With the reaction kinds tau (Eq. 7) is nonzero: its Laplacian part cancels
 * exactly (see FMGSR_TAU_SPLIT) and the reaction part R_H(I^ u) - I R_h(u)
 * is added to every coarse right-hand side. */
enum { FMGSR_OP_POISSON = 0, FMGSR_OP_CUBIC_REACTION = 1, FMGSR_OP_LINEAR_REACTION = 2 };

/* Arithmetic of the smoother.  FP64: everything in FP64.  FP32_RELAX: each
 * smoother call forms the FP64 residual once, runs its sweeps on an FP32
 * correction (exterior correction 0; the same iteration in exact
 * arithmetic) and adds it to the FP64 iterate; residuals, tau, transfers and
 * the coarsest solve stay FP64.  In fmgsr_solve the levels handled by the
 * single-workgroup coarse core (at most 2048 cells) also relax in FP64, and
 * FP32_RELAX with FMGSR_TAU_LITERAL returns FMGSR_ENOTSUP: literal tau applies
 * L_h to the iterate, which amplifies the FP32 rounding by ~n^2 into every
 * coarse right-hand side (at n = 2^16 the result misses a tenth of the
 * discretisation error by 2.4x). */
enum { FMGSR_FP64 = 0, FMGSR_FP32_RELAX = 1 };

/* Restriction I of right-hand sides and residuals (Eq. 6, Eq. 7).
 * FULLWEIGHT: full weighting, 1/2 of the transposed linear prolongation (the
 *   appendix's commented alternative); with the average solution restriction
 *   I^ it satisfies L_H I^ = I L_h exactly, which split tau relies on.
 * AVERAGE: the two-cell average, the appendix's choice for both
 *   restrictions (the paper's own transfer pair, Sec. 4); literal tau only
 *   (FMGSR_EINVAL with split tau, where that identity fails). */
enum { FMGSR_R_FULLWEIGHT = 0, FMGSR_R_AVERAGE = 1 };

typedef struct {
  int32_t kind;          /* FMGSR_OP_*                                        */
  const double *kappa;   /* fmgsr_solve / fmgsr_adjoint: [n] coefficient at
                            the cell centres (device), NULL for POISSON       */
} fmgsr_operator;

typedef struct {
  int32_t nu1;           /* pre-smoothing sweeps per smoother call (>= 0)     */
  int32_t nu2;           /* post-smoothing sweeps per smoother call (>= 0)    */
  int32_t sr_levels;     /* number k of SR levels, 0..levels-1.  1: the
                            finest level is an SR level (block smoother,
                            full update + compatible relaxation, never
                            stored); k >= 2: the k finest levels are (Sec. 4
                            studies 0-3), each pre-smoothed by the block
                            smoother and post-smoothed by the full update +
                            CR, the ones below the finest stored; split tau
                            only (literal: FMGSR_ENOTSUP); 0: plain FMG-FAS
                            with every level stored                          */
  int32_t tau_mode;      /* FMGSR_TAU_SPLIT or FMGSR_TAU_LITERAL              */
  void *workspace;       /* device scratch of >= fmgsr_workspace_bytes()
                            bytes, or NULL: the library then allocates and
                            frees it stream-ordered around the call            */
  size_t workspace_bytes;
  int32_t precision;     /* FMGSR_FP64 or FMGSR_FP32_RELAX                    */
  int32_t reserved;      /* must be 0                                         */
  double *functionals;   /* fmgsr_solve with sr_levels >= 1: NULL, or a device
                            array [2] that receives h sum u and h sum u^2 of
                            the finest-level result, accumulated segment by
                            segment while the SR up pass rebuilds u (Sec. 3.2:
                            the fine solution is only needed for functionals;
                            summation order fixed, so results repeat bit for
                            bit).  With functionals set, u_out may be NULL and
                            the fine solution is never written.  Needs a
                            segment core of at least 4 cells.                 */
  double *coarse_out;    /* fmgsr_solve with sr_levels = 1: NULL, or a device
                            array [n/2] that receives the level-(M-1)
                            solution of the final V-cycle, from which the SR
                            up pass rebuilds the finest level (Eq. 5, Fig. 5).
                            With f it is the PDE-compressed solution (Sec. 2.4)
                            that fmgsr_decompress expands on demand (Sec. 3.2,
                            method 2).  With coarse_out set, u_out (and
                            functionals) may be NULL: the SR up pass is then
                            skipped.  Other sr_levels: FMGSR_ENOTSUP.         */
  int32_t rhs_restriction; /* FMGSR_R_FULLWEIGHT (default) or FMGSR_R_AVERAGE */
  int32_t check_finite;  /* 0 (default), or 1: fmgsr_solve scans f before
                            solving and returns FMGSR_ENONFINITE, having
                            solved nothing, if it holds a NaN or Inf, and
                            scans the results (u_out, coarse_out,
                            functionals) afterwards, returning
                            FMGSR_ENONFINITE if one is not finite.  The call
                            then synchronises hip_stream (not capturable).   */
} fmgsr_options;

/* Defaults: V(2,1), sr_levels = 1, split tau, FP64, library-managed
 * workspace. */
void fmgsr_default_options(fmgsr_options *opt);

/* Bytes of device workspace fmgsr_solve needs for these sizes and options,
 * whatever the segments (0 if the arguments are invalid). */
size_t fmgsr_workspace_bytes(int64_t n, int32_t levels, const fmgsr_options *opt);

/* The same for these segments and buffer exactly (0 if invalid); never more
 * than fmgsr_workspace_bytes.  With one SR level, split tau, buffer >=
 * 2 nu1 - 1 and >= 2 nu2 and no functionals the SR passes run as the top
 * level of the vertical kernels and the restricted fine iterate (n/2
 * doubles) is never stored. */
size_t fmgsr_workspace_bytes_for(int64_t n, int32_t levels, int64_t n_segments, int32_t buffer,
                                 const fmgsr_options *opt);

/* Largest dynamic LDS (bytes) one workgroup of fmgsr_solve requests for
 * these sizes, segments and options (0 if invalid): the single-workgroup
 * coarse core holds the level stack of the coarsest levels (Fig. 1's exact
 * solve and the V-cycle bottoms), the segment kernels a register stage and
 * exchange buffer per thread.  fmgsr_solve grants each of those kernels the
 * device's per-workgroup LDS limit (at most 160 KiB) less the kernel's static
 * LDS, and returns FMGSR_EINVAL, before enqueuing anything, when a request
 * exceeds its kernel's grant; FMGSR_EDEVICE when a grant itself failed. */
size_t fmgsr_launch_lds_bytes(int64_t n, int32_t levels, int64_t n_segments, int32_t buffer,
                              const fmgsr_options *opt);

/*
 * fmgsr_solve -- one FMG-FAS-SR iteration (Fig. 3) for -u'' = f.
 *
 *   op          operator descriptor (NULL = Poisson).  The reaction kinds
 *               run as a batch of one problem (fmgsr_solve_batched: one
 *               workgroup, N0 <= 256) and return after the stream has
 *               finished the solve.
 *   f           [n] right-hand side at the cell centres of the finest level.
 *   g_left,
 *   g_right     Dirichlet values u(0), u(1).
 *   n           finest cells; n % 2^(levels-1) == 0 and N0 = n >> (levels-1)
 *               <= 1024.
 *   levels      number of grids, 1..40.
 *   n_segments  SR segments on each SR level (used when sr_levels >= 1):
 *               n % n_segments == 0, the core s = n / n_segments is even, and
 *               s + 2 (buffer + 2) <= 8192; on the k-th SR level below the
 *               finest the core is s / 2^k, which must be an even integer.
 *   buffer      buffer (halo) cells on each side of a segment, 0..1024; each
 *               segment is smoothed on [i s - buffer, (i+1) s + buffer)
 *               clipped to the domain, with the exterior frozen, and only its
 *               core is kept (additive block Jacobi, Sec. 3).
 *   opt         options (NULL = defaults); nu1, nu2 in 0..16; sr_levels in
 *               0..levels-1.
 *   u_out       [n] result: the finest-level solution after the cycle,
 *               written once as it is produced (Sec. 3.2, streaming); may be
 *               NULL when opt->functionals is set.
 *   hip_stream  stream to enqueue on.
 *
 * Smoother: red-black Gauss-Seidel (red = even cell index first, omega = 1).
 * Restrictions: solution = two-cell average, rhs/residual = full weighting.
 * Returns FMGSR_OK once enqueued.
 */
fmgsr_status fmgsr_solve(const fmgsr_operator *op, const double *f, double g_left,
                         double g_right, int64_t n, int32_t levels, int64_t n_segments,
                         int32_t buffer, const fmgsr_options *opt, double *u_out,
                         void *hip_stream);

/* Bytes of the static device scratch behind fmgsr_solve_noalloc (128 MiB on
 * every GPU the library runs on, held until the process ends): enough for
 * the workspace of n <= 2^22 with the default options. */
#define FMGSR_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/*
 * fmgsr_solve_noalloc -- fmgsr_solve for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine: its workspace is a static device array of
 * FMGSR_NOALLOC_SCRATCH_BYTES bytes, one per GPU, shared by every call on
 * that GPU.
 *
 * Arguments and results as fmgsr_solve, for the Poisson operator (op NULL or
 * FMGSR_OP_POISSON; the reaction kinds return FMGSR_ENOTSUP because their
 * batched plan allocates).  opt->workspace must be NULL and
 * opt->workspace_bytes 0 (else FMGSR_EINVAL).  Returns FMGSR_ENOMEM, before
 * enqueuing anything, when the solve's workspace
 * (fmgsr_workspace_bytes_for) exceeds FMGSR_NOALLOC_SCRATCH_BYTES.
 * Calls that overlap on one GPU (concurrent streams or host threads) race on
 * the shared scratch: serialise them.  The scratch keeps the last call's
 * contents; the solve writes every workspace cell before reading it.
 */
fmgsr_status fmgsr_solve_noalloc(const fmgsr_operator *op, const double *f, double g_left,
                                 double g_right, int64_t n, int32_t levels, int64_t n_segments,
                                 int32_t buffer, const fmgsr_options *opt, double *u_out,
                                 void *hip_stream);

/*
 * fmgsr_decompress -- PDE decompression (Sec. 3.2, method 2): the finest-level
 * solution on cells [lo, hi), expanded from the stored level-(M-1) solution
 * (fmgsr_options.coarse_out of a solve with one SR level) by the SR up pass
 * of the segments whose cores meet [lo, hi): full update Pi c (Eq. 5), then
 * nu2 x [Kaczmarz projection onto I^ u = c (Eq. 8, Fig. 5), red-black sweep]
 * on each extended patch with its exterior frozen.  Only local data is read:
 * the covering segments' patches of f and their coarse image.
 *
 *   coarse      [n/2] level-(M-1) solution (device).
 *   f           [n] finest right-hand side of the solve (device).
 *   g_left, g_right, n, n_segments, buffer
 *               as in the solve (n_segments divides n, even core).
 *   opt         nu2 and precision as in the solve (NULL = defaults); other
 *               fields ignored.
 *   lo, hi      0 <= lo <= hi <= n; hi == lo enqueues nothing.
 *   u_out       [hi - lo] receives u[lo..hi) (device).
 *
 * With the solve's segments, buffer and options the result equals that
 * solve's u_out on [lo, hi) bit for bit.  Asynchronous on hip_stream;
 * allocates nothing.
 */
fmgsr_status fmgsr_decompress(const double *coarse, const double *f, double g_left,
                              double g_right, int64_t n, int64_t n_segments, int32_t buffer,
                              const fmgsr_options *opt, int64_t lo, int64_t hi, double *u_out,
                              void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched solves: many independent problems of uneven size in ONE persistent
 * launch.  Every workgroup takes problems from an atomic queue (longest
 * first) and runs the whole FMG-FAS-SR iteration of each (Fig. 3); the
 * data-driven execution of Sec. 3 at problem granularity.
 *
 * Problem j has n_j fine cells (device arrays packed: its cells start at
 * offset_j), levels_j grids with N0_j = n_j >> (levels_j - 1) <= 256 coarsest
 * cells, Dirichlet values g[2j], g[2j+1], and (levels_j >= 2) an SR finest
 * level cut into segments of core s_j = n_j / segments_j with `buffer` cells
 * on each side (0..64).  A plan holds the descriptors, the launch shape and
 * the workspace (every problem's stored levels, about 5.5 n_j doubles), so
 * that executing it needs no allocation and no host-to-device copy.  When the
 * batch has fewer problems than resident workgroups, several workgroups
 * share each problem; they must all be resident at once, so such a plan
 * expects the device not to be shared with other long kernels (a bounded
 * wait turns a stall into the `stalled` flag instead of a hang).
 * ------------------------------------------------------------------------ */
typedef struct fmgsr_batch_s *fmgsr_batch;

typedef struct {
  int32_t threads;       /* workgroup size                                    */
  int32_t run;           /* cells per thread (window = threads * run)         */
  int32_t grid;          /* persistent workgroups                             */
  int32_t halo;          /* stored-level tile halo (cells)                    */
  int64_t lds_bytes;     /* LDS per workgroup                                 */
  int64_t workspace_bytes;
  int32_t group;         /* workgroups per problem (> 1 when the batch has
                            fewer problems than resident workgroups: they
                            split every large level's tiles and segments and
                            meet at a barrier between phases)                 */
  int32_t stalled;       /* 1 if a group barrier ever timed out (the results
                            of that execution are invalid); reading it
                            synchronises the device                           */
} fmgsr_batch_shape;

/*
 * fmgsr_batch_create -- validate a batch and build its plan (synchronous:
 * allocates device memory and uploads descriptors).
 *
 *   batch          number of problems, 1..2^24.
 *   n_host         [batch] fine cells per problem (host memory).
 *   offset_host    [batch] offsets (elements) into the packed arrays, or NULL
 *                  for back-to-back packing (prefix sums of n).
 *   levels_host    [batch] grids per problem (1..31).
 *   segments_host  [batch] SR segments per problem, or NULL: the library
 *                  picks the largest segment core N0 2^k whose extended patch
 *                  fits one workgroup window (threads x run cells: 256 x 4
 *                  when the batch has at least as many problems as CUs, else
 *                  512 x 8).  A given count must divide n_j, give an even
 *                  core and fit the largest window, 4096 cells (EINVAL
 *                  otherwise); the plan then takes a window it fits.
 *   buffer         SR buffer cells per side, 0..64.
 *   g_host         [2 batch] Dirichlet values (g_left, g_right) per problem,
 *                  or NULL for homogeneous data.
 *   op_kind        FMGSR_OP_*; kappa is passed at execution.
 *   opt            nu1, nu2 (0..16), precision; sr_levels must be 1,
 *                  tau_mode split and functionals NULL (others: ENOTSUP);
 *                  workspace ignored.
 *   out            receives the plan.
 */
fmgsr_status fmgsr_batch_create(int32_t batch, const int64_t *n_host, const int64_t *offset_host,
                                const int32_t *levels_host, const int64_t *segments_host,
                                int32_t buffer, const double *g_host, int32_t op_kind,
                                const fmgsr_options *opt, fmgsr_batch *out);

/* One FMG-FAS-SR iteration of every problem (asynchronous on hip_stream).
 * f_packed, kappa_packed (NULL for POISSON) and u_packed are device arrays
 * covering every problem's [offset_j, offset_j + n_j).  Executions of one
 * plan share its workspace: do not overlap them on different streams.  The
 * enqueued work is one reset kernel and one persistent kernel, so the call
 * can be captured into a HIP graph. */
fmgsr_status fmgsr_batch_solve(fmgsr_batch plan, const double *f_packed,
                               const double *kappa_packed, double *u_packed, void *hip_stream);

/* Adjoint of the cubic problem (plan made with FMGSR_OP_CUBIC_REACTION): for
 * a functional J(u) of the discrete solution u of -u'' + kappa u^3 = f,
 * lambda solves (L + diag(3 kappa u^2)) lambda = dJ/du with homogeneous
 * Dirichlet data (the matrix is symmetric), computed by one FMG-FAS-SR
 * iteration of the linear reaction problem with c = 3 kappa u_fwd^2 formed
 * on the fly on every level (nothing of the forward solve is stored but
 * u_fwd).  Outputs grad_f = lambda and grad_kappa = -u_fwd^3 lambda (either
 * may be NULL, not both). */
fmgsr_status fmgsr_batch_adjoint(fmgsr_batch plan, const double *kappa_packed,
                                 const double *u_fwd_packed, const double *dJdu_packed,
                                 double *grad_f_packed, double *grad_kappa_packed,
                                 void *hip_stream);

/* PDE compression of the batch (Sec. 2.4; Sec. 3.2): one FMG-FAS-SR
 * iteration that also keeps every problem's level-(M-1) solution V^{M-1}
 * (the last step's post-smoothed iterate below the SR level).  Problem j's
 * n_j/2 values go to coarse_packed[offset_j/2 .. offset_j/2 + n_j/2)
 * (integer division; problems of one grid keep nothing), so a packed
 * coarse array of half the packed length holds back-to-back problems.
 * u_packed as fmgsr_batch_solve, or NULL: then only V^{M-1} is produced
 * and the SR up pass is skipped.  The kept array together with f and kappa
 * determines the fine solution: fmgsr_batch_adjoint_compressed rebuilds it
 * from them.  Asynchronous on hip_stream; EINVAL for a non-device or
 * aliased array. */
fmgsr_status fmgsr_batch_solve_keep(fmgsr_batch plan, const double *f_packed,
                                    const double *kappa_packed, double *u_packed,
                                    double *coarse_packed, void *hip_stream);

/* fmgsr_batch_adjoint without u_fwd (Sec. 2.4: levels are recomputed, not
 * stored): wherever the adjoint needs 3 kappa u_fwd^2 on the finest level
 * (its forcing and both SR passes), u_fwd is rebuilt segment by segment by
 * the forward's own SR up pass (Eq. 5, Fig. 5) from f_fwd_packed, kappa and
 * coarse_fwd_packed (a fmgsr_batch_solve_keep of the same plan and inputs);
 * a window's buffer cells come from the neighbouring segments' rebuilds.
 * The rebuilt u_fwd equals the forward's bit for bit, so the gradients
 * equal fmgsr_batch_adjoint's on that forward's u.  Costs seven forward SR
 * up passes per adjoint; saves holding n doubles of u_fwd (the kept level
 * is n/2).  ENOTSUP unless the plan is cubic and every problem's segment
 * core is at least the window pad ((buffer + 2) rounded down to even). */
fmgsr_status fmgsr_batch_adjoint_compressed(fmgsr_batch plan, const double *kappa_packed,
                                            const double *f_fwd_packed,
                                            const double *coarse_fwd_packed,
                                            const double *dJdu_packed, double *grad_f_packed,
                                            double *grad_kappa_packed, void *hip_stream);

/* Project autotuner: times the plan's candidate launch shapes (workgroup
 * size 256 or 512, 4 or 8 cells per thread, workgroups per problem 1..16
 * when the batch is small) and segment sizes (the largest fitting core and
 * half of it, unless segments were given) on these inputs, keeps the fastest
 * and returns its time per solve in *ms_out (may be NULL).  With the
 * environment variable FMGSR_AUTOTUNE_LOG=1 every candidate's time is
 * printed to stderr.  Synchronises hip_stream;
 * u_scratch_packed is overwritten.  Segment sizes change the SR iterate
 * (within the method's accuracy); fmgsr_batch_query reports the choice. */
fmgsr_status fmgsr_batch_autotune(fmgsr_batch plan, const double *f_packed,
                                  const double *kappa_packed, double *u_scratch_packed,
                                  void *hip_stream, double *ms_out);

/* Launch shape and (if segments_out != NULL) the [batch] segment counts. */
fmgsr_status fmgsr_batch_query(fmgsr_batch plan, fmgsr_batch_shape *shape_out,
                               int64_t *segments_out);

/* Frees the plan's device memory (synchronises the device first). */
fmgsr_status fmgsr_batch_destroy(fmgsr_batch plan);

/* One-shot forms (create, execute, synchronise hip_stream, destroy). */
fmgsr_status fmgsr_solve_batched(int32_t batch, const int64_t *n_host, const int64_t *offset_host,
                                 const int32_t *levels_host, const int64_t *segments_host,
                                 int32_t buffer, const fmgsr_operator *op /* kappa packed like f */,
                                 const double *f_packed, const double *g_host,
                                 const fmgsr_options *opt, double *u_packed, void *hip_stream);

/* Adjoint of one cubic problem (op->kind = FMGSR_OP_CUBIC_REACTION, op->kappa
 * [n]).  u_fwd = the forward solution, or NULL: the forward iteration with
 * f, g_left, g_right is then run keeping only its level-(M-1) solution (a
 * temporary of n/2 doubles) and the adjoint rebuilds u_fwd from it
 * (fmgsr_batch_adjoint_compressed); where that does not apply (one grid,
 * segment cores shorter than the window pad) u_fwd is computed into a
 * temporary of n doubles.  dJ_du [n]; outputs as fmgsr_batch_adjoint.
 * Synchronous. */
fmgsr_status fmgsr_adjoint(const fmgsr_operator *op, const double *f, double g_left,
                           double g_right, int64_t n, int32_t levels, int64_t n_segments,
                           int32_t buffer, const fmgsr_options *opt, const double *u_fwd,
                           const double *dJ_du, double *grad_f, double *grad_kappa,
                           void *hip_stream);

/* Per-kernel timing for benchmarks.  Between fmgsr_profile_enable() and
 * fmgsr_profile_collect(), every kernel that fmgsr_solve launches whose name
 * contains `filter` (NULL or "" = every kernel) is bracketed by two HIP
 * events recorded on the same stream, and its algorithmic byte count (each
 * input read once, each output written once) is noted.  Profiling state is
 * process-wide; calls from several threads are serialised. */
typedef struct {
  char name[48];         /* kernel name                                     */
  int64_t launches;      /* launches recorded                               */
  double total_ms;       /* sum of event-measured durations                 */
  double algo_bytes;     /* sum of algorithmic bytes over the launches      */
} fmgsr_kernel_stat;

/* Start recording (discarding anything recorded before). */
fmgsr_status fmgsr_profile_enable(const char *filter);

/* Wait for the recorded events, write up to max_stats per-kernel totals
 * into stats (host memory), stop recording and return the number of kernel
 * kinds seen (negative fmgsr_status on failure). */
int32_t fmgsr_profile_collect(fmgsr_kernel_stat *stats, int32_t max_stats);

/* Human-readable name of a status code (static string). */
const char *fmgsr_status_string(int32_t status);

/* Library version string, e.g. "fmgsr 0.2 gfx950". */
const char *fmgsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMGSR_H */
