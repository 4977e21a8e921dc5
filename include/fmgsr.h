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
  FMGSR_ENOTSUP = -4   /* valid request this library does not implement     */
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

/* Operator kinds.  POISSON: -u'' (Sec. 4). */
enum { FMGSR_OP_POISSON = 0 };

typedef struct {
  int32_t kind;          /* FMGSR_OP_POISSON                                 */
  const double *kappa;   /* reserved for reaction terms; must be NULL        */
} fmgsr_operator;

typedef struct {
  int32_t nu1;           /* pre-smoothing sweeps per smoother call (>= 0)     */
  int32_t nu2;           /* post-smoothing sweeps per smoother call (>= 0)    */
  int32_t sr_levels;     /* 1: the finest level is an SR level (full update +
                            compatible relaxation, never stored); 0: plain
                            FMG-FAS with every level stored                    */
  int32_t tau_mode;      /* FMGSR_TAU_SPLIT or FMGSR_TAU_LITERAL              */
  void *workspace;       /* device scratch of >= fmgsr_workspace_bytes()
                            bytes, or NULL: the library then allocates and
                            frees it stream-ordered around the call            */
  size_t workspace_bytes;
} fmgsr_options;

/* Defaults: V(2,1), sr_levels = 1, split tau, library-managed workspace. */
void fmgsr_default_options(fmgsr_options *opt);

/* Bytes of device workspace fmgsr_solve needs for these sizes and options
 * (0 if the arguments are invalid). */
size_t fmgsr_workspace_bytes(int64_t n, int32_t levels, const fmgsr_options *opt);

/*
 * fmgsr_solve -- one FMG-FAS-SR iteration (Fig. 3) for -u'' = f.
 *
 *   op          operator descriptor (NULL = Poisson).
 *   f           [n] right-hand side at the cell centres of the finest level.
 *   g_left,
 *   g_right     Dirichlet values u(0), u(1).
 *   n           finest cells; n % 2^(levels-1) == 0 and N0 = n >> (levels-1)
 *               <= 1024.
 *   levels      number of grids, 1..40.
 *   n_segments  SR segments on the finest level (used when sr_levels = 1):
 *               n % n_segments == 0, the core s = n / n_segments is even, and
 *               s + 2 (buffer + 2) <= 8192.
 *   buffer      buffer (halo) cells on each side of a segment, 0..1024; each
 *               segment is smoothed on [i s - buffer, (i+1) s + buffer)
 *               clipped to the domain, with the exterior frozen, and only its
 *               core is kept (additive block Jacobi, Sec. 3).
 *   opt         options (NULL = defaults); nu1, nu2 in 0..16; sr_levels 0 or
 *               1 (1 needs levels >= 2).
 *   u_out       [n] result: the finest-level solution after the cycle,
 *               written once as it is produced (Sec. 3.2, streaming).
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

/* Library version string, e.g. "fmgsr 0.1 gfx950". */
const char *fmgsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FMGSR_H */
