/*
 * fmgsr_oracle_reaction.c -- plain FP64 CPU oracle for FMG-FAS-SR on the 1D
 * reaction-diffusion problems  -u'' + kappa(x) u^3 = f  (cubic) and
 * -u'' + c(x) u = f  (linear reaction; the adjoint of the cubic problem),
 * and for the adjoint gradients of a least-squares functional.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load or call this code.  It shares no
 * code, header, table or helper with the HIP library.  It reuses the transfer
 * operators of fmgsr_oracle.c (Pi, I^, I, P, Kaczmarz), which it calls through
 * their exported names.
 *
 * The paper (M. F. Adams, arXiv:1207.6720) states FAS for a general nonlinear
 * operator (Sec. 2.4, Eqs. 2, 3, 6, 7) and applies FMG-FAS-SR (Fig. 3) to
 * the Poisson problem of Sec. 4.  The reaction operators are additions of
 * this project.  Its readings, beyond R1-R8 of fmgsr_oracle.c:
 *  R13 Operator on a level with n cells and coefficient a (a_i at cell i):
 *        N(u)_i = (L u)_i + a_i u_i^3      (cubic)
 *        N(u)_i = (L u)_i + a_i u_i        (linear reaction)
 *      with L the Dirichlet finite-volume Laplacian of Sec. 4.  Kind 0 is
 *      the plain Poisson operator (a ignored).
 *  R14 Coarse coefficients: a^H = I^ a^h (two-cell average), so a one-cell
 *      child pair and its parent carry the same mean coefficient.
 *  R15 Smoother: red-black nonlinear Gauss-Seidel, one Newton step per point
 *      per visit (for the linear kinds this is exact point GS).  With
 *      q = a h^2, D = 2 inside, 3 at a boundary cell, 4 for a one-cell level
 *      and l, r the neighbours (ghost 2g at a boundary):
 *        cubic:  u_i <- ((F_i h^2 + (l + r)) + 2 q u_i^3) / (D + 3 q u_i^2)
 *        linear: u_i <- (F_i h^2 + (l + r)) / (D + q)
 *      Both reduce to the Poisson update when a = 0.
 *  R16 tau in split form: the Laplacian parts cancel exactly (R5), leaving
 *        f^H = I f^h + (R_H(I^ u) - I R_h(u)),   R(u)_i = a_i u_i^3 (or a_i u_i).
 *      The literal Eq. 7 (I(f - N_h u) + N_H(I^ u)) is a switch.
 *  R17 Coarsest level: Newton's method, each step an exact tridiagonal solve
 *      (Thomas) of the h^2-scaled Jacobian, from the incoming iterate (zero
 *      at the start of FMG).  Stop when max|delta| <= 1e-14 max|u|; or when
 *      max|delta| <= 1e-8 max|u| and the step failed to halve max|delta|
 *      (the rounding floor: the Jacobian's condition number grows like n^2,
 *      so the first test alone need not be reachable); or after 30 steps.
 *  R18 Adjoint: for J(u) with u solving N(u) = f, lambda solves
 *      (L + diag(3 kappa u^2)) lambda = dJ/du (homogeneous Dirichlet; the
 *      matrix is symmetric), and grad_f = lambda, grad_kappa = -u^3 lambda.
 *      The FMG-SR adjoint is one FMG-FAS-SR iteration of the linear-reaction
 *      problem with c = 3 kappa u^2.
 *
 * Floating point: fixed expression trees, compiled with -ffp-contract=off.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

#define RX_POISSON 0
#define RX_CUBIC 1
#define RX_LINEAR 2

/* Transfer operators of fmgsr_oracle.c. */
void orc_restrict_avg(const double *u, int64_t nf, double *out);
void orc_restrict_fw(const double *r, int64_t nf, double *out);
void orc_prolong_linear(const double *e, int64_t nc, double *out);
void orc_interp_fmg(const double *c, int64_t nc, double gL, double gR, double *out);
void orc_kaczmarz(double *u, int64_t n, int64_t lo, int64_t hi, const double *c);

typedef struct {
  int32_t nu1, nu2;     /* inner sweeps of the pre / post smoother            */
  int32_t nsr;          /* 0: plain FMG-FAS; 1: the finest level uses SR      */
  int32_t tau_mode;     /* 0: split (R16), 1: literal Eq. 7                   */
  int32_t tau_assembled; /* 0: tau of the SR level per patch, from each
                            segment's extended iterate (Fig. 3 step 4);
                            1: assembled from the global iterate             */
} orc_rx_options;

static double h2_of(int64_t n) { return 1.0 / ((double)n * (double)n); }

/* Reaction term R(u)_i (unscaled). */
static double reaction(int kind, double a, double u)
{
  if (kind == RX_CUBIC) return a * ((u * u) * u);
  if (kind == RX_LINEAR) return a * u;
  return 0.0;
}

/* N(u) = L u + R(u) on a level of n cells (R13). */
void orc_rx_apply(int kind, const double *a, const double *u, int64_t n, double gL, double gR,
                  double *out)
{
  double w = (double)n * (double)n;
  for (int64_t i = 0; i < n; ++i) {
    double l = (i > 0) ? u[i - 1] : 2.0 * gL - u[0];
    double r = (i < n - 1) ? u[i + 1] : 2.0 * gR - u[n - 1];
    double Lu = (2.0 * u[i] - (l + r)) * w;
    out[i] = Lu + reaction(kind, kind ? a[i] : 0.0, u[i]);
  }
}

/* Nonlinear Gauss-Seidel update of cell i (R15). */
static void ngs_point(int kind, const double *a, double *u, const double *F, int64_t n, int64_t i,
                      double h2, double gL, double gR)
{
  double l = (i > 0) ? u[i - 1] : 2.0 * gL;
  double r = (i < n - 1) ? u[i + 1] : 2.0 * gR;
  double D = (n == 1) ? 4.0 : ((i > 0 && i < n - 1) ? 2.0 : 3.0);
  double b = F[i] * h2 + (l + r);
  if (kind == RX_CUBIC) {
    double q = a[i] * h2;
    double uu = u[i] * u[i];
    u[i] = (b + 2.0 * q * (uu * u[i])) / (D + 3.0 * q * uu);
  } else if (kind == RX_LINEAR) {
    double q = a[i] * h2;
    u[i] = b / (D + q);
  } else {
    u[i] = b / D;
  }
}

/* Red-black sweep (red = even index first) over cells [lo,hi); cells
 * outside are read, never written. */
void orc_rx_ngs_sweep(int kind, const double *a, double *u, const double *F, int64_t n,
                      int64_t lo, int64_t hi, double gL, double gR)
{
  double h2 = h2_of(n);
  for (int colour = 0; colour < 2; ++colour)
    for (int64_t i = lo; i < hi; ++i)
      if ((i & 1) == colour) ngs_point(kind, a, u, F, n, i, h2, gL, gR);
}

/* Newton's method on N(u) = F (R17).  u holds the initial iterate on entry.
 * Returns the number of Newton steps taken in *iters.  rtol = 0 runs exactly
 * max_it steps. */
int orc_rx_newton(int kind, const double *a, const double *F, int64_t n, double gL, double gR,
                  double *u, int max_it, double rtol, int *iters)
{
  double h2 = h2_of(n);
  double *res = (double *)calloc((size_t)n, sizeof(double));
  double *dg = (double *)calloc((size_t)n, sizeof(double));
  double *cp = (double *)calloc((size_t)n, sizeof(double));
  double *dp = (double *)calloc((size_t)n, sizeof(double));
  if (!res || !dg || !cp || !dp) { free(res); free(dg); free(cp); free(dp); return ORC_ENOMEM; }
  int it = 0;
  double dprev = 0.0;
  for (; it < max_it; ++it) {
    /* h^2-scaled residual and Jacobian diagonal; off-diagonals are -1 */
    for (int64_t i = 0; i < n; ++i) {
      double l = (i > 0) ? u[i - 1] : 2.0 * gL;
      double r = (i < n - 1) ? u[i + 1] : 2.0 * gR;
      double D = (n == 1) ? 4.0 : ((i > 0 && i < n - 1) ? 2.0 : 3.0);
      double q = kind ? a[i] * h2 : 0.0;
      double Ru = 0.0, dR = 0.0;
      if (kind == RX_CUBIC) { Ru = q * ((u[i] * u[i]) * u[i]); dR = 3.0 * q * (u[i] * u[i]); }
      else if (kind == RX_LINEAR) { Ru = q * u[i]; dR = q; }
      res[i] = (F[i] * h2 + (l + r)) - (D * u[i] + Ru);
      dg[i] = D + dR;
    }
    /* Thomas: forward elimination, back substitution */
    cp[0] = (n > 1) ? -1.0 / dg[0] : 0.0;
    dp[0] = res[0] / dg[0];
    for (int64_t i = 1; i < n; ++i) {
      double m = dg[i] + cp[i - 1];
      cp[i] = (i < n - 1) ? -1.0 / m : 0.0;
      dp[i] = (res[i] + dp[i - 1]) / m;
    }
    double dmax = 0.0, umax = 0.0;
    double d = dp[n - 1];
    u[n - 1] = u[n - 1] + d;
    dmax = fabs(d);
    for (int64_t i = n - 2; i >= 0; --i) {
      d = dp[i] - cp[i] * d;
      u[i] = u[i] + d;
      if (fabs(d) > dmax) dmax = fabs(d);
    }
    for (int64_t i = 0; i < n; ++i) if (fabs(u[i]) > umax) umax = fabs(u[i]);
    if (rtol > 0.0 && (dmax <= rtol * umax ||
                       (it >= 1 && dmax <= 1e-8 * umax && dmax > 0.5 * dprev))) { ++it; break; }
    dprev = dmax;
  }
  if (iters) *iters = it;
  free(res); free(dg); free(cp); free(dp);
  return ORC_OK;
}

static int coarse_newton(int kind, const double *a, const double *F, int64_t n, double gL,
                         double gR, double *u)
{
  return orc_rx_newton(kind, a, F, n, gL, gR, u, 30, 1e-14, NULL);
}

/* ------------------------------------------------------------------------ */
/* Smoothing: whole level, or additive block Jacobi over segments (R4)      */
/* ------------------------------------------------------------------------ */

static void smooth_set(int kind, const double *a, double *u, const double *F, int64_t n,
                       int64_t lo, int64_t hi, int nu, const double *kc, double gL, double gR)
{
  for (int it = 0; it < nu; ++it) {
    if (kc) orc_kaczmarz(u, n, lo, hi, kc);
    orc_rx_ngs_sweep(kind, a, u, F, n, lo, hi, gL, gR);
  }
}

/* Every segment's extended patch starts from v, is smoothed with its
 * exterior frozen at v and contributes its core to out.  If patches != NULL
 * each segment's extended iterate is kept as a window of s + 2 pw cells
 * (pw = max(b, 2) + 1) around the core (cells outside the domain are 0). */
static int smooth_blocks(int kind, const double *a, const double *v, const double *F, int64_t n,
                         int64_t S, int64_t b, int nu, const double *kc, double gL, double gR,
                         double *out, double *patches, int order)
{
  int64_t s = n / S, pw = (b > 2 ? b : 2) + 1, ww = s + 2 * pw;
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  if (!w) return ORC_ENOMEM;
  memcpy(w, v, sizeof(double) * (size_t)n);
  for (int64_t k = 0; k < S; ++k) {
    int64_t i = order ? (S - 1 - k) : k;
    int64_t lo = i * s - b, hi = (i + 1) * s + b;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    int64_t wlo = i * s - pw, whi = (i + 1) * s + pw;
    int64_t clo = wlo < 0 ? 0 : wlo, chi = whi > n ? n : whi;
    memcpy(w + clo, v + clo, sizeof(double) * (size_t)(chi - clo));
    smooth_set(kind, a, w, F, n, lo, hi, nu, kc, gL, gR);
    memcpy(out + i * s, w + i * s, sizeof(double) * (size_t)s);
    if (patches) {
      double *p = patches + i * ww;
      for (int64_t j = wlo; j < whi; ++j) p[j - wlo] = (j >= 0 && j < n) ? w[j] : 0.0;
    }
    memcpy(w + clo, v + clo, sizeof(double) * (size_t)(chi - clo));
  }
  free(w);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* FAS coarse right-hand side (Eqs. 3, 6, 7; R16)                            */
/* ------------------------------------------------------------------------ */

/* FW restriction of one fine grid function at coarse cell J from the four
 * fine values 2J-1..2J+2 (v[0..3]); fine cells beyond the level use the
 * homogeneous reflection of I = 1/2 P^T. */
static double fw_at(const double v[4], int64_t J, int64_t nf)
{
  double rm = (2 * J - 1 >= 0) ? v[0] : -v[1];
  double rp = (2 * J + 2 < nf) ? v[3] : -v[2];
  return ((rm + rp) + 3.0 * (v[1] + v[2])) * 0.125;
}

/* Coarse rhs of coarse cell J from a fine iterate u (any layout: u_at gives
 * fine cell k, valid for k in [2J-1, 2J+2] inside the level), the fine rhs
 * Fh, the fine coefficient af and the coarse coefficient ac. */
typedef struct { const double *base; int64_t off; } view_t;
static double vat(view_t v, int64_t k) { return v.base[k - v.off]; }

static double coarse_rhs_at(int kind, int tau_mode, view_t u, const double *Fh, const double *af,
                            double ac, int64_t J, int64_t nf, double gL, double gR)
{
  int64_t nc = nf / 2;
  double fv[4], rv[4];
  for (int q = 0; q < 4; ++q) {
    int64_t k = 2 * J - 1 + q;
    if (k < 0 || k >= nf) { fv[q] = 0.0; rv[q] = 0.0; continue; }
    if (tau_mode == 0) {
      fv[q] = Fh[k];
      rv[q] = reaction(kind, kind ? af[k] : 0.0, vat(u, k));
    } else {
      /* literal: residual f - N_h(u) at fine cell k */
      double l = (k > 0) ? vat(u, k - 1) : 2.0 * gL - vat(u, 0);
      double r = (k < nf - 1) ? vat(u, k + 1) : 2.0 * gR - vat(u, nf - 1);
      double w = (double)nf * (double)nf;
      double Nu = (2.0 * vat(u, k) - (l + r)) * w + reaction(kind, kind ? af[k] : 0.0, vat(u, k));
      fv[q] = Fh[k] - Nu;
      rv[q] = 0.0;
    }
  }
  double uh = (vat(u, 2 * J) + vat(u, 2 * J + 1)) * 0.5;
  if (tau_mode == 0) {
    double IF = fw_at(fv, J, nf);
    double IR = fw_at(rv, J, nf);
    return IF + (reaction(kind, ac, uh) - IR);
  }
  double IRes = fw_at(fv, J, nf);
  double ul = (J > 0) ? (vat(u, 2 * J - 2) + vat(u, 2 * J - 1)) * 0.5 : 2.0 * gL - uh;
  double ur = (J < nc - 1) ? (vat(u, 2 * J + 2) + vat(u, 2 * J + 3)) * 0.5 : 2.0 * gR - uh;
  double wc = (double)nc * (double)nc;
  return IRes + ((2.0 * uh - (ul + ur)) * wc + reaction(kind, ac, uh));
}

/* ------------------------------------------------------------------------ */
/* FMG-FAS-SR (Fig. 3) for the reaction operators                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;
  double *u, *uhat, *F, *Q, *a;
} rlevel_t;

static void free_rlevels(rlevel_t *lv, int nl)
{
  if (!lv) return;
  for (int l = 0; l < nl; ++l) { free(lv[l].u); free(lv[l].uhat); free(lv[l].F); free(lv[l].Q); free(lv[l].a); }
  free(lv);
}

static rlevel_t *alloc_rlevels(int64_t n, int M)
{
  rlevel_t *lv = (rlevel_t *)calloc((size_t)(M + 1), sizeof(rlevel_t));
  if (!lv) return NULL;
  for (int l = 0; l <= M; ++l) {
    int64_t nl = n >> (M - l);
    lv[l].n = nl;
    lv[l].u = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].uhat = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].F = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].Q = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].a = (double *)calloc((size_t)nl, sizeof(double));
    if (!lv[l].u || !lv[l].uhat || !lv[l].F || !lv[l].Q || !lv[l].a) {
      free_rlevels(lv, M + 1);
      return NULL;
    }
  }
  return lv;
}

static int rx_validate(int kind, int64_t n, int levels, int64_t S, int64_t b,
                       const orc_rx_options *o)
{
  if (kind < 0 || kind > 2 || n < 1 || levels < 1 || levels > 40 || b < 0 || !o) return ORC_EINVAL;
  int M = levels - 1;
  if (n % ((int64_t)1 << M) != 0) return ORC_EINVAL;
  if (o->nu1 < 0 || o->nu2 < 0 || o->nsr < 0 || o->nsr > 1 || o->nsr > M) return ORC_EINVAL;
  if (o->tau_mode < 0 || o->tau_mode > 1) return ORC_EINVAL;
  if (o->tau_assembled < 0 || o->tau_assembled > 1) return ORC_EINVAL;
  if (o->nsr == 1 && (S < 1 || n % S != 0 || (n / S) % 2 != 0)) return ORC_EINVAL;
  return M;
}

/* FAS coarse rhs for the whole coarse level m from fine level m+1 (global
 * iterate). */
static void coarse_rhs_global(int kind, int tau_mode, rlevel_t *lv, int m, double gL, double gR)
{
  view_t u = { lv[m + 1].u, 0 };
  for (int64_t J = 0; J < lv[m].n; ++J)
    lv[m].Q[J] = coarse_rhs_at(kind, tau_mode, u, lv[m + 1].Q, lv[m + 1].a, lv[m].a[J], J,
                               lv[m + 1].n, gL, gR);
}

/* Per-patch coarse rhs on the SR level (Fig. 3 steps 3-5 from each
 * segment's extended iterate, on the core's coarse cells). */
static void coarse_rhs_patches(int kind, int tau_mode, rlevel_t *lv, int m, const double *patches,
                               int64_t S, int64_t b, double gL, double gR)
{
  int64_t nf = lv[m + 1].n, s = nf / S, pw = (b > 2 ? b : 2) + 1, ww = s + 2 * pw;
  for (int64_t i = 0; i < S; ++i) {
    view_t u = { patches + i * ww, i * s - pw };
    for (int64_t J = i * s / 2; J < (i + 1) * s / 2; ++J)
      lv[m].Q[J] = coarse_rhs_at(kind, tau_mode, u, lv[m + 1].Q, lv[m + 1].a, lv[m].a[J], J, nf,
                                 gL, gR);
  }
}

static int smooth_level(int kind, rlevel_t *lv, int l, int M, int nu, const orc_rx_options *o,
                        int64_t S, int64_t b, const double *kc, double gL, double gR,
                        double *patches, int order)
{
  int64_t n = lv[l].n;
  if (l == M && o->nsr == 1) {
    double *out = (double *)malloc(sizeof(double) * (size_t)n);
    if (!out) return ORC_ENOMEM;
    int st = smooth_blocks(kind, lv[l].a, lv[l].u, lv[l].Q, n, S, b, nu, kc, gL, gR, out,
                           patches, order);
    if (st == ORC_OK) memcpy(lv[l].u, out, sizeof(double) * (size_t)n);
    free(out);
    return st;
  }
  smooth_set(kind, lv[l].a, lv[l].u, lv[l].Q, n, 0, n, nu, kc, gL, gR);
  return ORC_OK;
}

/* One FMG-FAS-SR iteration (Fig. 3) for N(u) = f with coefficient `coef` on
 * the finest level (R13-R17).  Same schedule as orc_fmgsr_solve_ex:
 *   u^0 = Newton solve with f^0 = I^M f (from zero)
 *   for t = 1..M: u^t = Pi u^{t-1}; V-cycle from t with f^t, where on the
 *   way down f^{m} = I f^{m+1} + tau(u^{m+1}) and u^m starts from I^ u^{m+1};
 *   the coarsest level takes a Newton solve from I^ u^1; on the way up
 *   u^{m+1} += P(u^m - I^ u^{m+1}) (or, on the SR level, the full update
 *   Pi u^m and compatible relaxation), then nu2 sweeps. */
static int rx_fmgsr_solve_core(int kind, const double *f, const double *coef, double gL,
                               double gR, int64_t n, int levels, int64_t S, int64_t b,
                               const orc_rx_options *o, double *u_out, int order,
                               double *coarse_out);

int orc_rx_fmgsr_solve_ex(int kind, const double *f, const double *coef, double gL, double gR,
                          int64_t n, int levels, int64_t S, int64_t b, const orc_rx_options *o,
                          double *u_out, int order)
{
  return rx_fmgsr_solve_core(kind, f, coef, gL, gR, n, levels, S, b, o, u_out, order, NULL);
}

/* The same iteration, also returning the level-(M-1) solution it ends with
 * (the last step's post-smoothed iterate below the finest level, from which
 * the finest level's full update and compatible relaxation are made;
 * Sec. 2.4 keeps exactly this level).  coarse_out: n/2 values (M >= 1). */
int orc_rx_fmgsr_solve_keep(int kind, const double *f, const double *coef, double gL, double gR,
                            int64_t n, int levels, int64_t S, int64_t b, const orc_rx_options *o,
                            double *u_out, double *coarse_out)
{
  if (levels < 2 || !coarse_out) return ORC_EINVAL;
  return rx_fmgsr_solve_core(kind, f, coef, gL, gR, n, levels, S, b, o, u_out, 0, coarse_out);
}

static int rx_fmgsr_solve_core(int kind, const double *f, const double *coef, double gL,
                               double gR, int64_t n, int levels, int64_t S, int64_t b,
                               const orc_rx_options *o, double *u_out, int order,
                               double *coarse_out)
{
  int M = rx_validate(kind, n, levels, S, b, o);
  if (M < 0) return M;
  if (kind != RX_POISSON && !coef) return ORC_EINVAL;
  rlevel_t *lv = alloc_rlevels(n, M);
  if (!lv) return ORC_ENOMEM;
  memcpy(lv[M].F, f, sizeof(double) * (size_t)n);
  if (kind != RX_POISSON) memcpy(lv[M].a, coef, sizeof(double) * (size_t)n);
  for (int l = M - 1; l >= 0; --l) {
    orc_restrict_fw(lv[l + 1].F, lv[l + 1].n, lv[l].F);
    orc_restrict_avg(lv[l + 1].a, lv[l + 1].n, lv[l].a);
  }
  for (int l = 0; l <= M; ++l) memcpy(lv[l].Q, lv[l].F, sizeof(double) * (size_t)lv[l].n);

  int st = coarse_newton(kind, lv[0].a, lv[0].Q, lv[0].n, gL, gR, lv[0].u);
  double *patches = NULL;
  if (st == ORC_OK && o->nsr == 1) {
    int64_t pw = (b > 2 ? b : 2) + 1;
    patches = (double *)malloc(sizeof(double) * (size_t)(n + 2 * pw * S));
    if (!patches) st = ORC_ENOMEM;
  }
  for (int k = 0; k < M && st == ORC_OK; ++k) {
    int t = k + 1;
    orc_interp_fmg(lv[k].u, lv[k].n, gL, gR, lv[t].u);
    memcpy(lv[t].Q, lv[t].F, sizeof(double) * (size_t)lv[t].n);
    int sr_top = (t == M && o->nsr == 1);
    st = smooth_level(kind, lv, t, M, o->nu1, o, S, b, NULL, gL, gR, sr_top ? patches : NULL, order);
    int patches_level = sr_top ? t : -1;
    for (int m = k; m >= 0 && st == ORC_OK; --m) {
      orc_restrict_avg(lv[m + 1].u, lv[m + 1].n, lv[m].uhat);
      if (patches_level == m + 1 && !o->tau_assembled)
        coarse_rhs_patches(kind, o->tau_mode, lv, m, patches, S, b, gL, gR);
      else coarse_rhs_global(kind, o->tau_mode, lv, m, gL, gR);
      patches_level = -1;
      memcpy(lv[m].u, lv[m].uhat, sizeof(double) * (size_t)lv[m].n);
      if (m == 0) st = coarse_newton(kind, lv[0].a, lv[0].Q, lv[0].n, gL, gR, lv[0].u);
      else st = smooth_level(kind, lv, m, M, o->nu1, o, S, b, NULL, gL, gR, NULL, order);
    }
    for (int m = 0; m <= k && st == ORC_OK; ++m) {
      int64_t nc = lv[m].n, nf = lv[m + 1].n;
      if (m + 1 == M && o->nsr == 1) {
        orc_interp_fmg(lv[m].u, nc, gL, gR, lv[m + 1].u);
        st = smooth_level(kind, lv, m + 1, M, o->nu2, o, S, b, lv[m].u, gL, gR, NULL, order);
      } else {
        double *e = (double *)malloc(sizeof(double) * (size_t)nc);
        double *pe = (double *)malloc(sizeof(double) * (size_t)nf);
        if (!e || !pe) { free(e); free(pe); st = ORC_ENOMEM; break; }
        for (int64_t J = 0; J < nc; ++J) e[J] = lv[m].u[J] - lv[m].uhat[J];
        orc_prolong_linear(e, nc, pe);
        for (int64_t i = 0; i < nf; ++i) lv[m + 1].u[i] = lv[m + 1].u[i] + pe[i];
        free(e); free(pe);
        st = smooth_level(kind, lv, m + 1, M, o->nu2, o, S, b, NULL, gL, gR, NULL, order);
      }
    }
  }
  if (st == ORC_OK) memcpy(u_out, lv[M].u, sizeof(double) * (size_t)n);
  if (st == ORC_OK && coarse_out && M >= 1)
    memcpy(coarse_out, lv[M - 1].u, sizeof(double) * (size_t)lv[M - 1].n);
  free(patches);
  free_rlevels(lv, M + 1);
  return st;
}

int orc_rx_fmgsr_solve(int kind, const double *f, const double *coef, double gL, double gR,
                       int64_t n, int levels, int64_t S, int64_t b, const orc_rx_options *o,
                       double *u_out)
{
  return orc_rx_fmgsr_solve_ex(kind, f, coef, gL, gR, n, levels, S, b, o, u_out, 0);
}

/* One FAS V(nu1,nu2)-cycle (Fig. 1) on the plain hierarchy, u updated in
 * place: the tests iterate it to check that its fixed point is the discrete
 * solution, which pins the coarse right-hand side (a wrong tau moves the
 * fixed point). */
int orc_rx_fas_vcycle(int kind, double *u, const double *f, const double *coef, double gL,
                      double gR, int64_t n, int levels, const orc_rx_options *o)
{
  orc_rx_options og = *o;
  og.nsr = 0;
  int M = rx_validate(kind, n, levels, 1, 0, &og);
  if (M < 0) return M;
  if (kind != RX_POISSON && !coef) return ORC_EINVAL;
  rlevel_t *lv = alloc_rlevels(n, M);
  if (!lv) return ORC_ENOMEM;
  memcpy(lv[M].u, u, sizeof(double) * (size_t)n);
  memcpy(lv[M].F, f, sizeof(double) * (size_t)n);
  memcpy(lv[M].Q, f, sizeof(double) * (size_t)n);
  if (kind != RX_POISSON) memcpy(lv[M].a, coef, sizeof(double) * (size_t)n);
  for (int l = M - 1; l >= 0; --l) orc_restrict_avg(lv[l + 1].a, lv[l + 1].n, lv[l].a);
  int st = ORC_OK;
  for (int m = M; m >= 1 && st == ORC_OK; --m) {
    if (m == M) st = smooth_level(kind, lv, m, M, o->nu1, &og, 1, 0, NULL, gL, gR, NULL, 0);
    orc_restrict_avg(lv[m].u, lv[m].n, lv[m - 1].uhat);
    coarse_rhs_global(kind, o->tau_mode, lv, m - 1, gL, gR);
    memcpy(lv[m - 1].u, lv[m - 1].uhat, sizeof(double) * (size_t)lv[m - 1].n);
    if (m - 1 == 0) st = coarse_newton(kind, lv[0].a, lv[0].Q, lv[0].n, gL, gR, lv[0].u);
    else st = smooth_level(kind, lv, m - 1, M, o->nu1, &og, 1, 0, NULL, gL, gR, NULL, 0);
  }
  for (int m = 0; m < M && st == ORC_OK; ++m) {
    int64_t nc = lv[m].n, nf = lv[m + 1].n;
    double *e = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pe = (double *)malloc(sizeof(double) * (size_t)nf);
    if (!e || !pe) { free(e); free(pe); st = ORC_ENOMEM; break; }
    for (int64_t J = 0; J < nc; ++J) e[J] = lv[m].u[J] - lv[m].uhat[J];
    orc_prolong_linear(e, nc, pe);
    for (int64_t i = 0; i < nf; ++i) lv[m + 1].u[i] = lv[m + 1].u[i] + pe[i];
    free(e); free(pe);
    st = smooth_level(kind, lv, m + 1, M, o->nu2, &og, 1, 0, NULL, gL, gR, NULL, 0);
  }
  if (st == ORC_OK && M == 0) st = coarse_newton(kind, lv[0].a, f, n, gL, gR, lv[0].u);
  if (st == ORC_OK) memcpy(u, lv[M].u, sizeof(double) * (size_t)n);
  free_rlevels(lv, M + 1);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Adjoint (R18)                                                             */
/* ------------------------------------------------------------------------ */

/* c = 3 kappa u^2, the derivative of the cubic reaction term. */
static double *adjoint_coefficient(const double *kappa, const double *u, int64_t n)
{
  double *c = (double *)malloc(sizeof(double) * (size_t)n);
  if (!c) return NULL;
  for (int64_t i = 0; i < n; ++i) c[i] = 3.0 * kappa[i] * (u[i] * u[i]);
  return c;
}

static void gradients(const double *u, const double *lam, int64_t n, double *grad_f,
                      double *grad_kappa)
{
  for (int64_t i = 0; i < n; ++i) {
    if (grad_f) grad_f[i] = lam[i];
    if (grad_kappa) grad_kappa[i] = -(((u[i] * u[i]) * u[i]) * lam[i]);
  }
}

/* Direct adjoint: (L + diag(3 kappa u^2)) lambda = dJdu by one exact
 * tridiagonal solve (Newton on the linear problem converges in one step). */
int orc_rx_adjoint_direct(const double *kappa, const double *u, const double *dJdu, int64_t n,
                          double *grad_f, double *grad_kappa)
{
  double *c = adjoint_coefficient(kappa, u, n);
  double *lam = (double *)calloc((size_t)n, sizeof(double));
  if (!c || !lam) { free(c); free(lam); return ORC_ENOMEM; }
  int st = orc_rx_newton(RX_LINEAR, c, dJdu, n, 0.0, 0.0, lam, 3, 0.0, NULL);
  if (st == ORC_OK) gradients(u, lam, n, grad_f, grad_kappa);
  free(c); free(lam);
  return st;
}

/* FMG-SR adjoint: lambda from one FMG-FAS-SR iteration of the linear
 * reaction problem with c = 3 kappa u^2 and homogeneous boundary values. */
int orc_rx_fmgsr_adjoint(const double *kappa, const double *u, const double *dJdu, int64_t n,
                         int levels, int64_t S, int64_t b, const orc_rx_options *o,
                         double *grad_f, double *grad_kappa)
{
  double *c = adjoint_coefficient(kappa, u, n);
  double *lam = (double *)calloc((size_t)n, sizeof(double));
  if (!c || !lam) { free(c); free(lam); return ORC_ENOMEM; }
  int st = orc_rx_fmgsr_solve(RX_LINEAR, dJdu, c, 0.0, 0.0, n, levels, S, b, o, lam);
  if (st == ORC_OK) gradients(u, lam, n, grad_f, grad_kappa);
  free(c); free(lam);
  return st;
}
