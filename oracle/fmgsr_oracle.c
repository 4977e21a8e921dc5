/*
 * fmgsr_oracle.c -- plain, slow FP64 CPU oracle for one FMG-FAS iteration
 * with segmental refinement (SR) on the 1D model problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load or call this code.  It shares no
 * code, header, table or helper with the HIP library; the two are written
 * independently from the same paper:
 *   M. F. Adams, "A low memory, highly concurrent multigrid algorithm",
 *   arXiv:1207.6720.
 *
 * Problem (Sec. 4): -u'' = f on [0,1], Dirichlet values gL = u(0), gR = u(1),
 * second-order cell-centred finite volumes.  A level with n cells has
 * spacing h = 1/n and cell centres x_i = (i + 1/2) h, i = 0..n-1.  Cells
 * outside [0,n) are odd reflections about the boundary value:
 *   u_{-1-j} = 2 gL - u_j,   u_{n+j} = 2 gR - u_{n-1-j}.
 * With that ghost rule the boundary row of L has diagonal 3 (Sec. 4, and
 * the appendix's operator assembly).
 *
 * Readings of the paper taken here:
 *  R1  "levels" counts grids; the coarsest has N0 = n >> (levels-1) cells.
 *  R2  Solution restriction I^ = two-cell average (Sec. 2.4, Eq. 3 allows it
 *      to differ from the rhs restriction).  rhs/residual restriction I =
 *      full weighting = 1/2 (linear prolongation)^T by default; the two-cell
 *      average (the appendix's choice) is an option.
 *  R3  Smoother: red-black Gauss-Seidel, red = even global index, relaxed
 *      first; omega = 1.  Lexicographic symmetric GS (the appendix's choice)
 *      is an option.  nu counts inner sweeps of one smoother application.
 *  R4  SR levels use the additive block-Jacobi smoother of Sec. 3: segment i
 *      has core [i s, (i+1) s) and extended patch [i s - b, (i+1) s + b)
 *      clipped to the domain; the exterior is frozen at the incoming iterate.
 *      Non-SR levels use the same point smoother on the whole level.
 *  R5  tau (Eq. 7) is evaluated either literally, or "split": with R2's
 *      transfer pair L_H(I^ u) = I(L_h u) holds exactly, so the Laplacian
 *      part of tau is identically zero and f^H = I f^h.  Split is the default.
 *  R6  Literal tau on an SR level is evaluated per patch from the patch's
 *      extended iterate (Fig. 3, step 4), on the core's coarse cells.
 *  R7  The Kaczmarz update of Fig. 5 moves the fine iterate along the
 *      transpose of the restriction row (an exact projection onto
 *      I^ u^h = u^H, Eq. 8); the target is the current coarse iterate.
 *  R8  Coarsest level: exact solve (Thomas); for a one-cell level this is
 *      the single point update (F h^2 + (2gL + 2gR)) / 4.
 *
 * Floating point: every stencil is one fixed expression tree (written out
 * below); the file is compiled with -ffp-contract=off.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

typedef struct {
  int32_t nu1, nu2;        /* inner sweeps of the pre / post smoother       */
  int32_t nsr;             /* number of finest levels using full update +
                              compatible relaxation (0 = plain FMG-FAS)      */
  int32_t rhs_restrict;    /* 0: full weighting, 1: two-cell average (R2)   */
  int32_t tau_mode;        /* 0: split (R5), 1: literal Eq. 7               */
  int32_t smoother;        /* 0: red-black GS, 1: lexicographic symmetric GS */
  int32_t tau_assembled;   /* 0: per-patch tau on SR levels (R6), 1: global */
  int32_t block_all;       /* 0: blocks on SR levels only (R4);
                              >0: every non-coarsest level uses blocks with
                              this core size (the appendix's 2-cell blocks) */
} orc_options;

/* ------------------------------------------------------------------------ */
/* Level helpers                                                            */
/* ------------------------------------------------------------------------ */

/* Value of cell j of a level with n cells, j possibly outside [0,n): odd
 * reflection about the boundary value (Sec. 4 boundary treatment); applied
 * repeatedly when the level is narrower than the reach. */
static double cell(const double *u, int64_t n, int64_t j, double gL, double gR)
{
  if (j < 0) return 2.0 * gL - cell(u, n, -1 - j, gL, gR);
  if (j >= n) return 2.0 * gR - cell(u, n, 2 * n - 1 - j, gL, gR);
  return u[j];
}

static double inv_h2(int64_t n) { return (double)n * (double)n; }
static double h2_of(int64_t n) { return 1.0 / ((double)n * (double)n); }

/* (L u)_i = (2 u_i - (u_{i-1} + u_{i+1})) / h^2 with Dirichlet ghosts
 * (Sec. 4: second-order finite-volume Laplacian). */
void orc_apply_L(const double *u, int64_t n, double gL, double gR, double *out)
{
  double w = inv_h2(n);
  for (int64_t i = 0; i < n; ++i) {
    double l = (i > 0) ? u[i - 1] : 2.0 * gL - u[0];
    double r = (i < n - 1) ? u[i + 1] : 2.0 * gR - u[n - 1];
    out[i] = (2.0 * u[i] - (l + r)) * w;
  }
}

/* Solution restriction I^ (Sec. 2.4): average of the two children. */
void orc_restrict_avg(const double *u, int64_t nf, double *out)
{
  for (int64_t J = 0; J < nf / 2; ++J) out[J] = (u[2 * J] + u[2 * J + 1]) * 0.5;
}

/* Full-weighting restriction I = 1/2 P^T (P = linear prolongation below):
 * (I r)_J = ((r_{2J-1} + r_{2J+2}) + 3 (r_{2J} + r_{2J+1})) / 8, with the
 * homogeneous reflections r_{-1} = -r_0, r_{nf} = -r_{nf-1}. */
void orc_restrict_fw(const double *r, int64_t nf, double *out)
{
  for (int64_t J = 0; J < nf / 2; ++J) {
    double rm = (2 * J - 1 >= 0) ? r[2 * J - 1] : -r[0];
    double rp = (2 * J + 2 < nf) ? r[2 * J + 2] : -r[nf - 1];
    out[J] = ((rm + rp) + 3.0 * (r[2 * J] + r[2 * J + 1])) * 0.125;
  }
}

static void restrict_rhs(const double *r, int64_t nf, int mode, double *out)
{
  if (mode == 0) orc_restrict_fw(r, nf, out);
  else orc_restrict_avg(r, nf, out);
}

/* Linear (second-order) prolongation of a correction (Sec. 4; Eq. 4):
 * child 2J gets (3 e_J + e_{J-1}) / 4, child 2J+1 gets (3 e_J + e_{J+1}) / 4;
 * corrections carry no boundary data, so e_{-1} = -e_0, e_{nc} = -e_{nc-1}. */
void orc_prolong_linear(const double *e, int64_t nc, double *out)
{
  for (int64_t J = 0; J < nc; ++J) {
    double em = (J > 0) ? e[J - 1] : -e[0];
    double ep = (J < nc - 1) ? e[J + 1] : -e[nc - 1];
    out[2 * J] = (3.0 * e[J] + em) * 0.25;
    out[2 * J + 1] = (3.0 * e[J] + ep) * 0.25;
  }
}

/* Fourth-order FMG interpolation Pi (Sec. 2.3, Sec. 4): cubic Lagrange
 * interpolation through the four nearest coarse centres.  Child 2J lies a
 * quarter coarse cell left of centre J: weights (-5, 35, 105, -7)/128 on
 * J-2..J+1; child 2J+1 is the mirror image.  Coarse values beyond the
 * boundary are the Dirichlet reflections (cell()). */
void orc_interp_fmg(const double *c, int64_t nc, double gL, double gR, double *out)
{
  for (int64_t J = 0; J < nc; ++J) {
    double cm2 = cell(c, nc, J - 2, gL, gR), cm1 = cell(c, nc, J - 1, gL, gR);
    double c0 = c[J];
    double cp1 = cell(c, nc, J + 1, gL, gR), cp2 = cell(c, nc, J + 2, gL, gR);
    out[2 * J] = (((105.0 * c0 + 35.0 * cm1) - 7.0 * cp1) - 5.0 * cm2) * 0.0078125;
    out[2 * J + 1] = (((105.0 * c0 + 35.0 * cp1) - 7.0 * cm1) - 5.0 * cp2) * 0.0078125;
  }
}

/* One Gauss-Seidel point update of cell i (omega = 1): solve row i of
 * L u = F for u_i with the neighbours fixed. */
static void relax_point(double *u, const double *F, int64_t n, int64_t i,
                        double h2, double gL, double gR)
{
  double l = (i > 0) ? u[i - 1] : 2.0 * gL;
  double r = (i < n - 1) ? u[i + 1] : 2.0 * gR;
  double num = F[i] * h2 + (l + r);
  if (i > 0 && i < n - 1) u[i] = num * 0.5;
  else if (n == 1) u[i] = num / 4.0;
  else u[i] = num / 3.0;
}

/* Red-black GS sweep restricted to cells [lo,hi): red (even index) cells
 * first, then black.  Cells outside [lo,hi) are read, never written. */
void orc_rb_sweep(double *u, const double *F, int64_t n, int64_t lo, int64_t hi,
                  double gL, double gR)
{
  double h2 = h2_of(n);
  for (int colour = 0; colour < 2; ++colour)
    for (int64_t i = lo; i < hi; ++i)
      if ((i & 1) == colour) relax_point(u, F, n, i, h2, gL, gR);
}

/* Lexicographic GS sweep on [lo,hi), forward or backward (appendix smoother,
 * whose direction alternates between inner iterations). */
void orc_lex_sweep(double *u, const double *F, int64_t n, int64_t lo, int64_t hi,
                   int backward, double gL, double gR)
{
  double h2 = h2_of(n);
  if (!backward)
    for (int64_t i = lo; i < hi; ++i) relax_point(u, F, n, i, h2, gL, gR);
  else
    for (int64_t i = hi - 1; i >= lo; --i) relax_point(u, F, n, i, h2, gL, gR);
}

/* Kaczmarz (distributive) relaxation of Fig. 5 on [lo,hi) toward the coarse
 * iterate c: for every coarse cell J whose two children both lie in
 * [lo,hi), r = c_J - (I^ u)_J; with P(J,J) = (I^ I^T)_{JJ} = 1/2 the
 * correction t = 2r moves both children by r, after which (I^ u)_J = c_J
 * (Eq. 8) holds exactly. */
void orc_kaczmarz(double *u, int64_t n, int64_t lo, int64_t hi, const double *c)
{
  (void)n;
  int64_t J0 = (lo + 1) / 2;
  for (int64_t J = J0; 2 * J + 1 < hi; ++J) {
    double r = c[J] - (u[2 * J] + u[2 * J + 1]) * 0.5;
    u[2 * J] = u[2 * J] + r;
    u[2 * J + 1] = u[2 * J + 1] + r;
  }
}

/* Exact solve of the coarsest level (Fig. 1, "exact solve of coarsest
 * grid"): Thomas algorithm on h^2 L u = h^2 F + boundary terms. */
int orc_coarse_solve(const double *F, int64_t n, double gL, double gR, double *u)
{
  double h2 = h2_of(n);
  if (n == 1) { u[0] = (F[0] * h2 + (2.0 * gL + 2.0 * gR)) / 4.0; return ORC_OK; }
  double *cp = (double *)calloc((size_t)n, sizeof(double));
  double *dp = (double *)calloc((size_t)n, sizeof(double));
  if (!cp || !dp) { free(cp); free(dp); return ORC_ENOMEM; }
  /* forward elimination; sub- and super-diagonal entries are -1 */
  cp[0] = -1.0 / 3.0;
  dp[0] = (F[0] * h2 + 2.0 * gL) / 3.0;
  for (int64_t i = 1; i < n; ++i) {
    double diag = (i == n - 1) ? 3.0 : 2.0;
    double d = F[i] * h2;
    if (i == n - 1) d += 2.0 * gR;
    double m = diag + cp[i - 1];
    cp[i] = -1.0 / m;
    dp[i] = (d + dp[i - 1]) / m;
  }
  /* back substitution */
  u[n - 1] = dp[n - 1];
  for (int64_t i = n - 2; i >= 0; --i) u[i] = dp[i] - cp[i] * u[i + 1];
  free(cp); free(dp);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Smoother S of Sec. 3: point smoother on a set of cells                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  int smoother;     /* 0 red-black, 1 lexicographic symmetric */
} sweep_kind;

/* nu inner iterations of the point smoother on [lo,hi) (exterior frozen);
 * with kaczmarz != NULL each iteration starts with the Kaczmarz pass of
 * Fig. 5 (compatible relaxation on full-update levels, Sec. 3.1). */
static void smooth_set(double *u, const double *F, int64_t n, int64_t lo, int64_t hi,
                       int nu, int smoother, const double *kaczmarz_c,
                       double gL, double gR)
{
  for (int it = 0; it < nu; ++it) {
    if (kaczmarz_c) orc_kaczmarz(u, n, lo, hi, kaczmarz_c);
    if (smoother == 0) orc_rb_sweep(u, F, n, lo, hi, gL, gR);
    else orc_lex_sweep(u, F, n, lo, hi, it & 1, gL, gR);
  }
}

/* Additive block-Jacobi application of the smoother (Sec. 3; Sec. 4):
 * every segment's extended patch starts from the same incoming iterate v,
 * is smoothed with its exterior frozen at v, and contributes only its core
 * to out.  The result does not depend on the order of the segments; `order`
 * reverses the loop so the tests can check that.
 *
 * If patches != NULL the extended iterates of every segment are returned
 * there, each as a window of width s + 2*pw (pw = max(b,2) + 1) centred on
 * the core, for per-patch tau (R6).  Window cells outside the domain are 0. */
static int smooth_blocks_range(const double *v, const double *F, int64_t n, int64_t S,
                               int64_t b, int nu, int smoother, const double *kaczmarz_c,
                               double gL, double gR, double *out, double *patches, int order,
                               int64_t k_lo, int64_t k_hi)
{
  int64_t s = n / S;
  int64_t pw = (b > 2 ? b : 2) + 1;
  int64_t ww = s + 2 * pw;
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  if (!w) return ORC_ENOMEM;
  /* w holds the whole level so that cell indices stay global; only the
   * window around the current segment is refreshed from v each time. */
  memcpy(w, v, sizeof(double) * (size_t)n);
  for (int64_t k = k_lo; k < k_hi; ++k) {
    int64_t i = order ? (k_hi - 1 - (k - k_lo)) : k;
    int64_t lo = i * s - b, hi = (i + 1) * s + b;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    int64_t wlo = i * s - pw, whi = (i + 1) * s + pw;
    int64_t clo = wlo < 0 ? 0 : wlo, chi = whi > n ? n : whi;
    memcpy(w + clo, v + clo, sizeof(double) * (size_t)(chi - clo));
    smooth_set(w, F, n, lo, hi, nu, smoother, kaczmarz_c, gL, gR);
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

/* All S segments (the smoother of an SR level). */
static int smooth_blocks(const double *v, const double *F, int64_t n, int64_t S,
                         int64_t b, int nu, int smoother, const double *kaczmarz_c,
                         double gL, double gR, double *out, double *patches, int order)
{
  return smooth_blocks_range(v, F, n, S, b, nu, smoother, kaczmarz_c, gL, gR, out, patches,
                             order, 0, S);
}

/* ------------------------------------------------------------------------ */
/* FAS coarse right-hand side (Eqs. 3, 6, 7)                                */
/* ------------------------------------------------------------------------ */

/* Literal Eq. 7 assembled over the whole level:
 *   f^H = I f^h + tau,  tau = L_H(I^ u^h) - I(L_h u^h),
 * evaluated as I(f^h - L_h u^h) + L_H(I^ u^h) (the FAS residual restricted,
 * plus the coarse operator of the restricted solution, Eq. 2). */
static int literal_rhs_global(const double *u, const double *Fh, int64_t nf, int rmode,
                              double gL, double gR, double *FH)
{
  int64_t nc = nf / 2;
  double *r = (double *)malloc(sizeof(double) * (size_t)nf);
  double *uh = (double *)malloc(sizeof(double) * (size_t)nc);
  double *Lu = (double *)malloc(sizeof(double) * (size_t)nc);
  if (!r || !uh || !Lu) { free(r); free(uh); free(Lu); return ORC_ENOMEM; }
  orc_apply_L(u, nf, gL, gR, r);
  for (int64_t i = 0; i < nf; ++i) r[i] = Fh[i] - r[i];
  restrict_rhs(r, nf, rmode, FH);
  orc_restrict_avg(u, nf, uh);
  orc_apply_L(uh, nc, gL, gR, Lu);
  for (int64_t J = 0; J < nc; ++J) FH[J] = FH[J] + Lu[J];
  free(r); free(uh); free(Lu);
  return ORC_OK;
}

/* Literal Eq. 7 per patch (Fig. 3, steps 3-5; R6): for the core coarse
 * cells of segment i the same expression is evaluated from that segment's
 * extended iterate ubar_i (window of width s + 2 pw around the core). */
static void literal_rhs_patches(const double *patches, const double *Fh, int64_t nf,
                                int64_t S, int64_t b, int rmode, double gL, double gR,
                                double *FH)
{
  int64_t s = nf / S, pw = (b > 2 ? b : 2) + 1, ww = s + 2 * pw;
  int64_t nc = nf / 2;
  double w = inv_h2(nf), wc = inv_h2(nc);
  for (int64_t i = 0; i < S; ++i) {
    const double *p = patches + i * ww;
    int64_t wlo = i * s - pw;
#define UB(j) (p[(j) - wlo])
    for (int64_t J = i * s / 2; J < (i + 1) * s / 2; ++J) {
      /* residual f - L ubar at fine cells 2J-1 .. 2J+2 */
      double rr[4];
      for (int q = 0; q < 4; ++q) {
        int64_t k = 2 * J - 1 + q;
        if (k < 0 || k >= nf) { rr[q] = 0.0; continue; }
        double l = (k > 0) ? UB(k - 1) : 2.0 * gL - UB(0);
        double r = (k < nf - 1) ? UB(k + 1) : 2.0 * gR - UB(nf - 1);
        rr[q] = Fh[k] - (2.0 * UB(k) - (l + r)) * w;
      }
      double IR;
      if (rmode == 0) {
        double rm = (2 * J - 1 >= 0) ? rr[0] : -rr[1];
        double rp = (2 * J + 2 < nf) ? rr[3] : -rr[2];
        IR = ((rm + rp) + 3.0 * (rr[1] + rr[2])) * 0.125;
      } else {
        IR = (rr[1] + rr[2]) * 0.5;
      }
      /* coarse operator of the restricted patch iterate */
      double u0 = (UB(2 * J) + UB(2 * J + 1)) * 0.5;
      double ul = (J > 0) ? (UB(2 * J - 2) + UB(2 * J - 1)) * 0.5 : 2.0 * gL - u0;
      double ur = (J < nc - 1) ? (UB(2 * J + 2) + UB(2 * J + 3)) * 0.5 : 2.0 * gR - u0;
      FH[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
    }
#undef UB
  }
}

/* ------------------------------------------------------------------------ */
/* FMG-FAS-SR (Fig. 3)                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;      /* cells */
  double *u;      /* current iterate u^l                     */
  double *uhat;   /* restricted iterate I^ u^{l+1} (down leg) */
  double *F;      /* forcing f^l = I f^{l+1} (never changes)  */
  double *Q;      /* right-hand side in use (f^l + tau^l)     */
} level_t;

static void free_levels(level_t *lv, int nl)
{
  if (!lv) return;
  for (int l = 0; l < nl; ++l) { free(lv[l].u); free(lv[l].uhat); free(lv[l].F); free(lv[l].Q); }
  free(lv);
}

/* Validation shared by the solver entry points.  Returns M (levels-1) or a
 * negative status. */
static int validate(int64_t n, int levels, int64_t S, int64_t b, const orc_options *o)
{
  if (n < 1 || levels < 1 || levels > 40 || b < 0 || !o) return ORC_EINVAL;
  int M = levels - 1;
  if (n % ((int64_t)1 << M) != 0) return ORC_EINVAL;
  if (o->nu1 < 0 || o->nu2 < 0 || o->nsr < 0 || o->nsr > M) return ORC_EINVAL;
  if (o->rhs_restrict == 1 && o->tau_mode == 0) return ORC_EINVAL; /* split needs FW */
  if (o->block_all > 0) {
    if (o->block_all % 2 != 0) return ORC_EINVAL;
    for (int l = 1; l <= M; ++l)
      if ((n >> (M - l)) % o->block_all != 0) return ORC_EINVAL;
  } else if (o->nsr > 0) {
    if (S < 1) return ORC_EINVAL;
    for (int l = M - o->nsr + 1; l <= M; ++l) {
      int64_t nl = n >> (M - l);
      if (nl % S != 0 || (nl / S) % 2 != 0) return ORC_EINVAL;
    }
  }
  return M;
}

/* Segment count used on level l (0 = the point smoother on the whole
 * level): SR levels use S segments (R4); with block_all every
 * non-coarsest level uses blocks of block_all cells. */
static int64_t level_segments(const level_t *lv, int l, int M, const orc_options *o, int64_t S)
{
  if (l == 0) return 0;
  if (o->block_all > 0) return lv[l].n / o->block_all;
  if (l > M - o->nsr) return S;
  return 0;
}

/* Smoothing of level l with nu sweeps; kc != NULL selects compatible
 * relaxation (Fig. 5). */
static int smooth_level(level_t *lv, int l, int M, int nu, const orc_options *o,
                        int64_t S, int64_t b, const double *kc, double gL, double gR,
                        double *patches, int order)
{
  int64_t n = lv[l].n;
  int64_t segs = level_segments(lv, l, M, o, S);
  if (segs > 0) {
    double *out = (double *)malloc(sizeof(double) * (size_t)n);
    if (!out) return ORC_ENOMEM;
    int st = smooth_blocks(lv[l].u, lv[l].Q, n, segs, b, nu, o->smoother, kc, gL, gR,
                           out, patches, order);
    if (st == ORC_OK) memcpy(lv[l].u, out, sizeof(double) * (size_t)n);
    free(out);
    return st;
  }
  smooth_set(lv[l].u, lv[l].Q, n, 0, n, nu, o->smoother, kc, gL, gR);
  return ORC_OK;
}

/* One FMG-FAS-SR iteration (Fig. 3, with the readings R1-R8).
 *
 *   u^0 = exact solve with f^0
 *   for k = 0..M-1 (t = k+1 is the new finest level):
 *     1   u^t = Pi u^k                       FMG prolongation
 *     2   u^t = S^{nu1}(u^t, f^t)             (block Jacobi if SR level)
 *     for m = k..0 (pre-smoothing leg):
 *     3     uhat^m = I^ u^{m+1}               restrict solution
 *     4-5   Q^m = I Q^{m+1} + tau^m           (split: f^m; literal: Eq. 7)
 *           u^m = uhat^m, then S^{nu1} (exact solve if m = 0)
 *     for m = 0..k (post-smoothing leg):
 *           SR level m+1:   u^{m+1} = Pi u^m (Eq. 5), then nu2 x [Kaczmarz
 *                           toward u^m, point sweep] per segment (Fig. 5)
 *           otherwise:      u^{m+1} += P(u^m - uhat^m) (Eq. 4), S^{nu2}
 *   return u^M
 *
 * order = 1 processes segments in reverse (block-order invariance test).
 */
static int fmgsr_solve_core(const double *f, double gL, double gR, int64_t n, int levels,
                            int64_t S, int64_t b, const orc_options *o, double *u_out,
                            double *coarse_out, int order)
{
  int M = validate(n, levels, S, b, o);
  if (M < 0) return M;
  level_t *lv = (level_t *)calloc((size_t)(M + 1), sizeof(level_t));
  if (!lv) return ORC_ENOMEM;
  for (int l = 0; l <= M; ++l) {
    int64_t nl = n >> (M - l);
    lv[l].n = nl;
    lv[l].u = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].uhat = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].F = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].Q = (double *)calloc((size_t)nl, sizeof(double));
    if (!lv[l].u || !lv[l].uhat || !lv[l].F || !lv[l].Q) { free_levels(lv, M + 1); return ORC_ENOMEM; }
  }
  /* forcing on all levels (Sec. 3: "f defined on all levels") */
  memcpy(lv[M].F, f, sizeof(double) * (size_t)n);
  for (int l = M - 1; l >= 0; --l) restrict_rhs(lv[l + 1].F, lv[l + 1].n, o->rhs_restrict, lv[l].F);
  for (int l = 0; l <= M; ++l) memcpy(lv[l].Q, lv[l].F, sizeof(double) * (size_t)lv[l].n);

  int st = orc_coarse_solve(lv[0].Q, lv[0].n, gL, gR, lv[0].u);
  double *patches = NULL;
  if (st == ORC_OK && o->tau_mode == 1 && !o->tau_assembled &&
      level_segments(lv, M, M, o, S) > 0) {
    int64_t pw = (b > 2 ? b : 2) + 1;
    int64_t segs = level_segments(lv, M, M, o, S);
    patches = (double *)malloc(sizeof(double) * (size_t)(n + 2 * pw * segs));
    if (!patches) st = ORC_ENOMEM;
  }
  for (int k = 0; k < M && st == ORC_OK; ++k) {
    int t = k + 1;
    /* 1: FMG prolongation to the new finest level */
    orc_interp_fmg(lv[k].u, lv[k].n, gL, gR, lv[t].u);
    memcpy(lv[t].Q, lv[t].F, sizeof(double) * (size_t)lv[t].n);
    /* 2: smooth it; keep the extended patch iterates for per-patch tau */
    int keep = (patches && level_segments(lv, t, M, o, S) > 0);
    st = smooth_level(lv, t, M, o->nu1, o, S, b, NULL, gL, gR, keep ? patches : NULL, order);
    int patches_level = keep ? t : -1;
    /* pre-smoothing leg */
    for (int m = k; m >= 0 && st == ORC_OK; --m) {
      orc_restrict_avg(lv[m + 1].u, lv[m + 1].n, lv[m].uhat);
      if (o->tau_mode == 0) {
        memcpy(lv[m].Q, lv[m].F, sizeof(double) * (size_t)lv[m].n);
      } else if (patches_level == m + 1) {
        int64_t segs = level_segments(lv, m + 1, M, o, S);
        literal_rhs_patches(patches, lv[m + 1].Q, lv[m + 1].n, segs, b, o->rhs_restrict, gL, gR, lv[m].Q);
      } else {
        st = literal_rhs_global(lv[m + 1].u, lv[m + 1].Q, lv[m + 1].n, o->rhs_restrict, gL, gR, lv[m].Q);
        if (st != ORC_OK) break;
      }
      memcpy(lv[m].u, lv[m].uhat, sizeof(double) * (size_t)lv[m].n);
      if (m == 0) {
        st = orc_coarse_solve(lv[0].Q, lv[0].n, gL, gR, lv[0].u);
      } else {
        int keep2 = (patches && level_segments(lv, m, M, o, S) > 0);
        st = smooth_level(lv, m, M, o->nu1, o, S, b, NULL, gL, gR, keep2 ? patches : NULL, order);
        patches_level = keep2 ? m : -1;
      }
    }
    /* post-smoothing leg */
    for (int m = 0; m <= k && st == ORC_OK; ++m) {
      int64_t nc = lv[m].n, nf = lv[m + 1].n;
      if (m + 1 > M - o->nsr) {
        /* full update (Eq. 5) with the high-order interpolation, then
         * compatible relaxation toward u^m (Fig. 3 SR branch, Fig. 5) */
        orc_interp_fmg(lv[m].u, nc, gL, gR, lv[m + 1].u);
        st = smooth_level(lv, m + 1, M, o->nu2, o, S, b, lv[m].u, gL, gR, NULL, order);
      } else {
        /* correction (Eq. 4): u^{m+1} += P(u^m - I^ u^{m+1}) */
        double *e = (double *)malloc(sizeof(double) * (size_t)nc);
        double *pe = (double *)malloc(sizeof(double) * (size_t)nf);
        if (!e || !pe) { free(e); free(pe); st = ORC_ENOMEM; break; }
        for (int64_t J = 0; J < nc; ++J) e[J] = lv[m].u[J] - lv[m].uhat[J];
        orc_prolong_linear(e, nc, pe);
        for (int64_t i = 0; i < nf; ++i) lv[m + 1].u[i] = lv[m + 1].u[i] + pe[i];
        free(e); free(pe);
        st = smooth_level(lv, m + 1, M, o->nu2, o, S, b, NULL, gL, gR, NULL, order);
      }
    }
  }
  if (st == ORC_OK && M == 0) st = orc_coarse_solve(lv[0].Q, n, gL, gR, lv[0].u);
  if (st == ORC_OK && u_out) memcpy(u_out, lv[M].u, sizeof(double) * (size_t)n);
  if (st == ORC_OK && coarse_out && M >= 1)
    memcpy(coarse_out, lv[M - 1].u, sizeof(double) * (size_t)lv[M - 1].n);
  free(patches);
  free_levels(lv, M + 1);
  return st;
}

int orc_fmgsr_solve_ex(const double *f, double gL, double gR, int64_t n, int levels,
                       int64_t S, int64_t b, const orc_options *o, double *u_out, int order)
{
  return fmgsr_solve_core(f, gL, gR, n, levels, S, b, o, u_out, NULL, order);
}

int orc_fmgsr_solve(const double *f, double gL, double gR, int64_t n, int levels,
                    int64_t S, int64_t b, const orc_options *o, double *u_out)
{
  return orc_fmgsr_solve_ex(f, gL, gR, n, levels, S, b, o, u_out, 0);
}

/* The same iteration, also returning the level-(M-1) solution after the
 * final V-cycle (coarse_out, n/2 cells; levels >= 2).  With an SR finest
 * level that array and f determine the fine solution: the last step of the
 * cycle rebuilds it from them alone (Eq. 5 and Fig. 5), which is the PDE
 * compression of Sec. 2.4 that Sec. 3.2 proposes to store and expand on
 * demand. */
int orc_fmgsr_solve_keep(const double *f, double gL, double gR, int64_t n, int levels,
                         int64_t S, int64_t b, const orc_options *o, double *u_out,
                         double *coarse_out)
{
  if (levels < 2) return ORC_EINVAL;
  return fmgsr_solve_core(f, gL, gR, n, levels, S, b, o, u_out, coarse_out, 0);
}

/* PDE decompression (Sec. 3.2, method 2): the fine solution on cells
 * [lo, hi) from the stored level-(M-1) solution c (n/2 cells) and the fine
 * forcing f.  This is the SR branch of the final post-smoothing step of
 * Fig. 3 -- full update u = Pi c (Eq. 5), then nu2 times [Kaczmarz toward c,
 * point sweep] on each extended patch with its exterior frozen (Fig. 5) --
 * run only for the segments whose cores meet [lo, hi).  With the solve's S,
 * b and options the result equals the solve's finest level on [lo, hi).
 * out has hi - lo cells. */
int orc_fmgsr_decompress(const double *c, const double *f, double gL, double gR, int64_t n,
                         int64_t S, int64_t b, const orc_options *o, int64_t lo, int64_t hi,
                         double *out)
{
  if (!o || n < 2 || n % 2 != 0 || S < 1 || n % S != 0 || (n / S) % 2 != 0 || b < 0 ||
      o->nu2 < 0 || lo < 0 || hi > n || lo > hi)
    return ORC_EINVAL;
  if (lo == hi) return ORC_OK;
  int64_t s = n / S;
  double *ubar = (double *)malloc(sizeof(double) * (size_t)n);
  double *u = (double *)malloc(sizeof(double) * (size_t)n);
  if (!ubar || !u) { free(ubar); free(u); return ORC_ENOMEM; }
  orc_interp_fmg(c, n / 2, gL, gR, ubar);
  int st = smooth_blocks_range(ubar, f, n, S, b, o->nu2, o->smoother, c, gL, gR, u, NULL, 0,
                               lo / s, (hi - 1) / s + 1);
  if (st == ORC_OK) memcpy(out, u + lo, sizeof(double) * (size_t)(hi - lo));
  free(ubar);
  free(u);
  return st;
}

/* Additive block smoother as a stand-alone entry (tests of R4). */
int orc_smooth_blocks(const double *v, const double *F, int64_t n, int64_t S, int64_t b,
                      int nu, int smoother, const double *kaczmarz_c, double gL, double gR,
                      double *out, int order)
{
  if (n < 1 || S < 1 || n % S != 0 || b < 0 || nu < 0) return ORC_EINVAL;
  return smooth_blocks(v, F, n, S, b, nu, smoother, kaczmarz_c, gL, gR, out, NULL, order);
}

/* One FAS V(nu1,nu2)-cycle (Fig. 1) on the plain hierarchy (no SR, global
 * smoother): used by the tests to measure the cycle's error-reduction
 * factor.  u is updated in place on the finest level. */
int orc_fas_vcycle(double *u, const double *f, double gL, double gR, int64_t n, int levels,
                   const orc_options *o)
{
  int M = validate(n, levels, 1, 0, o);
  if (M < 0) return M;
  level_t *lv = (level_t *)calloc((size_t)(M + 1), sizeof(level_t));
  if (!lv) return ORC_ENOMEM;
  for (int l = 0; l <= M; ++l) {
    int64_t nl = n >> (M - l);
    lv[l].n = nl;
    lv[l].u = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].uhat = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].F = (double *)calloc((size_t)nl, sizeof(double));
    lv[l].Q = (double *)calloc((size_t)nl, sizeof(double));
    if (!lv[l].u || !lv[l].uhat || !lv[l].F || !lv[l].Q) { free_levels(lv, M + 1); return ORC_ENOMEM; }
  }
  memcpy(lv[M].u, u, sizeof(double) * (size_t)n);
  memcpy(lv[M].F, f, sizeof(double) * (size_t)n);
  for (int l = M - 1; l >= 0; --l) restrict_rhs(lv[l + 1].F, lv[l + 1].n, o->rhs_restrict, lv[l].F);
  memcpy(lv[M].Q, f, sizeof(double) * (size_t)n);
  int st = ORC_OK;
  orc_options og = *o;
  og.nsr = 0;
  for (int m = M; m >= 1 && st == ORC_OK; --m) {
    if (m == M) st = smooth_level(lv, m, M, o->nu1, &og, 1, 0, NULL, gL, gR, NULL, 0);
    orc_restrict_avg(lv[m].u, lv[m].n, lv[m - 1].uhat);
    if (o->tau_mode == 0) memcpy(lv[m - 1].Q, lv[m - 1].F, sizeof(double) * (size_t)lv[m - 1].n);
    else st = literal_rhs_global(lv[m].u, lv[m].Q, lv[m].n, o->rhs_restrict, gL, gR, lv[m - 1].Q);
    memcpy(lv[m - 1].u, lv[m - 1].uhat, sizeof(double) * (size_t)lv[m - 1].n);
    if (m - 1 == 0) st = orc_coarse_solve(lv[0].Q, lv[0].n, gL, gR, lv[0].u);
    else st = smooth_level(lv, m - 1, M, o->nu1, &og, 1, 0, NULL, gL, gR, NULL, 0);
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
    st = smooth_level(lv, m + 1, M, o->nu2, &og, 1, 0, NULL, gL, gR, NULL, 0);
  }
  if (st == ORC_OK && M == 0) st = orc_coarse_solve(f, n, gL, gR, lv[0].u);
  if (st == ORC_OK) memcpy(u, lv[M].u, sizeof(double) * (size_t)n);
  free_levels(lv, M + 1);
  return st;
}
