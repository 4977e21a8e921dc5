/*
 * oracle_driver.c -- drives every entry point of the CPU oracle
 * (oracle/fmgsr_oracle.c, oracle/fmgsr_oracle_reaction.c) on small grids and
 * on invalid arguments, for an AddressSanitizer + UndefinedBehaviorSanitizer
 * build (tests/test_sanitizers.py).  Any out-of-bounds access, leak, signed
 * overflow or other undefined behaviour aborts the run; the exit status is
 * 0 only if every call also returned the expected status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nu1, nu2, nsr, rhs_restrict, tau_mode, smoother, tau_assembled, block_all;
} orc_options;
typedef struct {
  int32_t nu1, nu2, nsr, tau_mode, tau_assembled;
} orc_rx_options;

void orc_apply_L(const double *u, int64_t n, double gL, double gR, double *out);
void orc_restrict_avg(const double *u, int64_t nf, double *out);
void orc_restrict_fw(const double *r, int64_t nf, double *out);
void orc_prolong_linear(const double *e, int64_t nc, double *out);
void orc_interp_fmg(const double *c, int64_t nc, double gL, double gR, double *out);
void orc_rb_sweep(double *u, const double *F, int64_t n, int64_t lo, int64_t hi, double gL,
                  double gR);
void orc_lex_sweep(double *u, const double *F, int64_t n, int64_t lo, int64_t hi, int backward,
                   double gL, double gR);
void orc_kaczmarz(double *u, int64_t n, int64_t lo, int64_t hi, const double *c);
int orc_coarse_solve(const double *F, int64_t n, double gL, double gR, double *u);
int orc_smooth_blocks(const double *v, const double *F, int64_t n, int64_t S, int64_t b, int nu,
                      int smoother, const double *kaczmarz_c, double gL, double gR, double *out,
                      int order);
int orc_fmgsr_solve_ex(const double *f, double gL, double gR, int64_t n, int levels, int64_t S,
                       int64_t b, const orc_options *o, double *u_out, int order);
int orc_fmgsr_solve_keep(const double *f, double gL, double gR, int64_t n, int levels,
                         int64_t S, int64_t b, const orc_options *o, double *u_out,
                         double *coarse_out);
int orc_fmgsr_decompress(const double *c, const double *f, double gL, double gR, int64_t n,
                         int64_t S, int64_t b, const orc_options *o, int64_t lo, int64_t hi,
                         double *out);
int orc_fas_vcycle(double *u, const double *f, double gL, double gR, int64_t n, int levels,
                   const orc_options *o);
void orc_rx_apply(int kind, const double *a, const double *u, int64_t n, double gL, double gR,
                  double *out);
void orc_rx_ngs_sweep(int kind, const double *a, double *u, const double *F, int64_t n,
                      int64_t lo, int64_t hi, double gL, double gR);
int orc_rx_newton(int kind, const double *a, const double *F, int64_t n, double gL, double gR,
                  double *u, int max_it, double rtol, int *iters);
int orc_rx_fmgsr_solve_ex(int kind, const double *f, const double *coef, double gL, double gR,
                          int64_t n, int levels, int64_t S, int64_t b, const orc_rx_options *o,
                          double *u_out, int order);
int orc_rx_fas_vcycle(int kind, double *u, const double *f, const double *coef, double gL,
                      double gR, int64_t n, int levels, const orc_rx_options *o);
int orc_rx_adjoint_direct(const double *kappa, const double *u, const double *dJdu, int64_t n,
                          double *grad_f, double *grad_kappa);
int orc_rx_fmgsr_adjoint(const double *kappa, const double *u, const double *dJdu, int64_t n,
                         int levels, int64_t S, int64_t b, const orc_rx_options *o,
                         double *grad_f, double *grad_kappa);

static int failures = 0;

static void expect(int got, int want, const char *what)
{
  if ((want == 0 && got != 0) || (want != 0 && got >= 0)) {
    fprintf(stderr, "%s: status %d\n", what, got);
    ++failures;
  }
}

/* exactly-sized heap arrays, so any overrun is reported */
static double *arr(int64_t n, double v)
{
  double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) p[i] = v + 0.01 * (double)((i * 7919) % 101);
  return p;
}

static void transfers(void)
{
  for (int64_t nc = 1; nc <= 9; ++nc) {
    double *c = arr(nc, 0.5), *f = arr(2 * nc, 0.0), *g = arr(2 * nc, 0.0), *r = arr(nc, 0.0);
    orc_interp_fmg(c, nc, 0.3, -0.2, f);
    orc_prolong_linear(c, nc, g);
    orc_restrict_avg(f, 2 * nc, r);
    orc_restrict_fw(g, 2 * nc, r);
    orc_apply_L(f, 2 * nc, 0.1, 0.2, g);
    free(c); free(f); free(g); free(r);
  }
}

static void smoothers(void)
{
  for (int64_t n = 1; n <= 12; ++n) {
    double *u = arr(n, 0.1), *F = arr(n, 1.0), *c = arr(n / 2 > 0 ? n / 2 : 1, 0.2);
    double *o = arr(n, 0.0);
    orc_rb_sweep(u, F, n, 0, n, 0.0, 1.0);
    orc_lex_sweep(u, F, n, 0, n, 1, 0.0, 1.0);
    if (n % 2 == 0) orc_kaczmarz(u, n, 0, n, c);
    expect(orc_coarse_solve(F, n, 0.5, 0.5, o), 0, "coarse_solve");
    for (int64_t S = 1; S <= n; ++S)
      if (n % S == 0) {
        expect(orc_smooth_blocks(u, F, n, S, 2, 2, 0, NULL, 0.0, 0.0, o, 0), 0, "blocks");
        if (n % 2 == 0 && (n / S) % 2 == 0)
          expect(orc_smooth_blocks(u, F, n, S, 1, 1, 1, c, 0.0, 0.0, o, 1), 0, "blocks cr");
      }
    free(u); free(F); free(c); free(o);
  }
}

static void solves(void)
{
  const int64_t ns[] = {1, 2, 4, 8, 24, 64, 96};
  for (size_t i = 0; i < sizeof(ns) / sizeof(ns[0]); ++i) {
    int64_t n = ns[i];
    int maxl = 1;
    while ((n >> maxl) >= 1 && (n % ((int64_t)1 << maxl)) == 0) ++maxl;
    double *f = arr(n, 2.0), *u = arr(n, 0.0), *c = arr(n / 2 > 0 ? n / 2 : 1, 0.0);
    for (int levels = 1; levels <= maxl; ++levels)
      for (int nsr = 0; nsr <= 2 && nsr < levels; ++nsr)
        for (int tau = 0; tau <= 1; ++tau)
          for (int sm = 0; sm <= 1; ++sm) {
            orc_options o = {2, 1, nsr, tau, tau, sm, 0, 0};
            int64_t S = (n >= 8) ? 2 : 1;
            int ok = (nsr == 0) || ((n >> (nsr - 1)) % S == 0 && ((n >> (nsr - 1)) / S) % 2 == 0);
            for (int k = 1; k < nsr && ok; ++k) ok = ((n >> k) % S == 0 && ((n >> k) / S) % 2 == 0);
            int st = orc_fmgsr_solve_ex(f, 0.1, -0.1, n, levels, S, 3, &o, u, sm);
            expect(st, ok ? 0 : -1, "fmgsr_solve_ex");
            if (ok && levels >= 2 && nsr == 1) {
              expect(orc_fmgsr_solve_keep(f, 0.1, -0.1, n, levels, S, 3, &o, u, c), 0, "keep");
              double *d = arr(n, 0.0);
              expect(orc_fmgsr_decompress(c, f, 0.1, -0.1, n, S, 3, &o, 0, n, d), 0, "decompress");
              expect(orc_fmgsr_decompress(c, f, 0.1, -0.1, n, S, 3, &o, n / 2, n / 2 + 1, d), 0,
                     "decompress one cell");
              for (int64_t j = 0; j < n; ++j)
                if (d[0] != d[0]) ++failures;
              free(d);
            }
            if (ok) expect(orc_fas_vcycle(u, f, 0.1, -0.1, n, levels, &o), 0, "vcycle");
          }
    /* paper mode: 2-cell blocks, average restriction, literal tau */
    if (n >= 8) {
      orc_options o = {1, 1, 1, 1, 1, 1, 1, 2};
      expect(orc_fmgsr_solve_ex(f, 0.0, 0.0, n, 3, 1, 2, &o, u, 0), 0, "paper mode");
    }
    free(f); free(u); free(c);
  }
  /* invalid arguments */
  double *f = arr(16, 1.0), *u = arr(16, 0.0), *c = arr(8, 0.0);
  orc_options o = {2, 1, 1, 0, 0, 0, 0, 0};
  expect(orc_fmgsr_solve_ex(f, 0, 0, 16, 6, 4, 2, &o, u, 0), -1, "too many levels");
  expect(orc_fmgsr_solve_ex(f, 0, 0, 16, 3, 3, 2, &o, u, 0), -1, "segments do not divide");
  expect(orc_fmgsr_solve_ex(f, 0, 0, 16, 3, 4, -1, &o, u, 0), -1, "negative buffer");
  expect(orc_fmgsr_solve_ex(f, 0, 0, 0, 1, 1, 0, &o, u, 0), -1, "empty");
  expect(orc_fmgsr_solve_keep(f, 0, 0, 16, 1, 1, 0, &o, u, c), -1, "keep needs two levels");
  expect(orc_fmgsr_decompress(c, f, 0, 0, 16, 4, 2, &o, 4, 3, u), -1, "reversed range");
  expect(orc_fmgsr_decompress(c, f, 0, 0, 16, 4, 2, &o, 0, 17, u), -1, "range past n");
  expect(orc_fmgsr_decompress(c, f, 0, 0, 16, 4, 2, &o, 3, 3, u), 0, "empty range");
  o.rhs_restrict = 1;
  expect(orc_fmgsr_solve_ex(f, 0, 0, 16, 3, 4, 2, &o, u, 0), -1, "split tau with average R");
  free(f); free(u); free(c);
}

static void reaction(void)
{
  const int64_t ns[] = {1, 2, 8, 40, 64};
  for (size_t i = 0; i < sizeof(ns) / sizeof(ns[0]); ++i) {
    int64_t n = ns[i];
    double *f = arr(n, 1.0), *a = arr(n, 1.0), *u = arr(n, 0.0), *t = arr(n, 0.0);
    double *gf = arr(n, 0.0), *gk = arr(n, 0.0);
    int it = 0;
    for (int kind = 0; kind <= 2; ++kind) {
      orc_rx_apply(kind, a, u, n, 0.1, 0.2, t);
      orc_rx_ngs_sweep(kind, a, u, f, n, 0, n, 0.1, 0.2);
      expect(orc_rx_newton(kind, a, f, n, 0.1, 0.2, u, 30, 1e-14, &it), 0, "newton");
      int maxl = 1;
      while ((n % ((int64_t)1 << maxl)) == 0 && (n >> maxl) >= 1) ++maxl;
      for (int levels = 1; levels <= maxl; ++levels)
        for (int tau = 0; tau <= 1; ++tau) {
          int nsr = (levels >= 2 && n >= 4) ? 1 : 0;
          orc_rx_options o = {2, 1, nsr, tau, 0};
          int64_t S = (n >= 8) ? 2 : 1;
          expect(orc_rx_fmgsr_solve_ex(kind, f, a, 0.0, 0.1, n, levels, S, 2, &o, u, 0), 0,
                 "rx solve");
          expect(orc_rx_fas_vcycle(kind, u, f, a, 0.0, 0.1, n, levels, &o), 0, "rx vcycle");
        }
    }
    expect(orc_rx_adjoint_direct(a, u, f, n, gf, gk), 0, "adjoint direct");
    orc_rx_options o = {2, 1, n >= 4 ? 1 : 0, 0, 0};
    expect(orc_rx_fmgsr_adjoint(a, u, f, n, n >= 4 ? 2 : 1, 1, 2, &o, gf, gk), 0,
           "adjoint fmgsr");
    orc_rx_options bad = {2, 1, 2, 0, 0};
    expect(orc_rx_fmgsr_solve_ex(1, f, a, 0, 0, n, 1, 1, 0, &bad, u, 0), -1, "rx nsr 2");
    free(f); free(a); free(u); free(t); free(gf); free(gk);
  }
}

int main(void)
{
  transfers();
  smoothers();
  solves();
  reaction();
  if (failures) {
    fprintf(stderr, "%d unexpected statuses\n", failures);
    return 1;
  }
  printf("oracle driver: all calls clean\n");
  return 0;
}
