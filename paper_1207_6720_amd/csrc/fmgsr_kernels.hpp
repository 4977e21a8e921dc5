// fmgsr_kernels.hpp -- gfx950 kernels of the FMG-FAS-SR solver (1D model
// problem, FP64).  Included by fmgsr.hip only.
//
// Data layout.  Every level is a contiguous FP64 array in HBM.  A tile kernel
// gives each workgroup a contiguous window of cells; each thread owns K
// consecutive cells of the window in registers ("run").  Red-black
// Gauss-Seidel then touches LDS only to pass one boundary value between
// neighbouring threads per half-sweep: red cells (even index) need the left
// neighbour's last (black) cell, black cells need the right neighbour's first
// (red) cell.  Windows overlap by a halo of redundantly computed cells, so a
// tile reproduces the whole-level sweep exactly on its core: after nu sweeps
// the cells within 2 nu of a window edge are stale, the rest equal what a
// sweep over the whole level computes (same operations on the same operands).
//
// Stencils (Sec. 4; appendix operator assembly), level with n cells, h = 1/n,
// Dirichlet values gL, gR entering through odd reflections about the faces:
//   point update   u_i <- (F_i h^2 + (u_{i-1} + u_{i+1})) / 2, boundary cells
//                  use 2 gL (2 gR) for the missing neighbour and divide by 3
//   Pi (FMG)       child 2J: (105 c_J + 35 c_{J-1} - 7 c_{J+1} - 5 c_{J-2})/128
//                  child 2J+1 mirrored (cubic interpolation, Sec. 2.3)
//   I^ (solution)  (u_{2J} + u_{2J+1}) / 2
//   I  (rhs, FW)   ((r_{2J-1} + r_{2J+2}) + 3 (r_{2J} + r_{2J+1})) / 8
//   P  (correction) child 2J: (3 e_J + e_{J-1}) / 4, child 2J+1 mirrored
// Each is one fixed expression tree; the library is built without FMA
// contraction so that the results are reproducible operation by operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmgsr {

constexpr int kRun = 16;          // cells per thread in tile kernels
constexpr int kTileThreads = 256; // threads per stored-level tile
constexpr int kSegMaxThreads = 512;

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double ld(const double* __restrict__ p, int64_t i, int64_t n) {
  return (i >= 0 && i < n) ? p[i] : 0.0;
}

// Coarse value at index J in [-2, nc+1], with the Dirichlet reflection
// u_{-1-j} = 2 gL - u_j, u_{nc+j} = 2 gR - u_{nc-1-j} applied as often as
// the (possibly one-cell) level requires.
__device__ __forceinline__ double coarse_at(const double* __restrict__ c, int64_t nc, int64_t J,
                                            double gL, double gR) {
  if (J >= 0 && J < nc) return c[J];
  if (J < 0) {
    const int64_t m = -1 - J;
    const double in = (m < nc) ? c[m] : 2.0 * gR - c[2 * nc - 1 - m];
    return 2.0 * gL - in;
  }
  const int64_t m = 2 * nc - 1 - J;
  const double in = (m >= 0) ? c[m] : 2.0 * gL - c[-1 - m];
  return 2.0 * gR - in;
}

__device__ __forceinline__ double interp_even(double cm2, double cm1, double c0, double cp1) {
  return (((105.0 * c0 + 35.0 * cm1) - 7.0 * cp1) - 5.0 * cm2) * 0.0078125;
}
__device__ __forceinline__ double interp_odd(double cm1, double c0, double cp1, double cp2) {
  return (((105.0 * c0 + 35.0 * cp1) - 7.0 * cm1) - 5.0 * cp2) * 0.0078125;
}

// Point Gauss-Seidel update of cell g (omega = 1) from its neighbours.
__device__ __forceinline__ double relax(double fj, double l, double r, int64_t g, int64_t n,
                                        double h2, double gL2, double gR2) {
  if (g > 0 && g < n - 1) return (fj * h2 + (l + r)) * 0.5;
  if (g == 0) l = gL2;
  if (g == n - 1) r = gR2;
  const double num = fj * h2 + (l + r);
  return (n == 1) ? num / 4.0 : num / 3.0;
}

// ---------------------------------------------------------------------------
// Register runs
// ---------------------------------------------------------------------------

// One half-sweep of colour C (0 = red = even index) over the run
// u[0..K) = cells g0..g0+K-1 (g0 even), updating only cells in [lo, hi).
// xbuf: one LDS slot per thread, a different buffer per colour so that a
// single barrier per half-sweep suffices.
template <int K, int C>
__device__ __forceinline__ void rb_half(double (&u)[K], const double (&f)[K], int64_t g0,
                                        int64_t lo, int64_t hi, int64_t n, double h2,
                                        double gL2, double gR2, double* xbuf) {
  const int t = threadIdx.x;
  xbuf[t] = (C == 0) ? u[K - 1] : u[0];
  __syncthreads();
  double nb = 0.0;
  if (C == 0) {
    if (t > 0) nb = xbuf[t - 1];
  } else {
    if (t + 1 < (int)blockDim.x) nb = xbuf[t + 1];
  }
#pragma unroll
  for (int j = C; j < K; j += 2) {
    const int64_t g = g0 + j;
    const double l = (j == 0) ? nb : u[j - 1];
    const double r = (j == K - 1) ? nb : u[j + 1];
    if (g >= lo && g < hi) u[j] = relax(f[j], l, r, g, n, h2, gL2, gR2);
  }
}

template <int K>
__device__ __forceinline__ void rb_sweeps(double (&u)[K], const double (&f)[K], int64_t g0,
                                          int nu, int64_t lo, int64_t hi, int64_t n,
                                          double gL, double gR, double* xr, double* xb) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  for (int s = 0; s < nu; ++s) {
    rb_half<K, 0>(u, f, g0, lo, hi, n, h2, gL2, gR2, xr);
    rb_half<K, 1>(u, f, g0, lo, hi, n, h2, gL2, gR2, xb);
  }
}

// u <- Pi c on the run (cells outside [0,n) are set to 0 and never used).
template <int K>
__device__ __forceinline__ void load_interp(double (&u)[K], int64_t g0, int64_t n,
                                            const double* __restrict__ c, double gL, double gR) {
  const int64_t nc = n >> 1;
  const int64_t J0 = g0 >> 1;  // g0 even (also when negative)
  double cv[K / 2 + 4];
#pragma unroll
  for (int q = 0; q < K / 2 + 4; ++q) {
    const int64_t J = J0 - 2 + q;
    cv[q] = (J >= -2 && J <= nc + 1) ? coarse_at(c, nc, J, gL, gR) : 0.0;
  }
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t g = g0 + 2 * p;
    const bool in = (g >= 0 && g < n);
    u[2 * p] = in ? interp_even(cv[p], cv[p + 1], cv[p + 2], cv[p + 3]) : 0.0;
    u[2 * p + 1] = in ? interp_odd(cv[p + 1], cv[p + 2], cv[p + 3], cv[p + 4]) : 0.0;
  }
}

// u <- I^ fine (two-cell average of the finer level).
template <int K>
__device__ __forceinline__ void load_restrict(double (&u)[K], int64_t g0, int64_t n,
                                              const double* __restrict__ fine) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t g = g0 + j;
    u[j] = (g >= 0 && g < n) ? (fine[2 * g] + fine[2 * g + 1]) * 0.5 : 0.0;
  }
}

template <int K>
__device__ __forceinline__ void load_direct(double (&u)[K], int64_t g0, int64_t n,
                                            const double* __restrict__ src) {
#pragma unroll
  for (int j = 0; j < K; ++j) u[j] = ld(src, g0 + j, n);
}

template <int K>
__device__ __forceinline__ void store_range(const double (&u)[K], int64_t g0, int64_t lo,
                                            int64_t hi, double* __restrict__ out) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int64_t g = g0 + j;
    if (g >= lo && g < hi) out[g] = u[j];
  }
}

// ---------------------------------------------------------------------------
// Stored-level visits
// ---------------------------------------------------------------------------

enum SourceKind : int { kSrcInterp = 0, kSrcRestrict = 1, kSrcDirect = 2 };

struct LevelArgs {
  int64_t n;          // cells on this level
  double gL, gR;
  int nu;             // sweeps
  int64_t core;       // core cells per workgroup
  int64_t halo;       // halo cells on each side (even, >= 2 nu)
  int src_kind;       // down visit: how the initial iterate is formed
  const double* src;  // down: coarser (Pi), finer (I^) or same-level array
  const double* pre;  // up: pre-smoothed iterate of this level
  const double* coarse;  // up: post-smoothed coarser level
  const double* rhs;  // right-hand side of this level
  double* out;        // result on the cores
};

// Down visit of a stored level (Fig. 3 steps 1-2, or restrict + smooth of
// the pre-smoothing leg): initial iterate from Pi / I^ / a copy, nu sweeps.
template <int K>
__global__ __launch_bounds__(kTileThreads) void k_level_down(LevelArgs a) {
  __shared__ double xr[kTileThreads], xb[kTileThreads];
  const int64_t tile_lo = (int64_t)blockIdx.x * a.core - a.halo;
  const int64_t tile_hi = tile_lo + (int64_t)blockDim.x * K;
  const int64_t g0 = tile_lo + (int64_t)threadIdx.x * K;
  double u[K], f[K];
#pragma unroll
  for (int j = 0; j < K; ++j) f[j] = ld(a.rhs, g0 + j, a.n);
  if (a.src_kind == kSrcInterp) load_interp<K>(u, g0, a.n, a.src, a.gL, a.gR);
  else if (a.src_kind == kSrcRestrict) load_restrict<K>(u, g0, a.n, a.src);
  else load_direct<K>(u, g0, a.n, a.src);
  const int64_t lo = tile_lo <= 0 ? 0 : tile_lo + 1;
  const int64_t hi = tile_hi >= a.n ? a.n : tile_hi - 1;
  rb_sweeps<K>(u, f, g0, a.nu, lo, hi, a.n, a.gL, a.gR, xr, xb);
  const int64_t clo = (int64_t)blockIdx.x * a.core;
  const int64_t chi = (clo + a.core < a.n) ? clo + a.core : a.n;
  store_range<K>(u, g0, clo, chi, a.out);
}

// Up visit of a stored level (Fig. 3 post-smoothing leg, Eq. 4):
// u = pre + P(coarse - I^ pre), then nu sweeps.
template <int K>
__global__ __launch_bounds__(kTileThreads) void k_level_up(LevelArgs a) {
  __shared__ double xr[kTileThreads], xb[kTileThreads];
  const int64_t n = a.n, nc = n >> 1;
  const int64_t tile_lo = (int64_t)blockIdx.x * a.core - a.halo;
  const int64_t tile_hi = tile_lo + (int64_t)blockDim.x * K;
  const int64_t g0 = tile_lo + (int64_t)threadIdx.x * K;
  const int64_t J0 = g0 >> 1;
  double u[K], f[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    f[j] = ld(a.rhs, g0 + j, n);
    u[j] = ld(a.pre, g0 + j, n);
  }
  // coarse error e_J = c_J - I^ pre, for J0-1 .. J0+K/2
  double e[K / 2 + 2];
#pragma unroll
  for (int q = 0; q < K / 2 + 2; ++q) {
    const int64_t J = J0 - 1 + q;
    double p0, p1;
    if (q == 0) { p0 = ld(a.pre, g0 - 2, n); p1 = ld(a.pre, g0 - 1, n); }
    else if (q == K / 2 + 1) { p0 = ld(a.pre, g0 + K, n); p1 = ld(a.pre, g0 + K + 1, n); }
    else { p0 = u[2 * (q - 1)]; p1 = u[2 * (q - 1) + 1]; }
    e[q] = (J >= 0 && J < nc) ? a.coarse[J] - (p0 + p1) * 0.5 : 0.0;
  }
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t J = J0 + p;
    if (J >= 0 && J < nc) {
      const double eJ = e[p + 1];
      const double em = (J > 0) ? e[p] : -eJ;
      const double ep = (J < nc - 1) ? e[p + 2] : -eJ;
      u[2 * p] = u[2 * p] + (3.0 * eJ + em) * 0.25;
      u[2 * p + 1] = u[2 * p + 1] + (3.0 * eJ + ep) * 0.25;
    }
  }
  const int64_t lo = tile_lo <= 0 ? 0 : tile_lo + 1;
  const int64_t hi = tile_hi >= n ? n : tile_hi - 1;
  rb_sweeps<K>(u, f, g0, a.nu, lo, hi, n, a.gL, a.gR, xr, xb);
  const int64_t clo = (int64_t)blockIdx.x * a.core;
  const int64_t chi = (clo + a.core < n) ? clo + a.core : n;
  store_range<K>(u, g0, clo, chi, a.out);
}

// ---------------------------------------------------------------------------
// Full-weighting restriction of the forcing (rhs hierarchy) and literal tau
// ---------------------------------------------------------------------------

// out[J] = I fine, J < nc.
__global__ void k_restrict_fw(const double* __restrict__ fine, int64_t nc, double* __restrict__ out) {
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int64_t nf = 2 * nc;
  const double rm = (J > 0) ? fine[2 * J - 1] : -fine[0];
  const double rp = (2 * J + 2 < nf) ? fine[2 * J + 2] : -fine[nf - 1];
  out[J] = ((rm + rp) + 3.0 * (fine[2 * J] + fine[2 * J + 1])) * 0.125;
}

// FAS coarse right-hand side, literal Eq. 7 assembled over a stored level:
//   Q_H = I(F_h - L_h u) + L_H(I^ u),  for J < nc.
__device__ __forceinline__ double fine_residual(const double* __restrict__ u,
                                                const double* __restrict__ F, int64_t k,
                                                int64_t nf, double w, double gL, double gR) {
  const double l = (k > 0) ? u[k - 1] : 2.0 * gL - u[0];
  const double r = (k < nf - 1) ? u[k + 1] : 2.0 * gR - u[nf - 1];
  return F[k] - (2.0 * u[k] - (l + r)) * w;
}

__global__ void k_tau_literal(const double* __restrict__ u, const double* __restrict__ F,
                              int64_t nc, double gL, double gR, double* __restrict__ out) {
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int64_t nf = 2 * nc;
  const double w = (double)nf * (double)nf, wc = (double)nc * (double)nc;
  const double r1 = fine_residual(u, F, 2 * J, nf, w, gL, gR);
  const double r2 = fine_residual(u, F, 2 * J + 1, nf, w, gL, gR);
  const double rm = (J > 0) ? fine_residual(u, F, 2 * J - 1, nf, w, gL, gR) : -r1;
  const double rp = (2 * J + 2 < nf) ? fine_residual(u, F, 2 * J + 2, nf, w, gL, gR) : -r2;
  const double IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
  const double u0 = (u[2 * J] + u[2 * J + 1]) * 0.5;
  const double ul = (J > 0) ? (u[2 * J - 2] + u[2 * J - 1]) * 0.5 : 2.0 * gL - u0;
  const double ur = (J < nc - 1) ? (u[2 * J + 2] + u[2 * J + 3]) * 0.5 : 2.0 * gR - u0;
  out[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
}

// ---------------------------------------------------------------------------
// SR level: segments with buffers (Sec. 3, Fig. 3; compatible relaxation
// Sec. 3.1, Fig. 5).  One workgroup per segment; the window starts `pad`
// cells left of the core (pad even, >= buffer + 1) so the frozen neighbours
// of the extended patch are inside it.
// ---------------------------------------------------------------------------

struct SegArgs {
  int64_t n;           // fine cells
  double gL, gR;
  int nu;
  int64_t s;           // core cells per segment
  int64_t buffer;      // buffer cells per side
  int64_t pad;         // window offset left of the core
  const double* coarse;  // level n/2 iterate (Pi source; Kaczmarz target)
  const double* f;       // fine right-hand side
  double* out;           // down: I^ of the smoothed cores [n/2]; up: u_out [n]
  double* q_out;         // down, literal tau: coarse rhs [n/2] (else nullptr)
};

// Down pass (Fig. 3 steps 1-5 fused): Pi, nu sweeps on the extended patch,
// then I^ (and literal tau) on the core's coarse cells.  The fine iterate
// never leaves registers.
template <int K>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_down(SegArgs a) {
  __shared__ double xr[kSegMaxThreads], xb[kSegMaxThreads];
  __shared__ double xl2[2 * kSegMaxThreads], xr2[2 * kSegMaxThreads];
  const int64_t n = a.n;
  const int64_t seg = blockIdx.x;
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t tile_lo = core_lo - a.pad;
  const int64_t g0 = tile_lo + (int64_t)threadIdx.x * K;
  double u[K], f[K];
#pragma unroll
  for (int j = 0; j < K; ++j) f[j] = ld(a.f, g0 + j, n);
  load_interp<K>(u, g0, n, a.coarse, a.gL, a.gR);
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  rb_sweeps<K>(u, f, g0, a.nu, lo, hi, n, a.gL, a.gR, xr, xb);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t g = g0 + 2 * p;
    if (g >= core_lo && g < core_hi) a.out[g >> 1] = (u[2 * p] + u[2 * p + 1]) * 0.5;
  }
  if (a.q_out == nullptr) return;  // uniform per launch
  // Literal tau per patch: needs two cells beyond the run on each side.
  const int t = threadIdx.x;
  xl2[2 * t] = u[K - 2];
  xl2[2 * t + 1] = u[K - 1];
  xr2[2 * t] = u[0];
  xr2[2 * t + 1] = u[1];
  __syncthreads();
  double w[K + 4];
  w[0] = (t > 0) ? xl2[2 * (t - 1)] : 0.0;
  w[1] = (t > 0) ? xl2[2 * (t - 1) + 1] : 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) w[j + 2] = u[j];
  w[K + 2] = (t + 1 < (int)blockDim.x) ? xr2[2 * (t + 1)] : 0.0;
  w[K + 3] = (t + 1 < (int)blockDim.x) ? xr2[2 * (t + 1) + 1] : 0.0;
  const int64_t nc = n >> 1;
  const double wf = (double)n * (double)n, wc = (double)nc * (double)nc;
  const double gL = a.gL, gR = a.gR;
  // w[m] holds cell g0 - 2 + m.  Residual F - L w at local offset m (cell k).
  auto res = [&](int m) -> double {
    const int64_t k = g0 - 2 + m;
    const double l = (k > 0) ? w[m - 1] : 2.0 * gL - w[m];
    const double r = (k < n - 1) ? w[m + 1] : 2.0 * gR - w[m];
    return ld(a.f, k, n) - (2.0 * w[m] - (l + r)) * wf;
  };
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t g = g0 + 2 * p;
    if (!(g >= core_lo && g < core_hi)) continue;
    const int64_t J = g >> 1;
    const int m = 2 * p + 2;  // offset of cell 2J
    const double r1 = res(m), r2 = res(m + 1);
    const double rm = (J > 0) ? res(m - 1) : -r1;
    const double rp = (2 * J + 2 < n) ? res(m + 2) : -r2;
    const double IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
    const double u0 = (w[m] + w[m + 1]) * 0.5;
    const double ul = (J > 0) ? (w[m - 2] + w[m - 1]) * 0.5 : 2.0 * gL - u0;
    const double ur = (J < nc - 1) ? (w[m + 2] + w[m + 3]) * 0.5 : 2.0 * gR - u0;
    a.q_out[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
  }
}

// Up pass (Fig. 3 SR branch): full update u = Pi c (Eq. 5), then nu times
// [Kaczmarz projection onto I^ u = c (Eq. 8, Fig. 5), red-black sweep] on
// the extended patch; the core streams to u_out.
template <int K>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_up(SegArgs a) {
  __shared__ double xr[kSegMaxThreads], xb[kSegMaxThreads];
  const int64_t n = a.n, nc = n >> 1;
  const int64_t seg = blockIdx.x;
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t tile_lo = core_lo - a.pad;
  const int64_t g0 = tile_lo + (int64_t)threadIdx.x * K;
  const int64_t J0 = g0 >> 1;
  double u[K], f[K], c[K / 2];
#pragma unroll
  for (int j = 0; j < K; ++j) f[j] = ld(a.f, g0 + j, n);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) c[p] = ld(a.coarse, J0 + p, nc);
  load_interp<K>(u, g0, n, a.coarse, a.gL, a.gR);
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * a.gL, gR2 = 2.0 * a.gR;
  for (int it = 0; it < a.nu; ++it) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      const int64_t g = g0 + 2 * p;
      if (g >= lo && g + 1 < hi) {
        const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
        u[2 * p] = u[2 * p] + r;
        u[2 * p + 1] = u[2 * p + 1] + r;
      }
    }
    rb_half<K, 0>(u, f, g0, lo, hi, n, h2, gL2, gR2, xr);
    rb_half<K, 1>(u, f, g0, lo, hi, n, h2, gL2, gR2, xb);
  }
  store_range<K>(u, g0, core_lo, core_hi < n ? core_hi : n, a.out);
}

// ---------------------------------------------------------------------------
// Coarse core: all levels with at most kCoreMaxCells cells, in one workgroup
// with the level stack resident in LDS.
// ---------------------------------------------------------------------------

constexpr int kCoreThreads = 1024;
constexpr int64_t kCoreMaxCells = 1024;
constexpr int64_t kMaxN0 = 1024;

struct CoreArgs {
  int top;             // coarse-core top level C (levels 0..C)
  int64_t n0;          // cells of level 0
  double gL, gR;
  int nu1, nu2;
  int literal;         // literal tau on the levels below C
  int mode;            // 0: FMG on levels 0..C; 1: V-cycle from a level-C guess
  int src_kind;        // mode 1: kSrcRestrict (from level C+1) or kSrcDirect
  const double* F;     // forcing hierarchy, level l at offset n0 (2^l - 1)
  const double* src;   // mode 1: level C+1 iterate or level-C initial iterate
  const double* rhs_top;  // mode 1: right-hand side of level C
  double* out;         // level-C result
};

__device__ __forceinline__ int64_t lvl_off(int64_t n0, int l) { return n0 * (((int64_t)1 << l) - 1); }

__device__ void core_rb(double* u, const double* q, int64_t n, double gL, double gR) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  for (int colour = 0; colour < 2; ++colour) {
    for (int64_t i = 2 * (int64_t)threadIdx.x + colour; i < n; i += 2 * (int64_t)blockDim.x) {
      const double l = (i > 0) ? u[i - 1] : 0.0;
      const double r = (i < n - 1) ? u[i + 1] : 0.0;
      u[i] = relax(q[i], l, r, i, n, h2, gL2, gR2);
    }
    __syncthreads();
  }
}

__device__ void core_interp(const double* c, int64_t nc, double* fine, double gL, double gR) {
  for (int64_t J = threadIdx.x; J < nc; J += blockDim.x) {
    const double cm2 = coarse_at(c, nc, J - 2, gL, gR), cm1 = coarse_at(c, nc, J - 1, gL, gR);
    const double c0 = c[J];
    const double cp1 = coarse_at(c, nc, J + 1, gL, gR), cp2 = coarse_at(c, nc, J + 2, gL, gR);
    fine[2 * J] = interp_even(cm2, cm1, c0, cp1);
    fine[2 * J + 1] = interp_odd(cm1, c0, cp1, cp2);
  }
  __syncthreads();
}

__device__ void core_restrict(const double* fine, int64_t nc, double* c) {
  for (int64_t J = threadIdx.x; J < nc; J += blockDim.x) c[J] = (fine[2 * J] + fine[2 * J + 1]) * 0.5;
  __syncthreads();
}

// Literal tau (Eq. 7) for the coarse core: qc = I(qf - L_f uf) + L_c(I^ uf).
__device__ void core_tau(const double* uf, const double* qf, int64_t nc, double* qc, double gL,
                         double gR) {
  const int64_t nf = 2 * nc;
  const double w = (double)nf * (double)nf, wc = (double)nc * (double)nc;
  for (int64_t J = threadIdx.x; J < nc; J += blockDim.x) {
    const double r1 = fine_residual(uf, qf, 2 * J, nf, w, gL, gR);
    const double r2 = fine_residual(uf, qf, 2 * J + 1, nf, w, gL, gR);
    const double rm = (J > 0) ? fine_residual(uf, qf, 2 * J - 1, nf, w, gL, gR) : -r1;
    const double rp = (2 * J + 2 < nf) ? fine_residual(uf, qf, 2 * J + 2, nf, w, gL, gR) : -r2;
    const double IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
    const double u0 = (uf[2 * J] + uf[2 * J + 1]) * 0.5;
    const double ul = (J > 0) ? (uf[2 * J - 2] + uf[2 * J - 1]) * 0.5 : 2.0 * gL - u0;
    const double ur = (J < nc - 1) ? (uf[2 * J + 2] + uf[2 * J + 3]) * 0.5 : 2.0 * gR - u0;
    qc[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
  }
  __syncthreads();
}

// Correction (Eq. 4) of the fine iterate (still the pre-smoothed one) from
// the post-smoothed coarse iterate: uf += P(uc - I^ uf).
__device__ void core_correct(const double* uc, int64_t nc, double* uf, double* e) {
  for (int64_t J = threadIdx.x; J < nc; J += blockDim.x)
    e[J] = uc[J] - (uf[2 * J] + uf[2 * J + 1]) * 0.5;
  __syncthreads();
  for (int64_t J = threadIdx.x; J < nc; J += blockDim.x) {
    const double eJ = e[J];
    const double em = (J > 0) ? e[J - 1] : -eJ;
    const double ep = (J < nc - 1) ? e[J + 1] : -eJ;
    uf[2 * J] = uf[2 * J] + (3.0 * eJ + em) * 0.25;
    uf[2 * J + 1] = uf[2 * J + 1] + (3.0 * eJ + ep) * 0.25;
  }
  __syncthreads();
}

// Exact solve of the coarsest level: one-cell closed form, else parallel
// cyclic reduction on h^2 L u = h^2 q + boundary terms (tridiagonal with -1
// off the diagonal, 2 inside, 3 at the ends).
__device__ void core_coarse_solve(double* u, const double* q, int64_t n, double gL, double gR,
                                  double* pa, double* pb, double* pc, double* pd) {
  const double h2 = 1.0 / ((double)n * (double)n);
  if (n == 1) {
    if (threadIdx.x == 0) u[0] = (q[0] * h2 + (2.0 * gL + 2.0 * gR)) / 4.0;
    __syncthreads();
    return;
  }
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    pa[i] = (i > 0) ? -1.0 : 0.0;
    pc[i] = (i < n - 1) ? -1.0 : 0.0;
    pb[i] = (i == 0 || i == n - 1) ? 3.0 : 2.0;
    double d = q[i] * h2;
    if (i == 0) d += 2.0 * gL;
    if (i == n - 1) d += 2.0 * gR;
    pd[i] = d;
  }
  __syncthreads();
  for (int64_t st = 1; st < n; st <<= 1) {
    // n <= kMaxN0 <= blockDim: one row per thread
    const int64_t i = threadIdx.x;
    double na = 0.0, nb = 1.0, ncv = 0.0, nd = 0.0;
    if (i < n) {
      double ai = pa[i], bi = pb[i], ci = pc[i], di = pd[i];
      double k1 = 0.0, k2 = 0.0;
      double am = 0.0, cm = 0.0, dm = 0.0, ap = 0.0, cp = 0.0, dp = 0.0;
      if (i - st >= 0) { k1 = ai / pb[i - st]; am = pa[i - st]; cm = pc[i - st]; dm = pd[i - st]; }
      if (i + st < n) { k2 = ci / pb[i + st]; ap = pa[i + st]; cp = pc[i + st]; dp = pd[i + st]; }
      na = -am * k1;
      ncv = -cp * k2;
      nb = (bi - cm * k1) - ap * k2;
      nd = (di - dm * k1) - dp * k2;
    }
    __syncthreads();
    if (i < n) { pa[i] = na; pb[i] = nb; pc[i] = ncv; pd[i] = nd; }
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) u[i] = pd[i] / pb[i];
  __syncthreads();
}

__global__ __launch_bounds__(kCoreThreads) void k_coarse_core(CoreArgs a) {
  extern __shared__ double sm[];
  const int C = a.top;
  const int64_t n0 = a.n0;
  const int64_t ntot = lvl_off(n0, C + 1);
  double* U = sm;                 // iterates, levels 0..C
  double* Q = sm + ntot;          // right-hand sides in use, levels 0..C
  double* E = Q + ntot;           // coarse error scratch
  const int64_t esz = (C > 0) ? (n0 << (C - 1)) : 1;
  double* PA = E + esz;
  double* PB = PA + n0;
  double* PC = PB + n0;
  double* PD = PC + n0;
  const double gL = a.gL, gR = a.gR;
  for (int64_t i = threadIdx.x; i < ntot; i += blockDim.x) Q[i] = a.F[i];
  const int64_t nC = n0 << C;
  if (a.mode == 1) {
    for (int64_t i = threadIdx.x; i < nC; i += blockDim.x) {
      Q[lvl_off(n0, C) + i] = a.rhs_top[i];
      U[lvl_off(n0, C) + i] = (a.src_kind == kSrcRestrict)
                                   ? (a.src[2 * i] + a.src[2 * i + 1]) * 0.5
                                   : a.src[i];
    }
  }
  __syncthreads();
  // V-cycle on levels 0..t, entered with u^t holding its initial iterate.
  auto vcycle = [&](int t) {
    if (t == 0) {
      core_coarse_solve(U, Q, n0, gL, gR, PA, PB, PC, PD);
      return;
    }
    for (int s = 0; s < a.nu1; ++s) core_rb(U + lvl_off(n0, t), Q + lvl_off(n0, t), n0 << t, gL, gR);
    for (int m = t - 1; m >= 0; --m) {
      const int64_t nm = n0 << m;
      double* um = U + lvl_off(n0, m);
      double* uf = U + lvl_off(n0, m + 1);
      if (a.literal) core_tau(uf, Q + lvl_off(n0, m + 1), nm, Q + lvl_off(n0, m), gL, gR);
      core_restrict(uf, nm, um);
      if (m == 0) core_coarse_solve(um, Q, n0, gL, gR, PA, PB, PC, PD);
      else
        for (int s = 0; s < a.nu1; ++s) core_rb(um, Q + lvl_off(n0, m), nm, gL, gR);
    }
    for (int m = 0; m < t; ++m) {
      const int64_t nm = n0 << m;
      core_correct(U + lvl_off(n0, m), nm, U + lvl_off(n0, m + 1), E);
      for (int s = 0; s < a.nu2; ++s)
        core_rb(U + lvl_off(n0, m + 1), Q + lvl_off(n0, m + 1), nm << 1, gL, gR);
    }
  };
  if (a.mode == 0) {
    core_coarse_solve(U, Q, n0, gL, gR, PA, PB, PC, PD);
    for (int t = 1; t <= C; ++t) {
      core_interp(U + lvl_off(n0, t - 1), n0 << (t - 1), U + lvl_off(n0, t), gL, gR);
      vcycle(t);
    }
  } else {
    vcycle(C);
  }
  for (int64_t i = threadIdx.x; i < nC; i += blockDim.x) a.out[i] = U[lvl_off(n0, C) + i];
}

}  // namespace fmgsr
