// fmgsr_kernels.hpp -- gfx950 kernels of the FMG-FAS-SR solver (1D model
// problem, FP64).  Included by fmgsr.hip only.
//
// Execution model.  A tile kernel gives each workgroup a contiguous window
// of W*K cells of a level; thread t owns the run of K consecutive cells
// [t K, t K + K) of the window in registers.  HBM is only touched through
// coalesced lane-per-element loops (lane i handles window cells i + k W)
// that go through a padded LDS stage; the smoothing itself runs on the
// register runs, and LDS only carries one boundary value per thread per
// half-sweep: red cells (even index) need the left neighbour's last cell,
// black cells the right neighbour's first.
//
// Vertical processing (Sec. 1, Sec. 3: the multigrid cycle is walked
// "vertically" through each patch).  A down kernel starts from the window
// of its top level, smooths, restricts the run in registers (I^ of the
// iterate, full weighting of the right-hand side) and continues on the next
// coarser level with half-length runs, writing every level's core once.  An
// up kernel walks the same levels bottom-up and writes only its top level.
// Windows overlap by a halo that absorbs the cells made stale by the window
// edge (the host sizes it), so every core value equals what a sweep over
// the whole level computes: same operations on the same operands.
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
// contraction so that results are reproducible operation by operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmgsr {

constexpr int kRun = 16;           // cells per thread at the top of a tile
constexpr int kTileThreads = 256;  // threads per stored-level tile
constexpr int kMaxFuse = 4;        // levels per vertical kernel
constexpr int kTileHalo = 64;      // window halo (cells of the top level)
constexpr int kSegRun = 8;         // cells per thread on the SR level
constexpr int kSegMaxThreads = 1024;

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
// Neighbour exchange: each thread publishes its first and last value and
// reads its left neighbour's last and right neighbour's first.  Two LDS
// buffers are used alternately, so one barrier per exchange suffices.
// ---------------------------------------------------------------------------
struct Xch {
  double* buf;  // 4 * W doubles
  int sel;
  __device__ void swap(double first, double last, double& left_last, double& right_first) {
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? 2 * W : 0);
    sel ^= 1;
    b[t] = first;
    b[W + t] = last;
    __syncthreads();
    left_last = (t > 0) ? b[W + t - 1] : 0.0;
    right_first = (t + 1 < W) ? b[t + 1] : 0.0;
  }
  // one value only: the left neighbour's `mine` (0 for the first thread)
  __device__ double from_left(double mine) {
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? 2 * W : 0);
    sel ^= 1;
    b[t] = mine;
    __syncthreads();
    return (t > 0) ? b[t - 1] : 0.0;
  }
  // the right neighbour's `mine` (0 for the last thread)
  __device__ double from_right(double mine) {
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? 2 * W : 0);
    sel ^= 1;
    b[t] = mine;
    __syncthreads();
    return (t + 1 < W) ? b[t + 1] : 0.0;
  }
};

// Per-run bounds in 32-bit local indices (0..K): updatable cells [jlo, jhi)
// and the run positions of the first and last cell of the level (-1 if the
// run does not hold them).
struct RunBounds {
  int jlo, jhi, jb0, jbn;
};

__device__ __forceinline__ RunBounds run_bounds(int64_t g0, int K, int64_t lo, int64_t hi,
                                                int64_t n) {
  RunBounds b;
  const int64_t a = lo - g0, c = hi - g0, z = -g0, e = n - 1 - g0;
  b.jlo = (int)(a < 0 ? 0 : (a > K ? K : a));
  b.jhi = (int)(c < 0 ? 0 : (c > K ? K : c));
  b.jb0 = (z >= 0 && z < K) ? (int)z : -1;
  b.jbn = (e >= 0 && e < K) ? (int)e : -1;
  return b;
}

// One half-sweep of colour C (0 = red = even index) over the run u[0..K)
// (first cell even), updating the cells [jlo, jhi) of the run.
template <int K, int C>
__device__ __forceinline__ void rb_half(double (&u)[K], const double (&f)[K], const RunBounds& rb,
                                        double h2, double gL2, double gR2, double bdiv, Xch& x) {
  double ll, rf;
  x.swap(u[0], u[K - 1], ll, rf);
#pragma unroll
  for (int j = C; j < K; j += 2) {
    double l = (j == 0) ? ll : u[j - 1];
    double r = (j == K - 1) ? rf : u[j + 1];
    double v;
    if (j != rb.jb0 && j != rb.jbn) {
      v = (f[j] * h2 + (l + r)) * 0.5;
    } else {
      if (j == rb.jb0) l = gL2;
      if (j == rb.jbn) r = gR2;
      v = (f[j] * h2 + (l + r)) / bdiv;
    }
    if (j >= rb.jlo && j < rb.jhi) u[j] = v;
  }
}

template <int K>
__device__ __forceinline__ void rb_sweeps(double (&u)[K], const double (&f)[K], int64_t g0,
                                          int nu, int64_t lo, int64_t hi, int64_t n,
                                          double gL, double gR, Xch& x) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  const double bdiv = (n == 1) ? 4.0 : 3.0;
  const RunBounds rb = run_bounds(g0, K, lo, hi, n);
  for (int s = 0; s < nu; ++s) {
    rb_half<K, 0>(u, f, rb, h2, gL2, gR2, bdiv, x);
    rb_half<K, 1>(u, f, rb, h2, gL2, gR2, bdiv, x);
  }
}

// ---------------------------------------------------------------------------
// LDS stage: window cell e lives at e + e / K (one pad slot per run, so a
// thread reading its run and lanes walking consecutive cells are both free
// of bank conflicts).
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ int sidx(int e) { return e + e / K; }

// stage -> registers: thread t takes cells [t K, t K + K)
template <int K>
__device__ __forceinline__ void stage_to_run(const double* st, double (&v)[K]) {
  const int base = threadIdx.x * (K + 1);
#pragma unroll
  for (int j = 0; j < K; ++j) v[j] = st[base + j];
}
template <int K>
__device__ __forceinline__ void run_to_stage(double* st, const double (&v)[K]) {
  const int base = threadIdx.x * (K + 1);
#pragma unroll
  for (int j = 0; j < K; ++j) st[base + j] = v[j];
}

// Coalesced load of window cells [0, W K) (cell e = global wlo + e, valid
// while e < wcount) into registers through the stage: v = val(global index)
// for cells in [0, n), 0 elsewhere.  All K loads are issued unconditionally
// (at a clamped, in-range index) before any is consumed, so their latencies
// overlap; the validity test only selects the value.
template <int K, class Fn>
__device__ __forceinline__ void load_run(double* st, double (&v)[K], int64_t wlo, int wcount,
                                         int64_t n, Fn val) {
  const int W = blockDim.x;
  double tmp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t g = wlo + threadIdx.x + k * W;
    tmp[k] = val(g < 0 ? 0 : (g >= n ? n - 1 : g));
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    const int64_t g = wlo + e;
    st[sidx<K>(e)] = (e < wcount && g >= 0 && g < n) ? tmp[k] : 0.0;
  }
  __syncthreads();
  stage_to_run<K>(st, v);
  __syncthreads();
}

// Registers -> coalesced store of window cells whose global index lies in
// [lo, hi).
template <int K>
__device__ __forceinline__ void store_run(double* st, const double (&v)[K], int64_t wlo,
                                          int64_t lo, int64_t hi, double* __restrict__ out) {
  const int W = blockDim.x;
  run_to_stage<K>(st, v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    const int64_t g = wlo + e;
    if (g >= lo && g < hi) out[g] = st[sidx<K>(e)];
  }
  __syncthreads();
}

// Pi of the coarse level into the runs.  The coarse cells under the run,
// c[0..K/2) = J0..J0+K/2-1, arrive as one coalesced load; the two coarse
// values on each side come from the neighbouring threads (window-edge
// threads read them from HBM), so Pi is exact on the whole window.  Cells
// beyond the domain use the Dirichlet reflections (nested for a one-cell
// level), cells outside [0, n) are set to 0.
template <int K>
__device__ __forceinline__ void interp_from_run(double (&u)[K], const double (&c)[K / 2],
                                                int64_t g0, int64_t n,
                                                const double* __restrict__ cg, double gL,
                                                double gR, Xch& x) {
  const int64_t nc = n >> 1;
  const int64_t J0 = g0 >> 1;
  double l1, r0, l2, r1;
  x.swap(c[0], c[K / 2 - 1], l1, r0);
  x.swap(c[1], c[K / 2 - 2], l2, r1);
  auto at = [&](int64_t j) { return cg[j < 0 ? 0 : (j >= nc ? nc - 1 : j)]; };
  if (threadIdx.x == 0) { l2 = at(J0 - 2); l1 = at(J0 - 1); }
  if (threadIdx.x == blockDim.x - 1) { r0 = at(J0 + K / 2); r1 = at(J0 + K / 2 + 1); }
  double e[K / 2 + 4];  // coarse J0-2 .. J0+K/2+1
  e[0] = l2;
  e[1] = l1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p + 2] = c[p];
  e[K / 2 + 2] = r0;
  e[K / 2 + 3] = r1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t J = J0 + p;
    const double r0p = e[p + 2];
    const double vm1 = (J >= 1) ? e[p + 1] : 2.0 * gL - r0p;
    const double vp1 = (J + 1 < nc) ? e[p + 3] : 2.0 * gR - r0p;
    const double vm2 = (J >= 2) ? e[p] : ((J == 1) ? 2.0 * gL - e[p + 1] : 2.0 * gL - vp1);
    const double vp2 = (J + 2 < nc) ? e[p + 4] : ((J + 2 == nc) ? 2.0 * gR - e[p + 3] : 2.0 * gR - vm1);
    const bool in = (J >= 0 && J < nc);
    u[2 * p] = in ? interp_even(vm2, vm1, r0p, vp1) : 0.0;
    u[2 * p + 1] = in ? interp_odd(vm1, r0p, vp1, vp2) : 0.0;
  }
}

// Pi of the coarse level into the window (coarse run loaded here).
template <int K>
__device__ __forceinline__ void load_interp_run(double* st, double (&v)[K], int64_t wlo,
                                                int wcount, int64_t n,
                                                const double* __restrict__ c, double gL,
                                                double gR, Xch& x) {
  // coarse cells under the window plus the two the last valid pairs reach
  double cr[K / 2];
  load_run<K / 2>(st, cr, wlo >> 1, (wcount + 1) / 2 + 2, n >> 1, [&](int64_t J) { return c[J]; });
  interp_from_run<K>(v, cr, wlo + (int64_t)threadIdx.x * K, n, c, gL, gR, x);
}

// I^ of the finer level (pairs read as one 16-byte load) into the window.
template <int K>
__device__ __forceinline__ void load_restrict_run(double* st, double (&v)[K], int64_t wlo,
                                                  int wcount, int64_t n,
                                                  const double* __restrict__ fine) {
  const double2* __restrict__ f2 = reinterpret_cast<const double2*>(fine);
  load_run<K>(st, v, wlo, wcount, n, [&](int64_t g) {
    const double2 p = f2[g];
    return (p.x + p.y) * 0.5;
  });
}

// In-register restriction of a run to the next coarser level:
// u1 = I^ u (local pairs), f1 = I f (full weighting; needs the neighbours'
// edge values).  g0 is the global index of u[0] on the finer level (nf cells).
template <int K>
__device__ __forceinline__ void restrict_runs(const double (&u)[K], const double (&f)[K],
                                              double (&u1)[K / 2], double (&f1)[K / 2],
                                              int64_t g0, int64_t nf, Xch& x) {
  double fl, fr;
  x.swap(f[0], f[K - 1], fl, fr);
  const RunBounds rb = run_bounds(g0, K, 0, nf, nf);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    u1[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
    double rm = (p == 0) ? fl : f[2 * p - 1];
    double rp = (p == K / 2 - 1) ? fr : f[2 * p + 2];
    if (2 * p == rb.jb0) rm = -f[2 * p];
    if (2 * p + 1 == rb.jbn) rp = -f[2 * p + 1];
    f1[p] = ((rm + rp) + 3.0 * (f[2 * p] + f[2 * p + 1])) * 0.125;
  }
}

// Same full weighting for a right-hand side only.
template <int K>
__device__ __forceinline__ void restrict_rhs_run(const double (&f)[K], double (&f1)[K / 2],
                                                 int64_t g0, int64_t nf, Xch& x) {
  double fl, fr;
  x.swap(f[0], f[K - 1], fl, fr);
  const RunBounds rb = run_bounds(g0, K, 0, nf, nf);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    double rm = (p == 0) ? fl : f[2 * p - 1];
    double rp = (p == K / 2 - 1) ? fr : f[2 * p + 2];
    if (2 * p == rb.jb0) rm = -f[2 * p];
    if (2 * p + 1 == rb.jbn) rp = -f[2 * p + 1];
    f1[p] = ((rm + rp) + 3.0 * (f[2 * p] + f[2 * p + 1])) * 0.125;
  }
}

// ---------------------------------------------------------------------------
// Interior fast paths.  A workgroup whose window lies inside the level with a
// margin (no domain boundary, no reflection, no clipping) takes these: loads
// and stores at plain offsets from one base pointer, Pi and full weighting
// without boundary cases, and red-black updates without per-cell tests.  An
// interior update is computed as fma(l + r, 1/2, F h^2 / 2): the product by
// 1/2 is exact, so this rounds exactly like (F h^2 + (l + r)) / 2 (for normal
// numbers; scaling by 2 commutes with rounding).  Cells at the window edge of
// a tile are updated from a missing neighbour instead of being frozen; they
// go stale at the same rate either way and the halo absorbs them.
// ---------------------------------------------------------------------------

// Coalesced load of window cells [0, W K) from base (all inside the level),
// through the stage, into the runs.  Cells e >= count read base[0] and are
// set to 0 (they lie past the part of the window in use).
template <int K, bool kAll>
__device__ __forceinline__ void load_run_fast(double* st, double (&v)[K],
                                              const double* __restrict__ base, int count) {
  const int W = blockDim.x;
  double tmp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    tmp[k] = base[(kAll || e < count) ? e : 0];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    st[sidx<K>(e)] = (kAll || e < count) ? tmp[k] : 0.0;
  }
  __syncthreads();
  stage_to_run<K>(st, v);
  __syncthreads();
}

// The same in two halves, so that several loads can be in flight together:
// issue_loads puts window cells [0, W K) from base into tmp (lane layout,
// cell threadIdx.x + k W in tmp[k]); stage_tmp moves them into the runs.
template <int K, bool kAll>
__device__ __forceinline__ void issue_loads(double (&tmp)[K], const double* __restrict__ base,
                                            int count) {
  const int W = blockDim.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    tmp[k] = base[(kAll || e < count) ? e : 0];
  }
}
template <int K, bool kAll>
__device__ __forceinline__ void stage_tmp(double* st, const double (&tmp)[K], double (&v)[K],
                                          int count) {
  const int W = blockDim.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    st[sidx<K>(e)] = (kAll || e < count) ? tmp[k] : 0.0;
  }
  __syncthreads();
  stage_to_run<K>(st, v);
  __syncthreads();
}

// Registers -> coalesced store of window cells [clo, chi) to base.
template <int K>
__device__ __forceinline__ void store_run_fast(double* st, const double (&v)[K],
                                               double* __restrict__ base, int clo, int chi) {
  const int W = blockDim.x;
  run_to_stage<K>(st, v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    if (e >= clo && e < chi) base[e] = st[sidx<K>(e)];
  }
  __syncthreads();
}

// Pi from the coarse run c (cells J0..J0+K/2-1 of this thread, cbase =
// address of J0 in HBM): two coarse cells on each side from the neighbours,
// from HBM at the window edges.  No boundary cases.
template <int K>
__device__ __forceinline__ void interp_fast(double (&u)[K], const double (&c)[K / 2],
                                            const double* __restrict__ cbase, Xch& x) {
  double l1, r0, l2, r1;
  x.swap(c[0], c[K / 2 - 1], l1, r0);
  x.swap(c[1], c[K / 2 - 2], l2, r1);
  if (threadIdx.x == 0) { l2 = cbase[-2]; l1 = cbase[-1]; }
  if (threadIdx.x == blockDim.x - 1) { r0 = cbase[K / 2]; r1 = cbase[K / 2 + 1]; }
  double e[K / 2 + 4];
  e[0] = l2;
  e[1] = l1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p + 2] = c[p];
  e[K / 2 + 2] = r0;
  e[K / 2 + 3] = r1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    u[2 * p] = interp_even(e[p], e[p + 1], e[p + 2], e[p + 3]);
    u[2 * p + 1] = interp_odd(e[p + 1], e[p + 2], e[p + 3], e[p + 4]);
  }
}

// Full weighting of a run (no boundary cases).
template <int K>
__device__ __forceinline__ void fw_fast(const double (&f)[K], double (&f1)[K / 2], Xch& x) {
  double fl, fr;
  x.swap(f[0], f[K - 1], fl, fr);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const double rm = (p == 0) ? fl : f[2 * p - 1];
    const double rp = (p == K / 2 - 1) ? fr : f[2 * p + 2];
    f1[p] = ((rm + rp) + 3.0 * (f[2 * p] + f[2 * p + 1])) * 0.125;
  }
}

// fh = F h^2 / 2 for the fused interior update.
template <int K>
__device__ __forceinline__ void half_scaled(const double (&f)[K], double (&fh)[K], int64_t n) {
  const double h2 = 1.0 / ((double)n * (double)n);
#pragma unroll
  for (int j = 0; j < K; ++j) fh[j] = (f[j] * h2) * 0.5;
}

// nu red-black sweeps updating every cell of the run.
template <int K>
__device__ __forceinline__ void rb_sweeps_fast(double (&u)[K], const double (&fh)[K], int nu,
                                               Xch& x) {
  for (int s = 0; s < nu; ++s) {
    const double ll = x.from_left(u[K - 1]);
#pragma unroll
    for (int j = 0; j < K; j += 2) u[j] = __builtin_fma((j == 0 ? ll : u[j - 1]) + u[j + 1], 0.5, fh[j]);
    const double rf = x.from_right(u[0]);
#pragma unroll
    for (int j = 1; j < K; j += 2) u[j] = __builtin_fma(u[j - 1] + (j == K - 1 ? rf : u[j + 1]), 0.5, fh[j]);
  }
}

// nu red-black sweeps updating the run cells [jlo, jhi) only (interior of
// the level; used on SR segments, whose extended patch ends inside threads).
template <int K>
__device__ __forceinline__ void rb_sweeps_masked(double (&u)[K], const double (&fh)[K], int nu,
                                                 int jlo, int jhi, Xch& x) {
  const bool all = (jlo == 0 && jhi == K);
  for (int s = 0; s < nu; ++s) {
    const double ll = x.from_left(u[K - 1]);
    if (all) {
#pragma unroll
      for (int j = 0; j < K; j += 2) u[j] = __builtin_fma((j == 0 ? ll : u[j - 1]) + u[j + 1], 0.5, fh[j]);
    } else {
#pragma unroll
      for (int j = 0; j < K; j += 2) {
        const double v = __builtin_fma((j == 0 ? ll : u[j - 1]) + u[j + 1], 0.5, fh[j]);
        if (j >= jlo && j < jhi) u[j] = v;
      }
    }
    const double rf = x.from_right(u[0]);
    if (all) {
#pragma unroll
      for (int j = 1; j < K; j += 2) u[j] = __builtin_fma(u[j - 1] + (j == K - 1 ? rf : u[j + 1]), 0.5, fh[j]);
    } else {
#pragma unroll
      for (int j = 1; j < K; j += 2) {
        const double v = __builtin_fma(u[j - 1] + (j == K - 1 ? rf : u[j + 1]), 0.5, fh[j]);
        if (j >= jlo && j < jhi) u[j] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Stored levels: vertical down / up kernels
// ---------------------------------------------------------------------------

enum SourceKind : int { kSrcInterp = 0, kSrcRestrict = 1, kSrcDirect = 2 };

struct VertArgs {
  int64_t n;             // cells on the top level of this kernel
  double gL, gR;
  int nu;                // sweeps per level
  int levels;            // levels walked by this kernel (1..kMaxFuse)
  int64_t core;          // top-level core cells per workgroup (divisible by 2^kMaxFuse)
  int64_t halo;          // top-level halo (divisible by 2^kMaxFuse)
  int src_kind;          // down: how the top-level iterate starts
  const double* src;     // down: coarser (Pi), finer (I^) or same-level array
  const double* rhs;     // right-hand side of the top level
  const double* coarse;  // up: post-smoothed level below the bottom level
  const double* pre[kMaxFuse];  // up: pre-smoothed iterates, index = levels below top
  double* out[kMaxFuse];        // down: U of each level; up: out[0] = top result
};

struct TileGeom {
  int64_t wlo;   // window start on this level
  int64_t g0;    // first cell of this thread's run
  int64_t lo, hi;  // updatable cells
  int64_t clo, chi;  // core cells (clipped)
  int64_t n;
};

__device__ __forceinline__ TileGeom tile_geom(const VertArgs& a, int i, int K) {
  TileGeom g;
  g.n = a.n >> i;
  const int64_t W = blockDim.x;
  g.wlo = ((int64_t)blockIdx.x * a.core - a.halo) >> i;
  const int64_t whi = g.wlo + W * K;
  g.g0 = g.wlo + (int64_t)threadIdx.x * K;
  g.lo = g.wlo <= 0 ? 0 : g.wlo + 1;
  g.hi = whi >= g.n ? g.n : whi - 1;
  g.clo = ((int64_t)blockIdx.x * a.core) >> i;
  const int64_t c1 = ((int64_t)blockIdx.x * a.core + a.core) >> i;
  g.chi = c1 < g.n ? c1 : g.n;
  return g;
}

template <int K, int I>
__device__ void down_level(const VertArgs& a, double* st, Xch& x, double (&u)[K],
                           const double (&f)[K]) {
  const TileGeom G = tile_geom(a, I, K);
  rb_sweeps<K>(u, f, G.g0, a.nu, G.lo, G.hi, G.n, a.gL, a.gR, x);
  store_run<K>(st, u, G.wlo, G.clo, G.chi, a.out[I]);
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (I + 1 < a.levels) {
      double u1[K / 2], f1[K / 2];
      restrict_runs<K>(u, f, u1, f1, G.g0, G.n, x);
      down_level<K / 2, I + 1>(a, st, x, u1, f1);
    }
  }
}

constexpr int64_t kInteriorMargin = 4 << kMaxFuse;  // cells kept from the domain ends

// Window of this workgroup on the top level: [wlo, wlo + W K).
__device__ __forceinline__ int64_t top_wlo(const VertArgs& a) {
  return (int64_t)blockIdx.x * a.core - a.halo;
}
__device__ __forceinline__ bool window_interior(int64_t wlo, int64_t cells, int64_t n) {
  return wlo >= kInteriorMargin && wlo + cells + kInteriorMargin <= n;
}

template <int K, int I>
__device__ void down_level_fast(const VertArgs& a, double* st, Xch& x, double (&u)[K],
                                double (&f)[K], int64_t wlo0) {
  const int64_t wlo = wlo0 >> I;
  double f1[K / 2];
  const bool more = (I + 1 < kMaxFuse && K >= 4) && (I + 1 < a.levels);
  if constexpr (I + 1 < kMaxFuse && K >= 4)
    if (more) fw_fast<K>(f, f1, x);
  half_scaled<K>(f, f, a.n >> I);
  rb_sweeps_fast<K>(u, f, a.nu, x);
  store_run_fast<K>(st, u, a.out[I] + wlo, (int)(a.halo >> I), (int)((a.halo + a.core) >> I));
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (more) {
      double u1[K / 2];
#pragma unroll
      for (int p = 0; p < K / 2; ++p) u1[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
      down_level_fast<K / 2, I + 1>(a, st, x, u1, f1, wlo0);
    }
  }
}

// Down leg over `levels` stored levels (Fig. 3 steps 1-2 on the top level,
// then restrict + smooth of the pre-smoothing leg), split tau: the coarse
// right-hand side is the full weighting of the finer one (the Laplacian
// part of tau is identically zero with I^ = average, I = full weighting).
template <int K>
__global__ __launch_bounds__(kTileThreads) void k_down(VertArgs a) {
  __shared__ double st[kTileThreads * (K + 1)];
  __shared__ double xb[4 * kTileThreads];
  Xch x{xb, 0};
  const int wcount = kTileThreads * K;
  const int64_t wlo0 = top_wlo(a);
  double u[K], f[K];
  if (window_interior(wlo0, wcount, a.n)) {
    double tf[K];
    issue_loads<K, true>(tf, a.rhs + wlo0, 0);  // rhs and source loads in flight together
    if (a.src_kind == kSrcInterp) {
      const double* cb = a.src + (wlo0 >> 1);
      double tc[K / 2], c[K / 2];
      issue_loads<K / 2, true>(tc, cb, 0);
      stage_tmp<K, true>(st, tf, f, 0);
      stage_tmp<K / 2, true>(st, tc, c, 0);
      interp_fast<K>(u, c, cb + threadIdx.x * (K / 2), x);
    } else if (a.src_kind == kSrcRestrict) {
      const double2* fb = reinterpret_cast<const double2*>(a.src) + wlo0;
      double tu[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double2 q = fb[threadIdx.x + k * kTileThreads];
        tu[k] = (q.x + q.y) * 0.5;
      }
      stage_tmp<K, true>(st, tf, f, 0);
      stage_tmp<K, true>(st, tu, u, 0);
    } else {
      double tu[K];
      issue_loads<K, true>(tu, a.src + wlo0, 0);
      stage_tmp<K, true>(st, tf, f, 0);
      stage_tmp<K, true>(st, tu, u, 0);
    }
    down_level_fast<K, 0>(a, st, x, u, f, wlo0);
    return;
  }
  const TileGeom G = tile_geom(a, 0, K);
  load_run<K>(st, f, G.wlo, wcount, G.n, [&](int64_t g) { return a.rhs[g]; });
  if (a.src_kind == kSrcInterp)
    load_interp_run<K>(st, u, G.wlo, wcount, G.n, a.src, a.gL, a.gR, x);
  else if (a.src_kind == kSrcRestrict)
    load_restrict_run<K>(st, u, G.wlo, wcount, G.n, a.src);
  else
    load_run<K>(st, u, G.wlo, wcount, G.n, [&](int64_t g) { return a.src[g]; });
  down_level<K, 0>(a, st, x, u, f);
}

// Up leg, level I of the kernel (I = 0 is the top).  On entry f holds this
// level's right-hand side; on return u holds its post-smoothed iterate.
template <int K, int I>
__device__ void up_level(const VertArgs& a, double* st, Xch& x, const double (&f)[K],
                         double (&u)[K]) {
  const TileGeom G = tile_geom(a, I, K);
  const int wcount = (int)blockDim.x * K;
  const int64_t nc = G.n >> 1;
  double c[K / 2];  // post-smoothed coarse iterate of this run's pairs
  bool done = false;
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (I + 1 < a.levels) {
      double f1[K / 2];
      restrict_rhs_run<K>(f, f1, G.g0, G.n, x);
      up_level<K / 2, I + 1>(a, st, x, f1, c);
      done = true;
    }
  }
  if (!done) {
    // bottom of the kernel: coarse iterate from HBM (coalesced via the stage)
    const int64_t cwlo = G.wlo >> 1;
    load_run<K / 2>(st, c, cwlo, wcount / 2, nc, [&](int64_t J) { return a.coarse[J]; });
  }
  // correction (Eq. 4): u = pre + P(c - I^ pre)
  load_run<K>(st, u, G.wlo, wcount, G.n, [&](int64_t g) { return a.pre[I][g]; });
  double e[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p] = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
  double el, er;
  x.swap(e[0], e[K / 2 - 1], el, er);
  // pairs of the run inside the level, and the first / last pair of the level
  const RunBounds pb = run_bounds(G.g0 >> 1, K / 2, 0, nc, nc);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    if (p >= pb.jlo && p < pb.jhi) {
      const double eJ = e[p];
      const double em = (p != pb.jb0) ? ((p == 0) ? el : e[p - 1]) : -eJ;
      const double ep = (p != pb.jbn) ? ((p == K / 2 - 1) ? er : e[p + 1]) : -eJ;
      u[2 * p] = u[2 * p] + (3.0 * eJ + em) * 0.25;
      u[2 * p + 1] = u[2 * p + 1] + (3.0 * eJ + ep) * 0.25;
    }
  }
  rb_sweeps<K>(u, f, G.g0, a.nu, G.lo, G.hi, G.n, a.gL, a.gR, x);
}

// tp holds this level's pre-smoothed iterate in flight (lane layout); the
// coarser levels' loads are issued before descending, so every HBM read of
// the kernel is outstanding at once.
template <int K, int I>
__device__ void up_level_fast(const VertArgs& a, double* st, Xch& x, double (&f)[K],
                              double (&u)[K], const double (&tp)[K], int64_t wlo0) {
  const int64_t wlo = wlo0 >> I;
  double c[K / 2];
  bool done = false;
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (I + 1 < a.levels) {
      double tp1[K / 2];
      issue_loads<K / 2, true>(tp1, a.pre[I + 1] + (wlo >> 1), 0);
      double f1[K / 2];
      fw_fast<K>(f, f1, x);
      up_level_fast<K / 2, I + 1>(a, st, x, f1, c, tp1, wlo0);
      done = true;
    }
  }
  if (!done) {
    double tc[K / 2];
    issue_loads<K / 2, true>(tc, a.coarse + (wlo >> 1), 0);
    stage_tmp<K / 2, true>(st, tc, c, 0);
  }
  half_scaled<K>(f, f, a.n >> I);
  stage_tmp<K, true>(st, tp, u, 0);
  double e[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p] = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
  double el, er;
  x.swap(e[0], e[K / 2 - 1], el, er);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const double em = (p == 0) ? el : e[p - 1];
    const double ep = (p == K / 2 - 1) ? er : e[p + 1];
    u[2 * p] = u[2 * p] + (3.0 * e[p] + em) * 0.25;
    u[2 * p + 1] = u[2 * p + 1] + (3.0 * e[p] + ep) * 0.25;
  }
  rb_sweeps_fast<K>(u, f, a.nu, x);
}

// Up leg over `levels` stored levels, bottom-up (Fig. 3 post-smoothing leg,
// Eq. 4); only the top level's core is written.  Lower right-hand sides are
// the full weighting of the top one (split tau).
template <int K>
__global__ __launch_bounds__(kTileThreads) void k_up(VertArgs a) {
  __shared__ double st[kTileThreads * (K + 1)];
  __shared__ double xb[4 * kTileThreads];
  Xch x{xb, 0};
  const int wcount = kTileThreads * K;
  const int64_t wlo0 = top_wlo(a);
  double u[K], f[K];
  if (window_interior(wlo0, wcount, a.n)) {
    double tf[K], tp[K];
    issue_loads<K, true>(tf, a.rhs + wlo0, 0);
    issue_loads<K, true>(tp, a.pre[0] + wlo0, 0);
    stage_tmp<K, true>(st, tf, f, 0);
    up_level_fast<K, 0>(a, st, x, f, u, tp, wlo0);
    store_run_fast<K>(st, u, a.out[0] + wlo0, (int)a.halo, (int)(a.halo + a.core));
    return;
  }
  const TileGeom G = tile_geom(a, 0, K);
  load_run<K>(st, f, G.wlo, wcount, G.n, [&](int64_t g) { return a.rhs[g]; });
  up_level<K, 0>(a, st, x, f, u);
  store_run<K>(st, u, G.wlo, G.clo, G.chi, a.out[0]);
}

// ---------------------------------------------------------------------------
// Forcing hierarchy: up to kMaxFuse full-weighting restrictions per launch
// ---------------------------------------------------------------------------

template <int K, int I>
__device__ void forcing_level(const VertArgs& a, double* st, Xch& x, const double (&f)[K]) {
  // f holds level I (I >= 1 are written); the next level is its restriction
  const TileGeom G = tile_geom(a, I, K);
  if constexpr (I > 0) store_run<K>(st, f, G.wlo, G.clo, G.chi, a.out[I - 1]);
  if constexpr (I < kMaxFuse && K >= 2) {
    if (I < a.levels) {
      double f1[K / 2];
      restrict_rhs_run<K>(f, f1, G.g0, G.n, x);
      forcing_level<K / 2, I + 1>(a, st, x, f1);
    }
  }
}

template <int K, int I>
__device__ void forcing_level_fast(const VertArgs& a, double* st, Xch& x, double (&f)[K],
                                   int64_t wlo0) {
  if constexpr (I > 0)
    store_run_fast<K>(st, f, a.out[I - 1] + (wlo0 >> I), (int)(a.halo >> I),
                      (int)((a.halo + a.core) >> I));
  if constexpr (I < kMaxFuse && K >= 2) {
    if (I < a.levels) {
      double f1[K / 2];
      fw_fast<K>(f, f1, x);
      forcing_level_fast<K / 2, I + 1>(a, st, x, f1, wlo0);
    }
  }
}

// a.rhs: level with a.n cells; writes a.levels coarser levels into
// out[0..levels) (out[i] = level i+1 below).
template <int K>
__global__ __launch_bounds__(kTileThreads) void k_forcing(VertArgs a) {
  __shared__ double st[kTileThreads * (K + 1)];
  __shared__ double xb[4 * kTileThreads];
  Xch x{xb, 0};
  const int64_t wlo0 = top_wlo(a);
  double f[K];
  if (window_interior(wlo0, kTileThreads * K, a.n)) {
    load_run_fast<K, true>(st, f, a.rhs + wlo0, 0);
    forcing_level_fast<K, 0>(a, st, x, f, wlo0);
    return;
  }
  const TileGeom G = tile_geom(a, 0, K);
  load_run<K>(st, f, G.wlo, kTileThreads * K, G.n, [&](int64_t g) { return a.rhs[g]; });
  forcing_level<K, 0>(a, st, x, f);
}

// ---------------------------------------------------------------------------
// Literal tau (Eq. 7) on a stored level: Q_H = I(F_h - L_h u) + L_H(I^ u)
// ---------------------------------------------------------------------------

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
// Sec. 3.1, Fig. 5).  One workgroup per segment; its window starts `pad`
// cells left of the core (pad even, >= buffer + 1) so the frozen neighbours
// of the extended patch are inside it; cells past the window are dead.
// ---------------------------------------------------------------------------

struct SegArgs {
  int64_t n;             // fine cells
  double gL, gR;
  int nu;
  int64_t s;             // core cells per segment
  int64_t buffer;        // buffer cells per side
  int64_t pad;           // window offset left of the core
  int win;               // window cells actually used (s + 2 pad)
  const double* coarse;  // level n/2 iterate (Pi source; Kaczmarz target)
  const double* f;       // fine right-hand side
  double* out;           // down: I^ of the smoothed cores [n/2]; up: u_out [n]
  double* q_out;         // down, literal tau: coarse rhs [n/2] (else nullptr)
};

// Down pass (Fig. 3 steps 1-5 fused): Pi, nu sweeps on the extended patch,
// then I^ (and literal tau) on the core's coarse cells.  The fine iterate
// never leaves the chip.
template <int K>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_down(SegArgs a) {
  extern __shared__ double sm[];
  const int W = blockDim.x;
  double* st = sm;                   // W (K+1)
  Xch x{sm + W * (K + 1), 0};        // 4 W
  const int64_t n = a.n, nc = n >> 1;
  const int64_t seg = blockIdx.x;
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t wlo = core_lo - a.pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  double u[K], f[K];
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  if (a.q_out == nullptr && window_interior(wlo, (int64_t)W * K, n)) {
    const double* cb = a.coarse + (wlo >> 1);
    double tf[K], tc[K / 2], c[K / 2];
    issue_loads<K, false>(tf, a.f + wlo, a.win);
    issue_loads<K / 2, false>(tc, cb, a.win / 2 + 2);
    stage_tmp<K, false>(st, tf, f, a.win);
    stage_tmp<K / 2, false>(st, tc, c, a.win / 2 + 2);
    interp_fast<K>(u, c, cb + threadIdx.x * (K / 2), x);
    half_scaled<K>(f, f, n);
    const RunBounds rb = run_bounds(g0, K, lo, hi, n);
    rb_sweeps_masked<K>(u, f, a.nu, rb.jlo, rb.jhi, x);
    double uc[K / 2];
#pragma unroll
    for (int p = 0; p < K / 2; ++p) uc[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
    store_run_fast<K / 2>(st, uc, a.out + (wlo >> 1), (int)(a.pad >> 1), (int)((a.pad + a.s) >> 1));
    return;
  }
  load_run<K>(st, f, wlo, a.win, n, [&](int64_t g) { return a.f[g]; });
  load_interp_run<K>(st, u, wlo, a.win, n, a.coarse, a.gL, a.gR, x);
  rb_sweeps<K>(u, f, g0, a.nu, lo, hi, n, a.gL, a.gR, x);
  double uc[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) uc[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
  store_run<K / 2>(st, uc, wlo >> 1, core_lo >> 1, core_hi >> 1, a.out);
  if (a.q_out == nullptr) return;  // uniform per launch
  // Literal tau per patch: two cells beyond the run on each side.
  double l1, r0, l2, r1;
  x.swap(u[0], u[K - 1], l1, r0);
  x.swap(u[1], u[K - 2], l2, r1);
  double w[K + 4];
  w[0] = l2;
  w[1] = l1;
#pragma unroll
  for (int j = 0; j < K; ++j) w[j + 2] = u[j];
  w[K + 2] = r0;
  w[K + 3] = r1;
  const double wf = (double)n * (double)n, wc = (double)nc * (double)nc;
  const double gL = a.gL, gR = a.gR;
  // w[m] holds cell g0 - 2 + m.  Residual F - L w at offset m.
  auto res = [&](int m) -> double {
    const int64_t k = g0 - 2 + m;
    const double l = (k > 0) ? w[m - 1] : 2.0 * gL - w[m];
    const double r = (k < n - 1) ? w[m + 1] : 2.0 * gR - w[m];
    return ld(a.f, k, n) - (2.0 * w[m] - (l + r)) * wf;
  };
  double q[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t g = g0 + 2 * p;
    const int64_t J = g >> 1;
    const int m = 2 * p + 2;  // offset of cell 2J
    q[p] = 0.0;
    if (g >= core_lo && g < core_hi) {
      const double ra = res(m), rb = res(m + 1);
      const double rm = (J > 0) ? res(m - 1) : -ra;
      const double rp = (2 * J + 2 < n) ? res(m + 2) : -rb;
      const double IR = ((rm + rp) + 3.0 * (ra + rb)) * 0.125;
      const double u0 = (w[m] + w[m + 1]) * 0.5;
      const double ul = (J > 0) ? (w[m - 2] + w[m - 1]) * 0.5 : 2.0 * gL - u0;
      const double ur = (J < nc - 1) ? (w[m + 2] + w[m + 3]) * 0.5 : 2.0 * gR - u0;
      q[p] = IR + (2.0 * u0 - (ul + ur)) * wc;
    }
  }
  store_run<K / 2>(st, q, wlo >> 1, core_lo >> 1, core_hi >> 1, a.q_out);
}

// Up pass (Fig. 3 SR branch): full update u = Pi c (Eq. 5), then nu times
// [Kaczmarz projection onto I^ u = c (Eq. 8, Fig. 5), red-black sweep] on
// the extended patch; the core streams to u_out.
template <int K>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_up(SegArgs a) {
  extern __shared__ double sm[];
  const int W = blockDim.x;
  double* st = sm;
  Xch x{sm + W * (K + 1), 0};
  const int64_t n = a.n, nc = n >> 1;
  const int64_t seg = blockIdx.x;
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t wlo = core_lo - a.pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  double u[K], f[K], c[K / 2];
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  if (window_interior(wlo, (int64_t)W * K, n)) {
    const double* cb = a.coarse + (wlo >> 1);
    double tf[K], tc[K / 2];
    issue_loads<K, false>(tf, a.f + wlo, a.win);
    issue_loads<K / 2, false>(tc, cb, a.win / 2 + 2);
    stage_tmp<K, false>(st, tf, f, a.win);
    stage_tmp<K / 2, false>(st, tc, c, a.win / 2 + 2);
    interp_fast<K>(u, c, cb + threadIdx.x * (K / 2), x);
    half_scaled<K>(f, f, n);
    const RunBounds rb = run_bounds(g0, K, lo, hi, n);
    const bool all = (rb.jlo == 0 && rb.jhi == K);
    for (int it = 0; it < a.nu; ++it) {
      if (all) {
#pragma unroll
        for (int p = 0; p < K / 2; ++p) {
          const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
          u[2 * p] = u[2 * p] + r;
          u[2 * p + 1] = u[2 * p + 1] + r;
        }
      } else {
#pragma unroll
        for (int p = 0; p < K / 2; ++p) {
          if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {
            const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
            u[2 * p] = u[2 * p] + r;
            u[2 * p + 1] = u[2 * p + 1] + r;
          }
        }
      }
      rb_sweeps_masked<K>(u, f, 1, rb.jlo, rb.jhi, x);
    }
    store_run_fast<K>(st, u, a.out + wlo, (int)a.pad, (int)(a.pad + a.s));
    return;
  }
  load_run<K>(st, f, wlo, a.win, n, [&](int64_t g) { return a.f[g]; });
  load_run<K / 2>(st, c, wlo >> 1, a.win / 2 + 2, nc, [&](int64_t J) { return a.coarse[J]; });
  interp_from_run<K>(u, c, g0, n, a.coarse, a.gL, a.gR, x);
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * a.gL, gR2 = 2.0 * a.gR;
  const double bdiv = (n == 1) ? 4.0 : 3.0;
  const RunBounds rb = run_bounds(g0, K, lo, hi, n);
  for (int it = 0; it < a.nu; ++it) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {  // both children in the patch
        const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
        u[2 * p] = u[2 * p] + r;
        u[2 * p + 1] = u[2 * p + 1] + r;
      }
    }
    rb_half<K, 0>(u, f, rb, h2, gL2, gR2, bdiv, x);
    rb_half<K, 1>(u, f, rb, h2, gL2, gR2, bdiv, x);
  }
  store_run<K>(st, u, wlo, core_lo, core_hi < n ? core_hi : n, a.out);
}

// ---------------------------------------------------------------------------
// Coarse core: all levels with at most kCoreMaxCells cells, in one workgroup
// with the level stack resident in LDS.  The coarse levels are tiny, so this
// kernel is bound by the latency of its chain of about a hundred dependent
// LDS phases; the code is kept compact (rolled loops, 32-bit indices, one
// call site per phase) so that each phase issues few instructions.
// ---------------------------------------------------------------------------

constexpr int kCoreThreads = 256;
constexpr int64_t kCoreMaxCells = 2048;
constexpr int64_t kMaxN0 = 1024;

struct CoreArgs {
  int top;             // coarse-core top level C (levels 0..C)
  int64_t n0;          // cells of level 0
  double gL, gR;
  int nu1, nu2;
  int literal;         // literal tau on the levels below C
  int mode;            // 0: FMG on levels 0..C; 1: V-cycle from a level-C guess
  int src_kind;        // mode 1: kSrcRestrict (from level C+1) or kSrcDirect
  const double* F[12]; // forcing of levels 0..C (C <= 11)
  const double* src;   // mode 1: level C+1 iterate or level-C initial iterate
  const double* rhs_top;  // mode 1: right-hand side of level C
  double* out;         // level-C result
};

__device__ __forceinline__ int lvl_off(int n0, int l) { return n0 * ((1 << l) - 1); }

// One red-black sweep of a level (n cells) in LDS.
__device__ __forceinline__ void core_rb(double* u, const double* q, int n, double gL2, double gR2) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double bdiv = (n == 1) ? 4.0 : 3.0;
#pragma unroll 1
  for (int colour = 0; colour < 2; ++colour) {
#pragma unroll 1
    for (int i = 2 * (int)threadIdx.x + colour; i < n; i += 2 * (int)blockDim.x) {
      double l = (i > 0) ? u[i - 1] : gL2;
      double r = (i < n - 1) ? u[i + 1] : gR2;
      const double num = q[i] * h2 + (l + r);
      u[i] = (i > 0 && i < n - 1) ? num * 0.5 : num / bdiv;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kCoreThreads) void k_coarse_core(CoreArgs a) {
  extern __shared__ double sm[];
  const int C = a.top;
  const int n0 = (int)a.n0;
  const int T = blockDim.x, tid = threadIdx.x;
  const int ntot = lvl_off(n0, C + 1);
  double* U = sm;                 // iterates, levels 0..C
  double* Q = sm + ntot;          // right-hand sides in use, levels 0..C
  double* E = Q + ntot;           // coarse error of the correction
  const int esz = (C > 0) ? (n0 << (C - 1)) : 0;
  double* PA = E + esz;           // parallel cyclic reduction, two buffers
  const double gL = a.gL, gR = a.gR, gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  const int nC = n0 << C;
  // inputs: all global loads of a level are issued before any is consumed
#pragma unroll 1
  for (int l = 0; l <= C; ++l) {
    const int nl = n0 << l;
    const double* Fl = (l == C && a.mode == 1) ? a.rhs_top : a.F[l];
    double v[kCoreMaxCells / kCoreThreads];
#pragma unroll
    for (int k = 0; k < (int)(kCoreMaxCells / kCoreThreads); ++k) {
      const int i = tid + k * T;
      v[k] = Fl[i < nl ? i : nl - 1];
    }
#pragma unroll
    for (int k = 0; k < (int)(kCoreMaxCells / kCoreThreads); ++k) {
      const int i = tid + k * T;
      if (i < nl) Q[lvl_off(n0, l) + i] = v[k];
    }
  }
  if (a.mode == 1) {
    double v[kCoreMaxCells / kCoreThreads];
#pragma unroll
    for (int k = 0; k < (int)(kCoreMaxCells / kCoreThreads); ++k) {
      int i = tid + k * T;
      i = i < nC ? i : nC - 1;
      v[k] = (a.src_kind == kSrcRestrict) ? (a.src[2 * i] + a.src[2 * i + 1]) * 0.5 : a.src[i];
    }
#pragma unroll
    for (int k = 0; k < (int)(kCoreMaxCells / kCoreThreads); ++k) {
      const int i = tid + k * T;
      if (i < nC) U[lvl_off(n0, C) + i] = v[k];
    }
  }
  __syncthreads();
  // FMG (mode 0): V-cycles on levels 0..t for t = 0..C, each entered with the
  // FMG interpolation of the level below; mode 1: one V-cycle on levels
  // 0..C.  V-cycle (Fig. 1): smooth and restrict from t down to 1, exact
  // solve of level 0, then correct (Eq. 4) and smooth back up to t.
#pragma unroll 1
  for (int t = (a.mode == 0) ? 0 : C; t <= C; ++t) {
    if (a.mode == 0 && t > 0) {
      const int nc = n0 << (t - 1);
      const double* c = U + lvl_off(n0, t - 1);
      double* fine = U + lvl_off(n0, t);
#pragma unroll 1
      for (int J = tid; J < nc; J += T) {
        const double cm2 = coarse_at(c, nc, J - 2, gL, gR), cm1 = coarse_at(c, nc, J - 1, gL, gR);
        const double c0 = c[J];
        const double cp1 = coarse_at(c, nc, J + 1, gL, gR), cp2 = coarse_at(c, nc, J + 2, gL, gR);
        fine[2 * J] = interp_even(cm2, cm1, c0, cp1);
        fine[2 * J + 1] = interp_odd(cm1, c0, cp1, cp2);
      }
      __syncthreads();
    }
    // down leg
#pragma unroll 1
    for (int m = t; m >= 1; --m) {
      const int nm = n0 << m, nc = nm >> 1;
      double* uf = U + lvl_off(n0, m);
      double* qf = Q + lvl_off(n0, m);
#pragma unroll 1
      for (int s = 0; s < a.nu1; ++s) core_rb(uf, qf, nm, gL2, gR2);
      double* uc = U + lvl_off(n0, m - 1);
      double* qc = Q + lvl_off(n0, m - 1);
      const double w = (double)nm * (double)nm, wc = (double)nc * (double)nc;
#pragma unroll 1
      for (int J = tid; J < nc; J += T) {
        const double u0 = (uf[2 * J] + uf[2 * J + 1]) * 0.5;
        if (a.literal) {  // Eq. 7 as written: I(q - L u) + L_c(I^ u)
          auto res = [&](int k) {
            const double l = (k > 0) ? uf[k - 1] : gL2 - uf[0];
            const double r = (k < nm - 1) ? uf[k + 1] : gR2 - uf[nm - 1];
            return qf[k] - (2.0 * uf[k] - (l + r)) * w;
          };
          const double r1 = res(2 * J), r2 = res(2 * J + 1);
          const double rm = (J > 0) ? res(2 * J - 1) : -r1;
          const double rp = (2 * J + 2 < nm) ? res(2 * J + 2) : -r2;
          const double IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
          const double ul = (J > 0) ? (uf[2 * J - 2] + uf[2 * J - 1]) * 0.5 : gL2 - u0;
          const double ur = (J < nc - 1) ? (uf[2 * J + 2] + uf[2 * J + 3]) * 0.5 : gR2 - u0;
          qc[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
        }
        uc[J] = u0;
      }
      __syncthreads();
    }
    // exact solve of level 0: one-cell closed form, else parallel cyclic
    // reduction on h^2 L u = h^2 q + boundary terms (tridiagonal with -1
    // off the diagonal, 2 inside, 3 at the ends); up to 64 unknowns in one
    // wavefront's registers with cross-lane shuffles, else through LDS.
    {
      const double h2 = 1.0 / ((double)n0 * (double)n0);
      if (n0 == 1) {
        if (tid == 0) U[0] = (Q[0] * h2 + (gL2 + gR2)) / 4.0;
      } else if (n0 <= 64) {
        if (tid < 64) {
          const int i = tid;
          const bool in = i < n0;
          double aa = (in && i > 0) ? -1.0 : 0.0;
          double cc = (in && i < n0 - 1) ? -1.0 : 0.0;
          double bb = in ? ((i == 0 || i == n0 - 1) ? 3.0 : 2.0) : 1.0;
          double dd = 0.0;
          if (in) {
            dd = Q[i] * h2;
            if (i == 0) dd += gL2;
            if (i == n0 - 1) dd += gR2;
          }
#pragma unroll 1
          for (int st = 1; st < n0; st <<= 1) {
            const bool hasm = (i - st >= 0), hasp = (i + st < n0);
            const int im = hasm ? i - st : i, ip = hasp ? i + st : i;
            const double am = __shfl(aa, im), bm = __shfl(bb, im), cm = __shfl(cc, im), dm = __shfl(dd, im);
            const double ap = __shfl(aa, ip), bp = __shfl(bb, ip), cp = __shfl(cc, ip), dp = __shfl(dd, ip);
            const double k1 = (in && hasm) ? aa / bm : 0.0;
            const double k2 = (in && hasp) ? cc / bp : 0.0;
            const double na = hasm ? -am * k1 : 0.0;
            const double nc2 = hasp ? -cp * k2 : 0.0;
            const double nb = (bb - (hasm ? cm * k1 : 0.0)) - (hasp ? ap * k2 : 0.0);
            const double nd = (dd - (hasm ? dm * k1 : 0.0)) - (hasp ? dp * k2 : 0.0);
            if (in) { aa = na; bb = nb; cc = nc2; dd = nd; }
          }
          if (in) U[i] = dd / bb;
        }
      } else {
        double *A = PA, *B = PA + n0, *Cc = PA + 2 * n0, *D = PA + 3 * n0;
        double *A2 = PA + 4 * n0, *B2 = PA + 5 * n0, *C2 = PA + 6 * n0, *D2 = PA + 7 * n0;
#pragma unroll 1
        for (int i = tid; i < n0; i += T) {
          A[i] = (i > 0) ? -1.0 : 0.0;
          Cc[i] = (i < n0 - 1) ? -1.0 : 0.0;
          B[i] = (i == 0 || i == n0 - 1) ? 3.0 : 2.0;
          double d = Q[i] * h2;
          if (i == 0) d += gL2;
          if (i == n0 - 1) d += gR2;
          D[i] = d;
        }
        __syncthreads();
#pragma unroll 1
        for (int st = 1; st < n0; st <<= 1) {
#pragma unroll 1
          for (int i = tid; i < n0; i += T) {
            const double ai = A[i], bi = B[i], ci = Cc[i], di = D[i];
            double k1 = 0.0, k2 = 0.0, am = 0.0, cm = 0.0, dm = 0.0, ap = 0.0, cp = 0.0, dp = 0.0;
            if (i - st >= 0) { k1 = ai / B[i - st]; am = A[i - st]; cm = Cc[i - st]; dm = D[i - st]; }
            if (i + st < n0) { k2 = ci / B[i + st]; ap = A[i + st]; cp = Cc[i + st]; dp = D[i + st]; }
            A2[i] = -am * k1;
            C2[i] = -cp * k2;
            B2[i] = (bi - cm * k1) - ap * k2;
            D2[i] = (di - dm * k1) - dp * k2;
          }
          __syncthreads();
          double* tmp;
          tmp = A; A = A2; A2 = tmp;
          tmp = B; B = B2; B2 = tmp;
          tmp = Cc; Cc = C2; C2 = tmp;
          tmp = D; D = D2; D2 = tmp;
        }
#pragma unroll 1
        for (int i = tid; i < n0; i += T) U[i] = D[i] / B[i];
      }
      __syncthreads();
    }
    // up leg
#pragma unroll 1
    for (int m = 0; m < t; ++m) {
      const int nc = n0 << m, nf = nc << 1;
      const double* uc = U + lvl_off(n0, m);
      double* uf = U + lvl_off(n0, m + 1);
#pragma unroll 1
      for (int J = tid; J < nc; J += T) E[J] = uc[J] - (uf[2 * J] + uf[2 * J + 1]) * 0.5;
      __syncthreads();
#pragma unroll 1
      for (int J = tid; J < nc; J += T) {
        const double eJ = E[J];
        const double em = (J > 0) ? E[J - 1] : -eJ;
        const double ep = (J < nc - 1) ? E[J + 1] : -eJ;
        uf[2 * J] = uf[2 * J] + (3.0 * eJ + em) * 0.25;
        uf[2 * J + 1] = uf[2 * J + 1] + (3.0 * eJ + ep) * 0.25;
      }
      __syncthreads();
#pragma unroll 1
      for (int s = 0; s < a.nu2; ++s) core_rb(uf, Q + lvl_off(n0, m + 1), nf, gL2, gR2);
    }
  }
#pragma unroll 1
  for (int i = tid; i < nC; i += T) a.out[i] = U[lvl_off(n0, C) + i];
}

}  // namespace fmgsr
