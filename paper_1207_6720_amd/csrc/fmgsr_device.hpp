// fmgsr_device.hpp -- device helpers shared by the gfx950 FMG-FAS-SR kernels
// (single-problem solver in fmgsr_kernels.hpp, batched reaction solver in
// fmgsr_batched.hip): stencils, the neighbour exchange, register runs and
// their coalesced LDS-staged loads and stores.
//
// Execution model.  A workgroup holds a contiguous window of W*K cells of a
// level; thread t owns the run of K consecutive cells [t K, t K + K) of the
// window in registers.  HBM is only touched through coalesced
// lane-per-element loops (lane i handles window cells i + k W) that go
// through a padded LDS stage; the smoothing itself runs on the register
// runs, and LDS only carries one boundary value per thread per half-sweep.
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

// Whole-wavefront shift by one lane (DPP wave_shr:1 / wave_shl:1, GFX9):
// from_left: lane i takes lane i-1's value, else lane i+1's; the lane without
// a source gets 0.
__device__ __forceinline__ double wave_shift(double v, bool from_left) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int rlo, rhi;
  if (from_left) {
    rlo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xF, 0xF, false);
    rhi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xF, 0xF, false);
  } else {
    rlo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xF, 0xF, false);
    rhi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xF, 0xF, false);
  }
  return __hiloint2double(rhi, rlo);
}

// ---------------------------------------------------------------------------
// Neighbour exchange: each thread publishes a few values of its run (its
// first and last, or four for the one-exchange sweeps and the FMG
// interpolation) and reads its neighbours'.
// Workgroups of several wavefronts go through LDS: two halves of the buffer
// are used alternately, so one barrier per exchange suffices.  A workgroup
// of one wavefront (`wave`) shifts the values across lanes in registers
// (DPP) instead: no LDS and no barrier; the wave barrier only keeps the
// compiler from moving the workgroup's LDS accesses across the exchange,
// which the multi-wavefront barrier also orders.
// ---------------------------------------------------------------------------
// Workgroups are dispatched to the chip's 8 XCDs in turn, and each XCD has
// its own L2.  xcd_block() renumbers the launch so that every XCD takes one
// contiguous range of block indices, in order: neighbouring tiles or
// segments, which share halo cells, then meet in one L2 instead of reading
// the shared cells from HBM twice.  A bijection on [0, gridDim.x) for any
// grid size.
__device__ __forceinline__ int64_t xcd_block() {
  constexpr int64_t kXcds = 8;
  const int64_t n = gridDim.x, b = blockIdx.x;
  const int64_t per = n / kXcds, rem = n % kXcds, x = b % kXcds, k = b / kXcds;
  return x * per + (x < rem ? x : rem) + k;
}

struct Xch {
  double* buf;  // two halves of `half` doubles (unused in wave mode)
  int sel;
  int half;     // >= 2 W for two-value exchanges, >= 4 W for four-value ones
  bool wave = false;
  __device__ __forceinline__ void swap(double first, double last, double& left_last, double& right_first) {
    if (wave) {
      __builtin_amdgcn_wave_barrier();
      left_last = wave_shift(last, true);
      right_first = wave_shift(first, false);
      return;
    }
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? half : 0);
    sel ^= 1;
    b[t] = first;
    b[W + t] = last;
    __syncthreads();
    left_last = (t > 0) ? b[W + t - 1] : 0.0;
    right_first = (t + 1 < W) ? b[t + 1] : 0.0;
  }
  // one value only: the left neighbour's `mine` (0 for the first thread)
  __device__ __forceinline__ double from_left(double mine) {
    if (wave) {
      __builtin_amdgcn_wave_barrier();
      return wave_shift(mine, true);
    }
    const int t = threadIdx.x;
    double* b = buf + (sel ? half : 0);
    sel ^= 1;
    b[t] = mine;
    __syncthreads();
    return (t > 0) ? b[t - 1] : 0.0;
  }
  // the right neighbour's `mine` (0 for the last thread)
  __device__ __forceinline__ double from_right(double mine) {
    if (wave) {
      __builtin_amdgcn_wave_barrier();
      return wave_shift(mine, false);
    }
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? half : 0);
    sel ^= 1;
    b[t] = mine;
    __syncthreads();
    return (t + 1 < W) ? b[t + 1] : 0.0;
  }

  // Exchange of four values per thread, for sweeps with one exchange each:
  // every thread publishes (first, second, last, extra) and reads its left
  // neighbour's last and its right neighbour's first, second and extra (0 at
  // the workgroup edges).
  __device__ __forceinline__ void swap(double first, double second, double last, double extra, double& l_last,
                       double& r_first, double& r_second, double& r_extra) {
    if (wave) {
      __builtin_amdgcn_wave_barrier();
      l_last = wave_shift(last, true);
      r_first = wave_shift(first, false);
      r_second = wave_shift(second, false);
      r_extra = wave_shift(extra, false);
      return;
    }
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? half : 0);
    sel ^= 1;
    b[t] = first;
    b[W + t] = second;
    b[2 * W + t] = last;
    b[3 * W + t] = extra;
    __syncthreads();
    l_last = (t > 0) ? b[2 * W + t - 1] : 0.0;
    const bool r = (t + 1 < W);
    r_first = r ? b[t + 1] : 0.0;
    r_second = r ? b[W + t + 1] : 0.0;
    r_extra = r ? b[3 * W + t + 1] : 0.0;
  }
  // two cells on each side: the left neighbour's last two (l1 = its last)
  // and the right neighbour's first two (r0 = its first)
  __device__ __forceinline__ void swap2(double c0, double c1, double cl1, double cl, double& l2, double& l1,
                        double& r0, double& r1) {
    if (wave) {
      __builtin_amdgcn_wave_barrier();
      l2 = wave_shift(cl1, true);
      l1 = wave_shift(cl, true);
      r0 = wave_shift(c0, false);
      r1 = wave_shift(c1, false);
      return;
    }
    const int W = blockDim.x, t = threadIdx.x;
    double* b = buf + (sel ? half : 0);
    sel ^= 1;
    b[t] = c0;
    b[W + t] = c1;
    b[2 * W + t] = cl1;
    b[3 * W + t] = cl;
    __syncthreads();
    const bool l = (t > 0), r = (t + 1 < W);
    l2 = l ? b[2 * W + t - 1] : 0.0;
    l1 = l ? b[3 * W + t - 1] : 0.0;
    r0 = r ? b[t + 1] : 0.0;
    r1 = r ? b[W + t + 1] : 0.0;
  }
};
// The four-value role of the same exchanger.  A kernel may also pass one
// object in both roles: consecutive exchanges of either kind then alternate
// between the two halves, which keeps one barrier per exchange enough.
using Xch4 = Xch;

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
// overlap; the validity test only selects the value.  issue_run and
// stage_run are its two halves, for callers that put several windows'
// loads in flight at once.
template <int K, class Fn>
__device__ __forceinline__ void issue_run(double (&tmp)[K], int64_t wlo, int64_t n, Fn val) {
  const int W = blockDim.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t g = wlo + threadIdx.x + k * W;
    tmp[k] = val(g < 0 ? 0 : (g >= n ? n - 1 : g));
  }
}
template <int K>
__device__ __forceinline__ void stage_run(double* st, const double (&tmp)[K], double (&v)[K],
                                          int64_t wlo, int wcount, int64_t n) {
  const int W = blockDim.x;
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
template <int K, class Fn>
__device__ __forceinline__ void load_run(double* st, double (&v)[K], int64_t wlo, int wcount,
                                         int64_t n, Fn val) {
  double tmp[K];
  issue_run<K>(tmp, wlo, n, val);
  stage_run<K>(st, tmp, v, wlo, wcount, n);
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

template <int K>
__device__ __forceinline__ void interp_from_e(double (&u)[K], const double (&e)[K / 2 + 4],
                                              int64_t J0, int64_t nc, double gL, double gR);

// Pi of the coarse level into the runs.  The coarse cells under the run,
// c[0..K/2) = J0..J0+K/2-1, arrive as one coalesced load; the two coarse
// values on each side come from the neighbouring threads (window-edge
// threads read them from HBM), so Pi is exact on the whole window.  Cells
// beyond the domain use the Dirichlet reflections (nested for a one-cell
// level), cells outside [0, n) are set to 0.
// The coarse values the window-edge threads read from HBM for Pi: thread
// 0's J0-2, J0-1 and the last thread's J0+K/2, J0+K/2+1 (clamped into the
// level), issued by edge_issue ahead of their use.
struct PiEdges {
  double a, b;
};
template <int K>
__device__ __forceinline__ PiEdges edge_issue(int64_t g0, int64_t n,
                                              const double* __restrict__ cg) {
  const int64_t nc = n >> 1;
  const int64_t J0 = g0 >> 1;
  auto at = [&](int64_t j) { return cg[j < 0 ? 0 : (j >= nc ? nc - 1 : j)]; };
  PiEdges e{0.0, 0.0};
  if (threadIdx.x == 0) { e.a = at(J0 - 2); e.b = at(J0 - 1); }
  if (threadIdx.x == blockDim.x - 1) { e.a = at(J0 + K / 2); e.b = at(J0 + K / 2 + 1); }
  return e;
}

// Pi from the run c and the edge values ed (edge_issue of the same g0).
template <int K>
__device__ __forceinline__ void interp_from_run_edges(double (&u)[K], const double (&c)[K / 2],
                                                      int64_t g0, int64_t n, const PiEdges& ed,
                                                      double gL, double gR, Xch& x) {
  const int64_t nc = n >> 1;
  const int64_t J0 = g0 >> 1;
  double l1, r0, l2, r1;
  x.swap(c[0], c[K / 2 - 1], l1, r0);
  x.swap(c[1], c[K / 2 - 2], l2, r1);
  if (threadIdx.x == 0) { l2 = ed.a; l1 = ed.b; }
  if (threadIdx.x == blockDim.x - 1) { r0 = ed.a; r1 = ed.b; }
  double e[K / 2 + 4];  // coarse J0-2 .. J0+K/2+1
  e[0] = l2;
  e[1] = l1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p + 2] = c[p];
  e[K / 2 + 2] = r0;
  e[K / 2 + 3] = r1;
  interp_from_e<K>(u, e, J0, nc, gL, gR);
}

template <int K>
__device__ __forceinline__ void interp_from_run(double (&u)[K], const double (&c)[K / 2],
                                                int64_t g0, int64_t n,
                                                const double* __restrict__ cg, double gL,
                                                double gR, Xch& x) {
  interp_from_run_edges<K>(u, c, g0, n, edge_issue<K>(g0, n, cg), gL, gR, x);
}

// Pi of the coarse values e[m] = cell J0 - 2 + m (m < K/2 + 4) into the run
// of fine cells 2 J0 .. 2 J0 + K - 1 of a level with 2 nc cells.  Values of
// e outside [0, nc) are never read (Dirichlet reflections instead, nested
// for a one-cell level); fine cells outside the level become 0.
template <int K>
__device__ __forceinline__ void interp_from_e(double (&u)[K], const double (&e)[K / 2 + 4],
                                              int64_t J0, int64_t nc, double gL, double gR) {
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
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  double tc[K / 2], cr[K / 2];
  issue_run<K / 2>(tc, wlo >> 1, n >> 1, [&](int64_t J) { return c[J]; });
  const PiEdges ed = edge_issue<K>(g0, n, c);
  stage_run<K / 2>(st, tc, cr, wlo >> 1, (wcount + 1) / 2 + 2, n >> 1);
  interp_from_run_edges<K>(v, cr, g0, n, ed, gL, gR, x);
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

// Same full weighting for a right-hand side only.  avg (uniform per launch):
// the two-cell average instead, the rhs restriction of the paper's appendix.
template <int K>
__device__ __forceinline__ void restrict_rhs_run(const double (&f)[K], double (&f1)[K / 2],
                                                 int64_t g0, int64_t nf, Xch& x,
                                                 bool avg = false) {
  if (avg) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) f1[p] = (f[2 * p] + f[2 * p + 1]) * 0.5;
    return;
  }
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

// Registers -> coalesced store of window cells [clo, chi) to base.  trail =
// false leaves out the closing barrier: only for the workgroup's last use of
// the stage, or when a barrier comes before its next write.
template <int K>
__device__ __forceinline__ void store_run_fast(double* st, const double (&v)[K],
                                               double* __restrict__ base, int clo, int chi,
                                               bool trail = true) {
  const int W = blockDim.x;
  run_to_stage<K>(st, v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    if (e >= clo && e < chi) base[e] = st[sidx<K>(e)];
  }
  if (trail) __syncthreads();
}

// Two windows staged at once (kAll layout of issue_loads) through two stage
// buffers, with one barrier and no closing one: the caller's next step must
// be an exchange (whose barrier orders these reads before any later write).
template <int K1, int K2>
__device__ __forceinline__ void stage_two(double* st1, const double (&t1)[K1], double (&v1)[K1],
                                          double* st2, const double (&t2)[K2], double (&v2)[K2]) {
  const int W = blockDim.x;
#pragma unroll
  for (int k = 0; k < K1; ++k) st1[sidx<K1>(threadIdx.x + k * W)] = t1[k];
#pragma unroll
  for (int k = 0; k < K2; ++k) st2[sidx<K2>(threadIdx.x + k * W)] = t2[k];
  __syncthreads();
  stage_to_run<K1>(st1, v1);
  stage_to_run<K2>(st2, v2);
}

// Pi from the coarse run c (cells J0..J0+K/2-1 of this thread, cbase =
// address of J0 in HBM): two coarse cells on each side from the neighbours,
// from HBM at the window edges.  No boundary cases.
template <int K>
__device__ __forceinline__ void interp_ring(double (&u)[K], const double (&c)[K / 2],
                                            const double* __restrict__ cbase, double l2,
                                            double l1, double r0, double r1) {
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
template <int K>
__device__ __forceinline__ void interp_fast(double (&u)[K], const double (&c)[K / 2],
                                            const double* __restrict__ cbase, Xch& x) {
  double l1, r0, l2, r1;
  x.swap(c[0], c[K / 2 - 1], l1, r0);
  x.swap(c[1], c[K / 2 - 2], l2, r1);
  interp_ring<K>(u, c, cbase, l2, l1, r0, r1);
}
// The same with one exchange of two cells per side (halves of >= 4 W).
template <int K>
__device__ __forceinline__ void interp_fast1(double (&u)[K], const double (&c)[K / 2],
                                             const double* __restrict__ cbase, Xch4& x4) {
  double l2, l1, r0, r1;
  x4.swap2(c[0], c[1], c[K / 2 - 2], c[K / 2 - 1], l2, l1, r0, r1);
  interp_ring<K>(u, c, cbase, l2, l1, r0, r1);
}

// Full weighting of a run (no boundary cases); avg as in restrict_rhs_run.
template <int K>
__device__ __forceinline__ void fw_fast(const double (&f)[K], double (&f1)[K / 2], Xch& x,
                                        bool avg = false) {
  if (avg) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) f1[p] = (f[2 * p] + f[2 * p + 1]) * 0.5;
    return;
  }
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

// nu red-black sweeps over the run cells [jlo, jhi) with ONE exchange per
// sweep (interior of the level; fh = F h^2 / 2).  The black update of the
// run's last cell needs the right neighbour's first (red) cell after its
// red update; that value is recomputed here from the same operands the
// neighbour uses (its left value is this run's last cell, its right value
// its own second cell, its fh its first), so the result is bitwise the same
// as with an exchange between the two half-sweeps.  nb_upd: whether the
// neighbour's first cell is updated at all (inside the patch).
template <int K>
__device__ __forceinline__ void rb_sweeps_x1(double (&u)[K], const double (&fh)[K], int nu,
                                             int jlo, int jhi, bool nb_upd, Xch4& x) {
  const bool all = (jlo == 0 && jhi == K);
  for (int s = 0; s < nu; ++s) {
    double ll, r0, r1, fK;
    x.swap(u[0], u[1], u[K - 1], fh[0], ll, r0, r1, fK);
#pragma unroll
    for (int j = 0; j < K; j += 2) {
      const double v = __builtin_fma((j == 0 ? ll : u[j - 1]) + u[j + 1], 0.5, fh[j]);
      if (all || (j >= jlo && j < jhi)) u[j] = v;
    }
    const double uK = nb_upd ? __builtin_fma(u[K - 1] + r1, 0.5, fK) : r0;
#pragma unroll
    for (int j = 1; j < K; j += 2) {
      const double v = __builtin_fma(u[j - 1] + (j == K - 1 ? uK : u[j + 1]), 0.5, fh[j]);
      if (all || (j >= jlo && j < jhi)) u[j] = v;
    }
  }
}

}  // namespace fmgsr
