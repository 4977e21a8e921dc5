// fmgsr_kernels.hpp -- gfx950 kernels of the single-problem FMG-FAS-SR
// solver (1D Poisson, FP64).  Included by fmgsr.hip only; the device
// helpers (stencils, exchange, register runs, staged loads) are in
// fmgsr_device.hpp.
//
// Vertical processing (Sec. 1, Sec. 3: the multigrid cycle is walked
// "vertically" through each patch).  A down kernel starts from the window
// of its top level, smooths, restricts the run in registers (I^ of the
// iterate, full weighting of the right-hand side) and continues on the next
// coarser level with half-length runs, writing every level's core once.  An
// up kernel walks the same levels bottom-up and writes only its top level.
// Windows overlap by a halo that absorbs the cells made stale by the window
// edge (the host sizes it), so every core value equals what a sweep over
// the whole level computes: same operations on the same operands.  The
// same holds for the pre-smoothed iterates an up kernel rebuilds in its
// window instead of reading them (src / deep in VertArgs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmgsr_device.hpp"

namespace fmgsr {

// ---------------------------------------------------------------------------
// FP32 relaxation (correction form).  One smoother call forms the FP64
// residual once, runs its sweeps on an FP32 correction d (d = 0 on cells
// that are not updated) and adds d to the FP64 iterate.  In exact arithmetic
// this is the same Gauss-Seidel iteration: with u = u0 + d the point update
// becomes d_i <- (d_{i-1} + d_{i+1} + res_i) / D, res = F h^2 + (l + r) - D u0
// (boundary ghosts in res, homogeneous ghosts for d).
// ---------------------------------------------------------------------------

// Interior runs (no domain boundary in the window): fh = F h^2 / 2, cells
// [jlo, jhi) of the run updated.
template <int K>
__device__ __forceinline__ void cf_sweeps_fast(double (&u)[K], const double (&fh)[K], int nu,
                                               int jlo, int jhi, bool nb_upd, Xch& x, Xch4& x4) {
  if (nu <= 0) return;
  double ll, rf;
  x.swap(u[0], u[K - 1], ll, rf);
  float rh[K], d[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double l = (j == 0) ? ll : u[j - 1];
    const double r = (j == K - 1) ? rf : u[j + 1];
    rh[j] = (float)(__builtin_fma(l + r, 0.5, fh[j]) - u[j]);  // res / 2
    d[j] = 0.0f;
  }
  // one exchange per sweep: the right neighbour's first (red) correction is
  // recomputed from the same operands (see rb_sweeps_x1)
  for (int s = 0; s < nu; ++s) {
    double dl0d, d0, d1, rK;
    x4.swap((double)d[0], (double)d[1], (double)d[K - 1], (double)rh[0], dl0d, d0, d1, rK);
    const float dl0 = (float)dl0d;
#pragma unroll
    for (int j = 0; j < K; j += 2) {
      const float v = __builtin_fmaf((j == 0 ? dl0 : d[j - 1]) + d[j + 1], 0.5f, rh[j]);
      if (j >= jlo && j < jhi) d[j] = v;
    }
    const float dK = nb_upd ? __builtin_fmaf(d[K - 1] + (float)d1, 0.5f, (float)rK) : (float)d0;
#pragma unroll
    for (int j = 1; j < K; j += 2) {
      const float v = __builtin_fmaf(d[j - 1] + (j == K - 1 ? dK : d[j + 1]), 0.5f, rh[j]);
      if (j >= jlo && j < jhi) d[j] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j >= jlo && j < jhi) u[j] = u[j] + (double)d[j];
}

// General runs (domain boundaries, clipped windows): f = F, cells [lo, hi)
// of the level updated.
template <int K>
__device__ __forceinline__ void cf_sweeps(double (&u)[K], const double (&f)[K], int64_t g0,
                                          int nu, int64_t lo, int64_t hi, int64_t n, double gL,
                                          double gR, Xch& x) {
  if (nu <= 0) return;
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  const double bdiv = (n == 1) ? 4.0 : 3.0;
  const RunBounds rb = run_bounds(g0, K, lo, hi, n);
  double ll, rf;
  x.swap(u[0], u[K - 1], ll, rf);
  float rq[K], w[K], d[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double l = (j == 0) ? ll : u[j - 1];
    double r = (j == K - 1) ? rf : u[j + 1];
    double D = 2.0;
    if (j == rb.jb0) { l = gL2; D = bdiv; }
    if (j == rb.jbn) { r = gR2; D = bdiv; }
    const double res = (f[j] * h2 + (l + r)) - D * u[j];
    rq[j] = (float)(res / D);
    w[j] = (float)(1.0 / D);
    d[j] = 0.0f;
  }
  for (int s = 0; s < nu; ++s) {
    const float dl0 = (float)x.from_left((double)d[K - 1]);
#pragma unroll
    for (int j = 0; j < K; j += 2) {
      float dl = (j == 0) ? dl0 : d[j - 1];
      float dr = d[j + 1];
      if (j == rb.jb0) dl = 0.0f;
      if (j == rb.jbn) dr = 0.0f;
      const float v = __builtin_fmaf(dl + dr, w[j], rq[j]);
      if (j >= rb.jlo && j < rb.jhi) d[j] = v;
    }
    const float dr0 = (float)x.from_right((double)d[0]);
#pragma unroll
    for (int j = 1; j < K; j += 2) {
      float dl = d[j - 1];
      float dr = (j == K - 1) ? dr0 : d[j + 1];
      if (j == rb.jb0) dl = 0.0f;
      if (j == rb.jbn) dr = 0.0f;
      const float v = __builtin_fmaf(dl + dr, w[j], rq[j]);
      if (j >= rb.jlo && j < rb.jhi) d[j] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j >= rb.jlo && j < rb.jhi) u[j] = u[j] + (double)d[j];
}

// Smoother dispatch on the arithmetic of the relaxation (interior runs:
// one exchange per sweep).
template <int K, bool F32>
__device__ __forceinline__ void smooth_fast(double (&u)[K], const double (&fh)[K], int nu, Xch& x,
                                            Xch4& x4) {
  if constexpr (F32) cf_sweeps_fast<K>(u, fh, nu, 0, K, true, x, x4);
  else rb_sweeps_x1<K>(u, fh, nu, 0, K, true, x4);
}
template <int K, bool F32>
__device__ __forceinline__ void smooth_masked(double (&u)[K], const double (&fh)[K], int nu,
                                              int jlo, int jhi, bool nb_upd, Xch& x, Xch4& x4) {
  if constexpr (F32) cf_sweeps_fast<K>(u, fh, nu, jlo, jhi, nb_upd, x, x4);
  else rb_sweeps_x1<K>(u, fh, nu, jlo, jhi, nb_upd, x4);
}
template <int K, bool F32>
__device__ __forceinline__ void smooth_general(double (&u)[K], const double (&f)[K], int64_t g0,
                                               int nu, int64_t lo, int64_t hi, int64_t n,
                                               double gL, double gR, Xch& x) {
  if constexpr (F32) cf_sweeps<K>(u, f, g0, nu, lo, hi, n, gL, gR, x);
  else rb_sweeps<K>(u, f, g0, nu, lo, hi, n, gL, gR, x);
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
  const double* src;     // down: coarser (Pi), finer (I^) or same-level array;
                         // up: the level below's FMG iterate when the top
                         // level's pre-smoothed iterate is rebuilt here (Pi,
                         // then nu_pre sweeps, as the down kernel made it)
                         // instead of read from pre[0]; else null
  int nu_pre;            // up with src: the down leg's sweeps per level
  const double* rhs;     // right-hand side of the top level
  const double* coarse;  // up: post-smoothed level below the bottom level
  const double* pre[kMaxFuse];  // up: pre-smoothed iterates, index = levels below top
  int sr_top;            // up: the top level is an unstored SR level, rebuilt by
                         // the full update from the level below and compatible
                         // relaxation (pre[0] unused)
  double* part;          // up, SR top: per-tile (sum u, sum u^2) of the top core,
                         // or nullptr
  double* out[kMaxFuse];        // down: U of each level (null: not stored);
                                // up: out[0] = top result
  // tile of workgroup b: tile0 + b, plus gap from b = gap_at on (a launch
  // over a subset of the tiles); tile: the result, set by the kernel
  int64_t tile0, gap_at, gap, tile;
  int ravg;              // forcing: rhs restriction = two-cell average
  int deep;              // a down / up pair over the same levels whose up
                         // kernel rebuilds, on interior tiles, the pre-smoothed
                         // iterates of levels 0..levels-2 from src (down:
                         // those levels are stored only by tiles next to a
                         // tile on the general path, whose up kernel reads them)
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
  g.wlo = (a.tile * a.core - a.halo) >> i;
  const int64_t whi = g.wlo + W * K;
  g.g0 = g.wlo + (int64_t)threadIdx.x * K;
  g.lo = g.wlo <= 0 ? 0 : g.wlo + 1;
  g.hi = whi >= g.n ? g.n : whi - 1;
  g.clo = (a.tile * a.core) >> i;
  const int64_t c1 = (a.tile * a.core + a.core) >> i;
  g.chi = c1 < g.n ? c1 : g.n;
  return g;
}

// Runs of the general path on a level whose run starts and size are
// multiples of K (uniform per launch): the level's first cell can only be
// a run's cell 0 and its last cell a run's cell K-1.
struct EdgeRun {
  bool b0, bn;      // this run holds the level's first / last cell
  double fb0, fbn;  // F h^2 of those two cells
  double gL2, gR2;  // the boundary terms of their closures: 2 gL, 2 gR
};

// fh = F h^2 / 2 of the run and its EdgeRun (g0: first cell of the run).
template <int K>
__device__ __forceinline__ EdgeRun edge_run(const double (&f)[K], double (&fh)[K], int64_t g0,
                                            int64_t n, double gL, double gR) {
  const double h2 = 1.0 / ((double)n * (double)n);
  EdgeRun e;
  e.b0 = (g0 == 0);
  e.bn = (g0 + K == n);
  e.fb0 = f[0] * h2;
  e.fbn = f[K - 1] * h2;
  e.gL2 = 2.0 * gL;
  e.gR2 = 2.0 * gR;
#pragma unroll
  for (int j = 0; j < K; ++j) fh[j] = (f[j] * h2) * 0.5;
  return e;
}

// nu red-black sweeps over such a run: every cell takes the interior
// update, then the level's first (red) and last (black) cell are recomputed
// with their boundary closure (ghost value 2 g - u), in the operation order
// of the per-cell form, so the level's cells come out bitwise as with it.
// Cells outside the level and at the window's edges take values from
// undefined neighbours; as on interior tiles only halo cells depend on them,
// and the boundary closures read none.
template <int K>
__device__ __forceinline__ void rb_sweeps_edge(double (&u)[K], const double (&fh)[K], int nu,
                                               const EdgeRun& e, Xch& x) {
  for (int s = 0; s < nu; ++s) {
    const double ll = x.from_left(u[K - 1]);
#pragma unroll
    for (int j = 0; j < K; j += 2) u[j] = __builtin_fma((j == 0 ? ll : u[j - 1]) + u[j + 1], 0.5, fh[j]);
    if (e.b0) u[0] = (e.fb0 + (e.gL2 + u[1])) / 3.0;
    const double rf = x.from_right(u[0]);
#pragma unroll
    for (int j = 1; j < K; j += 2) u[j] = __builtin_fma(u[j - 1] + (j == K - 1 ? rf : u[j + 1]), 0.5, fh[j]);
    if (e.bn) u[K - 1] = (e.fbn + (u[K - 2] + e.gR2)) / 3.0;
  }
}

// Whether the level's runs start at multiples of K and its size is one
// (uniform per launch): the general path's FP64 sweeps then take the
// interior update with two boundary fix-ups (rb_sweeps_edge).
__device__ __forceinline__ bool edge_aligned(const TileGeom& G, int K) {
  return G.n % K == 0 && G.wlo % K == 0;
}

template <int K, int I, bool F32, bool E = false>
__device__ __forceinline__ void down_level(const VertArgs& a, double* st, Xch& x, double (&u)[K],
                           const double (&f)[K]) {
  const TileGeom G = tile_geom(a, I, K);
  if constexpr (!F32 && !E) {
    if (edge_aligned(G, K)) {
      down_level<K, I, F32, true>(a, st, x, u, f);
      return;
    }
  }
  if constexpr (E) {
    double f1[K / 2], fh[K];
    const bool more = (I + 1 < kMaxFuse && K >= 4) && (I + 1 < a.levels);
    if (more) restrict_rhs_run<K>(f, f1, G.g0, G.n, x);
    const EdgeRun e = edge_run<K>(f, fh, G.g0, G.n, a.gL, a.gR);
    rb_sweeps_edge<K>(u, fh, a.nu, e, x);
    if (a.out[I]) store_run<K>(st, u, G.wlo, G.clo, G.chi, a.out[I]);  // null: SR level
    if constexpr (I + 1 < kMaxFuse && K >= 4) {
      if (more) {
        double u1[K / 2];
#pragma unroll
        for (int p = 0; p < K / 2; ++p) u1[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
        down_level<K / 2, I + 1, F32>(a, st, x, u1, f1);
      }
    }
    return;
  }
  smooth_general<K, F32>(u, f, G.g0, a.nu, G.lo, G.hi, G.n, a.gL, a.gR, x);
  if (a.out[I]) store_run<K>(st, u, G.wlo, G.clo, G.chi, a.out[I]);  // null: SR level
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (I + 1 < a.levels) {
      double u1[K / 2], f1[K / 2];
      restrict_runs<K>(u, f, u1, f1, G.g0, G.n, x);
      down_level<K / 2, I + 1, F32>(a, st, x, u1, f1);
    }
  }
}

constexpr int64_t kInteriorMargin = 4 << kMaxFuse;  // cells kept from the domain ends

__device__ __forceinline__ int64_t tile_index(const VertArgs& a) {
  const int64_t b = xcd_block();
  return a.tile0 + b + (b >= a.gap_at ? a.gap : 0);
}

// Window of this workgroup on the top level: [wlo, wlo + W K).
__device__ __forceinline__ int64_t top_wlo(const VertArgs& a) {
  return a.tile * a.core - a.halo;
}
__device__ __forceinline__ bool window_interior(int64_t wlo, int64_t cells, int64_t n) {
  return wlo >= kInteriorMargin && wlo + cells + kInteriorMargin <= n;
}

// A deep pair's down kernel leaves out the levels between its top and its
// bottom on interior tiles whose neighbours are interior too.
__device__ __forceinline__ bool deep_skips(const VertArgs& a, int I, int64_t wlo0, int64_t wc) {
  if (!a.deep || I == 0 || I + 1 >= a.levels) return false;
  return window_interior(wlo0 - a.core, wc, a.n) && window_interior(wlo0 + a.core, wc, a.n);
}

template <int K, int I, bool F32>
__device__ __forceinline__ void down_level_fast(const VertArgs& a, double* st, Xch& x, Xch4& x4, double (&u)[K],
                                double (&f)[K], int64_t wlo0) {
  const int64_t wlo = wlo0 >> I;
  double f1[K / 2];
  const bool more = (I + 1 < kMaxFuse && K >= 4) && (I + 1 < a.levels);
  if constexpr (I + 1 < kMaxFuse && K >= 4)
    if (more) fw_fast<K>(f, f1, x);
  half_scaled<K>(f, f, a.n >> I);
  smooth_fast<K, F32>(u, f, a.nu, x, x4);
  // null: a level never stored (uniform per launch)
  if (a.out[I] && !deep_skips(a, I, wlo0, (int64_t)blockDim.x * (K << I)))
    store_run_fast<K>(st, u, a.out[I] + wlo, (int)(a.halo >> I), (int)((a.halo + a.core) >> I),
                      more);  // the last level's store is the stage's last use
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (more) {
      double u1[K / 2];
#pragma unroll
      for (int p = 0; p < K / 2; ++p) u1[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
      down_level_fast<K / 2, I + 1, F32>(a, st, x, x4, u1, f1, wlo0);
    }
  }
}

// ---------------------------------------------------------------------------
// Forcing hierarchy: up to kMaxFuse full-weighting restrictions per launch
// ---------------------------------------------------------------------------

template <int K, int I>
__device__ void forcing_level(const VertArgs& a, double* st, Xch& x, const double (&f)[K]) {
  // f holds level I (I >= 1 are written); the next level is its restriction
  const TileGeom G = tile_geom(a, I, K);
  if constexpr (I > 0)
    if (a.out[I - 1]) store_run<K>(st, f, G.wlo, G.clo, G.chi, a.out[I - 1]);  // null: not stored
  if constexpr (I < kMaxFuse && K >= 2) {
    if (I < a.levels) {
      double f1[K / 2];
      restrict_rhs_run<K>(f, f1, G.g0, G.n, x, a.ravg);
      forcing_level<K / 2, I + 1>(a, st, x, f1);
    }
  }
}

template <int K, int I>
__device__ void forcing_level_fast(const VertArgs& a, double* st, Xch& x, double (&f)[K],
                                   int64_t wlo0) {
  if constexpr (I > 0)
    if (a.out[I - 1])  // null: not stored (uniform per launch)
      store_run_fast<K>(st, f, a.out[I - 1] + (wlo0 >> I), (int)(a.halo >> I),
                        (int)((a.halo + a.core) >> I));
  if constexpr (I < kMaxFuse && K >= 2) {
    if (I < a.levels) {
      double f1[K / 2];
      fw_fast<K>(f, f1, x, a.ravg);
      forcing_level_fast<K / 2, I + 1>(a, st, x, f1, wlo0);
    }
  }
}

// a.rhs: level with a.n cells; writes a.levels coarser levels into
// out[0..levels) (out[i] = level i+1 below).
// One forcing tile (a.tile set): load, then the restriction chain.
template <int K, int T>
__device__ __forceinline__ void forcing_tile(const VertArgs& a, double* st, Xch& x) {
  const int64_t wlo0 = top_wlo(a);
  double f[K];
  if (window_interior(wlo0, T * K, a.n)) {
    load_run_fast<K, true>(st, f, a.rhs + wlo0, 0);
    forcing_level_fast<K, 0>(a, st, x, f, wlo0);
    return;
  }
  const TileGeom G = tile_geom(a, 0, K);
  load_run<K>(st, f, G.wlo, T * K, G.n, [&](int64_t g) { return a.rhs[g]; });
  forcing_level<K, 0>(a, st, x, f);
}

template <int K, int T>
__global__ __launch_bounds__(T) void k_forcing(VertArgs a) {
  __shared__ double st[T * (K + 1)];
  __shared__ double xb[T == 64 ? 1 : 4 * T];
  Xch x{xb, 0, 2 * T, T == 64};
  a.tile = tile_index(a);
  forcing_tile<K, T>(a, st, x);
}

// Down leg over `levels` stored levels (Fig. 3 steps 1-2 on the top level,
// then restrict + smooth of the pre-smoothing leg), split tau: the coarse
// right-hand side is the full weighting of the finer one (the Laplacian
// part of tau is identically zero with I^ = average, I = full weighting).
// OCC wavefronts per SIMD: 3 (at most 168 VGPRs, a few spilled; 51 KB of LDS
// per 256-thread workgroup) for launches of many tiles, 2 (no spills; a
// second stage buffer lets the rhs and the interpolation source share one
// barrier) for the latency-bound small ones.  T threads per workgroup: 256,
// or one wavefront (64), whose exchanges are lane shifts.
template <int K, bool F32, int OCC, int T>
__global__ __launch_bounds__(T, OCC) void k_down(VertArgs a) {
  __shared__ double st[T * (K + 1)];
  __shared__ double st2[OCC == 2 ? T * (K / 2 + 1) : 1];
  __shared__ double xb[T == 64 ? 1 : 8 * T];
  Xch x{xb, 0, 4 * T, T == 64};
  Xch4& x4 = x;  // one exchanger in both roles
  const int wcount = T * K;
  a.tile = tile_index(a);
  const int64_t wlo0 = top_wlo(a);
  double u[K], f[K];
  if (window_interior(wlo0, wcount, a.n)) {
    double tf[K];
    issue_loads<K, true>(tf, a.rhs + wlo0, 0);  // rhs and source loads in flight together
    if (a.src_kind == kSrcInterp) {
      const double* cb = a.src + (wlo0 >> 1);
      double tc[K / 2], c[K / 2];
      issue_loads<K / 2, true>(tc, cb, 0);
      if constexpr (OCC == 2) {
        stage_two<K, K / 2>(st, tf, f, st2, tc, c);
      } else {
        stage_tmp<K, true>(st, tf, f, 0);
        stage_tmp<K / 2, true>(st, tc, c, 0);
      }
      interp_fast1<K>(u, c, cb + threadIdx.x * (K / 2), x4);
    } else if (a.src_kind == kSrcRestrict) {
      const double2* fb = reinterpret_cast<const double2*>(a.src) + wlo0;
      double tu[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double2 q = fb[threadIdx.x + k * T];
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
    down_level_fast<K, 0, F32>(a, st, x, x4, u, f, wlo0);
    return;
  }
  // edge tile: the rhs, the source and Pi's edge values in flight together
  const TileGeom G = tile_geom(a, 0, K);
  double tf[K];
  issue_run<K>(tf, G.wlo, G.n, [&](int64_t g) { return a.rhs[g]; });
  if (a.src_kind == kSrcInterp) {
    double tc[K / 2], c[K / 2];
    issue_run<K / 2>(tc, G.wlo >> 1, G.n >> 1, [&](int64_t J) { return a.src[J]; });
    const PiEdges ed = edge_issue<K>(G.g0, G.n, a.src);
    stage_run<K>(st, tf, f, G.wlo, wcount, G.n);
    stage_run<K / 2>(st, tc, c, G.wlo >> 1, (wcount + 1) / 2 + 2, G.n >> 1);
    interp_from_run_edges<K>(u, c, G.g0, G.n, ed, a.gL, a.gR, x);
  } else {
    double tu[K];
    if (a.src_kind == kSrcRestrict) {
      const double2* __restrict__ f2 = reinterpret_cast<const double2*>(a.src);
      issue_run<K>(tu, G.wlo, G.n, [&](int64_t g) {
        const double2 q = f2[g];
        return (q.x + q.y) * 0.5;
      });
    } else {
      issue_run<K>(tu, G.wlo, G.n, [&](int64_t g) { return a.src[g]; });
    }
    stage_run<K>(st, tf, f, G.wlo, wcount, G.n);
    stage_run<K>(st, tu, u, G.wlo, wcount, G.n);
  }
  down_level<K, 0, F32>(a, st, x, u, f);
}

// Up leg, level I of the kernel (I = 0 is the top).  On entry f holds this
// level's right-hand side; on return u holds its post-smoothed iterate.
template <int K, int I, bool F32, bool E = false>
__device__ __forceinline__ void up_level(const VertArgs& a, double* st, Xch& x, const double (&f)[K],
                         double (&u)[K]) {
  const TileGeom G = tile_geom(a, I, K);
  if constexpr (!F32 && !E) {
    if (edge_aligned(G, K)) {
      up_level<K, I, F32, true>(a, st, x, f, u);
      return;
    }
  }
  const int wcount = (int)blockDim.x * K;
  const int64_t nc = G.n >> 1;
  double c[K / 2];  // post-smoothed coarse iterate of this run's pairs
  bool done = false;
  if constexpr (I + 1 < kMaxFuse && K >= 4) {
    if (I + 1 < a.levels) {
      double f1[K / 2];
      restrict_rhs_run<K>(f, f1, G.g0, G.n, x);
      up_level<K / 2, I + 1, F32>(a, st, x, f1, c);
      done = true;
    }
  }
  if (!done) {
    // bottom of the kernel: coarse iterate from HBM (coalesced via the stage)
    const int64_t cwlo = G.wlo >> 1;
    load_run<K / 2>(st, c, cwlo, wcount / 2, nc, [&](int64_t J) { return a.coarse[J]; });
  }
  if (I == 0 && a.sr_top) {
    // SR top level (Eq. 5, Fig. 5): u = Pi c, then nu x [Kaczmarz onto
    // I^ u = c, red-black sweep]; the window-edge neighbours' coarse values
    // are unknown here (they only feed halo cells)
    double l1, r0, l2, r1;
    x.swap(c[0], c[K / 2 - 1], l1, r0);
    x.swap(c[1], c[K / 2 - 2], l2, r1);
    double e[K / 2 + 4];
    e[0] = l2;
    e[1] = l1;
#pragma unroll
    for (int p = 0; p < K / 2; ++p) e[p + 2] = c[p];
    e[K / 2 + 2] = r0;
    e[K / 2 + 3] = r1;
    interp_from_e<K>(u, e, G.g0 >> 1, nc, a.gL, a.gR);
    const RunBounds rb = run_bounds(G.g0, K, G.lo, G.hi, G.n);
    const double h2 = 1.0 / ((double)G.n * (double)G.n);
    const double gL2 = 2.0 * a.gL, gR2 = 2.0 * a.gR;
    const double bdiv = (G.n == 1) ? 4.0 : 3.0;
    for (int it = 0; it < a.nu; ++it) {
#pragma unroll
      for (int p = 0; p < K / 2; ++p) {
        if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {  // both children updatable
          const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
          u[2 * p] = u[2 * p] + r;
          u[2 * p + 1] = u[2 * p + 1] + r;
        }
      }
      if constexpr (F32) {
        cf_sweeps<K>(u, f, G.g0, 1, G.lo, G.hi, G.n, a.gL, a.gR, x);
      } else {
        rb_half<K, 0>(u, f, rb, h2, gL2, gR2, bdiv, x);
        rb_half<K, 1>(u, f, rb, h2, gL2, gR2, bdiv, x);
      }
    }
    return;
  }
  // correction (Eq. 4): u = pre + P(c - I^ pre)
  double fh[E ? K : 1];
  EdgeRun eg{};
  if constexpr (E) eg = edge_run<K>(f, fh, G.g0, G.n, a.gL, a.gR);
  bool rebuilt = false;
  if constexpr (I == 0) {
    if (a.src) {
      // the pre-smoothed top level, rebuilt exactly as the down kernel made
      // it in the same window; its stale edge cells stay outside the core's
      // reach
      load_interp_run<K>(st, u, G.wlo, wcount, G.n, a.src, a.gL, a.gR, x);
      if constexpr (E) rb_sweeps_edge<K>(u, fh, a.nu_pre, eg, x);
      else smooth_general<K, F32>(u, f, G.g0, a.nu_pre, G.lo, G.hi, G.n, a.gL, a.gR, x);
      rebuilt = true;
    }
  }
  if (!rebuilt) load_run<K>(st, u, G.wlo, wcount, G.n, [&](int64_t g) { return a.pre[I][g]; });
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
  if constexpr (E) rb_sweeps_edge<K>(u, fh, a.nu, eg, x);
  else smooth_general<K, F32>(u, f, G.g0, a.nu, G.lo, G.hi, G.n, a.gL, a.gR, x);
}

// Interior runs, fh = F h^2 / 2 of the level, c = its post-smoothed coarse
// iterate.  SR top level (Eq. 5, Fig. 5): u = Pi c, then nu x [Kaczmarz onto
// I^ u = c, sweep].
template <int K, bool F32>
__device__ __forceinline__ void sr_top_fast(const VertArgs& a, Xch& x, Xch4& x4, double (&fh)[K],
                                            double (&u)[K], const double (&c)[K / 2]) {
  double l2, l1, r0, r1;
  x4.swap2(c[0], c[1], c[K / 2 - 2], c[K / 2 - 1], l2, l1, r0, r1);
  double ec[K / 2 + 4];
  ec[0] = l2;
  ec[1] = l1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) ec[p + 2] = c[p];
  ec[K / 2 + 2] = r0;
  ec[K / 2 + 3] = r1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    u[2 * p] = interp_even(ec[p], ec[p + 1], ec[p + 2], ec[p + 3]);
    u[2 * p + 1] = interp_odd(ec[p + 1], ec[p + 2], ec[p + 3], ec[p + 4]);
  }
  for (int it = 0; it < a.nu; ++it) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
      u[2 * p] = u[2 * p] + r;
      u[2 * p + 1] = u[2 * p + 1] + r;
    }
    smooth_fast<K, F32>(u, fh, 1, x, x4);
  }
}

// Correction (Eq. 4) u = pre + P(c - I^ pre) of interior runs (u holds pre
// on entry), then the post-sweeps.
template <int K, bool F32>
__device__ __forceinline__ void correct_fast(const VertArgs& a, Xch& x, Xch4& x4, double (&fh)[K],
                                             double (&u)[K], const double (&c)[K / 2]) {
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
  smooth_fast<K, F32>(u, fh, a.nu, x, x4);
}

// tp holds this level's pre-smoothed iterate in flight (lane layout); the
// coarser levels' loads are issued before descending, so every HBM read of
// the kernel is outstanding at once.
template <int K, int I, bool F32>
__device__ __forceinline__ void up_level_fast(const VertArgs& a, double* st, Xch& x, Xch4& x4, double (&f)[K],
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
      up_level_fast<K / 2, I + 1, F32>(a, st, x, x4, f1, c, tp1, wlo0);
      done = true;
    }
  }
  if (!done) {
    double tc[K / 2];
    issue_loads<K / 2, true>(tc, a.coarse + (wlo >> 1), 0);
    stage_tmp<K / 2, true>(st, tc, c, 0);
  }
  half_scaled<K>(f, f, a.n >> I);
  if constexpr (I == 0) {
    if (a.sr_top) {
      sr_top_fast<K, F32>(a, x, x4, f, u, c);
      return;
    }
  }
  bool rebuilt = false;
  if constexpr (I == 0) {
    if (a.src) {
      // rebuilt pre-smoothed top level (tp[0, K/2) holds the Pi source run)
      const double* cb = a.src + (wlo0 >> 1);
      double tc[K / 2], cs[K / 2];
#pragma unroll
      for (int k = 0; k < K / 2; ++k) tc[k] = tp[k];
      stage_tmp<K / 2, true>(st, tc, cs, 0);
      interp_fast1<K>(u, cs, cb + threadIdx.x * (K / 2), x4);
      smooth_fast<K, F32>(u, f, a.nu_pre, x, x4);
      rebuilt = true;
    }
  }
  if (!rebuilt) stage_tmp<K, true>(st, tp, u, 0);
  correct_fast<K, F32>(a, x, x4, f, u, c);
}

// Deep pair, interior tile: level I < L - 1 of the up kernel, which first
// redoes the down kernel's work on this level (the same window and code, so
// the same bits wherever they reach the core): u enters with the level's
// starting iterate (Pi on the top, I^ of the level above below it), f with
// its right-hand side.  The bottom level L - 1 takes its pre-smoothed
// iterate (tb) and the coarse iterate below it (tc) from HBM, loaded at the
// start of the kernel.  u leaves with the level's post-smoothed iterate.
template <int K, int I, int L, bool F32, int KB>
__device__ __forceinline__ void deep_level(const VertArgs& a, double* st, Xch& x, Xch4& x4, double (&f)[K],
                           double (&u)[K], const double (&tb)[KB], const double (&tc)[KB / 2]) {
  double f1[K / 2], c[K / 2];
  fw_fast<K>(f, f1, x);
  half_scaled<K>(f, f, a.n >> I);
  smooth_fast<K, F32>(u, f, a.nu_pre, x, x4);  // the pre-smoothed iterate
#pragma unroll
  for (int p = 0; p < K / 2; ++p) c[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
  if constexpr (I + 2 < L) {
    deep_level<K / 2, I + 1, L, F32, KB>(a, st, x, x4, f1, c, tb, tc);
  } else {
    static_assert(K / 2 == KB, "bottom run");
    double cb[KB / 2];
    half_scaled<KB>(f1, f1, a.n >> (I + 1));
    stage_two<KB, KB / 2>(st, tb, c, st + (int)blockDim.x * (KB + 1), tc, cb);
    correct_fast<KB, F32>(a, x, x4, f1, c, cb);
  }
  // c: the post-smoothed iterate of level I + 1
  if constexpr (I == 0) {
    if (a.sr_top) {
      sr_top_fast<K, F32>(a, x, x4, f, u, c);
      return;
    }
  }
  correct_fast<K, F32>(a, x, x4, f, u, c);
}

// kSt2: stage the rhs and the interpolation source at once through st and
// st2; else one after the other through st.
template <int K, int L, bool F32, bool kSt2>
__device__ __forceinline__ void deep_tile(const VertArgs& a, double* st, double* st2, Xch& x,
                                          Xch4& x4, double (&f)[K], double (&u)[K], int64_t wlo0) {
  constexpr int KB = K >> (L - 1);
  double tf[K], ts[K / 2], tb[KB], tc[KB / 2];
  const double* cb = a.src + (wlo0 >> 1);
  issue_loads<K, true>(tf, a.rhs + wlo0, 0);
  issue_loads<K / 2, true>(ts, cb, 0);
  issue_loads<KB, true>(tb, a.pre[L - 1] + (wlo0 >> (L - 1)), 0);
  issue_loads<KB / 2, true>(tc, a.coarse + (wlo0 >> L), 0);
  double cs[K / 2];
  if constexpr (kSt2) {
    stage_two<K, K / 2>(st, tf, f, st2, ts, cs);
  } else {
    stage_tmp<K, true>(st, tf, f, 0);
    stage_tmp<K / 2, true>(st, ts, cs, 0);
  }
  interp_fast1<K>(u, cs, cb + threadIdx.x * (K / 2), x4);
  deep_level<K, 0, L, F32, KB>(a, st, x, x4, f, u, tb, tc);
}

// Sums of the core cells [a, b) of this thread's run (run-local indices),
// in cell order, then over each wavefront by a fixed shuffle tree, then over
// the wavefronts in order; thread 0 writes (sum u, sum u^2) of the
// workgroup's core (an SR segment or a vertical tile) to part[2 slot].
// The order never depends on scheduling.
__device__ __forceinline__ void wave_sum2(double& s1, double& s2) {
  for (int o = 32; o > 0; o >>= 1) {
    s1 = s1 + __shfl_down(s1, o);
    s2 = s2 + __shfl_down(s2, o);
  }
}

template <int K>
__device__ __forceinline__ void segment_sums(const double (&u)[K], int a, int b, double* st,
                                             double* __restrict__ part, int64_t slot) {
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j >= a && j < b) { s1 = s1 + u[j]; s2 = s2 + u[j] * u[j]; }
  wave_sum2(s1, s2);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { st[w] = s1; st[32 + w] = s2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t1 = st[0], t2 = st[32];
    for (int i = 1; i < nw; ++i) { t1 = t1 + st[i]; t2 = t2 + st[32 + i]; }
    part[2 * slot] = t1;
    part[2 * slot + 1] = t2;
  }
}

// Up leg over `levels` stored levels, bottom-up (Fig. 3 post-smoothing leg,
// Eq. 4); only the top level's core is written.  Lower right-hand sides are
// the full weighting of the top one (split tau).
template <int K, bool F32, int T>
__global__ __launch_bounds__(T) void k_up(VertArgs a) {
  __shared__ double st[T * (K + 1)];
  __shared__ double st2[T * (K / 2 + 1)];
  __shared__ double xb[T == 64 ? 1 : 4 * T];
  __shared__ double xb4[T == 64 ? 1 : 8 * T];
  Xch x{xb, 0, 2 * T, T == 64};
  Xch4 x4{xb4, 0, 4 * T, T == 64};
  const int wcount = T * K;
  a.tile = tile_index(a);
  const int64_t wlo0 = top_wlo(a);
  double u[K], f[K];
  if (window_interior(wlo0, wcount, a.n)) {
    if (a.deep) {
      if (a.levels == 4) deep_tile<K, 4, F32, true>(a, st, st2, x, x4, f, u, wlo0);
      else deep_tile<K, 3, F32, true>(a, st, st2, x, x4, f, u, wlo0);
    } else {
      double tf[K], tp[K];
      issue_loads<K, true>(tf, a.rhs + wlo0, 0);
      if (a.src) {  // Pi source run of the rebuilt top level, in tp[0, K/2)
        const double* cb = a.src + (wlo0 >> 1);
#pragma unroll
        for (int k = 0; k < K / 2; ++k) tp[k] = cb[threadIdx.x + k * T];
      } else if (!a.sr_top) {
        issue_loads<K, true>(tp, a.pre[0] + wlo0, 0);
      }
      stage_tmp<K, true>(st, tf, f, 0);
      up_level_fast<K, 0, F32>(a, st, x, x4, f, u, tp, wlo0);
    }
    if (a.out[0])  // null: functionals only, the fine solution is not written
      store_run_fast<K>(st, u, a.out[0] + wlo0, (int)a.halo, (int)(a.halo + a.core),
                        false);  // segment_sums opens with a barrier
    if (a.part) {
      const int e0 = (int)threadIdx.x * K;
      segment_sums<K>(u, (int)a.halo - e0, (int)(a.halo + a.core) - e0, st, a.part, a.tile);
    }
    return;
  }
  const TileGeom G = tile_geom(a, 0, K);
  load_run<K>(st, f, G.wlo, wcount, G.n, [&](int64_t g) { return a.rhs[g]; });
  up_level<K, 0, F32>(a, st, x, f, u);
  if (a.out[0]) store_run<K>(st, u, G.wlo, G.clo, G.chi, a.out[0]);
  if (a.part) {
    const int64_t c0 = G.clo - G.g0, c1 = G.chi - G.g0;
    segment_sums<K>(u, (int)(c0 < 0 ? 0 : (c0 > K ? K : c0)), (int)(c1 < 0 ? 0 : (c1 > K ? K : c1)),
                    st, a.part, a.tile);
  }
}

// Interior tiles of a deep up launch alone (the edge tiles take k_up): 166
// VGPRs, so three wavefronts share a SIMD (FP32 relaxation: 182 VGPRs, two).
template <int K, bool F32, int T>
__global__ __launch_bounds__(T, F32 ? 2 : 3) void k_up_wide(VertArgs a) {
  __shared__ double st[T * (K + 1)];
  __shared__ double xb[T == 64 ? 1 : 8 * T];
  Xch x{xb, 0, 4 * T, T == 64};
  Xch4& x4 = x;  // one exchanger in both roles
  a.tile = tile_index(a);
  const int64_t wlo0 = top_wlo(a);
  if (!window_interior(wlo0, T * K, a.n)) return;  // the host launches interior tiles only
  double u[K], f[K];
  if (a.levels == 4) deep_tile<K, 4, F32, false>(a, st, st, x, x4, f, u, wlo0);
  else deep_tile<K, 3, F32, false>(a, st, st, x, x4, f, u, wlo0);
  if (a.out[0])
    store_run_fast<K>(st, u, a.out[0] + wlo0, (int)a.halo, (int)(a.halo + a.core), false);
  if (a.part) {
    const int e0 = (int)threadIdx.x * K;
    segment_sums<K>(u, (int)a.halo - e0, (int)(a.halo + a.core) - e0, st, a.part, a.tile);
  }
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

// ravg: the rhs restriction is the two-cell average instead of full weighting.
__global__ void k_tau_literal(const double* __restrict__ u, const double* __restrict__ F,
                              int64_t nc, double gL, double gR, int ravg,
                              double* __restrict__ out) {
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int64_t nf = 2 * nc;
  const double w = (double)nf * (double)nf, wc = (double)nc * (double)nc;
  const double r1 = fine_residual(u, F, 2 * J, nf, w, gL, gR);
  const double r2 = fine_residual(u, F, 2 * J + 1, nf, w, gL, gR);
  double IR;
  if (ravg) {
    IR = (r1 + r2) * 0.5;
  } else {
    const double rm = (J > 0) ? fine_residual(u, F, 2 * J - 1, nf, w, gL, gR) : -r1;
    const double rp = (2 * J + 2 < nf) ? fine_residual(u, F, 2 * J + 2, nf, w, gL, gR) : -r2;
    IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
  }
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
  const double* direct;  // down, several SR levels: the patch iterate is this
                         // level-n array (I^ of the finer SR level) instead of
                         // Pi coarse; nullptr otherwise
  const double* f;       // fine right-hand side
  double* out;           // down: I^ of the smoothed cores [n/2]; up: u_out or nullptr
  double* q_out;         // down, literal tau: coarse rhs [n/2] (else nullptr)
  int ravg;              // literal tau: rhs restriction = two-cell average
  double* part;          // up: per-segment (sum u, sum u^2) of the core, or nullptr
  // up: workgroup b runs segment seg0 + b and writes its core cells g in
  // [out_lo, out_hi) to out[g - out_lo] (a solve: 0, 0, n; a decompression:
  // the requested range)
  int64_t seg0, out_lo, out_hi;
};


// Down pass (Fig. 3 steps 1-5 fused): Pi, nu sweeps on the extended patch,
// then I^ (and literal tau) on the core's coarse cells.  The fine iterate
// never leaves the chip.  With a.direct the patch starts from that array
// instead of Pi: an SR level below the finest one, pre-smoothed in blocks
// from the restricted iterate of the level above (Sec. 4's runs with two
// and three SR levels).
template <int K, bool F32>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_down(SegArgs a) {
  extern __shared__ double sm[];
  const int W = blockDim.x;
  double* st = sm;                   // W (K+1)
  Xch x{sm + W * (K + 1), 0, 2 * W};        // 4 W
  const int64_t n = a.n, nc = n >> 1;
  const int64_t seg = xcd_block();
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t wlo = core_lo - a.pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  double u[K], f[K];
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  if (a.q_out == nullptr && window_interior(wlo, (int64_t)W * K, n)) {
    double tf[K];
    issue_loads<K, false>(tf, a.f + wlo, a.win);
    if (a.direct) {  // uniform per launch
      double tu[K];
      issue_loads<K, false>(tu, a.direct + wlo, a.win);
      stage_tmp<K, false>(st, tf, f, a.win);
      stage_tmp<K, false>(st, tu, u, a.win);
    } else {
      const double* cb = a.coarse + (wlo >> 1);
      double tc[K / 2], c[K / 2];
      issue_loads<K / 2, false>(tc, cb, a.win / 2 + 2);
      stage_tmp<K, false>(st, tf, f, a.win);
      stage_tmp<K / 2, false>(st, tc, c, a.win / 2 + 2);
      interp_fast<K>(u, c, cb + threadIdx.x * (K / 2), x);
    }
    half_scaled<K>(f, f, n);
    const RunBounds rb = run_bounds(g0, K, lo, hi, n);
    Xch4 x4{st, 0, 4 * W};  // the stage is idle during the sweeps (8 W <= W (K + 1) doubles)
    smooth_masked<K, F32>(u, f, a.nu, rb.jlo, rb.jhi, g0 + K >= lo && g0 + K < hi, x, x4);
    __syncthreads();  // last exchange read before the stage is reused
    double uc[K / 2];
#pragma unroll
    for (int p = 0; p < K / 2; ++p) uc[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
    store_run_fast<K / 2>(st, uc, a.out + (wlo >> 1), (int)(a.pad >> 1), (int)((a.pad + a.s) >> 1));
    return;
  }
  load_run<K>(st, f, wlo, a.win, n, [&](int64_t g) { return a.f[g]; });
  if (a.direct) load_run<K>(st, u, wlo, a.win, n, [&](int64_t g) { return a.direct[g]; });
  else load_interp_run<K>(st, u, wlo, a.win, n, a.coarse, a.gL, a.gR, x);
  smooth_general<K, F32>(u, f, g0, a.nu, lo, hi, n, a.gL, a.gR, x);
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
      double IR;
      if (a.ravg) {
        IR = (ra + rb) * 0.5;
      } else {
        const double rm = (J > 0) ? res(m - 1) : -ra;
        const double rp = (2 * J + 2 < n) ? res(m + 2) : -rb;
        IR = ((rm + rp) + 3.0 * (ra + rb)) * 0.125;
      }
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
// Registers -> coalesced store of the window cells whose global index lies in
// [lo, hi), cell g to out[g - out_lo].
template <int K>
__device__ __forceinline__ void store_run_at(double* st, const double (&v)[K], int64_t wlo,
                                             int64_t lo, int64_t hi, double* __restrict__ out,
                                             int64_t out_lo) {
  const int W = blockDim.x;
  run_to_stage<K>(st, v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * W;
    const int64_t g = wlo + e;
    if (g >= lo && g < hi) out[g - out_lo] = st[sidx<K>(e)];
  }
  __syncthreads();
}

template <int K, bool F32>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr_up(SegArgs a) {
  extern __shared__ double sm[];
  const int W = blockDim.x;
  double* st = sm;
  Xch x{sm + W * (K + 1), 0, 2 * W};
  const int64_t n = a.n, nc = n >> 1;
  const int64_t seg = a.seg0 + xcd_block();
  // cells of this segment's core that are written
  const int64_t wr_lo = seg * a.s > a.out_lo ? seg * a.s : a.out_lo;
  const int64_t wr_hi = (seg + 1) * a.s < a.out_hi ? (seg + 1) * a.s : a.out_hi;
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
    const bool nb_upd = g0 + K >= lo && g0 + K < hi;
    Xch4 x4{st, 0, 4 * W};  // the stage is idle during the sweeps (8 W <= W (K + 1) doubles)
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
      smooth_masked<K, F32>(u, f, 1, rb.jlo, rb.jhi, nb_upd, x, x4);
    }
    __syncthreads();  // last exchange read before the stage is reused
    if (a.out) store_run_at<K>(st, u, wlo, wr_lo, wr_hi, a.out, a.out_lo);
    if (a.part) {
      const int e0 = (int)threadIdx.x * K;
      segment_sums<K>(u, (int)a.pad - e0, (int)(a.pad + a.s) - e0, st, a.part, seg - a.seg0);
    }
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
    if constexpr (F32) {
      cf_sweeps<K>(u, f, g0, 1, lo, hi, n, a.gL, a.gR, x);
    } else {
      rb_half<K, 0>(u, f, rb, h2, gL2, gR2, bdiv, x);
      rb_half<K, 1>(u, f, rb, h2, gL2, gR2, bdiv, x);
    }
  }
  if (a.out) store_run_at<K>(st, u, wlo, wr_lo, wr_hi, a.out, a.out_lo);
  if (a.part) {
    const int64_t c0 = core_lo - g0, c1 = (core_hi < n ? core_hi : n) - g0;
    segment_sums<K>(u, (int)(c0 < 0 ? 0 : (c0 > K ? K : c0)), (int)(c1 < 0 ? 0 : (c1 > K ? K : c1)),
                    st, a.part, seg - a.seg0);
  }
}

// ---------------------------------------------------------------------------
// Two unstored SR levels (M and M-1): the finest segment passes rebuild the
// level-(M-1) iterate they need from V^{M-2} instead of reading it.
//
// V^{M-1} is, per level-(M-1) segment j, the compatible relaxation of
// Pi V^{M-2} on j's patch (Eq. 5, Fig. 5).  A level-M segment i needs it on
// the coarse image of its window plus Pi's reach: the core of level-(M-1)
// segment i and pad/2 + 2 cells on each side, which belong to segments
// i-R .. i+R (R = 1 unless the cores are tiny).  The workgroup holds a
// level-(M-1) window of s/2 + 2 p1 cells around that core and runs the
// relaxation 2R + 1 times on it, once with each of those segments' patches
// (exterior frozen at Pi V^{M-2}), keeping each run's result in that
// segment's zone.  A relaxation sweep reaches 3 cells per iteration
// (Kaczmarz pairs and a red-black sweep), so p1 >= pad/2 + 2 + 3 nu2 + 2
// keeps every kept cell exact; the window edges' stale cells are never read.
// When b >= 2 nu2 the block relaxation's cores equal the unsegmented
// relaxation bit for bit (the patch edges' influence does not reach the
// cores), so one run over the whole window serves every zone (R = 0).
// ---------------------------------------------------------------------------
struct Seg2Args {
  int64_t n;             // level-M cells
  double gL, gR;
  int nu1, nu2;          // level-M pre-sweeps (down); CR iterations
  int64_t s;             // level-M core cells per segment (level M-1: s / 2)
  int64_t S;             // segments
  int R;                 // level-(M-1) segments needed on each side; 0: one
                         // run over the whole window (b >= 2 nu2)
  int64_t buffer;        // buffer cells per side on both levels
  int64_t pad;           // level-M window offset left of the core
  int win;               // level-M window cells, s + 2 pad
  int64_t p1;            // level-(M-1) window offset left of the core (even)
  int win1;              // level-(M-1) window cells, s / 2 + 2 p1
  const double* v2;      // V^{M-2} [n/4]
  const double* f1;      // forcing of level M-1 [n/2]
  const double* f;       // fine right-hand side [n]
  double* out;           // down: I^ of the smoothed level-M cores [n/2];
                         // up: u_out [n] or nullptr
  double* part;          // up: per-segment (sum u, sum u^2), or nullptr
};

// One CR iteration pass count nu on a run: nu x [Kaczmarz projection of the
// pairs inside [lo, hi) onto c (Eq. 8), red-black sweep on [lo, hi)].
template <int K, bool F32>
__device__ __forceinline__ void cr_run(double (&u)[K], const double (&f)[K],
                                       const double (&c)[K / 2], int64_t g0, int nu, int64_t lo,
                                       int64_t hi, int64_t n, double gL, double gR, Xch& x) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  const double bdiv = (n == 1) ? 4.0 : 3.0;
  const RunBounds rb = run_bounds(g0, K, lo, hi, n);
  for (int it = 0; it < nu; ++it) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {  // both children in the patch
        const double r = c[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
        u[2 * p] = u[2 * p] + r;
        u[2 * p + 1] = u[2 * p + 1] + r;
      }
    }
    if constexpr (F32) {
      cf_sweeps<K>(u, f, g0, 1, lo, hi, n, gL, gR, x);
    } else {
      rb_half<K, 0>(u, f, rb, h2, gL2, gR2, bdiv, x);
      rb_half<K, 1>(u, f, rb, h2, gL2, gR2, bdiv, x);
    }
  }
}

// Up pass on interior windows: every level-(M-1) load in flight at once,
// one exchange per sweep.  (The down pass keeps the general code: there the
// one-exchange sweeps' extra registers cost half the resident workgroups,
// more than they save; measured.)
template <int K, bool F32>
__device__ void sr2_up_interior(const Seg2Args& a, double* st, Xch& x) {
  constexpr int K1 = K / 2;
  const int W = blockDim.x;
  const int64_t n = a.n, n1 = n >> 1;
  const int64_t seg = xcd_block();
  const int64_t s1 = a.s >> 1;
  const int64_t w1lo = seg * s1 - a.p1;
  const int64_t g1 = w1lo + (int64_t)threadIdx.x * K1;
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t wlo = core_lo - a.pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  const int64_t J0 = g0 >> 1;
  const int64_t lo = core_lo - a.buffer, hi = core_hi + a.buffer;  // inside the level
  const double* cb = a.v2 + (w1lo >> 1);
  double tF[K1], tc[K1 / 2];
  issue_loads<K1, false>(tF, a.f1 + w1lo, a.win1);
  issue_loads<K1 / 2, false>(tc, cb, a.win1 / 2 + 2);
  double F1[K1], c2[K1 / 2], u0[K1], v1[K1];
  stage_tmp<K1, false>(st, tF, F1, a.win1);
  stage_tmp<K1 / 2, false>(st, tc, c2, a.win1 / 2 + 2);
  interp_fast<K1>(u0, c2, cb + threadIdx.x * (K1 / 2), x);
  half_scaled<K1>(F1, F1, n1);
  Xch4 x4{st, 0, 4 * W};  // the stage is idle during the sweeps (8 W <= W (K + 1) doubles)
#pragma unroll
  for (int j = 0; j < K1; ++j) v1[j] = u0[j];
  for (int r = -a.R; r <= a.R; ++r) {
    const int64_t sj = seg + r;
    if (sj < 0 || sj >= a.S) continue;
    double u[K1];
#pragma unroll
    for (int j = 0; j < K1; ++j) u[j] = u0[j];
    int64_t plo = (sj * s1 - a.buffer > 0) ? sj * s1 - a.buffer : 0;
    int64_t phi = ((sj + 1) * s1 + a.buffer < n1) ? (sj + 1) * s1 + a.buffer : n1;
    if (a.R == 0) { plo = w1lo; phi = w1lo + a.win1; }  // interior: inside the level
    const RunBounds rb = run_bounds(g1, K1, plo, phi, n1);
    const bool nb_upd = g1 + K1 >= plo && g1 + K1 < phi;
    for (int it = 0; it < a.nu2; ++it) {
#pragma unroll
      for (int p = 0; p < K1 / 2; ++p) {
        if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {
          const double d = c2[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
          u[2 * p] = u[2 * p] + d;
          u[2 * p + 1] = u[2 * p + 1] + d;
        }
      }
      smooth_masked<K1, F32>(u, F1, 1, rb.jlo, rb.jhi, nb_upd, x, x4);
    }
    const int64_t zlo = (r == -a.R) ? INT64_MIN : sj * s1;
    const int64_t zhi = (r == a.R) ? INT64_MAX : (sj + 1) * s1;
#pragma unroll
    for (int j = 0; j < K1; ++j)
      if (g1 + j >= zlo && g1 + j < zhi) v1[j] = u[j];
  }
  double tf[K];  // in flight while V^{M-1} goes through the stage
  issue_loads<K, false>(tf, a.f + wlo, a.win);
  __syncthreads();  // last exchange through the stage read
  run_to_stage<K1>(st, v1);
  __syncthreads();
  double e[K / 2 + 4];
#pragma unroll
  for (int m = 0; m < K / 2 + 4; ++m) {
    int64_t idx = J0 - 2 + m - w1lo;
    idx = idx < 0 ? 0 : (idx >= (int64_t)K1 * W ? (int64_t)K1 * W - 1 : idx);
    e[m] = st[sidx<K1>((int)idx)];
  }
  __syncthreads();
  double u[K], f[K];
  stage_tmp<K, false>(st, tf, f, a.win);
  interp_from_e<K>(u, e, J0, n1, a.gL, a.gR);
  half_scaled<K>(f, f, n);
  const RunBounds rb = run_bounds(g0, K, lo, hi, n);
  const bool nb_upd = g0 + K >= lo && g0 + K < hi;
  {
    for (int it = 0; it < a.nu2; ++it) {
#pragma unroll
      for (int p = 0; p < K / 2; ++p) {
        if (2 * p >= rb.jlo && 2 * p + 1 < rb.jhi) {
          const double d = e[p + 2] - (u[2 * p] + u[2 * p + 1]) * 0.5;
          u[2 * p] = u[2 * p] + d;
          u[2 * p + 1] = u[2 * p + 1] + d;
        }
      }
      smooth_masked<K, F32>(u, f, 1, rb.jlo, rb.jhi, nb_upd, x, x4);
    }
    __syncthreads();
    if (a.out) store_run_fast<K>(st, u, a.out + wlo, (int)a.pad, (int)(a.pad + a.s));
    if (a.part) {
      const int e0 = (int)threadIdx.x * K;
      segment_sums<K>(u, (int)a.pad - e0, (int)(a.pad + a.s) - e0, st, a.part, seg);
    }
  }
}

template <int K, bool F32, bool UP>
__global__ __launch_bounds__(kSegMaxThreads) void k_sr2(Seg2Args a) {
  constexpr int K1 = K / 2;  // level-(M-1) cells per thread
  extern __shared__ double sm[];
  const int W = blockDim.x;
  double* st = sm;                   // W (K+1)
  Xch x{sm + W * (K + 1), 0, 2 * W};        // 4 W
  const int64_t n = a.n, n1 = n >> 1, n2 = n >> 2;
  const int64_t seg = xcd_block();
  const int64_t s1 = a.s >> 1;
  if constexpr (UP) {
    const int64_t wlo_m = seg * a.s - a.pad;
    if (window_interior(seg * s1 - a.p1, (int64_t)W * K1, n1) &&
        window_interior(wlo_m, (int64_t)W * K, n)) {
      sr2_up_interior<K, F32>(a, st, x);
      return;
    }
  }
  // ---- level M-1: V^{M-1} on [w1lo, w1lo + K1 W) ----
  const int64_t w1lo = seg * s1 - a.p1;
  const int64_t g1 = w1lo + (int64_t)threadIdx.x * K1;
  double F1[K1], c2[K1 / 2], u0[K1], v1[K1];
  load_run<K1>(st, F1, w1lo, a.win1, n1, [&](int64_t g) { return a.f1[g]; });
  load_run<K1 / 2>(st, c2, w1lo >> 1, a.win1 / 2 + 2, n2, [&](int64_t J) { return a.v2[J]; });
  interp_from_run<K1>(u0, c2, g1, n1, a.v2, a.gL, a.gR, x);
#pragma unroll
  for (int j = 0; j < K1; ++j) v1[j] = u0[j];
  for (int r = -a.R; r <= a.R; ++r) {
    const int64_t sj = seg + r;  // uniform per workgroup
    if (sj < 0 || sj >= a.S) continue;
    double u[K1];
#pragma unroll
    for (int j = 0; j < K1; ++j) u[j] = u0[j];
    int64_t lo = (sj * s1 - a.buffer > 0) ? sj * s1 - a.buffer : 0;
    int64_t hi = ((sj + 1) * s1 + a.buffer < n1) ? (sj + 1) * s1 + a.buffer : n1;
    if (a.R == 0) {  // the whole window, clipped to the level
      lo = w1lo > 0 ? w1lo : 0;
      hi = (w1lo + a.win1 < n1) ? w1lo + a.win1 : n1;
    }
    cr_run<K1, F32>(u, F1, c2, g1, a.nu2, lo, hi, n1, a.gL, a.gR, x);
    // this run's zone: its core, extended outwards for the outermost runs
    const int64_t zlo = (r == -a.R) ? INT64_MIN : sj * s1;
    const int64_t zhi = (r == a.R) ? INT64_MAX : (sj + 1) * s1;
#pragma unroll
    for (int j = 0; j < K1; ++j)
      if (g1 + j >= zlo && g1 + j < zhi) v1[j] = u[j];
  }
  // ---- level M: Pi V^{M-1} on the segment window ----
  run_to_stage<K1>(st, v1);
  __syncthreads();
  const int64_t core_lo = seg * a.s, core_hi = core_lo + a.s;
  const int64_t wlo = core_lo - a.pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  const int64_t J0 = g0 >> 1;
  double e[K / 2 + 4];
#pragma unroll
  for (int m = 0; m < K / 2 + 4; ++m) {
    int64_t idx = J0 - 2 + m - w1lo;  // window-local level-(M-1) cell
    idx = idx < 0 ? 0 : (idx >= (int64_t)K1 * W ? (int64_t)K1 * W - 1 : idx);
    e[m] = st[sidx<K1>((int)idx)];
  }
  __syncthreads();
  double u[K], f[K], c[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) c[p] = e[p + 2];
  interp_from_e<K>(u, e, J0, n1, a.gL, a.gR);
  load_run<K>(st, f, wlo, a.win, n, [&](int64_t g) { return a.f[g]; });
  const int64_t lo = (core_lo - a.buffer > 0) ? core_lo - a.buffer : 0;
  const int64_t hi = (core_hi + a.buffer < n) ? core_hi + a.buffer : n;
  if constexpr (!UP) {
    smooth_general<K, F32>(u, f, g0, a.nu1, lo, hi, n, a.gL, a.gR, x);
    double uc[K / 2];
#pragma unroll
    for (int p = 0; p < K / 2; ++p) uc[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
    store_run<K / 2>(st, uc, wlo >> 1, core_lo >> 1, core_hi >> 1, a.out);
  } else {
    cr_run<K, F32>(u, f, c, g0, a.nu2, lo, hi, n, a.gL, a.gR, x);
    if (a.out) store_run<K>(st, u, wlo, core_lo, core_hi < n ? core_hi : n, a.out);
    if (a.part) {
      const int64_t c0 = core_lo - g0, c1 = (core_hi < n ? core_hi : n) - g0;
      segment_sums<K>(u, (int)(c0 < 0 ? 0 : (c0 > K ? K : c0)),
                      (int)(c1 < 0 ? 0 : (c1 > K ? K : c1)), st, a.part, seg);
    }
  }
}

// Functionals of the fine solution from the per-segment sums (fixed order:
// each thread walks a strided set of segments in order, then the shuffle
// tree and the wavefronts in order): out[0] = h sum u, out[1] = h sum u^2.
__global__ __launch_bounds__(1024) void k_functionals(const double* __restrict__ part,
                                                      int64_t S, double h,
                                                      double* __restrict__ out) {
  __shared__ double r[64];
  const int t = threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = t; i < S; i += 1024) {
    const double2 p = reinterpret_cast<const double2*>(part)[i];
    s1 = s1 + p.x;
    s2 = s2 + p.y;
  }
  wave_sum2(s1, s2);
  if ((t & 63) == 0) { r[t >> 6] = s1; r[32 + (t >> 6)] = s2; }
  __syncthreads();
  if (t == 0) {
    double t1 = r[0], t2 = r[32];
    for (int i = 1; i < 16; ++i) { t1 = t1 + r[i]; t2 = t2 + r[32 + i]; }
    out[0] = h * t1;
    out[1] = h * t2;
  }
}

// ---------------------------------------------------------------------------
// Coarse core: all levels with at most kCoreMaxCells cells, in one workgroup
// with the level stack resident in LDS.  The coarse levels are tiny, so this
// kernel is bound by the latency of its chain of about a hundred dependent
// LDS phases; the code is kept compact (rolled loops, 32-bit indices, one
// call site per phase) so that each phase issues few instructions.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Non-finite check (fmgsr_options.check_finite): a grid-stride scan that sets
// *flag (cleared beforehand by k_clear_flag, not a memset, so the pair is
// also safe inside a captured graph) when any of the n values is NaN or Inf.
// Every thread that finds one writes the same value; no atomics are needed.
// ---------------------------------------------------------------------------
__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ x, int64_t n,
                                                   int* flag) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;
}

constexpr int kCoreThreads = 512;
constexpr int64_t kCoreMaxCells = 2048;
constexpr int64_t kMaxN0 = 1024;

struct CoreArgs {
  int top;             // coarse-core top level C (levels 0..C)
  int64_t n0;          // cells of level 0
  double gL, gR;
  int nu1, nu2;
  int literal;         // literal tau on the levels below C
  int ravg;            // literal tau: rhs restriction = two-cell average
  int mode;            // 0: FMG on levels 0..C; 1: V-cycle from a level-C guess
  int src_kind;        // mode 1: kSrcRestrict (from level C+1) or kSrcDirect
  const double* F[12]; // forcing of levels 0..C (C <= 11)
  const double* src;   // mode 1: level C+1 iterate or level-C initial iterate
  const double* rhs_top;  // mode 1: right-hand side of level C
  double* out;         // level-C result
};

__device__ __forceinline__ int lvl_off(int n0, int l) { return n0 * ((1 << l) - 1); }

// One red-black sweep of a level of n cells (n even) in LDS, in one phase:
// the thread that owns the pairs (2J, 2J+1), J = tid + k T, reads the old
// iterate from src and writes the new one to dst, a separate buffer, so no
// barrier separates the colours.  Its black cell's right neighbour, the
// next pair's red cell, is recomputed here from the same operands its owner
// uses, so dst is bitwise the result of the red then black half-sweeps.
// With the pair's final values the same phase can also produce
//   rc:  I^ of the level (the next coarser level's start, n/2 cells), and
//   e:   the correction e = u - I^ ufine of this level (ufine: the finer
//        level's pre-smoothed iterate), read by the next finer level.
__device__ __forceinline__ void core_sweep(const double* src, double* dst, const double* q, int n,
                                           double gL2, double gR2, double* rc = nullptr,
                                           double* e = nullptr, const double* ufine = nullptr) {
  const double h2 = 1.0 / ((double)n * (double)n);
  const double bdiv = (n == 1) ? 4.0 : 3.0;
#pragma unroll 1
  for (int J = threadIdx.x; 2 * J < n; J += blockDim.x) {
    const int i0 = 2 * J, i1 = i0 + 1;
    const double lft = (i0 > 0) ? src[i0 - 1] : gL2;
    const double b_old = src[i1];
    const double num0 = q[i0] * h2 + (lft + b_old);
    const double r0 = (i0 > 0) ? num0 * 0.5 : num0 / bdiv;
    double rgt = gR2;
    if (i1 < n - 1) {  // the next pair's red cell, an interior cell
      const double num2 = q[i0 + 2] * h2 + (b_old + src[i0 + 3]);
      rgt = num2 * 0.5;
    }
    const double num1 = q[i1] * h2 + (r0 + rgt);
    const double b1 = (i1 < n - 1) ? num1 * 0.5 : num1 / bdiv;
    dst[i0] = r0;
    dst[i1] = b1;
    if (rc) rc[J] = (r0 + b1) * 0.5;
    if (e) {
      e[i0] = r0 - (ufine[2 * i0] + ufine[2 * i0 + 1]) * 0.5;
      e[i1] = b1 - (ufine[2 * i1] + ufine[2 * i1 + 1]) * 0.5;
    }
  }
  __syncthreads();
}

// Levels of at most 64 cells run on the first wavefront alone, one cell per
// lane, with neighbours from DPP wavefront shifts (no LDS round trip and no
// workgroup barrier per half-sweep).  Same expression trees as the LDS code.
__device__ __forceinline__ double dpp_shift(double v, bool from_left) {
  // wave_shr:1 (lane i takes lane i-1) or wave_shl:1 (lane i takes lane i+1);
  // lanes without a source get 0
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

// nu red-black sweeps of a level of n <= 64 cells held one per lane.
__device__ __forceinline__ double wave_rb(double u, double q, int n, int nu, double gL2,
                                          double gR2) {
  const int i = threadIdx.x;
  const double h2 = 1.0 / ((double)n * (double)n);
  const double bdiv = (n == 1) ? 4.0 : 3.0;
#pragma unroll 1
  for (int s = 0; s < nu; ++s) {
#pragma unroll
    for (int colour = 0; colour < 2; ++colour) {
      const double lv = dpp_shift(u, true), rv = dpp_shift(u, false);
      if (i < n && (i & 1) == colour) {
        const double l = (i > 0) ? lv : gL2;
        const double r = (i < n - 1) ? rv : gR2;
        const double num = q * h2 + (l + r);
        u = (i > 0 && i < n - 1) ? num * 0.5 : num / bdiv;
      }
    }
  }
  return u;
}

// Down leg of a V-cycle on levels top..1 (top <= the last level of at most
// 64 cells), first wavefront only: sweeps, then I^ into the next level.  The
// pre-smoothed iterates go to U (the up leg needs them); level 0 gets I^ of
// level 1 as the solve's start.  Split tau: Q is the forcing.
__device__ void wave_down(double* U, const double* Q, int n0, int top, int nu1, double gL2,
                          double gR2) {
  const int i = threadIdx.x;
  int n = n0 << top;
  double u = (i < n) ? U[lvl_off(n0, top) + i] : 0.0;
#pragma unroll 1
  for (int m = top; m >= 1; --m, n >>= 1) {
    const double q = (i < n) ? Q[lvl_off(n0, m) + i] : 0.0;
    u = wave_rb(u, q, n, nu1, gL2, gR2);
    if (i < n) U[lvl_off(n0, m) + i] = u;
    const int j0 = (2 * i < n) ? 2 * i : 0, j1 = (2 * i + 1 < n) ? 2 * i + 1 : 0;
    const double a0 = __shfl(u, j0), a1 = __shfl(u, j1);
    u = (i < n / 2) ? (a0 + a1) * 0.5 : 0.0;
  }
  if (i < n0) U[i] = u;
}

// Up leg on levels 1..top (first wavefront): correction from the level
// below (Eq. 4, e = u^{m} - I^ u^{m+1}_pre), then nu2 sweeps; level top's
// result goes to U.
__device__ void wave_up(double* U, const double* Q, int n0, int top, int nu2, double gL2,
                        double gR2) {
  const int i = threadIdx.x;
  int nc = n0;
  double uc = (i < nc) ? U[i] : 0.0;
#pragma unroll 1
  for (int m = 0; m < top; ++m, nc <<= 1) {
    const int nf = nc << 1;
    const double up = (i < nf) ? U[lvl_off(n0, m + 1) + i] : 0.0;  // pre-smoothed
    const int j0 = (2 * i < nf) ? 2 * i : 0, j1 = (2 * i + 1 < nf) ? 2 * i + 1 : 0;
    const double p0 = __shfl(up, j0), p1 = __shfl(up, j1);
    const double e = (i < nc) ? uc - (p0 + p1) * 0.5 : 0.0;
    const int J = i >> 1;
    const double eJ = __shfl(e, J < nc ? J : 0);
    const double eL = __shfl(e, (J > 0 && J - 1 < nc) ? J - 1 : 0);
    const double eR = __shfl(e, (J + 1 < nc) ? J + 1 : 0);
    double u = up;
    if (i < nf) {
      if ((i & 1) == 0) {
        const double em = (J > 0) ? eL : -eJ;
        u = up + (3.0 * eJ + em) * 0.25;
      } else {
        const double ep = (J < nc - 1) ? eR : -eJ;
        u = up + (3.0 * eJ + ep) * 0.25;
      }
    }
    const double q = (i < nf) ? Q[lvl_off(n0, m + 1) + i] : 0.0;
    uc = wave_rb(u, q, nf, nu2, gL2, gR2);
  }
  if (i < (n0 << top)) U[lvl_off(n0, top) + i] = uc;
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
  double* TMP = PA + 8 * n0;      // the sweeps' second buffer (level C's size)
  const double gL = a.gL, gR = a.gR, gL2 = 2.0 * gL, gR2 = 2.0 * gR;
  const int nC = n0 << C;
  int lw = -1;  // last level of at most 64 cells (first-wavefront levels)
  while (lw + 1 <= C && (n0 << (lw + 1)) <= 64) ++lw;
  // inputs: every global load of the kernel is issued before any is
  // consumed (one HBM round trip instead of one per level).  The level stack
  // in LDS is the flattened index q of (level l, cell i), q = lvl_off(l) + i;
  // each lane finds its level from q and its pointer in a small LDS table.
  __shared__ const double* lp[12];
  if (tid <= C) lp[tid] = (tid == C && a.mode == 1) ? a.rhs_top : a.F[tid];
  __syncthreads();
  constexpr int kQ = (int)(2 * kCoreMaxCells / kCoreThreads);  // ntot < 2 kCoreMaxCells
  constexpr int kV = (int)(kCoreMaxCells / kCoreThreads);
  double vq[kQ], vs[kV];
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int q = tid + k * T;
    const int qq = q < ntot ? q : 0;
    const int l = 31 - __clz(qq / n0 + 1);
    vq[k] = lp[l][qq - lvl_off(n0, l)];
  }
  if (a.mode == 1) {
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      int i = tid + k * T;
      i = i < nC ? i : nC - 1;
      vs[k] = (a.src_kind == kSrcRestrict) ? (a.src[2 * i] + a.src[2 * i + 1]) * 0.5 : a.src[i];
    }
  }
#pragma unroll
  for (int k = 0; k < kQ; ++k) {
    const int q = tid + k * T;
    if (q < ntot) Q[q] = vq[k];
  }
  if (a.mode == 1) {
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      const int i = tid + k * T;
      if (i < nC) U[lvl_off(n0, C) + i] = vs[k];
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
    // down leg: levels above 64 cells on the whole workgroup, the rest on
    // the first wavefront (split tau)
    const int wtop = (lw >= 1 && !a.literal) ? min(t, lw) : 0;
#pragma unroll 1
    for (int m = t; m >= wtop + 1 && m >= 1; --m) {
      const int nm = n0 << m, nc = nm >> 1;
      double* uf = U + lvl_off(n0, m);
      double* qf = Q + lvl_off(n0, m);
      double* uc = U + lvl_off(n0, m - 1);
      double* qc = Q + lvl_off(n0, m - 1);
      // nu1 sweeps alternating between the level and TMP (an odd count
      // ends with a copy back); split tau: the last sweep also restricts
      const bool fused = !a.literal && a.nu1 > 0;
#pragma unroll 1
      for (int s = 0; s < a.nu1; ++s) {
        const bool even = (s % 2 == 0);
        core_sweep(even ? uf : TMP, even ? TMP : uf, qf, nm, gL2, gR2,
                   (fused && s == a.nu1 - 1) ? uc : nullptr);
      }
      if (a.nu1 % 2 == 1) {
#pragma unroll 1
        for (int i = tid; i < nm; i += T) uf[i] = TMP[i];
        __syncthreads();
      }
      if (fused) continue;
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
          double IR;
          if (a.ravg) {
            IR = (r1 + r2) * 0.5;
          } else {
            const double rm = (J > 0) ? res(2 * J - 1) : -r1;
            const double rp = (2 * J + 2 < nm) ? res(2 * J + 2) : -r2;
            IR = ((rm + rp) + 3.0 * (r1 + r2)) * 0.125;
          }
          const double ul = (J > 0) ? (uf[2 * J - 2] + uf[2 * J - 1]) * 0.5 : gL2 - u0;
          const double ur = (J < nc - 1) ? (uf[2 * J + 2] + uf[2 * J + 3]) * 0.5 : gR2 - u0;
          qc[J] = IR + (2.0 * u0 - (ul + ur)) * wc;
        }
        uc[J] = u0;
      }
      __syncthreads();
    }
    if (wtop >= 1) {
      if (tid < 64) wave_down(U, Q, n0, wtop, a.nu1, gL2, gR2);
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
    if (wtop >= 1) {
      if (tid < 64) wave_up(U, Q, n0, wtop, a.nu2, gL2, gR2);
      __syncthreads();
    }
    // up leg; e = u^m - I^ u^{m+1} comes from level m's last sweep when it
    // has one, else from its own phase
    bool have_e = false;
#pragma unroll 1
    for (int m = wtop; m < t; ++m) {
      const int nc = n0 << m, nf = nc << 1;
      const double* uc = U + lvl_off(n0, m);
      double* uf = U + lvl_off(n0, m + 1);
      if (!have_e) {
#pragma unroll 1
        for (int J = tid; J < nc; J += T) E[J] = uc[J] - (uf[2 * J] + uf[2 * J + 1]) * 0.5;
        __syncthreads();
      }
      // the corrected iterate goes to the buffer from which the nu2 sweeps,
      // alternating, end in the level
      double* cd = (a.nu2 % 2 == 1) ? TMP : uf;
      double* co = (a.nu2 % 2 == 1) ? uf : TMP;
#pragma unroll 1
      for (int J = tid; J < nc; J += T) {
        const double eJ = E[J];
        const double em = (J > 0) ? E[J - 1] : -eJ;
        const double ep = (J < nc - 1) ? E[J + 1] : -eJ;
        cd[2 * J] = uf[2 * J] + (3.0 * eJ + em) * 0.25;
        cd[2 * J + 1] = uf[2 * J + 1] + (3.0 * eJ + ep) * 0.25;
      }
      __syncthreads();
      // the last sweep also forms the next level's e (level m+1 against m+2)
      const bool next_e = (m + 1 < t) && a.nu2 > 0;
#pragma unroll 1
      for (int s = 0; s < a.nu2; ++s) {
        const bool even = (s % 2 == 0);
        core_sweep(even ? cd : co, even ? co : cd, Q + lvl_off(n0, m + 1), nf, gL2, gR2, nullptr,
                   (next_e && s == a.nu2 - 1) ? E : nullptr, U + lvl_off(n0, m + 2));
      }
      have_e = next_e;
    }
  }
#pragma unroll 1
  for (int i = tid; i < nC; i += T) a.out[i] = U[lvl_off(n0, C) + i];
}

}  // namespace fmgsr
