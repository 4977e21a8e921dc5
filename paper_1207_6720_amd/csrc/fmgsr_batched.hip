// fmgsr_batched.hip -- batched FMG-FAS-SR for the 1D reaction-diffusion
// operators (Poisson, -u'' + kappa u^3, -u'' + c u) on gfx950, and the adjoint
// solve built on it.
//
// One persistent launch solves a whole batch of independent problems of
// uneven size.  Every workgroup takes problems from an atomic queue in
// longest-first order and runs the complete FMG-FAS-SR iteration of Fig. 3
// for each: no data crosses workgroups, so the only synchronisation is the
// workgroup barrier between the phases of one problem.  This is the paper's
// data-driven execution (Sec. 3: work proceeds as soon as its inputs are
// ready) at the granularity of problems.
//
// Per problem (levels 0..M, level l with n0 2^l cells; level M is the SR
// level and is never stored):
//   forcing     R^l = I R^{l+1} (R^M = f), A^l = I^ A^{l+1} (A^M = kappa, or
//               3 kappa u_fwd^2 for the adjoint)
//   coarse      Newton on level 0, each step a PCR tridiagonal solve in LDS
//   step t<M    down visits t..1 (smooth, store U^l, coarse rhs Q^{l-1} =
//               I F + R_H(I^ u) - I R_h(u)), coarse Newton, up visits 1..t
//               (V^l = U^l + P(V^{l-1} - I^ U^l), smooth)
//   step M      SR down pass per segment (Pi V^{M-1}, smooth, write I^ of the
//               core to Uh and the core's coarse rhs to Q^{M-1}), V-cycle on
//               the stored levels, SR up pass per segment (Pi, nu2 x
//               [Kaczmarz, sweep], core to the output)
// Stored-level visits walk the level in halo-exact register tiles (every
// core equals a whole-level sweep); each visit reads arrays it does not
// write, so the tiles of one visit are independent.  The legs visit the
// stored levels two at a time (down: from the top; up: from the bottom),
// the lower level of a pair worked from registers (down_visit2,
// up_visit2).
//
// Smoothing (nonlinear red-black Gauss-Seidel, one Newton step per point):
//   cubic   u_i <- ((F_i h^2 + (l + r)) + 2 q u_i^3) / (D + 3 q u_i^2)
//   linear  u_i <- (F_i h^2 + (l + r)) / (D + q),   q = a_i h^2
// with D = 2 (3 at a boundary cell, 4 on a one-cell level).  In the FP32
// relaxation mode each smoothing call forms the FP64 residual once, runs the
// sweeps on an FP32 correction d (exterior d = 0) with the equivalent update
//   d_i <- ((d_l + d_r) + r_i + q d_i^2 (2 w + u_i)) / (D + 3 q w^2),  w = u_i + d_i
// and adds d to u in FP64; residuals, tau and the coarse solve stay FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "fmgsr.h"
#include "fmgsr_device.hpp"

namespace fmgsr {
namespace bt {

constexpr int kOpPoisson = 0, kOpCubic = 1, kOpLinear = 2;
constexpr int kF64 = 0, kF32 = 1;
constexpr int kMaxBatchN0 = 256;     // coarsest level solved in LDS
constexpr int kMaxThreads = 512;
constexpr int64_t kLvlAlign = 32;    // doubles: level arrays start 256-byte aligned
constexpr int kMaxPad = 66;          // SR window pad for the largest buffer (64)

enum Src : int { kZero = 0, kInterp = 1, kRestrict = 2, kDirect = 3 };

struct Prob {
  int64_t n;      // fine cells
  int64_t off;    // offset of the problem in the packed f / kappa / u arrays
  int64_t ws;     // offset (doubles) of its workspace slab
  int64_t seg;    // SR segment core (fine cells)
  int64_t coff;   // offset of its level-(M-1) solution in a packed coarse array
  int32_t M;      // levels - 1
  int32_t n0;     // coarsest cells
  double gL, gR;
};

struct Args {
  const Prob* probs;
  const int32_t* order;  // queue position -> problem
  int32_t batch;
  int32_t* queue;
  const double* f;       // packed right-hand sides (adjoint: dJ/du)
  const double* kappa;   // packed coefficient (null for Poisson)
  const double* ufwd;    // adjoint: packed forward solution (coefficient 3 kappa u^2)
  double* u;             // packed result (adjoint: grad_f = lambda), may be null
  double* gk;            // adjoint: packed grad_kappa = -u^3 lambda, may be null
  double* ws;
  double* vkeep;         // forward: packed level-(M-1) solution out, or null
  const double* ffwd;    // adjoint without u_fwd: the forward's packed rhs
  const double* vfwd;    // ... and its kept level-(M-1) solution
  int nu1, nu2, buffer, halo;
  int halo2;             // halo of the two-level (fused) visits
  int region;            // doubles of the LDS stage / coarse-solve region
  int adjoint;           // 1: homogeneous boundary values (adjoint solve)
  int group;             // workgroups cooperating on one problem (G)
  int32_t* bars;         // [2 batch] per-problem barrier (count, generation)
  int32_t* status;       // set to 1 if a group barrier timed out
};

__host__ __device__ inline int64_t lvl_size(int64_t n0, int l) {
  return ((n0 << l) + kLvlAlign - 1) / kLvlAlign * kLvlAlign;
}
__host__ __device__ inline int64_t lvl_off(int64_t n0, int l) {
  int64_t o = 0;
  for (int m = 0; m < l; ++m) o += lvl_size(n0, m);
  return o;
}
// Slab of one problem: R, A, U, V, Q (levels 0..M-1 each), then Uh (n/2).
__host__ __device__ inline int64_t slab_doubles(int64_t n0, int M) {
  const int64_t h = lvl_off(n0, M);
  return 5 * h + (M > 0 ? lvl_size(n0, M - 1) : 0);
}

// Per-problem view used by the device code.
struct Ctx {
  int64_t n, n0, seg;
  int M;
  double gL, gR;
  const double* f;
  const double* kap;
  const double* uf;
  double* uo;
  double* gk;
  double *R, *A, *U, *V, *Q, *Uh;
  int64_t hier;  // doubles per hierarchy array
  int member, G; // this workgroup's rank in the problem's group, group size
  int32_t* bar;  // the problem's barrier (count, generation)
  int32_t* status;
  double* vk;          // forward: the last step's V^{M-1} goes here (null: workspace)
  const double* ff;    // adjoint rebuild: forward rhs, kept V^{M-1} (null: u_fwd given)
  const double* vf;
  double gLf, gRf;     // forward boundary values
  double* eb;          // LDS, 2 * kMaxPad doubles: window cells of neighbour patches
  __device__ __forceinline__ int64_t nl(int l) const { return n0 << l; }
  __device__ __forceinline__ int64_t off(int l) const { return lvl_off(n0, l); }
  // fine-level coefficient: kappa, or 3 kappa u_fwd^2 for the adjoint
  __device__ __forceinline__ double coef_fine(int64_t g) const {
    if (!kap) return 0.0;
    if (uf) { const double v = uf[g]; return (3.0 * kap[g]) * (v * v); }
    return kap[g];
  }
};

__device__ __forceinline__ Ctx make_ctx(const Prob& p, const Args& a) {
  Ctx c;
  c.n = p.n; c.n0 = p.n0; c.seg = p.seg; c.M = p.M;
  c.gL = a.adjoint ? 0.0 : p.gL;
  c.gR = a.adjoint ? 0.0 : p.gR;
  c.f = a.f + p.off;
  c.kap = a.kappa ? a.kappa + p.off : nullptr;
  c.uf = a.ufwd ? a.ufwd + p.off : nullptr;
  c.uo = a.u ? a.u + p.off : nullptr;
  c.gk = a.gk ? a.gk + p.off : nullptr;
  c.hier = lvl_off(p.n0, p.M);
  double* s = a.ws + p.ws;
  c.R = s; c.A = s + c.hier; c.U = s + 2 * c.hier; c.V = s + 3 * c.hier; c.Q = s + 4 * c.hier;
  c.Uh = s + 5 * c.hier;
  c.G = a.group;
  c.member = 0;
  c.bar = nullptr;
  c.status = a.status;
  c.vk = (a.vkeep && p.M >= 1) ? a.vkeep + p.coff : nullptr;
  c.ff = a.ffwd ? a.ffwd + p.off : nullptr;
  c.vf = (a.vfwd && p.M >= 1) ? a.vfwd + p.coff : nullptr;
  c.gLf = p.gL;
  c.gRf = p.gR;
  c.eb = nullptr;
  return c;
}

// The forward problem's view for rebuilding u_fwd: its rhs, kappa as the
// coefficient, its boundary values, no outputs.
__device__ __forceinline__ Ctx forward_ctx(const Ctx& c) {
  Ctx f = c;
  f.f = c.ff;
  f.uf = nullptr;
  f.uo = nullptr;
  f.gk = nullptr;
  f.gL = c.gLf;
  f.gR = c.gRf;
  return f;
}

// ---------------------------------------------------------------------------
// Loads in two halves (issue all, then stage), so that the HBM latencies of
// all arrays of a tile overlap.  Cell e of the window has global index
// wlo + e; values outside [0, n) or beyond wcount become 0.
// ---------------------------------------------------------------------------
template <int K, class Fn>
__device__ __forceinline__ void issue(double (&tmp)[K], int64_t wlo, int64_t n, Fn val) {
  const int W = blockDim.x;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t g = wlo + threadIdx.x + k * W;
    tmp[k] = val(g < 0 ? 0 : (g >= n ? n - 1 : g));
  }
}
template <int K>
__device__ __forceinline__ void stage(double* st, const double (&tmp)[K], double (&v)[K],
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

// A window of a level: cells wlo .. wlo + cnt - 1 of a level with n cells;
// local cell e is inside the level when lo <= e <= hi.  Loads and stores go
// through a uniform base pointer (base + wlo) with 32-bit lane offsets.
struct Win {
  int64_t wlo;
  int lo, hi, cnt;
};
__device__ __forceinline__ Win make_win(int64_t wlo, int cnt, int64_t n) {
  Win w;
  w.wlo = wlo;
  w.cnt = cnt;
  w.lo = wlo < 0 ? (int)(-wlo) : 0;
  const int64_t h = n - 1 - wlo;
  w.hi = h > 0x3fffffff ? 0x3fffffff : (int)h;
  return w;
}
__device__ __forceinline__ int clampe(int e, const Win& w) { return min(max(e, w.lo), w.hi); }

// threadIdx.x through an empty asm statement: per-lane offsets are then
// recomputed at each use instead of being hoisted out of the tile loops and
// kept live (which costs dozens of VGPRs across the smoothing).
__device__ __forceinline__ int lane_id() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__device__ __forceinline__ bool inside(int e, const Win& w) { return e < w.cnt && e >= w.lo && e <= w.hi; }

template <int K>
__device__ __forceinline__ void ld_win(double (&tmp)[K], const double* __restrict__ base,
                                       const Win& w) {
  const double* __restrict__ p = base + w.wlo;
  const int t = lane_id();
#pragma unroll
  for (int k = 0; k < K; ++k) tmp[k] = p[clampe(t + k * blockDim.x, w)];
}
// cell pairs 2g, 2g+1 of the finer level (one 16-byte load each)
template <int K>
__device__ __forceinline__ void ld_win_pairs(double2 (&tmp)[K], const double* __restrict__ fine,
                                             const Win& w) {
  const double2* __restrict__ p = reinterpret_cast<const double2*>(fine + 2 * w.wlo);
  const int t = lane_id();
#pragma unroll
  for (int k = 0; k < K; ++k) tmp[k] = p[clampe(t + k * blockDim.x, w)];
}
// loaded lane values -> stage -> runs; cells outside the level become 0
template <int K>
__device__ __forceinline__ void stage_win(double* st, const double (&tmp)[K], double (&v)[K],
                                          const Win& w) {
  const int t = lane_id();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = t + k * blockDim.x;
    st[sidx<K>(e)] = inside(e, w) ? tmp[k] : 0.0;
  }
  __syncthreads();
  stage_to_run<K>(st, v);
  __syncthreads();
}
// runs -> stage -> coalesced store of the window cells whose level index is
// in [clo, chi)
template <int K>
__device__ __forceinline__ void store_win(double* st, const double (&v)[K],
                                          double* __restrict__ base, int64_t wlo, int64_t clo,
                                          int64_t chi) {
  run_to_stage<K>(st, v);
  __syncthreads();
  double* __restrict__ q = base + wlo;
  const int a = (int)(clo - wlo), b = (int)(chi - wlo);
  const int t = lane_id();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = t + k * blockDim.x;
    if (e >= a && e < b) q[e] = st[sidx<K>(e)];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Smoothing on register runs
// ---------------------------------------------------------------------------
struct SweepGeom {
  RunBounds rb;
  double h2, gL2, gR2, bdiv;
};

__device__ __forceinline__ SweepGeom sweep_geom(int64_t g0, int K, int64_t lo, int64_t hi,
                                                int64_t n, double gL, double gR) {
  SweepGeom s;
  s.rb = run_bounds(g0, K, lo, hi, n);
  s.h2 = 1.0 / ((double)n * (double)n);
  s.gL2 = 2.0 * gL;
  s.gR2 = 2.0 * gR;
  s.bdiv = (n == 1) ? 4.0 : 3.0;
  return s;
}

// One FP64 half-sweep of colour C (0 = red = even) over the run.
template <int K, int C, int OP>
__device__ __forceinline__ void ngs_half(double (&u)[K], const double (&F)[K],
                                         const double (&a)[K], const SweepGeom& s, Xch& x) {
  double ll, rf;
  x.swap(u[0], u[K - 1], ll, rf);
#pragma unroll
  for (int j = C; j < K; j += 2) {
    double l = (j == 0) ? ll : u[j - 1];
    double r = (j == K - 1) ? rf : u[j + 1];
    double D = 2.0;
    const bool bnd = (j == s.rb.jb0 || j == s.rb.jbn);
    if (j == s.rb.jb0) { l = s.gL2; D = s.bdiv; }
    if (j == s.rb.jbn) { r = s.gR2; D = s.bdiv; }
    const double b = F[j] * s.h2 + (l + r);
    double v;
    if constexpr (OP == kOpCubic) {
      const double q = a[j] * s.h2;
      const double uu = u[j] * u[j];
      v = (b + (2.0 * q) * (uu * u[j])) / (D + (3.0 * q) * uu);
    } else if constexpr (OP == kOpLinear) {
      const double q = a[j] * s.h2;
      v = b / (D + q);
    } else {
      v = bnd ? b / D : b * 0.5;
    }
    if (j >= s.rb.jlo && j < s.rb.jhi) u[j] = v;
  }
}

// One FP32 half-sweep of the correction d (correction form).
template <int K, int C, int OP>
__device__ __forceinline__ void cf_half(float (&d)[K], const float (&r)[K], const float (&q)[K],
                                        const float (&ut)[K], const SweepGeom& s, float bdiv,
                                        Xch& x) {
  double lld, rfd;
  x.swap((double)d[0], (double)d[K - 1], lld, rfd);
  const float ll = (float)lld, rf = (float)rfd;
#pragma unroll
  for (int j = C; j < K; j += 2) {
    float l = (j == 0) ? ll : d[j - 1];
    float rr = (j == K - 1) ? rf : d[j + 1];
    float D = 2.0f;
    if (j == s.rb.jb0) { l = 0.0f; D = bdiv; }
    if (j == s.rb.jbn) { rr = 0.0f; D = bdiv; }
    float num = (l + rr) + r[j];
    float den = D;
    if constexpr (OP == kOpCubic) {
      const float w = ut[j] + d[j];
      num = num + q[j] * ((d[j] * d[j]) * (2.0f * w + ut[j]));
      den = D + (3.0f * q[j]) * (w * w);
    } else if constexpr (OP == kOpLinear) {
      den = D + q[j];
    }
    const float v = num * __builtin_amdgcn_rcpf(den);
    if (j >= s.rb.jlo && j < s.rb.jhi) d[j] = v;
  }
}

// nu sweeps over the cells [rb.jlo, rb.jhi) of the run; cells outside are
// frozen.
template <int K, int OP, int PREC>
__device__ __forceinline__ void smooth(double (&u)[K], const double (&F)[K], const double (&a)[K],
                                       const SweepGeom& s, int nu, Xch& x) {
  if (nu <= 0) return;
  if constexpr (PREC == kF64) {
    for (int it = 0; it < nu; ++it) {
      ngs_half<K, 0, OP>(u, F, a, s, x);
      ngs_half<K, 1, OP>(u, F, a, s, x);
    }
  } else {
    // FP64 residual r = F h^2 - h^2 N(u), once per call
    double ll, rf;
    x.swap(u[0], u[K - 1], ll, rf);
    float r[K], q[K], ut[K], d[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double l = (j == 0) ? ll : u[j - 1];
      double rr = (j == K - 1) ? rf : u[j + 1];
      double D = 2.0;
      if (j == s.rb.jb0) { l = s.gL2; D = s.bdiv; }
      if (j == s.rb.jbn) { rr = s.gR2; D = s.bdiv; }
      double Ru = 0.0, qd = 0.0;
      if constexpr (OP == kOpCubic) { qd = a[j] * s.h2; Ru = qd * ((u[j] * u[j]) * u[j]); }
      else if constexpr (OP == kOpLinear) { qd = a[j] * s.h2; Ru = qd * u[j]; }
      const double res = (F[j] * s.h2 + (l + rr)) - (D * u[j] + Ru);
      r[j] = (float)res;
      q[j] = (float)qd;
      ut[j] = (float)u[j];
      d[j] = 0.0f;
    }
    const float bd = (float)s.bdiv;
    for (int it = 0; it < nu; ++it) {
      cf_half<K, 0, OP>(d, r, q, ut, s, bd, x);
      cf_half<K, 1, OP>(d, r, q, ut, s, bd, x);
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (j >= s.rb.jlo && j < s.rb.jhi) u[j] = u[j] + (double)d[j];
  }
}

template <int OP>
__device__ __forceinline__ double reaction(double a, double u) {
  if constexpr (OP == kOpCubic) return a * ((u * u) * u);
  else if constexpr (OP == kOpLinear) return a * u;
  else return 0.0;
}

// Coarse right-hand side (split tau) of the run's pairs:
//   Q_J = I F + (R_H(a^H, I^ u) - I R_h(a, u)),  a^H = I^ a.
// g0 = global index of the run's first cell on a level of nf cells.
template <int K, int OP>
__device__ __forceinline__ void coarse_rhs(const double (&u)[K], const double (&F)[K],
                                           const double (&a)[K], double (&Qc)[K / 2], int64_t g0,
                                           int64_t nf, Xch& x) {
  double rv[K];
#pragma unroll
  for (int j = 0; j < K; ++j) rv[j] = reaction<OP>(a[j], u[j]);
  double Fl, Fr, Rl, Rr;
  x.swap(F[0], F[K - 1], Fl, Fr);
  x.swap(rv[0], rv[K - 1], Rl, Rr);
  const RunBounds rb = run_bounds(g0, K, 0, nf, nf);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    double fm = (p == 0) ? Fl : F[2 * p - 1];
    double fp = (p == K / 2 - 1) ? Fr : F[2 * p + 2];
    double rm = (p == 0) ? Rl : rv[2 * p - 1];
    double rp = (p == K / 2 - 1) ? Rr : rv[2 * p + 2];
    if (2 * p == rb.jb0) { fm = -F[2 * p]; rm = -rv[2 * p]; }
    if (2 * p + 1 == rb.jbn) { fp = -F[2 * p + 1]; rp = -rv[2 * p + 1]; }
    const double IF = ((fm + fp) + 3.0 * (F[2 * p] + F[2 * p + 1])) * 0.125;
    const double IR = ((rm + rp) + 3.0 * (rv[2 * p] + rv[2 * p + 1])) * 0.125;
    const double uh = (u[2 * p] + u[2 * p + 1]) * 0.5;
    const double ac = (a[2 * p] + a[2 * p + 1]) * 0.5;
    Qc[p] = IF + (reaction<OP>(ac, uh) - IR);
  }
}

// Tiling of a stored level of n cells by windows of W = T K cells.
struct Tiling {
  int64_t core, ntiles, halo;
  int wcount;
};
__device__ __forceinline__ Tiling tiling(int64_t n, int K, int halo) {
  Tiling t;
  const int64_t W = (int64_t)blockDim.x * K;
  if (n <= W) { t.core = n; t.ntiles = 1; t.halo = 0; t.wcount = (int)n; }
  else { t.core = W - 2 * halo; t.ntiles = (n + t.core - 1) / t.core; t.halo = halo; t.wcount = (int)W; }
  return t;
}

// ---------------------------------------------------------------------------
// Level visits
// ---------------------------------------------------------------------------

// Down visit of stored level l: the iterate starts from src (Pi of the
// coarser V, I^ of the finer U, or a copy), nu1 sweeps with F, the core is
// stored to U^l and (reaction operators) the coarse rhs to Q^{l-1}.
template <int K, int OP, int PREC>
__device__ __forceinline__ void down_visit(const Ctx& c, const Args& ar, int l, int src_kind, const double* src,
                           const double* F, double* st, Xch& x) {
  const int64_t n = c.nl(l);
  const double* A = c.A + c.off(l);
  double* Uo = c.U + c.off(l);
  double* Qo = (OP != kOpPoisson) ? c.Q + c.off(l - 1) : nullptr;
  const Tiling tl = tiling(n, K, ar.halo);
  const int64_t first = (tl.ntiles == 1) ? 0 : c.member, stride = (tl.ntiles == 1) ? 1 : c.G;
  for (int64_t ti = first; ti < tl.ntiles; ti += stride) {
    const int64_t clo = ti * tl.core, chi = min(clo + tl.core, n);
    const int64_t wlo = clo - tl.halo;
    const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
    double u[K], Fr[K], a[K];
    double tu[K], tf[K], ta[K];
    double2 tp[K];
    double tc[K / 2];
    const Win wf = make_win(wlo, tl.wcount, n);
    const Win wc = make_win(wlo >> 1, (tl.wcount + 1) / 2 + 2, n >> 1);
    if (src_kind == kInterp) ld_win<K / 2>(tc, src, wc);
    else if (src_kind == kRestrict) ld_win_pairs<K>(tp, src, wf);
    else ld_win<K>(tu, src, wf);
    ld_win<K>(tf, F, wf);
    if constexpr (OP != kOpPoisson) ld_win<K>(ta, A, wf);
    if (src_kind == kInterp) {
      double cr[K / 2];
      stage_win<K / 2>(st, tc, cr, wc);
      interp_from_run<K>(u, cr, g0, n, src, c.gL, c.gR, x);
    } else {
      if (src_kind == kRestrict) {
#pragma unroll
        for (int k = 0; k < K; ++k) tu[k] = (tp[k].x + tp[k].y) * 0.5;
      }
      stage_win<K>(st, tu, u, wf);
    }
    stage_win<K>(st, tf, Fr, wf);
    if constexpr (OP != kOpPoisson) stage_win<K>(st, ta, a, wf);
    else {
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] = 0.0;
    }
    const SweepGeom sg = sweep_geom(g0, K, max(wlo, (int64_t)0), min(wlo + tl.wcount, n), n,
                                    c.gL, c.gR);
    smooth<K, OP, PREC>(u, Fr, a, sg, ar.nu1, x);
    store_win<K>(st, u, Uo, wlo, clo, chi);
    if constexpr (OP != kOpPoisson) {
      double qc[K / 2];
      coarse_rhs<K, OP>(u, Fr, a, qc, g0, n, x);
      store_win<K / 2>(st, qc, Qo, wlo >> 1, clo >> 1, chi >> 1);
    }
  }
  __syncthreads();
}

// Up visit of stored level l: V^l = U^l + P(V^{l-1} - I^ U^l), nu2 sweeps.
// Coarse-grid correction (Eq. 4) of a run: u += P(cv - I^ u), homogeneous
// reflections at the level's ends; g0 = the run's first cell, nc = coarse
// cells of the level.
template <int K>
__device__ __forceinline__ void correct_run(double (&u)[K], const double (&cv)[K / 2], int64_t g0,
                                            int64_t nc, Xch& x) {
  double e[K / 2];
#pragma unroll
  for (int p = 0; p < K / 2; ++p) e[p] = cv[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
  double el, er;
  x.swap(e[0], e[K / 2 - 1], el, er);
  const int64_t J0 = g0 >> 1;
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    const int64_t J = J0 + p;
    double em = (p == 0) ? el : e[p - 1];
    double ep = (p == K / 2 - 1) ? er : e[p + 1];
    if (J == 0) em = -e[p];
    if (J == nc - 1) ep = -e[p];
    u[2 * p] = u[2 * p] + (3.0 * e[p] + em) * 0.25;
    u[2 * p + 1] = u[2 * p + 1] + (3.0 * e[p] + ep) * 0.25;
  }
}

// Vout: where V^l goes (null: the workspace).
template <int K, int OP, int PREC>
__device__ __forceinline__ void up_visit(const Ctx& c, const Args& ar, int l, const double* F, double* st,
                         Xch& x, double* Vout = nullptr) {
  const int64_t n = c.nl(l), nc = n >> 1;
  const double* A = c.A + c.off(l);
  const double* Up = c.U + c.off(l);
  const double* Vc = c.V + c.off(l - 1);
  double* Vo = Vout ? Vout : c.V + c.off(l);
  const Tiling tl = tiling(n, K, ar.halo);
  const int64_t first = (tl.ntiles == 1) ? 0 : c.member, stride = (tl.ntiles == 1) ? 1 : c.G;
  for (int64_t ti = first; ti < tl.ntiles; ti += stride) {
    const int64_t clo = ti * tl.core, chi = min(clo + tl.core, n);
    const int64_t wlo = clo - tl.halo;
    const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
    double u[K], Fr[K], a[K], cv[K / 2];
    double tu[K], tf[K], ta[K], tc[K / 2];
    const Win wf = make_win(wlo, tl.wcount, n);
    const Win wc = make_win(wlo >> 1, (tl.wcount + 1) / 2, nc);
    ld_win<K>(tu, Up, wf);
    ld_win<K / 2>(tc, Vc, wc);
    ld_win<K>(tf, F, wf);
    if constexpr (OP != kOpPoisson) ld_win<K>(ta, A, wf);
    stage_win<K>(st, tu, u, wf);
    stage_win<K / 2>(st, tc, cv, wc);
    stage_win<K>(st, tf, Fr, wf);
    if constexpr (OP != kOpPoisson) stage_win<K>(st, ta, a, wf);
    else {
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] = 0.0;
    }
    correct_run<K>(u, cv, g0, nc, x);
    const SweepGeom sg = sweep_geom(g0, K, max(wlo, (int64_t)0), min(wlo + tl.wcount, n), n,
                                    c.gL, c.gR);
    smooth<K, OP, PREC>(u, Fr, a, sg, ar.nu2, x);
    store_win<K>(st, u, Vo, wlo, clo, chi);
  }
  __syncthreads();
}

// Full weighting of a run's rhs pairs, I F (the Poisson forcing restriction,
// same expression and boundary reflections as forcing_level).
template <int K>
__device__ __forceinline__ void fw_run(const double (&F)[K], double (&Fc)[K / 2], int64_t g0,
                                       int64_t nf, Xch& x) {
  double Fl, Fr;
  x.swap(F[0], F[K - 1], Fl, Fr);
  const RunBounds rb = run_bounds(g0, K, 0, nf, nf);
#pragma unroll
  for (int p = 0; p < K / 2; ++p) {
    double fm = (p == 0) ? Fl : F[2 * p - 1];
    double fp = (p == K / 2 - 1) ? Fr : F[2 * p + 2];
    if (2 * p == rb.jb0) fm = -F[2 * p];
    if (2 * p + 1 == rb.jbn) fp = -F[2 * p + 1];
    Fc[p] = ((fm + fp) + 3.0 * (F[2 * p] + F[2 * p + 1])) * 0.125;
  }
}

// Two stored levels per tile visit (vertical fusion): the tiles of level l
// carry a halo of ar.halo2 cells, enough for both levels' sweeps, so the
// level-(l-1) half of every window is exact on its core.  Each fused value
// is formed by the same expression as in the one-level visits, so results
// are bit-for-bit those of two separate visits.
//
// Down: level l as down_visit (src, F, A; nu1 sweeps; U^l and Q^{l-1}
// stored), then level l-1 from registers: its iterate I^ u, its rhs Q^{l-1}
// (Poisson: I F), its coefficient I^ a; nu1 sweeps; U^{l-1} and Q^{l-2}
// stored.  Saves reading level l-1's source, rhs and coefficient.
template <int K, int OP, int PREC>
__device__ __forceinline__ void down_visit2(const Ctx& c, const Args& ar, int l, int src_kind,
                                            const double* src, const double* F, double* st,
                                            Xch& x) {
  const int64_t n = c.nl(l), n1 = n >> 1;
  const double* A = c.A + c.off(l);
  double* Uo = c.U + c.off(l);
  double* U1 = c.U + c.off(l - 1);
  double* Qo = (OP != kOpPoisson) ? c.Q + c.off(l - 1) : nullptr;
  double* Q1 = (OP != kOpPoisson) ? c.Q + c.off(l - 2) : nullptr;
  const Tiling tl = tiling(n, K, ar.halo2);
  const int64_t first = (tl.ntiles == 1) ? 0 : c.member, stride = (tl.ntiles == 1) ? 1 : c.G;
  for (int64_t ti = first; ti < tl.ntiles; ti += stride) {
    const int64_t clo = ti * tl.core, chi = min(clo + tl.core, n);
    const int64_t wlo = clo - tl.halo;
    const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
    double u[K], Fr[K], a[K];
    {
      double tu[K], tf[K], ta[K];
      double2 tp[K];
      double tc[K / 2];
      const Win wf = make_win(wlo, tl.wcount, n);
      const Win wc = make_win(wlo >> 1, (tl.wcount + 1) / 2 + 2, n >> 1);
      if (src_kind == kInterp) ld_win<K / 2>(tc, src, wc);
      else if (src_kind == kRestrict) ld_win_pairs<K>(tp, src, wf);
      else ld_win<K>(tu, src, wf);
      ld_win<K>(tf, F, wf);
      if constexpr (OP != kOpPoisson) ld_win<K>(ta, A, wf);
      if (src_kind == kInterp) {
        double cr[K / 2];
        stage_win<K / 2>(st, tc, cr, wc);
        interp_from_run<K>(u, cr, g0, n, src, c.gL, c.gR, x);
      } else {
        if (src_kind == kRestrict) {
#pragma unroll
          for (int k = 0; k < K; ++k) tu[k] = (tp[k].x + tp[k].y) * 0.5;
        }
        stage_win<K>(st, tu, u, wf);
      }
      stage_win<K>(st, tf, Fr, wf);
      if constexpr (OP != kOpPoisson) stage_win<K>(st, ta, a, wf);
      else {
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = 0.0;
      }
    }
    const SweepGeom sg = sweep_geom(g0, K, max(wlo, (int64_t)0), min(wlo + tl.wcount, n), n,
                                    c.gL, c.gR);
    smooth<K, OP, PREC>(u, Fr, a, sg, ar.nu1, x);
    store_win<K>(st, u, Uo, wlo, clo, chi);
    // level l-1 from the runs of level l
    double u1[K / 2], f1[K / 2], a1[K / 2];
    if constexpr (OP != kOpPoisson) {
      coarse_rhs<K, OP>(u, Fr, a, f1, g0, n, x);
      store_win<K / 2>(st, f1, Qo, wlo >> 1, clo >> 1, chi >> 1);
    } else {
      fw_run<K>(Fr, f1, g0, n, x);
    }
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      u1[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
      a1[p] = (a[2 * p] + a[2 * p + 1]) * 0.5;
    }
    const int64_t wlo1 = wlo >> 1, g1 = g0 >> 1;
    const int wcount1 = tl.wcount / 2;
    const SweepGeom sg1 = sweep_geom(g1, K / 2, max(wlo1, (int64_t)0), min(wlo1 + wcount1, n1),
                                     n1, c.gL, c.gR);
    smooth<K / 2, OP, PREC>(u1, f1, a1, sg1, ar.nu1, x);
    store_win<K / 2>(st, u1, U1, wlo1, clo >> 1, chi >> 1);
    if constexpr (OP != kOpPoisson) {
      double q1[K / 4];
      coarse_rhs<K / 2, OP>(u1, f1, a1, q1, g1, n1, x);
      store_win<K / 4>(st, q1, Q1, wlo1 >> 1, clo >> 2, chi >> 2);
    }
  }
  __syncthreads();
}

// Up: level l-1 as up_visit (U^{l-1}, V^{l-2}, F^{l-1}, A^{l-1}; correction
// and nu2 sweeps) into registers, then level l with that V^{l-1} as its
// coarse iterate; only V^l is stored (to Vout when given).  Saves writing and
// reading V^{l-1}.
template <int K, int OP, int PREC>
__device__ __forceinline__ void up_visit2(const Ctx& c, const Args& ar, int l, const double* F1,
                                          const double* F, double* st, Xch& x,
                                          double* Vout = nullptr) {
  const int64_t n = c.nl(l), n1 = n >> 1, n2 = n1 >> 1;
  const double* A = c.A + c.off(l);
  const double* A1 = c.A + c.off(l - 1);
  const double* Up = c.U + c.off(l);
  const double* Up1 = c.U + c.off(l - 1);
  const double* Vc = c.V + c.off(l - 2);
  double* Vo = Vout ? Vout : c.V + c.off(l);
  const Tiling tl = tiling(n, K, ar.halo2);
  const int64_t first = (tl.ntiles == 1) ? 0 : c.member, stride = (tl.ntiles == 1) ? 1 : c.G;
  for (int64_t ti = first; ti < tl.ntiles; ti += stride) {
    const int64_t clo = ti * tl.core, chi = min(clo + tl.core, n);
    const int64_t wlo = clo - tl.halo;
    const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
    const int64_t wlo1 = wlo >> 1, g1 = g0 >> 1;
    const int wcount1 = tl.wcount / 2;
    // level l-1
    double v1[K / 2];
    {
      double u[K / 2], Fr[K / 2], a[K / 2], cv[K / 4];
      double tu[K / 2], tf[K / 2], ta[K / 2], tc[K / 4];
      const Win wf = make_win(wlo1, wcount1, n1);
      const Win wc = make_win(wlo1 >> 1, (wcount1 + 1) / 2, n2);
      ld_win<K / 2>(tu, Up1, wf);
      ld_win<K / 4>(tc, Vc, wc);
      ld_win<K / 2>(tf, F1, wf);
      if constexpr (OP != kOpPoisson) ld_win<K / 2>(ta, A1, wf);
      stage_win<K / 2>(st, tu, u, wf);
      stage_win<K / 4>(st, tc, cv, wc);
      stage_win<K / 2>(st, tf, Fr, wf);
      if constexpr (OP != kOpPoisson) stage_win<K / 2>(st, ta, a, wf);
      else {
#pragma unroll
        for (int j = 0; j < K / 2; ++j) a[j] = 0.0;
      }
      correct_run<K / 2>(u, cv, g1, n2, x);
      const SweepGeom sg = sweep_geom(g1, K / 2, max(wlo1, (int64_t)0),
                                      min(wlo1 + wcount1, n1), n1, c.gL, c.gR);
      smooth<K / 2, OP, PREC>(u, Fr, a, sg, ar.nu2, x);
#pragma unroll
      for (int j = 0; j < K / 2; ++j) v1[j] = u[j];
    }
    // level l
    double u[K], Fr[K], a[K];
    {
      double tu[K], tf[K], ta[K];
      const Win wf = make_win(wlo, tl.wcount, n);
      ld_win<K>(tu, Up, wf);
      ld_win<K>(tf, F, wf);
      if constexpr (OP != kOpPoisson) ld_win<K>(ta, A, wf);
      stage_win<K>(st, tu, u, wf);
      stage_win<K>(st, tf, Fr, wf);
      if constexpr (OP != kOpPoisson) stage_win<K>(st, ta, a, wf);
      else {
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = 0.0;
      }
    }
    correct_run<K>(u, v1, g0, n1, x);
    const SweepGeom sg = sweep_geom(g0, K, max(wlo, (int64_t)0), min(wlo + tl.wcount, n), n,
                                    c.gL, c.gR);
    smooth<K, OP, PREC>(u, Fr, a, sg, ar.nu2, x);
    store_win<K>(st, u, Vo, wlo, clo, chi);
  }
  __syncthreads();
}

// SR up pass of segment i (Eq. 5, Fig. 5) on staged runs: ubar = Pi of the
// coarse run cr (V^{M-1} under the window, Vc for the edge values), then
// nu2 x [Kaczmarz projection of the patch's full pairs onto I^ ubar =
// V^{M-1}, one sweep].
template <int K, int OP, int PREC>
__device__ __forceinline__ void sr_up_runs(const Ctx& c, const Args& ar, const double* Vc,
                                           int64_t i, const double (&cr)[K / 2],
                                           const double (&Fr)[K], const double (&a)[K],
                                           double (&u)[K], Xch& x) {
  const int64_t n = c.n, s = c.seg;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const int64_t wlo = i * s - pad;
  const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
  interp_from_run<K>(u, cr, g0, n, Vc, c.gL, c.gR, x);
  const int64_t lo = max(i * s - ar.buffer, (int64_t)0), hi = min((i + 1) * s + ar.buffer, n);
  const SweepGeom sg = sweep_geom(g0, K, lo, hi, n, c.gL, c.gR);
  for (int it = 0; it < ar.nu2; ++it) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      const int64_t g = g0 + 2 * p;
      if (g >= lo && g + 1 < hi) {
        const double r = cr[p] - (u[2 * p] + u[2 * p + 1]) * 0.5;
        u[2 * p] = u[2 * p] + r;
        u[2 * p + 1] = u[2 * p + 1] + r;
      }
    }
    smooth<K, OP, PREC>(u, Fr, a, sg, 1, x);
  }
}

// u_fwd on the window of segment j, exact on its core [j s, (j+1) s): the
// forward's SR up pass of that segment again (cf = forward_ctx), from its
// rhs, kappa and kept V^{M-1}.  Same window, same code, so the same bits.
template <int K, int PREC>
__device__ __forceinline__ void fwd_patch(const Ctx& cf, const Args& ar, int64_t j,
                                          double (&w)[K], double* st, Xch& x) {
  const int64_t n = cf.n, nc = n >> 1, s = cf.seg;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const int wcount = (int)(s + 2 * pad);
  const int64_t wlo = j * s - pad;
  double Fr[K], a[K], cr[K / 2];
  double tf[K], ta[K], tc[K / 2];
  const Win wf = make_win(wlo, wcount, n);
  const Win wc = make_win(wlo >> 1, (wcount + 1) / 2 + 2, nc);
  ld_win<K / 2>(tc, cf.vf, wc);
  ld_win<K>(tf, cf.f, wf);
  ld_win<K>(ta, cf.kap, wf);
  stage_win<K / 2>(st, tc, cr, wc);
  stage_win<K>(st, tf, Fr, wf);
  stage_win<K>(st, ta, a, wf);
  sr_up_runs<K, kOpCubic, PREC>(cf, ar, cf.vf, j, cr, Fr, a, w, x);
}

// u_fwd on the whole window of segment i (inside the domain): the core
// from patch i's own rebuild, the pad cells on each side from the
// neighbouring patches' cores (they hold them since pad <= s), passed
// through the LDS buffer c.eb.
template <int K, int PREC>
__device__ __forceinline__ void fwd_window(const Ctx& c, const Args& ar, int64_t i, double (&w)[K], double* st,
                           Xch& x) {
  const Ctx cf = forward_ctx(c);
  const int64_t s = c.seg, S = c.n / s;
  const int pad = (ar.buffer + 2) & ~1;
  const int t0 = (int)threadIdx.x * K;  // window cell of w[0]
  if (i > 0) {
    // window i-1 cell e + s = window i cell e, e < pad
    fwd_patch<K, PREC>(cf, ar, i - 1, w, st, x);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int e = t0 + j - (int)s;
      if (e >= 0 && e < pad) c.eb[e] = w[j];
    }
  }
  if (i + 1 < S) {
    // window i+1 cell e - s = window i cell e, pad + s <= e < 2 pad + s
    fwd_patch<K, PREC>(cf, ar, i + 1, w, st, x);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int e = t0 + j;  // = (window i cell) - s
      if (e >= pad && e < 2 * pad) c.eb[e] = w[j];
    }
  }
  fwd_patch<K, PREC>(cf, ar, i, w, st, x);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int e = t0 + j;
    if (i > 0 && e < pad) w[j] = c.eb[e];
    if (i + 1 < S && e >= pad + (int)s && e < 2 * pad + (int)s) w[j] = c.eb[e - (int)s];
  }
  __syncthreads();
}

// Inputs of the SR passes on segment i, as staged runs: the coarse run cr
// of Vc, the rhs Fr and the coefficient a (kappa; for the adjoint 3 kappa
// u_fwd^2, with u_fwd read from ufwd or rebuilt into w; Poisson: 0).
template <int K, int OP, int PREC, bool RB>
__device__ __forceinline__ void sr_inputs(const Ctx& c, const Args& ar, const double* Vc, int64_t i,
                                          double (&cr)[K / 2], double (&Fr)[K], double (&a)[K],
                                          double (&w)[K], double* st, Xch& x) {
  const int64_t n = c.n, nc = n >> 1, s = c.seg;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const int wcount = (int)(s + 2 * pad);
  const int64_t wlo = i * s - pad;
  if constexpr (RB) fwd_window<K, PREC>(c, ar, i, w, st, x);
  double tf[K], ta[K], tw[K], tc[K / 2];
  const Win wf = make_win(wlo, wcount, n);
  const Win wc = make_win(wlo >> 1, (wcount + 1) / 2 + 2, nc);
  ld_win<K / 2>(tc, Vc, wc);
  ld_win<K>(tf, c.f, wf);
  if constexpr (OP != kOpPoisson) {
    ld_win<K>(ta, c.kap, wf);
    if (c.uf) ld_win<K>(tw, c.uf, wf);
  }
  stage_win<K / 2>(st, tc, cr, wc);
  stage_win<K>(st, tf, Fr, wf);
  if constexpr (OP != kOpPoisson) {
    if (c.uf) {
#pragma unroll
      for (int k = 0; k < K; ++k) ta[k] = (3.0 * ta[k]) * (tw[k] * tw[k]);
    }
    stage_win<K>(st, ta, a, wf);
    if constexpr (RB) {
#pragma unroll
      for (int j = 0; j < K; ++j) a[j] = (3.0 * a[j]) * (w[j] * w[j]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < K; ++j) a[j] = 0.0;
  }
}

// SR down pass (Fig. 3 at the finest level, per segment): ubar = Pi V^{M-1}
// on the extended patch, nu1 sweeps with the exterior frozen, I^ of the core
// to Uh and (reaction operators) the core's coarse rhs to Q^{M-1}.
template <int K, int OP, int PREC, bool RB>
__device__ __forceinline__ void sr_down(const Ctx& c, const Args& ar, double* st, Xch& x) {
  const int64_t n = c.n, s = c.seg, S = n / s;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const double* Vc = c.V + c.off(c.M - 1);
  double* Qo = (OP != kOpPoisson) ? c.Q + c.off(c.M - 1) : nullptr;
  for (int64_t i = c.member; i < S; i += c.G) {
    const int64_t wlo = i * s - pad;
    const int64_t g0 = wlo + (int64_t)threadIdx.x * K;
    double u[K], Fr[K], a[K], cr[K / 2], w[K];
    sr_inputs<K, OP, PREC, RB>(c, ar, Vc, i, cr, Fr, a, w, st, x);
    interp_from_run<K>(u, cr, g0, n, Vc, c.gL, c.gR, x);
    const int64_t lo = max(i * s - ar.buffer, (int64_t)0), hi = min((i + 1) * s + ar.buffer, n);
    const SweepGeom sg = sweep_geom(g0, K, lo, hi, n, c.gL, c.gR);
    smooth<K, OP, PREC>(u, Fr, a, sg, ar.nu1, x);
    double uh[K / 2];
#pragma unroll
    for (int p = 0; p < K / 2; ++p) uh[p] = (u[2 * p] + u[2 * p + 1]) * 0.5;
    store_win<K / 2>(st, uh, c.Uh, wlo >> 1, (i * s) >> 1, ((i + 1) * s) >> 1);
    if constexpr (OP != kOpPoisson) {
      double qc[K / 2];
      coarse_rhs<K, OP>(u, Fr, a, qc, g0, n, x);
      store_win<K / 2>(st, qc, Qo, wlo >> 1, (i * s) >> 1, ((i + 1) * s) >> 1);
    }
  }
  __syncthreads();
}

// SR up pass (Eq. 5, Fig. 5, per segment), core to the output.  V^{M-1} is
// read from the kept array when the forward keeps it.  For the adjoint the
// output is lambda (grad_f) and grad_kappa = -u_fwd^3 lambda.
template <int K, int OP, int PREC, bool RB>
__device__ __forceinline__ void sr_up(const Ctx& c, const Args& ar, double* st, Xch& x) {
  const int64_t n = c.n, s = c.seg, S = n / s;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const int wcount = (int)(s + 2 * pad);
  const double* Vc = c.vk ? c.vk : c.V + c.off(c.M - 1);
  for (int64_t i = c.member; i < S; i += c.G) {
    const int64_t wlo = i * s - pad;
    double u[K], Fr[K], a[K], cr[K / 2], w[K];
    sr_inputs<K, OP, PREC, RB>(c, ar, Vc, i, cr, Fr, a, w, st, x);
    sr_up_runs<K, OP, PREC>(c, ar, Vc, i, cr, Fr, a, u, x);
    if (c.uo) store_win<K>(st, u, c.uo, wlo, i * s, (i + 1) * s);
    if (c.gk) {
      if constexpr (!RB) {
        const Win wf = make_win(wlo, wcount, n);
        double tw2[K];
        ld_win<K>(tw2, c.uf, wf);
        stage_win<K>(st, tw2, w, wf);
      }
#pragma unroll
      for (int j = 0; j < K; ++j) w[j] = -(((w[j] * w[j]) * w[j]) * u[j]);
      store_win<K>(st, w, c.gk, wlo, i * s, (i + 1) * s);
    }
  }
  __syncthreads();
}

// Adjoint without u_fwd: A^{M-1} = I^ (3 kappa u_fwd^2) on each segment's
// core, u_fwd rebuilt by the forward's SR up pass of that segment (its core
// is exact, and the pairs of the core are all the level-(M-1) cells it
// covers).
template <int K, int PREC>
__device__ __forceinline__ void coef_top(const Ctx& c, const Args& ar, double* st, Xch& x) {
  const int64_t n = c.n, s = c.seg, S = n / s;
  const int64_t pad = (ar.buffer + 2) & ~1;
  const int wcount = (int)(s + 2 * pad);
  const Ctx cf = forward_ctx(c);
  double* Ac = c.A + c.off(c.M - 1);
  for (int64_t i = c.member; i < S; i += c.G) {
    const int64_t wlo = i * s - pad;
    double w[K], kr[K], ta[K], ac[K / 2];
    fwd_patch<K, PREC>(cf, ar, i, w, st, x);
    const Win wf = make_win(wlo, wcount, n);
    ld_win<K>(ta, c.kap, wf);
    stage_win<K>(st, ta, kr, wf);
#pragma unroll
    for (int p = 0; p < K / 2; ++p) {
      const double a0 = (3.0 * kr[2 * p]) * (w[2 * p] * w[2 * p]);
      const double a1 = (3.0 * kr[2 * p + 1]) * (w[2 * p + 1] * w[2 * p + 1]);
      ac[p] = (a0 + a1) * 0.5;
    }
    store_win<K / 2>(st, ac, Ac, wlo >> 1, (i * s) >> 1, ((i + 1) * s) >> 1);
  }
  __syncthreads();
}

// Forcing of level l: R^l = I R^{l+1}, A^l = I^ A^{l+1} (R^M = f, A^M = the
// fine coefficient), cells J = first*T + tid, stepping by stride*T.
template <int OP>
__device__ __forceinline__ void forcing_level(const Ctx& c, int l, int first, int stride) {
  const int T = blockDim.x;
  const int64_t nf = c.nl(l + 1), ncl = c.nl(l);
  const bool top = (l + 1 == c.M);
  const double* Ff = top ? c.f : c.R + c.off(l + 1);
  const double* Af = c.A + c.off(l + 1);
  double* Rc = c.R + c.off(l);
  double* Ac = c.A + c.off(l);
  for (int64_t J = (int64_t)first * T + threadIdx.x; J < ncl; J += (int64_t)stride * T) {
    const double f0 = Ff[2 * J], f1 = Ff[2 * J + 1];
    const double rm = (2 * J - 1 >= 0) ? Ff[2 * J - 1] : -f0;
    const double rp = (2 * J + 2 < nf) ? Ff[2 * J + 2] : -f1;
    Rc[J] = ((rm + rp) + 3.0 * (f0 + f1)) * 0.125;
    if constexpr (OP != kOpPoisson) {
      if (!(top && c.vf)) {  // rebuilt u_fwd: coef_top writes A^{M-1}
        const double a0 = top ? c.coef_fine(2 * J) : Af[2 * J];
        const double a1 = top ? c.coef_fine(2 * J + 1) : Af[2 * J + 1];
        Ac[J] = (a0 + a1) * 0.5;
      }
    }
  }
  __syncthreads();
}

// Barrier of the G workgroups solving one problem: arrive on the problem's
// counter, the last arriver advances the generation.  Writes before the
// barrier are released at agent scope and acquired after it.  The wait is
// bounded; on expiry the status flag is set and false is returned (the
// caller abandons the problem, so every wave still reaches its exit).
__device__ __forceinline__ bool group_sync(const Ctx& c) {
  if (c.G == 1) {
    __syncthreads();
    return true;
  }
  // every wave waits for its own stores, so the release below covers the
  // whole workgroup's writes
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    int32_t* cnt = c.bar;
    int32_t* gen = c.bar + 1;
    const int32_t g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const int32_t arrived = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    if (arrived == c.G - 1) {
      __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int64_t spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(4);
        if (++spins > (int64_t)1 << 24) {
          __hip_atomic_store(c.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = 0;
          break;
        }
      }
    }
    __threadfence();
    ok = good;
  }
  __syncthreads();
  const bool r = ok != 0;
  __syncthreads();
  return r;
}

// Phase sequencing for a group: a barrier separates phases, except between
// two consecutive phases that member 0 runs alone.  Returns whether this
// workgroup takes part in the phase; `alive` turns false after a barrier
// timeout.
struct Phases {
  bool started = false, prev_solo = false, alive = true;
  __device__ __forceinline__ bool begin(const Ctx& c, bool solo) {
    if (!alive) return false;
    if (c.G > 1 && started && !(prev_solo && solo)) alive = group_sync(c);
    started = true;
    prev_solo = solo;
    return alive && (!solo || c.member == 0);
  }
};

__device__ __forceinline__ void wg_max2(double& a, double& b, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a = fmax(a, __shfl_xor(a, o));
    b = fmax(b, __shfl_xor(b, o));
  }
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[w] = a; red[16 + w] = b; }
  __syncthreads();
  a = red[0];
  b = red[16];
  for (int i = 1; i < nw; ++i) { a = fmax(a, red[i]); b = fmax(b, red[16 + i]); }
  __syncthreads();
}

// Coarsest level: Newton's method, each step one PCR solve of the h^2-scaled
// tridiagonal Jacobian in LDS.  Stop when max|d| <= 1e-14 max|u|, or when
// max|d| <= 1e-8 max|u| and the step failed to halve max|d| (rounding
// floor), or after 30 steps.  src: kZero (start of FMG), kRestrict (I^ of
// U^1) or kDirect (Uh).  F and A: rhs and coefficient (fine arrays when the
// problem has one level).
template <int OP>
__device__ __forceinline__ void coarse_visit(const Ctx& c, int src_kind, const double* src, const double* F,
                             const double* A, bool fine, double* out, double* lds, double* red) {
  const int T = blockDim.x;
  const int64_t n = c.n0;
  const int nn = (int)n;
  const double h2 = 1.0 / ((double)n * (double)n);
  double* u = lds;
  double* Fv = u + nn;
  double* q = Fv + nn;
  double* P0 = q + nn;          // a, b, c, d of buffer 0
  double* P1 = P0 + 4 * nn;     // buffer 1
  for (int i = threadIdx.x; i < nn; i += T) {
    u[i] = (src_kind == kZero) ? 0.0
         : (src_kind == kRestrict) ? (src[2 * i] + src[2 * i + 1]) * 0.5 : src[i];
    Fv[i] = F[i];
    q[i] = (OP == kOpPoisson) ? 0.0 : (fine ? c.coef_fine(i) : A[i]) * h2;
  }
  __syncthreads();
  const double gL2 = 2.0 * c.gL, gR2 = 2.0 * c.gR;
  double dprev = 0.0;
  for (int it = 0; it < 30; ++it) {
    for (int i = threadIdx.x; i < nn; i += T) {
      const double l = (i > 0) ? u[i - 1] : gL2;
      const double r = (i < nn - 1) ? u[i + 1] : gR2;
      const double D = (nn == 1) ? 4.0 : ((i > 0 && i < nn - 1) ? 2.0 : 3.0);
      double Ru = 0.0, dR = 0.0;
      if constexpr (OP == kOpCubic) { Ru = q[i] * ((u[i] * u[i]) * u[i]); dR = 3.0 * q[i] * (u[i] * u[i]); }
      else if constexpr (OP == kOpLinear) { Ru = q[i] * u[i]; dR = q[i]; }
      P0[i] = (i > 0) ? -1.0 : 0.0;
      P0[nn + i] = D + dR;
      P0[2 * nn + i] = (i < nn - 1) ? -1.0 : 0.0;
      P0[3 * nn + i] = (Fv[i] * h2 + (l + r)) - (D * u[i] + Ru);
    }
    __syncthreads();
    double* cur = P0;
    double* nxt = P1;
    for (int sd = 1; sd < nn; sd <<= 1) {
      for (int i = threadIdx.x; i < nn; i += T) {
        const double ai = cur[i], bi = cur[nn + i], ci = cur[2 * nn + i], di = cur[3 * nn + i];
        double na = 0.0, nb = bi, nc2 = 0.0, nd = di;
        if (i - sd >= 0) {
          const int k = i - sd;
          const double al = -ai / cur[nn + k];
          na = al * cur[k];
          nb = nb + al * cur[2 * nn + k];
          nd = nd + al * cur[3 * nn + k];
        }
        if (i + sd < nn) {
          const int k = i + sd;
          const double ga = -ci / cur[nn + k];
          nc2 = ga * cur[2 * nn + k];
          nb = nb + ga * cur[k];
          nd = nd + ga * cur[3 * nn + k];
        }
        nxt[i] = na; nxt[nn + i] = nb; nxt[2 * nn + i] = nc2; nxt[3 * nn + i] = nd;
      }
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
    double dmax = 0.0, umax = 0.0;
    for (int i = threadIdx.x; i < nn; i += T) {
      const double d = cur[3 * nn + i] / cur[nn + i];
      u[i] = u[i] + d;
      dmax = fmax(dmax, fabs(d));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nn; i += T) umax = fmax(umax, fabs(u[i]));
    wg_max2(dmax, umax, red);
    if (dmax <= 1e-14 * umax || (it >= 1 && dmax <= 1e-8 * umax && dmax > 0.5 * dprev)) break;
    dprev = dmax;
  }
  for (int i = threadIdx.x; i < nn; i += T) out[i] = u[i];
  __syncthreads();
}

// The whole FMG-FAS-SR iteration of one problem (by the group's member
// c.member; levels of at most one window are run by member 0 alone).
template <int K, int OP, int PREC, bool RB>
__device__ __forceinline__ void solve_problem(const Ctx& c, const Args& ar, double* st, Xch& x, double* red) {
  const int M = c.M;
  const int64_t W = (int64_t)blockDim.x * K;
  Phases ph;
  if (M == 0) {
    // one level: the exact (Newton) solve on the fine grid
    if (!ph.begin(c, true)) return;
    double* out = c.uo ? c.uo : c.U;
    Ctx ca = c;
    if constexpr (RB) {
      {
        // adjoint without u_fwd: the forward's exact solve again, into the
        // second half of the workspace slab
        double* uw = c.U + lvl_size(c.n0, 0);
        const Ctx cf = forward_ctx(c);
        coarse_visit<kOpCubic>(cf, kZero, nullptr, cf.f, nullptr, true, uw, st, red);
        ca.uf = uw;
      }
    }
    coarse_visit<OP>(ca, kZero, nullptr, ca.f, nullptr, true, out, st, red);
    if (ca.gk) {
      for (int64_t i = threadIdx.x; i < ca.n; i += blockDim.x) {
        const double w = ca.uf[i];
        ca.gk[i] = -(((w * w) * w) * out[i]);
      }
    }
    __syncthreads();
    return;
  }
  for (int l = M - 1; l >= 0; --l) {
    if constexpr (RB) {
      // adjoint without u_fwd: A^{M-1} from the rebuilt u_fwd, per segment
      if (l == M - 1 && ph.begin(c, false)) coef_top<K, PREC>(c, ar, st, x);
    }
    const bool solo = c.nl(l) <= W;
    if (ph.begin(c, solo)) forcing_level<OP>(c, l, solo ? 0 : c.member, solo ? 1 : c.G);
  }
  const double* Fsrc = (OP == kOpPoisson) ? c.R : c.Q;   // rhs of inner levels
  // FMG start: level 0 from zero with the original rhs
  if (ph.begin(c, true)) coarse_visit<OP>(c, kZero, nullptr, c.R, c.A, false, c.V, st, red);
  for (int t = 1; t <= M; ++t) {
    const bool sr = (t == M);
    int top;
    if (sr) {
      if (ph.begin(c, false)) sr_down<K, OP, PREC, RB>(c, ar, st, x);
      top = M - 1;
    } else {
      top = t;
    }
    // down leg: two levels per visit from the top, a single one at the bottom
    for (int l = top; l >= 1;) {
      int sk;
      const double* src;
      if (l == top && !sr) { sk = kInterp; src = c.V + c.off(l - 1); }
      else if (l == top) { sk = kDirect; src = c.Uh; }
      else { sk = kRestrict; src = c.U + c.off(l + 1); }
      const double* F = (l == top && !sr) ? c.R + c.off(l) : Fsrc + c.off(l);
      if (l >= 2) {
        if (ph.begin(c, c.nl(l) <= W)) down_visit2<K, OP, PREC>(c, ar, l, sk, src, F, st, x);
        l -= 2;
      } else {
        if (ph.begin(c, c.nl(l) <= W)) down_visit<K, OP, PREC>(c, ar, l, sk, src, F, st, x);
        l -= 1;
      }
    }
    {
      int sk;
      const double* src;
      if (top >= 1) { sk = kRestrict; src = c.U + c.off(1); }
      else { sk = kDirect; src = c.Uh; }   // M == 1: level 0 is the top
      const double* F = (top == 0 && !sr) ? c.R : Fsrc;
      // the last step's V^{M-1} (level 0 when M == 1) to the kept array
      double* out = (sr && top == 0 && c.vk) ? c.vk : c.V;
      if (ph.begin(c, true)) coarse_visit<OP>(c, sk, src, F, c.A, false, out, st, red);
    }
    // up leg: two levels per visit from the bottom (only the upper one's V
    // is stored), a single one at the top
    for (int l = 1; l <= top;) {
      if (l + 1 <= top) {
        const int h = l + 1;
        const double* F = (h == top && !sr) ? c.R + c.off(h) : Fsrc + c.off(h);
        double* Vout = (sr && h == top) ? c.vk : nullptr;
        if (ph.begin(c, c.nl(h) <= W))
          up_visit2<K, OP, PREC>(c, ar, h, Fsrc + c.off(l), F, st, x, Vout);
        l += 2;
      } else {
        const double* F = (l == top && !sr) ? c.R + c.off(l) : Fsrc + c.off(l);
        double* Vout = (sr && l == top) ? c.vk : nullptr;
        if (ph.begin(c, c.nl(l) <= W)) up_visit<K, OP, PREC>(c, ar, l, F, st, x, Vout);
        l += 1;
      }
    }
    // compression only (a kept V^{M-1} and no fine output): no SR up pass
    if (sr && (c.uo || c.gk) && ph.begin(c, false)) sr_up<K, OP, PREC, RB>(c, ar, st, x);
  }
}

// RB: the adjoint that rebuilds u_fwd (OP = linear with c = 3 kappa u_fwd^2).
template <int K, int OP, int PREC, bool RB>
__global__ __launch_bounds__(kMaxThreads) void k_batched(Args a) {
  extern __shared__ double lds[];
  double* st = lds;                                  // a.region >= T (K + 1) doubles
  double* red = lds + a.region;                      // 32 doubles
  Xch x{red + 32, 0, 2 * (int)blockDim.x};  // 4 T doubles, then 2 kMaxPad (Ctx::eb)
  __shared__ int next;
  for (;;) {
    // slot -> (queue position, member): the G members of a problem are
    // consecutive slots, so all of them are taken by running workgroups
    if (threadIdx.x == 0) next = atomicAdd(a.queue, 1);
    __syncthreads();
    const int slot = next;
    __syncthreads();
    const int p = slot / a.group;
    if (p >= a.batch) break;
    const int qp = a.order[p];
    const Prob pr = a.probs[qp];
    Ctx c = make_ctx(pr, a);
    c.eb = red + 32 + 4 * (int)blockDim.x;
    c.member = slot % a.group;
    c.bar = a.bars + 2 * (int64_t)qp;
    solve_problem<K, OP, PREC, RB>(c, a, st, x, red);
  }
}

// Zero the queue counter and the per-problem barriers (a kernel rather than
// a memset, so that a captured graph replays it reliably).
__global__ void k_queue_reset(int32_t* q, int32_t* bars, int64_t nbars) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *q = 0;
  if (i < nbars) bars[i] = 0;
}

}  // namespace bt
}  // namespace fmgsr

// ===========================================================================
// Host side: plans, launch, autotuner, C ABI
// ===========================================================================
#include "fmgsr_host.hpp"

using fmgsr::bt::Prob;

struct fmgsr_batch_s {
  int device = 0;
  int32_t batch = 0;
  int op = 0, prec = 0, nu1 = 2, nu2 = 1, buffer = 0, halo = 0;
  int K = 8, T = 256, grid = 0, group = 1;
  int grid_rb = 0;                // persistent grid of the adjoint that rebuilds u_fwd
  int region = 0;                 // doubles of the LDS stage / coarse region
  size_t lds = 0;
  int n0max = 1;
  bool auto_segments = true;
  std::vector<int64_t> n, off, levels_v, segs;
  std::vector<double> g;
  std::vector<int32_t> order;
  Prob* d_probs = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_queue = nullptr;     // [0] queue, [1] status, [2..] barriers (2 per problem)
  double* d_ws = nullptr;
  int64_t ws_doubles = 0;
  double algo_bytes = 0.0;          // algorithmic bytes of one solve (profiling)
  double algo_bytes_adjoint = 0.0;  // ... of one adjoint solve
  double algo_bytes_keep = 0.0;     // ... of a forward solve that only keeps V^{M-1}
  double algo_bytes_adjoint_rebuild = 0.0;  // ... of an adjoint that rebuilds u_fwd
};

namespace fmgsr {
namespace bt {
namespace {

// Cells per thread: 4 (fewer registers, three resident workgroups per CU;
// best for many small problems) or 8 (wider windows, fewer tiles; best for
// few large problems split over groups).  The window of a segment patch is
// at most kMaxThreads * kMaxRun cells.
constexpr int kMaxRun = 8;
constexpr int kMaxGroup = 16;

int64_t pad_of(int buffer) { return (buffer + 2) & ~1; }

// Algorithmic bytes of one problem's FMG-FAS-SR iteration as the kernel
// schedules it: every array a visit reads counted once per visit, every
// array it writes once (8 bytes per cell).  `reaction`: coefficient arrays
// and coarse right-hand sides exist; `adjoint`: the fine coefficient is
// formed from kappa and u_fwd and grad_kappa is written too.
// `keep_only`: the SR up pass is skipped (a forward that only keeps
// V^{M-1}); `rebuild`: an adjoint that rebuilds u_fwd instead of reading it
// (seven forward SR up passes over rhs, kappa and V^{M-1}: one per segment
// for A^{M-1}, three per segment in each SR pass).
double model_bytes(int64_t n, int64_t n0, int M, bool reaction, bool adjoint,
                   bool keep_only = false, bool rebuild = false) {
  const double r = reaction ? 1.0 : 0.0;
  const double fine_coef = reaction ? ((adjoint && !rebuild) ? 2.0 : 1.0) : 0.0;  // kappa (+ u_fwd)
  auto nl = [&](int l) { return (double)(n0 << l); };
  double b = 0.0;
  if (M == 0)
    return 8.0 * (double)n * (2.0 + fine_coef + (adjoint ? 1.0 : 0.0) + (rebuild ? 3.0 : 0.0));
  // forcing: level l from level l+1
  for (int l = M - 1; l >= 0; --l) {
    const double nf = nl(l + 1);
    b += 8.0 * nf * (1.0 + (l + 1 == M ? fine_coef : r)) + 8.0 * nl(l) * (1.0 + r);
  }
  auto down = [&](int l, int src) {  // src: 0 interp, 1 restrict, 2 direct
    const double m = nl(l);
    const double sb = src == 0 ? 0.5 * m : (src == 1 ? 2.0 * m : m);
    return 8.0 * (sb + m * (1.0 + r) + m + 0.5 * m * r);
  };
  auto up = [&](int l) { const double m = nl(l); return 8.0 * (m + 0.5 * m + m * (1.0 + r) + m); };
  // two-level visits: the lower level of a down pair reads nothing and
  // writes U (and Q); an up pair reads both levels' U, F, A and the coarse
  // V below, and writes the upper level's V only
  auto down2 = [&](int l, int src) { const double m = nl(l - 1); return down(l, src) + 8.0 * (m + 0.5 * m * r); };
  auto up2 = [&](int h) {
    const double a = nl(h - 1), m = nl(h);
    return 8.0 * (0.5 * a + a + a * (1.0 + r) + m + m * (1.0 + r) + m);
  };
  auto legs = [&](int top, int src_top) {
    double s = 0.0;
    for (int l = top; l >= 1;) {
      const int src = (l == top) ? src_top : 1;
      if (l >= 2) { s += down2(l, src); l -= 2; }
      else { s += down(l, src); l -= 1; }
    }
    for (int l = 1; l <= top;) {
      if (l + 1 <= top) { s += up2(l + 1); l += 2; }
      else { s += up(l); l += 1; }
    }
    return s;
  };
  for (int t = 1; t < M; ++t) b += legs(t, 0);
  const double N = (double)n;
  b += 8.0 * (0.5 * N + N * (1.0 + fine_coef) + 0.5 * N + 0.5 * N * r);  // SR down
  b += legs(M - 1, 2);
  if (!keep_only) b += 8.0 * (0.5 * N + N * (1.0 + fine_coef) + N + (adjoint ? N : 0.0));  // SR up
  if (rebuild) b += 7.0 * 8.0 * (0.5 * N + 2.0 * N);
  return b;
}

// Largest segment core n0 2^k (even, dividing n) whose extended patch fits a
// window of W cells; `halve` > 0 halves it that many times (autotuner).
int64_t auto_core(int64_t n, int M, int64_t n0, int buffer, int64_t W, int halve) {
  int64_t best = 0;
  for (int k = 0; k <= M; ++k) {
    const int64_t s = n0 << k;
    if (s % 2 != 0) continue;
    if (s + 2 * pad_of(buffer) > W) break;
    best = s;
  }
  for (int i = 0; i < halve && best > 2 && (best / 2) % 2 == 0 && n % (best / 2) == 0; ++i)
    best /= 2;
  return best;
}

// op: kOp*, or kOpRebuild for the adjoint that rebuilds u_fwd.
constexpr int kOpRebuild = 3;
template <int K>
const void* kernel_ptr_k(int op, int prec) {
  if (prec == kF64) {
    if (op == kOpRebuild) return (const void*)k_batched<K, kOpLinear, kF64, true>;
    if (op == kOpCubic) return (const void*)k_batched<K, kOpCubic, kF64, false>;
    if (op == kOpLinear) return (const void*)k_batched<K, kOpLinear, kF64, false>;
    return (const void*)k_batched<K, kOpPoisson, kF64, false>;
  }
  if (op == kOpRebuild) return (const void*)k_batched<K, kOpLinear, kF32, true>;
  if (op == kOpCubic) return (const void*)k_batched<K, kOpCubic, kF32, false>;
  if (op == kOpLinear) return (const void*)k_batched<K, kOpLinear, kF32, false>;
  return (const void*)k_batched<K, kOpPoisson, kF32, false>;
}

const void* kernel_ptr(int op, int prec, int K) {
  return K == 4 ? kernel_ptr_k<4>(op, prec) : kernel_ptr_k<8>(op, prec);
}

hipError_t launch(const Args& a, int op, int prec, int K, int grid, int T, size_t lds,
                  hipStream_t s) {
  void* args[] = {const_cast<Args*>(&a)};
  if (hipLaunchKernel(kernel_ptr(op, prec, K), dim3(grid), dim3(T), args, lds, s) != hipSuccess)
    return hipGetLastError();
  return hipGetLastError();
}

void free_plan_device(fmgsr_batch_s* b) {
  if (b->d_probs) (void)hipFree(b->d_probs);
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_ws) (void)hipFree(b->d_ws);
  b->d_probs = nullptr; b->d_order = nullptr; b->d_queue = nullptr; b->d_ws = nullptr;
  (void)hipGetLastError();
}

// (Re)build the descriptors for the plan's shape and segment choice and
// upload them; allocates on first use.
fmgsr_status build_plan(fmgsr_batch_s* b, int T, int K, int halve, int group_cap = kMaxGroup) {
  const int64_t W = (int64_t)T * K;
  const int64_t pad = pad_of(b->buffer);
  std::vector<Prob> pr(b->batch);
  int64_t ws = 0;
  double bytes = 0.0;
  for (int j = 0; j < b->batch; ++j) {
    Prob& p = pr[j];
    p.n = b->n[j];
    p.off = b->off[j];
    p.M = (int32_t)(b->levels_v[j] - 1);
    p.n0 = (int32_t)(p.n >> p.M);
    p.gL = b->g[2 * j];
    p.gR = b->g[2 * j + 1];
    if (p.M >= 1) {
      int64_t s;
      if (b->auto_segments) s = auto_core(p.n, p.M, p.n0, b->buffer, W, halve);
      else s = p.n / b->segs[j];
      if (s < 2 || s % 2 != 0 || p.n % s != 0 || s + 2 * pad > W) return FMGSR_EINVAL;
      p.seg = s;
    } else {
      p.seg = 0;
    }
    p.coff = p.off / 2;
    p.ws = ws;
    // one level: room for the result and a rebuilt forward solution
    ws += std::max<int64_t>(slab_doubles(p.n0, p.M), 2 * lvl_size(p.n0, 0));
    bytes += model_bytes(p.n, p.n0, p.M, b->op != kOpPoisson, false);
  }
  if (b->auto_segments)
    for (int j = 0; j < b->batch; ++j) b->segs[j] = pr[j].M >= 1 ? pr[j].n / pr[j].seg : 1;

  // launch shape
  b->T = T;
  b->K = K;
  b->region = std::max(T * (K + 1), 11 * b->n0max);
  b->lds = sizeof(double) * ((size_t)b->region + 32 + 4 * (size_t)T + 2 * kMaxPad);
  if (b->lds > 160 * 1024) return FMGSR_EINVAL;
  size_t lds_limit = 0;  // the device's opt-in limit per workgroup
  if (fmgsr::device_lds_limit(&lds_limit) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  if (b->lds > lds_limit) return FMGSR_EINVAL;
  const void* kp = kernel_ptr(b->op, b->prec, K);
  if (hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kp, T, b->lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  per_cu = std::max(per_cu, 1);
  // fewer problems than resident workgroups: split each problem over a group
  const int64_t cap = (int64_t)per_cu * cus;
  b->group = (b->batch < cap) ? (int)std::min<int64_t>(group_cap, cap / b->batch) : 1;
  b->grid = (int)std::min<int64_t>((int64_t)b->batch * b->group, cap);
  // the adjoint that rebuilds u_fwd runs its own kernel: its persistent grid
  // is what of this one stays resident (at least a group, for the barriers)
  b->grid_rb = b->grid;
  if (b->op == kOpCubic) {
    const void* kr = kernel_ptr(kOpRebuild, b->prec, K);
    int per_cu_rb = 0;
    if (hipFuncSetAttribute(kr, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_rb, kr, T, b->lds) != hipSuccess) {
      (void)hipGetLastError();
      return FMGSR_EDEVICE;
    }
    const int64_t cap_rb = (int64_t)std::max(per_cu_rb, 1) * cus;
    b->grid_rb = (int)std::max<int64_t>(std::min<int64_t>(b->grid, cap_rb), b->group);
  }
  b->algo_bytes = bytes;
  double adj = 0.0, adj_rb = 0.0, keep = 0.0;
  for (const Prob& p : pr) {
    adj += model_bytes(p.n, p.n0, p.M, true, true);
    adj_rb += model_bytes(p.n, p.n0, p.M, true, true, false, true);
    keep += model_bytes(p.n, p.n0, p.M, b->op != kOpPoisson, false, true);
  }
  b->algo_bytes_adjoint = adj;
  b->algo_bytes_adjoint_rebuild = adj_rb;
  b->algo_bytes_keep = keep;

  if (!b->d_probs) {
    if (hipMalloc((void**)&b->d_probs, sizeof(Prob) * b->batch) != hipSuccess ||
        hipMalloc((void**)&b->d_order, sizeof(int32_t) * b->batch) != hipSuccess ||
        hipMalloc((void**)&b->d_queue, sizeof(int32_t) * (2 + 2 * (size_t)b->batch)) != hipSuccess) {
      free_plan_device(b);
      return FMGSR_ENOMEM;
    }
    if (hipMemset(b->d_queue, 0, sizeof(int32_t) * (2 + 2 * (size_t)b->batch)) != hipSuccess) {
      (void)hipGetLastError();
      return FMGSR_EDEVICE;
    }
  }
  if (ws > b->ws_doubles) {
    if (b->d_ws) (void)hipFree(b->d_ws);
    b->d_ws = nullptr;
    if (hipMalloc((void**)&b->d_ws, sizeof(double) * (size_t)std::max<int64_t>(ws, 1)) != hipSuccess) {
      (void)hipGetLastError();
      b->ws_doubles = 0;
      return FMGSR_ENOMEM;
    }
    b->ws_doubles = ws;
  }
  if (hipMemcpy(b->d_probs, pr.data(), sizeof(Prob) * b->batch, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_order, b->order.data(), sizeof(int32_t) * b->batch, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  return FMGSR_OK;
}

// An adjoint that rebuilds u_fwd takes each window's pad cells from the
// neighbouring segments' cores: every segment core must be at least the pad.
bool rebuild_fits(const fmgsr_batch_s* b) {
  const int64_t pad = pad_of(b->buffer);
  for (int j = 0; j < b->batch; ++j)
    if (b->levels_v[j] > 1 && b->n[j] / b->segs[j] < pad) return false;
  return true;
}

// Extra inputs and outputs of an execution: the kept level-(M-1) solutions
// (forward: written; adjoint without u_fwd: the forward rhs and them, read).
struct Keep {
  double* vkeep = nullptr;
  const double* ffwd = nullptr;
  const double* vfwd = nullptr;
};

fmgsr_status execute(fmgsr_batch_s* b, int op, bool adjoint, const double* f, const double* kappa,
                     const double* ufwd, double* u, double* gk, hipStream_t s,
                     const Keep& kp = Keep()) {
  Args a;
  a.vkeep = kp.vkeep;
  a.ffwd = kp.ffwd;
  a.vfwd = kp.vfwd;
  a.probs = b->d_probs;
  a.order = b->d_order;
  a.batch = b->batch;
  a.queue = b->d_queue;
  a.f = f;
  a.kappa = kappa;
  a.ufwd = ufwd;
  a.u = u;
  a.gk = gk;
  a.ws = b->d_ws;
  a.nu1 = b->nu1;
  a.nu2 = b->nu2;
  a.buffer = b->buffer;
  a.halo = b->halo;
  a.halo2 = 4 * b->halo;
  a.region = b->region;
  a.adjoint = adjoint ? 1 : 0;
  a.group = b->group;
  a.status = b->d_queue + 1;
  a.bars = b->d_queue + 2;
  if (op != b->op) {
    const void* kf = kernel_ptr(op, b->prec, b->K);
    if (hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds) != hipSuccess) {
      (void)hipGetLastError();
      return FMGSR_EDEVICE;
    }
  }
  const double bytes = !adjoint ? (u ? b->algo_bytes : b->algo_bytes_keep)
                                 : (kp.vfwd ? b->algo_bytes_adjoint_rebuild : b->algo_bytes_adjoint);
  ProfScope ps(adjoint ? "k_batched_adjoint" : "k_batched", bytes, s);
  const int64_t nbars = 2 * (int64_t)b->batch;
  hipLaunchKernelGGL(k_queue_reset, dim3((unsigned)((nbars + 255) / 256)), dim3(256), 0, s,
                     b->d_queue, b->d_queue + 2, nbars);
  if (hipGetLastError() != hipSuccess) return FMGSR_EDEVICE;
  const int grid = (op == kOpRebuild) ? b->grid_rb : b->grid;
  if (launch(a, op, b->prec, b->K, grid, b->T, b->lds, s) != hipSuccess) return FMGSR_EDEVICE;
  return FMGSR_OK;
}

}  // namespace
}  // namespace bt
}  // namespace fmgsr

using namespace fmgsr;

extern "C" {

fmgsr_status fmgsr_batch_create(int32_t batch, const int64_t* n_host, const int64_t* offset_host,
                                const int32_t* levels_host, const int64_t* segments_host,
                                int32_t buffer, const double* g_host, int32_t op_kind,
                                const fmgsr_options* opt, fmgsr_batch* out) {
  if (!out) return FMGSR_EINVAL;
  *out = nullptr;
  if (batch < 1 || batch > (1 << 24) || !n_host || !levels_host) return FMGSR_EINVAL;
  if (buffer < 0 || buffer > 64) return FMGSR_EINVAL;
  if (op_kind < FMGSR_OP_POISSON || op_kind > FMGSR_OP_LINEAR_REACTION) return FMGSR_EINVAL;
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  if (o.nu1 < 0 || o.nu1 > 16 || o.nu2 < 0 || o.nu2 > 16) return FMGSR_EINVAL;
  if (o.precision != FMGSR_FP64 && o.precision != FMGSR_FP32_RELAX) return FMGSR_EINVAL;
  if (o.reserved != 0) return FMGSR_EINVAL;
  if (o.check_finite != 0 && o.check_finite != 1) return FMGSR_EINVAL;
  if (o.rhs_restriction != FMGSR_R_FULLWEIGHT && o.rhs_restriction != FMGSR_R_AVERAGE)
    return FMGSR_EINVAL;
  if (o.tau_mode != FMGSR_TAU_SPLIT || o.functionals || o.coarse_out || o.check_finite ||
      o.rhs_restriction != FMGSR_R_FULLWEIGHT)
    return FMGSR_ENOTSUP;
  auto* b = new (std::nothrow) fmgsr_batch_s;
  if (!b) return FMGSR_ENOMEM;
  b->batch = batch;
  b->op = op_kind;
  b->prec = o.precision;
  b->nu1 = o.nu1;
  b->nu2 = o.nu2;
  b->buffer = buffer;
  b->halo = ((2 * std::max(o.nu1, o.nu2) + 4) + 1) & ~1;
  b->auto_segments = (segments_host == nullptr);
  b->n.resize(batch); b->off.resize(batch); b->levels_v.resize(batch); b->segs.assign(batch, 1);
  b->g.assign(2 * (size_t)batch, 0.0);
  int64_t run = 0;
  for (int j = 0; j < batch; ++j) {
    const int64_t n = n_host[j];
    const int32_t L = levels_host[j];
    if (n < 1 || L < 1 || L > 31) { delete b; return FMGSR_EINVAL; }
    const int M = L - 1;
    if (n % ((int64_t)1 << M) != 0 || (n >> M) > bt::kMaxBatchN0) { delete b; return FMGSR_EINVAL; }
    if (M >= 1 && o.sr_levels != 1) { delete b; return FMGSR_ENOTSUP; }
    b->n[j] = n;
    b->levels_v[j] = L;
    b->off[j] = offset_host ? offset_host[j] : run;
    if (b->off[j] < 0) { delete b; return FMGSR_EINVAL; }
    run += n;
    b->n0max = std::max<int>(b->n0max, (int)(n >> M));
    if (segments_host && M >= 1) {
      const int64_t sg = segments_host[j];
      if (sg < 1 || n % sg != 0) { delete b; return FMGSR_EINVAL; }
      const int64_t s = n / sg;
      if (s % 2 != 0 || s + 2 * bt::pad_of(buffer) > (int64_t)bt::kMaxThreads * bt::kMaxRun) {
        delete b;
        return FMGSR_EINVAL;
      }
      b->segs[j] = sg;
    }
    if (g_host) { b->g[2 * j] = g_host[2 * j]; b->g[2 * j + 1] = g_host[2 * j + 1]; }
  }
  // longest first
  b->order.resize(batch);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int32_t x, int32_t y) { return b->n[x] > b->n[y]; });
  if (hipGetDevice(&b->device) != hipSuccess) { (void)hipGetLastError(); delete b; return FMGSR_EDEVICE; }
  // default shape: small batches (fewer problems than CUs) get the wide
  // window (512 threads x 8 cells) and groups of workgroups; large batches
  // one 256 x 4 workgroup per problem, three per CU (the autotuner refines
  // both)
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return FMGSR_EDEVICE;
  }
  fmgsr_status st = batch < cus ? bt::build_plan(b, 512, 8, 0, 4) : bt::build_plan(b, 256, 4, 0, 4);
  if (st == FMGSR_EINVAL) st = bt::build_plan(b, 256, 8, 0, 4);
  if (st == FMGSR_EINVAL) st = bt::build_plan(b, 512, 8, 0, 4);
  if (st != FMGSR_OK) { bt::free_plan_device(b); delete b; return st; }
  *out = b;
  return FMGSR_OK;
}

fmgsr_status fmgsr_batch_solve(fmgsr_batch b, const double* f_packed, const double* kappa_packed,
                               double* u_packed, void* hip_stream) {
  if (!b || !is_device_ptr(f_packed) || !is_device_ptr(u_packed)) return FMGSR_EINVAL;
  if (b->op == FMGSR_OP_POISSON ? kappa_packed != nullptr : !is_device_ptr(kappa_packed))
    return FMGSR_EINVAL;
  if ((const void*)f_packed == (const void*)u_packed) return FMGSR_EINVAL;
  return bt::execute(b, b->op, false, f_packed, kappa_packed, nullptr, u_packed, nullptr,
                     (hipStream_t)hip_stream);
}

fmgsr_status fmgsr_batch_adjoint(fmgsr_batch b, const double* kappa_packed,
                                 const double* u_fwd_packed, const double* dJdu_packed,
                                 double* grad_f_packed, double* grad_kappa_packed,
                                 void* hip_stream) {
  if (!b) return FMGSR_EINVAL;
  if (b->op != FMGSR_OP_CUBIC_REACTION) return FMGSR_ENOTSUP;
  if (!is_device_ptr(kappa_packed) || !is_device_ptr(u_fwd_packed) || !is_device_ptr(dJdu_packed))
    return FMGSR_EINVAL;
  if (!grad_f_packed && !grad_kappa_packed) return FMGSR_EINVAL;
  if ((grad_f_packed && !is_device_ptr(grad_f_packed)) ||
      (grad_kappa_packed && !is_device_ptr(grad_kappa_packed)))
    return FMGSR_EINVAL;
  return bt::execute(b, bt::kOpLinear, true, dJdu_packed, kappa_packed, u_fwd_packed,
                     grad_f_packed, grad_kappa_packed, (hipStream_t)hip_stream);
}

fmgsr_status fmgsr_batch_solve_keep(fmgsr_batch b, const double* f_packed,
                                    const double* kappa_packed, double* u_packed,
                                    double* coarse_packed, void* hip_stream) {
  if (!b || !is_device_ptr(f_packed) || !is_device_ptr(coarse_packed)) return FMGSR_EINVAL;
  if (u_packed && !is_device_ptr(u_packed)) return FMGSR_EINVAL;
  if (b->op == FMGSR_OP_POISSON ? kappa_packed != nullptr : !is_device_ptr(kappa_packed))
    return FMGSR_EINVAL;
  if ((const void*)f_packed == (const void*)u_packed ||
      (const void*)f_packed == (const void*)coarse_packed ||
      (const void*)u_packed == (const void*)coarse_packed)
    return FMGSR_EINVAL;
  bt::Keep kp;
  kp.vkeep = coarse_packed;
  return bt::execute(b, b->op, false, f_packed, kappa_packed, nullptr, u_packed, nullptr,
                     (hipStream_t)hip_stream, kp);
}

fmgsr_status fmgsr_batch_adjoint_compressed(fmgsr_batch b, const double* kappa_packed,
                                            const double* f_fwd_packed,
                                            const double* coarse_fwd_packed,
                                            const double* dJdu_packed, double* grad_f_packed,
                                            double* grad_kappa_packed, void* hip_stream) {
  if (!b) return FMGSR_EINVAL;
  if (b->op != FMGSR_OP_CUBIC_REACTION) return FMGSR_ENOTSUP;
  if (!is_device_ptr(kappa_packed) || !is_device_ptr(f_fwd_packed) ||
      !is_device_ptr(coarse_fwd_packed) || !is_device_ptr(dJdu_packed))
    return FMGSR_EINVAL;
  if (!grad_f_packed && !grad_kappa_packed) return FMGSR_EINVAL;
  if ((grad_f_packed && !is_device_ptr(grad_f_packed)) ||
      (grad_kappa_packed && !is_device_ptr(grad_kappa_packed)))
    return FMGSR_EINVAL;
  if (!bt::rebuild_fits(b)) return FMGSR_ENOTSUP;
  bt::Keep kp;
  kp.ffwd = f_fwd_packed;
  kp.vfwd = coarse_fwd_packed;
  return bt::execute(b, bt::kOpRebuild, true, dJdu_packed, kappa_packed, nullptr, grad_f_packed,
                     grad_kappa_packed, (hipStream_t)hip_stream, kp);
}

fmgsr_status fmgsr_batch_autotune(fmgsr_batch b, const double* f_packed, const double* kappa_packed,
                                  double* u_scratch_packed, void* hip_stream, double* ms_out) {
  if (!b) return FMGSR_EINVAL;
  hipStream_t s = (hipStream_t)hip_stream;
  const int shapes[2] = {256, 512};
  const int runs[2] = {4, 8};
  const int halves = b->auto_segments ? 2 : 1;
  const int gcaps[5] = {1, 2, 4, 8, 16};
  const char* env = std::getenv("FMGSR_AUTOTUNE_LOG");
  const bool log = env && env[0] && env[0] != '0';
  double best = 1e300;
  int bestT = b->T, bestK = b->K, bestH = 0, bestG = bt::kMaxGroup;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  fmgsr_status st = FMGSR_OK;
  for (int T : shapes) {
   for (int K : runs) {
    for (int h = 0; h < halves && st == FMGSR_OK; ++h) {
     int last_group = -1;
     for (int gc : gcaps) {
      if (st != FMGSR_OK) break;
      fmgsr_status bs = bt::build_plan(b, T, K, h, gc);
      if (bs == FMGSR_OK && b->group == last_group) continue;  // same group size as before
      last_group = b->group;
      if (bs == FMGSR_EINVAL) continue;  // shape does not fit these problems
      if (bs != FMGSR_OK) { st = bs; break; }
      st = fmgsr_batch_solve(b, f_packed, kappa_packed, u_scratch_packed, hip_stream);  // warm
      if (st != FMGSR_OK) break;
      const int reps = 3;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && st == FMGSR_OK; ++r)
        st = fmgsr_batch_solve(b, f_packed, kappa_packed, u_scratch_packed, hip_stream);
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        (void)hipGetLastError();
        st = FMGSR_EDEVICE;
        break;
      }
      if (log)
        std::fprintf(stderr, "fmgsr autotune: threads %d run %d segment-halving %d group %d: %.3f ms\n",
                     T, K, h, b->group, ms / reps);
      if (ms / reps < best) { best = ms / reps; bestT = T; bestK = K; bestH = h; bestG = gc; }
     }
    }
   }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FMGSR_OK) return st;
  st = bt::build_plan(b, bestT, bestK, bestH, bestG);
  if (st == FMGSR_OK && ms_out) *ms_out = best;
  return st;
}

fmgsr_status fmgsr_batch_query(fmgsr_batch b, fmgsr_batch_shape* shape, int64_t* segments_out) {
  if (!b) return FMGSR_EINVAL;
  if (shape) {
    shape->threads = b->T;
    shape->run = b->K;
    shape->grid = b->grid;
    shape->halo = b->halo;
    shape->lds_bytes = (int64_t)b->lds;
    shape->workspace_bytes = b->ws_doubles * (int64_t)sizeof(double);
    shape->group = b->group;
    int32_t stalled = 0;
    if (hipMemcpy(&stalled, b->d_queue + 1, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      return FMGSR_EDEVICE;
    }
    shape->stalled = stalled;
  }
  if (segments_out)
    for (int j = 0; j < b->batch; ++j) segments_out[j] = b->segs[j];
  return FMGSR_OK;
}

fmgsr_status fmgsr_batch_destroy(fmgsr_batch b) {
  if (!b) return FMGSR_EINVAL;
  (void)hipDeviceSynchronize();
  bt::free_plan_device(b);
  delete b;
  return FMGSR_OK;
}

fmgsr_status fmgsr_solve_batched(int32_t batch, const int64_t* n_host, const int64_t* offset_host,
                                 const int32_t* levels_host, const int64_t* segments_host,
                                 int32_t buffer, const fmgsr_operator* op, const double* f_packed,
                                 const double* g_host, const fmgsr_options* opt, double* u_packed,
                                 void* hip_stream) {
  const int32_t kind = op ? op->kind : FMGSR_OP_POISSON;
  fmgsr_batch b = nullptr;
  fmgsr_status st = fmgsr_batch_create(batch, n_host, offset_host, levels_host, segments_host,
                                       buffer, g_host, kind, opt, &b);
  if (st != FMGSR_OK) return st;
  st = fmgsr_batch_solve(b, f_packed, op ? op->kappa : nullptr, u_packed, hip_stream);
  if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) {
    (void)hipGetLastError();
    if (st == FMGSR_OK) st = FMGSR_EDEVICE;
  }
  fmgsr_batch_destroy(b);
  return st;
}

fmgsr_status fmgsr_adjoint(const fmgsr_operator* op, const double* f, double g_left,
                           double g_right, int64_t n, int32_t levels, int64_t n_segments,
                           int32_t buffer, const fmgsr_options* opt, const double* u_fwd,
                           const double* dJ_du, double* grad_f, double* grad_kappa,
                           void* hip_stream) {
  if (!op || op->kind != FMGSR_OP_CUBIC_REACTION) return FMGSR_ENOTSUP;
  const int64_t nn = n;
  const double g[2] = {g_left, g_right};
  fmgsr_batch b = nullptr;
  fmgsr_status st = fmgsr_batch_create(1, &nn, nullptr, &levels, n_segments > 0 ? &n_segments : nullptr,
                                       buffer, g, FMGSR_OP_CUBIC_REACTION, opt, &b);
  if (st != FMGSR_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  double* tmp = nullptr;
  if (!u_fwd && levels > 1 && bt::rebuild_fits(b)) {
    // compressed: keep the forward's level-(M-1) solution only (n/2
    // doubles) and rebuild u_fwd inside the adjoint
    if (hipMalloc((void**)&tmp, sizeof(double) * (size_t)(n / 2)) != hipSuccess) {
      (void)hipGetLastError();
      fmgsr_batch_destroy(b);
      return FMGSR_ENOMEM;
    }
    st = fmgsr_batch_solve_keep(b, f, op->kappa, nullptr, tmp, hip_stream);
    if (st == FMGSR_OK)
      st = fmgsr_batch_adjoint_compressed(b, op->kappa, f, tmp, dJ_du, grad_f, grad_kappa,
                                          hip_stream);
  } else {
    if (!u_fwd) {
      if (hipMalloc((void**)&tmp, sizeof(double) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        fmgsr_batch_destroy(b);
        return FMGSR_ENOMEM;
      }
      st = fmgsr_batch_solve(b, f, op->kappa, tmp, hip_stream);
      u_fwd = tmp;
    }
    if (st == FMGSR_OK)
      st = fmgsr_batch_adjoint(b, op->kappa, u_fwd, dJ_du, grad_f, grad_kappa, hip_stream);
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    if (st == FMGSR_OK) st = FMGSR_EDEVICE;
  }
  if (tmp) (void)hipFree(tmp);
  fmgsr_batch_destroy(b);
  return st;
}

}  // extern "C"
