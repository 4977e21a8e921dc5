// fmgsr.hip -- C ABI (include/fmgsr.h) and launch schedule of the gfx950
// FMG-FAS-SR solver.
//
// Schedule of one FMG cycle (Fig. 3) on levels 0..M (M = levels - 1):
//   forcing hierarchy   F^l = I F^{l+1}, l = M-1..0 (F^M = f), up to four
//                       levels per launch
//   coarse core         levels 0..C (C = largest level <= M - max(1, nSR)
//                       with at most kCoreMaxCells cells) in one workgroup:
//                       the FMG cycles up to level C, then one V-cycle bottom
//                       per later step
//   step t = C+1..M     vertical down kernels over levels t..C+1 (up to four
//                       levels each), coarse core, vertical up kernels over
//                       levels C+1..t
// A stored level keeps two arrays: U (pre-smoothed iterate, written by the
// down leg, read by the up leg) and V (post-smoothed iterate; the FMG
// result of step t that step t+1 interpolates from).  Separate arrays keep
// every launch free of read/write overlap between workgroups.  The finest
// SR level (t = M, sr_levels >= 1) is never stored: its down pass writes only
// I^ of the smoothed cores (Uh) and its up pass streams the cores to u_out.
// With split tau and one SR level both SR passes are the top levels of the
// first down and the last up kernel.  The top up kernel of a step rebuilds
// the pre-smoothed iterates the down kernel made on its levels above the
// bottom one (Pi of V^{t-1} and the same sweeps in the same window), so
// those are not stored ("deep pairs").  The vertical kernels run
// one-wavefront tiles whose exchanges are lane shifts.  Launches of many
// tiles run their interior tiles at three wavefronts per SIMD (k_down's
// register-capped variant; k_up_wide, with the edge tiles in a second launch
// of k_up).
// With sr_levels = k >= 2 the levels M-k+1 .. M-1 are SR levels too (the
// semantics of Sec. 4's runs with two and three SR levels): wherever they
// are visited, their pre-smoothing is the block smoother (segment kernels
// with the same segment count, so cores halve per level) started from I^ of
// the SR level above, and their post-smoothing is the full update Pi + CR;
// their V arrays are stored for the next FMG step.
// With literal tau every stored level is its own launch, preceded by the
// tau kernel that forms its right-hand side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fmgsr.h"
#include "fmgsr_host.hpp"
#include "fmgsr_kernels.hpp"

namespace fmgsr {

// ---------------------------------------------------------------------------
// Optional per-launch timing (fmgsr_profile_*), shared by every entry point
// ---------------------------------------------------------------------------
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_filter;
std::vector<ProfRecord> g_prof;

ProfScope::ProfScope(const char* name, double bytes, hipStream_t s) : st(s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  if (!g_prof_filter.empty() && std::string(name).find(g_prof_filter) == std::string::npos) return;
  if (hipEventCreate(&rec.start) != hipSuccess) return;
  if (hipEventCreate(&rec.stop) != hipSuccess) { (void)hipEventDestroy(rec.start); return; }
  rec.name = name;
  rec.bytes = bytes;
  on = (hipEventRecord(rec.start, st) == hipSuccess);
}

ProfScope::~ProfScope() {
  if (!on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (hipEventRecord(rec.stop, st) == hipSuccess) g_prof.push_back(rec);
}

bool is_device_ptr(const void* ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

hipError_t device_lds_limit(size_t* bytes) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static size_t cache[kMaxDev] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  if (dev >= 0 && dev < kMaxDev && cache[dev]) {
    *bytes = cache[dev];
    return hipSuccess;
  }
  int v = 0;
  e = hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev);
  if (e != hipSuccess) return e;
  *bytes = (size_t)(v > 0 ? v : 0);
  if (dev >= 0 && dev < kMaxDev) cache[dev] = *bytes;
  return hipSuccess;
}

}  // namespace fmgsr

namespace fmgsr {
namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kLevelAlign = 32;  // doubles: every level array starts 256-byte aligned

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Offset (doubles) of level l in a hierarchy array holding levels 0..l-1.
int64_t lvl_off_ws(int64_t n0, int l) {
  int64_t off = 0;
  for (int m = 0; m < l; ++m) off += ((n0 << m) + kLevelAlign - 1) / kLevelAlign * kLevelAlign;
  return off;
}

// Stale cells (counted from a window edge) on each level of a vertical
// kernel walking `d` levels with nu sweeps per level.  The window edge cell
// is never updated, so every half-sweep spreads staleness by one cell; I^
// halves it, full weighting of the rhs and the neighbour exchange at the
// window edge add one coarse cell, P reaches one coarse cell further.
bool down_fits(int nu, int d, int64_t halo) {
  int64_t inv = 0, rinv = 0;
  for (int i = 0; i < d; ++i) {
    if (i > 0) {
      rinv = (rinv + 2) / 2;
      inv = std::max((inv + 1) / 2, rinv);
    }
    inv += 2 * nu;
    if ((halo >> i) < inv) return false;  // core of level i starts halo >> i cells in
  }
  return true;
}

bool up_fits(int nu, int d, int64_t halo) {
  // bottom level: the exchanged coarse error of the edge pair is unknown
  int64_t inv = 2 + 2 * nu;
  for (int i = d - 2; i >= 0; --i) inv = 2 * (inv + 1) + 2 * nu;
  return halo >= inv;  // only the top level's core is written
}

// Up kernel whose top level is an SR level (full update Pi from the level
// below, then nu x [Kaczmarz, sweep]): Pi reaches two coarse cells, and each
// relaxation iteration spreads staleness by three (the pair and the sweep).
bool sr_up_fits(int nu, int d, int64_t halo) {
  int64_t inv = 2 + 2 * nu;
  for (int i = d - 2; i >= 1; --i) inv = 2 * (inv + 1) + 2 * nu;
  inv = 2 * (inv + 2) + 3 * nu;
  return halo >= inv;
}

// Vertical kernels run one-wavefront tiles (64 threads x kRun cells, less
// the halo): their neighbour exchanges are lane shifts, with no LDS round
// trip and no workgroup barrier, and each wavefront walks its tile at its
// own pace.
constexpr int kVertThreads = 64;
// Top levels of at least this many cells (768 tiles of the 256-thread shape)
// take the three-wavefronts-per-SIMD down kernel, and deep up launches run
// their interior tiles on k_up_wide (one more launch for the edge tiles);
// smaller launches are bound by one tile's latency, which the down kernel's
// spills would lengthen.
constexpr int64_t kWideCells = 768 * ((int64_t)kRun * 256 - 2 * kTileHalo);

// Up kernel that rebuilds its top level's pre-smoothed iterate (Pi of the
// level below's FMG iterate, then the down leg's nu1 sweeps) instead of
// reading it: the rebuild is stale in 2 nu1 cells plus Pi's two-cell reach,
// which enter the correction through I^ (pairs) and P (one coarse cell more).
bool rebuild_up_fits(int nu1, int nu2, int d, int64_t halo) {
  if (d < 2) return false;
  int64_t inv = 2 + 2 * nu2;
  for (int i = d - 2; i >= 1; --i) inv = 2 * (inv + 1) + 2 * nu2;
  const int64_t pre = (2 * (int64_t)nu1 + 2 + 1) / 2;
  inv = 2 * (std::max(inv, pre) + 1) + 2 * nu2;
  return halo >= inv;
}

// Deep pair: the up kernel also rebuilds the pre-smoothed iterates of levels
// 1..d-2 (the bottom one still comes from HBM).  The rebuilt level i is stale
// in the down leg's cells s_i from the window edge (down_fits), which enter
// the correction through I^ and P like the rebuilt top level's.  sr: the top
// level is the SR level (full update; its own iterate is not needed).
bool deep_fits(int nu1, int nu2, int d, int64_t halo, bool sr) {
  if (d < 3 || !down_fits(nu1, d, halo)) return false;
  int64_t s[kMaxFuse];
  int64_t dinv = 0, rinv = 0;
  for (int i = 0; i < d; ++i) {
    if (i > 0) {
      rinv = (rinv + 2) / 2;
      dinv = std::max((dinv + 1) / 2, rinv);
    }
    dinv += 2 * nu1;
    s[i] = dinv;
  }
  s[0] += 2;  // Pi's reach
  int64_t inv = 2 + 2 * nu2;
  for (int i = d - 2; i >= 1; --i) inv = 2 * (std::max(inv, (s[i] + 1) / 2) + 1) + 2 * nu2;
  inv = sr ? 2 * (inv + 2) + 3 * nu2 : 2 * (std::max(inv, (s[0] + 1) / 2) + 1) + 2 * nu2;
  return halo >= inv;
}

int fuse_depth(bool up, int nu) {
  for (int d = kMaxFuse; d > 1; --d)
    if (up ? up_fits(nu, d, kTileHalo) : down_fits(nu, d, kTileHalo)) return d;
  return 1;
}

struct Plan {
  int64_t n = 0, n0 = 0;
  int M = 0, C = 0;
  int nu1 = 2, nu2 = 1, nsr = 1, literal = 0;
  bool f32 = false;  // FP32 relaxation (correction form) on stored and SR levels
  int d_down = 1, d_up = 1;
  int d_srup = 0;  // levels of an up kernel topped by the SR level (0: none fit)
  bool functionals = false;
  // the final level-(M-1) solution goes to the caller (PDE compression)
  bool keep_coarse = false;
  int ravg = 0;  // literal tau with the two-cell average as rhs restriction
  // one SR level whose segment passes are exact as the top level of the
  // vertical kernels (set with the segments)
  bool fuse_down = false, fuse_up = false;
  int64_t S = 1, s = 0, b = 0, pad = 0;
  int seg_threads = 0;
  // sr_levels >= 2: levels M and M-1 are never stored; the finest segment
  // passes rebuild level M-1 on a window of s/2 + 2 p1 cells
  int64_t p1 = 0;
  int R = 1;
  int seg2_threads = 0;
  // workspace layout (byte offsets)
  size_t off_flag = 0, off_F = 0, off_U = 0, off_V = 0, off_Uh = 0, off_Q = 0, off_Utop = 0,
         off_P = 0, total = 0;
};

// Geometry, options and workspace layout (segment arguments excluded).
fmgsr_status make_plan(int64_t n, int32_t levels, const fmgsr_options& o, Plan* p) {
  if (n < 1 || levels < 1 || levels > 40) return FMGSR_EINVAL;
  const int M = levels - 1;
  if ((n % ((int64_t)1 << M)) != 0) return FMGSR_EINVAL;
  const int64_t n0 = n >> M;
  if (n0 > kMaxN0) return FMGSR_EINVAL;
  if (o.nu1 < 0 || o.nu1 > 16 || o.nu2 < 0 || o.nu2 > 16) return FMGSR_EINVAL;
  if (o.sr_levels < 0 || o.sr_levels > M) return FMGSR_EINVAL;
  // per-patch literal tau exists for the finest SR level only
  if (o.sr_levels > 1 && o.tau_mode == FMGSR_TAU_LITERAL) return FMGSR_ENOTSUP;
  if (o.tau_mode != FMGSR_TAU_SPLIT && o.tau_mode != FMGSR_TAU_LITERAL) return FMGSR_EINVAL;
  if (o.precision != FMGSR_FP64 && o.precision != FMGSR_FP32_RELAX) return FMGSR_EINVAL;
  if (o.reserved != 0) return FMGSR_EINVAL;
  if (o.check_finite != 0 && o.check_finite != 1) return FMGSR_EINVAL;
  if (o.rhs_restriction != FMGSR_R_FULLWEIGHT && o.rhs_restriction != FMGSR_R_AVERAGE)
    return FMGSR_EINVAL;
  // split tau rests on L_H I^ = I L_h, which holds for full weighting only
  if (o.rhs_restriction == FMGSR_R_AVERAGE && o.tau_mode != FMGSR_TAU_LITERAL) return FMGSR_EINVAL;
  p->ravg = (o.rhs_restriction == FMGSR_R_AVERAGE);
  p->f32 = (o.precision == FMGSR_FP32_RELAX);
  p->functionals = (o.functionals != nullptr);
  p->keep_coarse = (o.coarse_out != nullptr);
  if (p->keep_coarse && M < 1) return FMGSR_EINVAL;
  // the compressed form is the level below the one SR level
  if (p->keep_coarse && o.sr_levels != 1) return FMGSR_ENOTSUP;
  // literal tau differentiates the iterate (L_h u), amplifying the FP32
  // rounding of the relaxation by ~n^2 into every coarse right-hand side
  if (p->f32 && o.tau_mode == FMGSR_TAU_LITERAL) return FMGSR_ENOTSUP;
  p->n = n;
  p->n0 = n0;
  p->M = M;
  p->nu1 = o.nu1;
  p->nu2 = o.nu2;
  p->nsr = o.sr_levels;
  p->literal = (o.tau_mode == FMGSR_TAU_LITERAL);
  p->d_down = p->literal ? 1 : fuse_depth(false, o.nu1);
  p->d_up = p->literal ? 1 : fuse_depth(true, o.nu2);
  for (int d = kMaxFuse; d >= 2 && p->d_srup == 0; --d)
    if (sr_up_fits(o.nu2, d, kTileHalo)) p->d_srup = d;
  // coarse core top level
  int C = 0;
  const int cmax = M - std::max(o.sr_levels, 1);  // SR levels stay above the core
  while (C + 1 <= cmax && (n0 << (C + 1)) <= kCoreMaxCells) ++C;
  p->C = C;
  // workspace layout
  const size_t hier = (size_t)(M >= 1 ? lvl_off_ws(n0, M) : 0) * sizeof(double);  // levels 0..M-1
  // with two or more SR levels, V holds levels 0..M-2 only and U levels
  // 0..M-2 plus I^ of level M-1 (n/4 cells) in level M-1's place
  const bool two = (o.sr_levels >= 2);
  const size_t hierV = two ? (size_t)lvl_off_ws(n0, M - 1) * sizeof(double) : hier;
  const size_t hierU = two ? hierV + (size_t)(n >> 2) * sizeof(double) : hier;
  size_t off = 0;
  p->off_flag = off; off = align_up(off + sizeof(int));  // non-finite flag
  p->off_F = off; off = align_up(off + hier);
  p->off_U = off; off = align_up(off + hierU);
  p->off_V = off; off = align_up(off + hierV);
  p->off_Q = off; off = align_up(off + (p->literal ? hier : 0));
  p->off_Utop = off; off = align_up(off + (p->nsr == 0 && M >= 1 ? (size_t)n * sizeof(double) : 0));
  // per-tile functional partials of the SR-topped up kernel (2 per tile)
  const int64_t tile_core = (int64_t)kRun * kVertThreads - 2 * kTileHalo;
  p->off_P = off;
  off = align_up(off + (p->nsr >= 1 ? (size_t)(2 * ((n + tile_core - 1) / tile_core) + 2) * sizeof(double) : 0));
  // Uh last: plan_bytes() leaves it out when the segments never use it
  p->off_Uh = off; off = align_up(off + (p->nsr ? (size_t)(n / 2) * sizeof(double) : 0));
  p->total = std::max<size_t>(off, kAlign);
  return FMGSR_OK;
}

// Segments of the SR levels: the same count on each, core s_l = n_l /
// n_segments (even on every SR level), window of s + 2 pad cells per
// workgroup on the finest, pad = even >= buffer + 1.
fmgsr_status plan_segments(int64_t n_segments, int32_t buffer, Plan* p) {
  if (p->nsr == 0) return FMGSR_OK;
  if (buffer < 0 || buffer > 1024) return FMGSR_EINVAL;
  if (n_segments < 1 || p->n % n_segments != 0) return FMGSR_EINVAL;
  const int64_t s = p->n / n_segments;
  if (s < 2 || (s & 1)) return FMGSR_EINVAL;
  for (int k = 1; k < p->nsr; ++k) {
    const int64_t nk = p->n >> k;
    if (nk % n_segments != 0 || (nk / n_segments) < 2 || ((nk / n_segments) & 1)) return FMGSR_EINVAL;
  }
  const int64_t pad = ((int64_t)buffer + 2) & ~(int64_t)1;
  const int64_t cells = s + 2 * pad;
  if (cells > (int64_t)kSegRun * kSegMaxThreads) return FMGSR_EINVAL;
  const int64_t thr = (cells + kSegRun - 1) / kSegRun;
  p->S = n_segments;
  p->s = s;
  p->b = buffer;
  p->pad = pad;
  p->seg_threads = (int)((thr + 63) / 64 * 64);
  // One SR level, split tau: with b >= 2 nu1 - 1 the block smoother's cores
  // equal global red-black sweeps bit for bit, and with b >= 2 nu2 the
  // blocked compatible relaxation's cores equal the unsegmented one, so the
  // SR down / up passes are exact as the top level of a vertical kernel.
  p->fuse_down = p->nsr == 1 && !p->literal && buffer >= 2 * (int64_t)p->nu1 - 1 &&
                 p->d_down >= 2 && p->M - 1 > p->C;
  // (kept coarse solution: the up leg stores level M-1 and the segment pass
  // expands it)
  p->fuse_up = p->fuse_down && buffer >= 2 * (int64_t)p->nu2 && !p->keep_coarse &&
               std::min(p->d_srup, p->M - p->C) >= 2;
  if (p->nsr >= 2) {
    // level-(M-1) margin: pad/2 + 2 cells for Pi's reach from the level-M
    // window, 3 per CR iteration of stale cells from the window edges, even
    p->p1 = ((pad / 2 + 3 * (int64_t)p->nu2 + 6) + 1) & ~(int64_t)1;
    // b >= 2 nu2: the level-(M-1) relaxation's cores do not see the segment
    // edges, and one run over the window serves all zones; else one run per
    // segment the window reaches
    p->R = (buffer >= 2 * p->nu2) ? 0 : (int)((pad / 2 + 2 + s / 2 - 1) / (s / 2));
    const int64_t cells1 = s / 2 + 2 * p->p1;
    const int64_t thr1 = std::max(thr, (cells1 + kSegRun / 2 - 1) / (kSegRun / 2));
    if (thr1 > kSegMaxThreads) return FMGSR_EINVAL;
    p->seg2_threads = (int)((thr1 + 63) / 64 * 64);
    if (p->seg2_threads > kSegMaxThreads) return FMGSR_EINVAL;
  }
  return FMGSR_OK;
}

// FMG step t (a stored level) rebuilds its top level's pre-smoothed iterate
// inside its top up kernel, and its top down kernel never stores it.  Needs
// split tau; both top kernels walk two or more levels (so the next down
// kernel and the coarse core read lower levels only, and no up kernel of the
// step writes V^{t-1}, the rebuild's source, before the top one); and the
// rebuild's stale edge cells stay outside the top core's reach.
bool rebuild_top(const Plan& p, int t) {
  if (p.literal || t > p.M || t < p.C + 2) return false;
  if (p.nsr >= 1 && t > p.M - p.nsr) return false;  // an SR level
  const int dd = std::min(p.d_down, t - p.C), du = std::min(p.d_up, t - p.C);
  return dd >= 2 && rebuild_up_fits(p.nu1, p.nu2, du, kTileHalo);
}

// Workspace these segments actually use: the restricted SR iterate Uh (the
// last region of the layout, after every region the solve may need) is
// only needed by the segment passes (also for their functional partials);
// without SR levels, the finest pre-smoothed iterate Utop (then the last
// non-empty region) only when the finest step does not rebuild it.
size_t plan_bytes(const Plan& p) {
  if (p.nsr == 0)
    return (p.M >= 1 && rebuild_top(p, p.M)) ? std::max<size_t>(p.off_Utop, kAlign) : p.total;
  const bool uh = p.nsr >= 2 || (p.nsr == 1 && !(p.fuse_down && p.fuse_up));
  return uh ? p.total : std::max<size_t>(p.off_Uh, kAlign);
}

// Dynamic LDS (bytes) of one workgroup of each kernel that takes it: the
// coarse core holds its level stack (iterates, right-hand sides, correction),
// the cyclic-reduction buffers and the sweeps' second buffer (level C); the
// segment kernels a stage of K + 1 and an exchange of 4 doubles per thread.
size_t core_lds(const Plan& p) {
  const int64_t ntot = p.n0 * (((int64_t)1 << (p.C + 1)) - 1);
  const int64_t esz = (p.C > 0) ? (p.n0 << (p.C - 1)) : 0;
  return (size_t)(2 * ntot + esz + 8 * p.n0 + (p.n0 << p.C)) * sizeof(double);
}
size_t seg_lds(int threads) { return (size_t)threads * (kSegRun + 1 + 4) * sizeof(double); }

// The largest dynamic LDS any launch of this plan requests (segment kernels
// counted whenever the plan has SR levels).
size_t plan_lds(const Plan& p) {
  size_t m = core_lds(p);
  if (p.nsr >= 1) m = std::max(m, seg_lds(p.seg_threads));
  if (p.nsr >= 2) m = std::max(m, seg_lds(p.seg2_threads));
  return m;
}

// Upper bound of the LDS one workgroup may hold on gfx950 (static + dynamic).
constexpr size_t kMaxLds = 160 * 1024;

// Dynamic LDS a kernel may be granted: the device's per-workgroup limit
// (capped at kMaxLds) less the kernel's own static LDS.  The runtime refuses
// a grant that, added to the static part, exceeds the limit (the coarse core
// keeps a small static table, so a flat 160 KiB grant is refused for it).
size_t lds_grant(size_t limit, size_t static_bytes) {
  const size_t cap = std::min(limit, kMaxLds);
  return static_bytes < cap ? cap - static_bytes : 0;
}

// Grants the dynamic-LDS attribute to every kernel that takes dynamic LDS
// (once per device; each call's return code is checked and a failure is
// remembered and reported by every solve on that device), then checks that
// this plan's requests fit the grants, so an oversized request becomes an
// error code instead of a launch the device cannot honour.
fmgsr_status check_lds(const Plan& p) {
  constexpr int kMaxDev = 64;
  struct Grants {
    bool done = false;
    hipError_t err = hipSuccess;
    size_t core = 0, seg = 0;
  };
  static std::mutex mu;
  static Grants grants[kMaxDev];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(mu);
  Grants& g = grants[dev];
  if (!g.done) {
    g.done = true;
    size_t limit = 0;
    g.err = device_lds_limit(&limit);
    auto grant = [&](const void* k, size_t* granted) {
      if (g.err != hipSuccess) return;
      hipFuncAttributes fa;
      g.err = hipFuncGetAttributes(&fa, k);
      if (g.err != hipSuccess) return;
      const size_t v = lds_grant(limit, fa.sharedSizeBytes);
      g.err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)v);
      if (g.err == hipSuccess) *granted = std::min(*granted, v);
    };
    size_t core = SIZE_MAX, seg = SIZE_MAX;
    grant((const void*)k_coarse_core, &core);
    const void* segk[] = {(const void*)k_sr_down<kSegRun, false>, (const void*)k_sr_up<kSegRun, false>,
                          (const void*)k_sr_down<kSegRun, true>, (const void*)k_sr_up<kSegRun, true>,
                          (const void*)k_sr2<kSegRun, false, false>, (const void*)k_sr2<kSegRun, false, true>,
                          (const void*)k_sr2<kSegRun, true, false>, (const void*)k_sr2<kSegRun, true, true>};
    for (const void* k : segk) grant(k, &seg);
    if (g.err != hipSuccess) (void)hipGetLastError();
    g.core = core;
    g.seg = seg;
  }
  if (g.err != hipSuccess) return FMGSR_EDEVICE;
  if (core_lds(p) > g.core) return FMGSR_EINVAL;
  if (p.nsr >= 1 && seg_lds(p.seg_threads) > g.seg) return FMGSR_EINVAL;
  if (p.nsr >= 2 && seg_lds(p.seg2_threads) > g.seg) return FMGSR_EINVAL;
  return FMGSR_OK;
}

struct Ctx {
  const Plan* p;
  hipStream_t st;
  double gL, gR;
  const double* f;
  double* u_out;
  double* functionals = nullptr;  // [2] device: h sum u, h sum u^2 of the result
  double* coarse_out = nullptr;   // [n/2] device: the final level-(M-1) solution
  double *F, *U, *V, *Uh, *Q, *Utop;
  double* P;  // per-tile functional partials
  fmgsr_status err = FMGSR_OK;

  double* lv(double* base, int l) const { return base + lvl_off_ws(p->n0, l); }
  int64_t nl(int l) const { return p->n0 << l; }
  const double* forcing(int l) const { return l == p->M ? f : lv(F, l); }

  void check() {
    if (hipGetLastError() != hipSuccess) err = FMGSR_EDEVICE;
  }

  // Core cells of a tile of T threads (kRun cells each, less the halo on
  // both sides).
  static int64_t tile_core(int T) { return (int64_t)kRun * T - 2 * kTileHalo; }

  VertArgs vargs(int top, int levels, int nu, int T = kVertThreads) const {
    VertArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = nl(top);
    a.gL = gL;
    a.gR = gR;
    a.nu = nu;
    a.levels = levels;
    a.core = tile_core(T);
    a.halo = kTileHalo;
    return a;
  }

  // Down leg over levels top..top-levels+1.
  // deep: paired with a deep up kernel, which rebuilds levels top-1 ..
  // top-levels+2 (interior tiles do not store them)
  void down_launch(int top, int levels, int src_kind, const double* src, const double* rhs,
                   double* top_out, bool deep = false) {
    VertArgs a = vargs(top, levels, p->nu1);
    a.src_kind = src_kind;
    a.src = src;
    a.rhs = rhs;
    a.deep = deep;
    double bytes = 0.0;
    for (int i = 0; i < levels; ++i) {
      a.out[i] = (i == 0) ? top_out : lv(U, top - i);
      const bool skipped = deep && i >= 1 && i + 1 < levels;
      if (a.out[i] && !skipped) bytes += (double)nl(top - i) * 8.0;  // U written
    }
    const double nb = (double)a.n * 8.0;
    bytes += nb + (src_kind == kSrcInterp ? nb * 0.5 : src_kind == kSrcRestrict ? nb * 2.0 : nb);
    const int64_t blocks = (a.n + a.core - 1) / a.core;
    const bool wide = a.n >= kWideCells;
    ProfScope ps("k_down", bytes, st);
    constexpr int T = kVertThreads;
    const dim3 g((unsigned)blocks), b(T);
    if (p->f32 && wide) hipLaunchKernelGGL((k_down<kRun, true, 3, T>), g, b, 0, st, a);
    else if (p->f32) hipLaunchKernelGGL((k_down<kRun, true, 2, T>), g, b, 0, st, a);
    else if (wide) hipLaunchKernelGGL((k_down<kRun, false, 3, T>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_down<kRun, false, 2, T>), g, b, 0, st, a);
    check();
  }

  // Up leg over levels top-levels+1..top; result of the top level to out.
  // top_pre == nullptr: the top level is the SR level (full update + CR)
  // Top level: sr_top: the SR level (full update from the level below and
  // compatible relaxation); else rebuild_src != nullptr: its pre-smoothed
  // iterate is rebuilt from that FMG iterate of the level below; else read
  // from top_pre.  deep: levels top-1 .. top-levels+2 are rebuilt as well
  // (from rebuild_src, also with sr_top).
  void up_launch(int top, int levels, const double* rhs, const double* coarse,
                 const double* top_pre, double* out, const double* rebuild_src = nullptr,
                 bool sr_top = false, bool deep = false) {
    VertArgs a = vargs(top, levels, p->nu2);
    a.rhs = rhs;
    a.coarse = coarse;
    a.src = rebuild_src;
    a.nu_pre = p->nu1;
    a.sr_top = sr_top;
    a.deep = deep;
    if (rebuild_src || sr_top) top_pre = nullptr;
    double bytes = rebuild_src ? (double)nl(top - 1) * 8.0 : 0.0;  // Pi source read
    for (int i = 0; i < levels; ++i) {
      a.pre[i] = (i == 0) ? top_pre : lv(U, top - i);
      const bool rebuilt = deep && i + 1 < levels;
      if (a.pre[i] && !rebuilt) bytes += (double)nl(top - i) * 8.0;  // pre read
    }
    bytes += (double)a.n * (out ? 16.0 : 8.0) + (double)nl(top - levels) * 8.0;  // rhs, out; coarse
    a.out[0] = out;
    if (a.sr_top && functionals) a.part = P;
    const int64_t blocks = (a.n + a.core - 1) / a.core;
    ProfScope ps("k_up", bytes, st);
    int64_t b_lo = 0, b_hi = -1;
    if (deep && a.n >= kWideCells) interior_tiles(a, kVertThreads, &b_lo, &b_hi);
    up_kernels<kVertThreads>(a, blocks, b_lo, b_hi);
    check();
  }

  // The up launch of tile shape T: interior tiles [b_lo, b_hi] on the
  // three-wavefronts-per-SIMD kernel and the edge tiles on k_up, or every
  // tile on k_up when b_hi < b_lo.
  template <int T>
  void up_kernels(const VertArgs& a, int64_t blocks, int64_t b_lo, int64_t b_hi) {
    if (b_hi >= b_lo) {
      VertArgs w = a;
      w.tile0 = b_lo;
      VertArgs e = a;
      e.gap_at = b_lo;
      e.gap = b_hi - b_lo + 1;
      const dim3 gw((unsigned)(b_hi - b_lo + 1)), ge((unsigned)(blocks - e.gap)), tb(T);
      if (p->f32) {
        hipLaunchKernelGGL((k_up_wide<kRun, true, T>), gw, tb, 0, st, w);
        hipLaunchKernelGGL((k_up<kRun, true, T>), ge, tb, 0, st, e);
      } else {
        hipLaunchKernelGGL((k_up_wide<kRun, false, T>), gw, tb, 0, st, w);
        hipLaunchKernelGGL((k_up<kRun, false, T>), ge, tb, 0, st, e);
      }
    } else if (p->f32) {
      hipLaunchKernelGGL((k_up<kRun, true, T>), dim3((unsigned)blocks), dim3(T), 0, st, a);
    } else {
      hipLaunchKernelGGL((k_up<kRun, false, T>), dim3((unsigned)blocks), dim3(T), 0, st, a);
    }
  }

  // The tiles whose window lies inside the level (window_interior on the
  // device), [b_lo, b_hi]; empty when b_hi < b_lo.
  static void interior_tiles(const VertArgs& a, int T, int64_t* b_lo, int64_t* b_hi) {
    const int64_t wc = (int64_t)T * kRun;
    auto inside = [&](int64_t b) {
      const int64_t wlo = b * a.core - a.halo;
      return b >= 0 && wlo >= kInteriorMargin && wlo + wc + kInteriorMargin <= a.n;
    };
    int64_t lo = (kInteriorMargin + a.halo + a.core - 1) / a.core;
    int64_t hi = (a.n - wc - kInteriorMargin + a.halo) >= 0 ? (a.n - wc - kInteriorMargin + a.halo) / a.core : -1;
    // the closed forms, checked against the predicate itself
    if (hi < lo || !inside(lo) || inside(lo - 1) || !inside(hi) || inside(hi + 1)) {
      *b_lo = 0;
      *b_hi = -1;
      return;
    }
    *b_lo = lo;
    *b_hi = hi;
  }

  // Forcing of levels src_level-1 .. src_level-levels from level src_level
  // (256-thread tiles: a plain restriction chain has no exchange-bound
  // phases, and its larger windows re-read fewer halo cells).
  void forcing_launch(int src_level, int levels) {
    VertArgs a = vargs(src_level, levels, 0, kTileThreads);
    a.rhs = forcing(src_level);
    a.ravg = p->ravg;
    double bytes = (double)a.n * 8.0;
    for (int i = 0; i < levels; ++i) {
      a.out[i] = lv(F, src_level - 1 - i);
      bytes += (double)nl(src_level - 1 - i) * 8.0;
    }
    const int64_t blocks = (a.n + a.core - 1) / a.core;
    ProfScope ps("k_forcing", bytes, st);
    hipLaunchKernelGGL((k_forcing<kRun, kTileThreads>), dim3((unsigned)blocks), dim3(kTileThreads), 0,
                       st, a);
    check();
  }

  void tau_launch(const double* ufine, const double* Ffine, int lcoarse, double* out) {
    const int64_t nc = nl(lcoarse);
    const int thr = 256;
    ProfScope ps("k_tau_literal", (double)nc * 8.0 * 5.0, st);  // u, F: 2 nc each; out: nc
    hipLaunchKernelGGL(k_tau_literal, dim3((unsigned)((nc + thr - 1) / thr)), dim3(thr), 0, st,
                       ufine, Ffine, nc, gL, gR, p->ravg, out);
    check();
  }

  void core_launch(int mode, int src_kind, const double* src, const double* rhs_top,
                   double* out = nullptr) {
    CoreArgs a;
    std::memset(&a, 0, sizeof(a));
    a.top = p->C;
    a.n0 = p->n0;
    a.gL = gL;
    a.gR = gR;
    a.nu1 = p->nu1;
    a.nu2 = p->nu2;
    a.literal = p->literal;
    a.ravg = p->ravg;
    a.mode = mode;
    a.src_kind = src_kind;
    for (int l = 0; l <= p->C; ++l) a.F[l] = forcing(l);
    a.src = src;
    a.rhs_top = rhs_top;
    a.out = out ? out : (p->M >= 1) ? lv(V, p->C) : u_out;
    const int64_t ntot = p->n0 * (((int64_t)1 << (p->C + 1)) - 1);
    const size_t lds = core_lds(*p);
    const int64_t nC = p->n0 << p->C;
    double bytes = (double)ntot * 8.0 + (double)nC * 8.0;  // forcing levels, result
    if (mode == 1) bytes += (double)nC * 8.0 * (src_kind == kSrcRestrict ? 3.0 : 2.0);
    ProfScope ps("k_coarse_core", bytes, st);
    hipLaunchKernelGGL(k_coarse_core, dim3(1), dim3(kCoreThreads), lds, st, a);
    check();
  }

  // Segment pass over SR level l: down (coarse = Pi source, or direct =
  // the level's restricted iterate) writes I^ of the cores to out (and the
  // literal coarse rhs to q_out); up writes the cores to out.
  void seg_launch(int l, bool up, const double* coarse, const double* direct, double* out,
                  double* q_out) {
    SegArgs a;
    std::memset(&a, 0, sizeof(a));
    const bool finest = (l == p->M);
    if (up && finest && functionals) a.part = Uh;  // Uh is dead once the down pass has been consumed
    a.n = nl(l);
    a.gL = gL;
    a.gR = gR;
    a.nu = up ? p->nu2 : p->nu1;
    a.s = p->s >> (p->M - l);
    a.buffer = p->b;
    a.pad = p->pad;
    a.win = (int)(a.s + 2 * p->pad);
    a.coarse = coarse;
    a.direct = direct;
    a.f = forcing(l);
    a.out = out;
    a.q_out = q_out;
    a.ravg = p->ravg;
    a.seg0 = 0;
    a.out_lo = 0;
    a.out_hi = a.n;
    const int64_t thr = (a.win + kSegRun - 1) / kSegRun;
    const int threads = finest ? p->seg_threads : (int)((thr + 63) / 64 * 64);
    const double nb = (double)a.n * 8.0;
    // source (Pi: n/2, direct: n) and f read; down writes n/2 (+ n/2 literal
    // tau), up writes n
    const double src = direct ? nb : nb * 0.5;
    const double bytes = up ? nb * 2.5 : nb + src + nb * 0.5 + (q_out ? nb * 0.5 : 0.0);
    const size_t lds = seg_lds(threads);
    ProfScope ps(up ? "k_sr_up" : "k_sr_down", bytes, st);
    const dim3 g((unsigned)p->S), b(threads);
    if (up && p->f32) hipLaunchKernelGGL((k_sr_up<kSegRun, true>), g, b, lds, st, a);
    else if (up) hipLaunchKernelGGL((k_sr_up<kSegRun, false>), g, b, lds, st, a);
    else if (p->f32) hipLaunchKernelGGL((k_sr_down<kSegRun, true>), g, b, lds, st, a);
    else hipLaunchKernelGGL((k_sr_down<kSegRun, false>), g, b, lds, st, a);
    check();
  }

  // Finest segment pass with level M-1 unstored: rebuilds V^{M-1} from
  // V^{M-2} per segment, then the level-M down (I^ of the cores to Uh) or
  // up (cores to u_out, functionals) pass.
  void seg2_launch(bool up) {
    Seg2Args a;
    std::memset(&a, 0, sizeof(a));
    const int M = p->M;
    a.n = p->n;
    a.gL = gL;
    a.gR = gR;
    a.nu1 = p->nu1;
    a.nu2 = p->nu2;
    a.s = p->s;
    a.S = p->S;
    a.R = p->R;
    a.buffer = p->b;
    a.pad = p->pad;
    a.win = (int)(p->s + 2 * p->pad);
    a.p1 = p->p1;
    a.win1 = (int)(p->s / 2 + 2 * p->p1);
    a.v2 = lv(V, M - 2);
    a.f1 = lv(F, M - 1);
    a.f = f;
    a.out = up ? u_out : Uh;
    if (up && functionals) a.part = Uh;
    const double nb = (double)p->n * 8.0;
    // V^{M-2} n/4, F^{M-1} n/2 and f n read; down writes n/2, up writes n
    const double bytes = nb * 1.75 + (up ? (u_out ? nb : 0.0) : nb * 0.5);
    const int threads = p->seg2_threads;
    const size_t lds = seg_lds(threads);
    ProfScope ps(up ? "k_sr2_up" : "k_sr2_down", bytes, st);
    const dim3 g((unsigned)p->S), b(threads);
    if (up && p->f32) hipLaunchKernelGGL((k_sr2<kSegRun, true, true>), g, b, lds, st, a);
    else if (up) hipLaunchKernelGGL((k_sr2<kSegRun, false, true>), g, b, lds, st, a);
    else if (p->f32) hipLaunchKernelGGL((k_sr2<kSegRun, true, false>), g, b, lds, st, a);
    else hipLaunchKernelGGL((k_sr2<kSegRun, false, false>), g, b, lds, st, a);
    check();
  }

  void run() {
    const Plan& P = *p;
    const int M = P.M, C = P.C;
    if (M == 0) {  // a single grid: exact solve
      core_launch(0, kSrcDirect, nullptr, nullptr);
      return;
    }
    // forcing on all levels
    for (int l = M; l > 0; l -= kMaxFuse) forcing_launch(l, std::min(kMaxFuse, l));
    // FMG cycles on the coarse core levels
    core_launch(0, kSrcDirect, nullptr, nullptr);
    const int sr_lo = M - P.nsr + 1;  // lowest SR level (M + 1: none)
    for (int t = C + 1; t <= M && err == FMGSR_OK; ++t) {
      const bool sr = (P.nsr >= 1 && t >= sr_lo);
      double* Ut = (t == M) ? Utop : lv(U, t);
      auto U_of = [&](int l) -> double* { return l == t ? Ut : lv(U, l); };
      // right-hand side in use on level l during this step
      auto rhs_of = [&](int l) -> const double* {
        if (l == t) return forcing(t);
        return P.literal ? lv(Q, l) : lv(F, l);
      };
      // I^ of the smoothed SR level l+1 (the start of level l's down visit):
      // Uh below the finest level; below an SR level l+1 < M, the U array of
      // level l+1, which SR levels do not otherwise use
      auto H = [&](int l) -> double* { return l == M - 1 ? Uh : lv(U, l + 1); };
      // with two or more SR levels, level M-1 is never stored either: the
      // finest passes rebuild it from V^{M-2}
      const bool two = (P.nsr >= 2);
      // post-smoothed iterate of level l in this step: the final step's
      // level-(M-1) solution goes to the caller's array when it is kept
      auto Vout = [&](int l) -> double* {
        return (t == M && l == M - 1 && coarse_out) ? coarse_out : lv(V, l);
      };
      // One SR level with split tau and b >= 2 nu1 - 1: the block smoother's
      // cores equal global red-black sweeps bit for bit, so the SR down pass
      // (Pi, sweeps, I^ of the cores) is the top level of an ordinary
      // vertical down kernel whose level-M output is simply not stored; the
      // restricted iterate never goes through HBM.
      const bool fused_down = sr && t == M && P.fuse_down;
      // one SR level with both passes inside the vertical kernels: a deep
      // pair when both SR-topped kernels walk the same levels
      const int dsr_n = std::min(P.d_srup, M - C);
      // with FP32 relaxation only where the interior tiles take k_up_wide:
      // the general up kernel then runs one wavefront per SIMD and has no
      // latency left to hide the extra sweeps in
      const bool deep_ok = !P.f32 || nl(t) >= kWideCells;
      const bool deep_sr = fused_down && P.fuse_up && deep_ok && dsr_n == std::min(P.d_down, M - C) &&
                           deep_fits(P.nu1, P.nu2, dsr_n, kTileHalo, true);
      // the top up kernel rebuilds level t's pre-smoothed iterate, and with
      // a deep pair the next levels' as well
      const bool rebuild = !sr && rebuild_top(P, t);
      const int dtop_n = std::min(P.d_down, t - C);
      const bool deep_stored = rebuild && deep_ok && dtop_n == std::min(P.d_up, t - C) &&
                               deep_fits(P.nu1, P.nu2, dtop_n, kTileHalo, false);
      int top = t;  // highest stored level of this step
      int dtop = t;  // top of the vertical down leg
      if (sr && !fused_down) {
        if (two && t == M) seg2_launch(false);
        else seg_launch(t, false, lv(V, t - 1), nullptr, H(t - 1), P.literal ? lv(Q, t - 1) : nullptr);
        for (int l = t - 1; l >= sr_lo; --l) seg_launch(l, false, nullptr, H(l), H(l - 1), nullptr);
        top = dtop = sr_lo - 1;
      } else if (fused_down) {
        top = M - 1;
      }
      // pre-smoothing leg: levels dtop..C+1
      for (int hi = dtop; hi >= C + 1;) {
        const int d = std::min(P.d_down, hi - C);
        int src_kind;
        const double* src;
        if (hi == t) { src_kind = kSrcInterp; src = lv(V, t - 1); }
        else if (sr && !fused_down && hi == top) { src_kind = kSrcDirect; src = H(top); }
        else { src_kind = kSrcRestrict; src = U_of(hi + 1); }
        if (P.literal && src_kind == kSrcRestrict) tau_launch(U_of(hi + 1), rhs_of(hi + 1), hi, lv(Q, hi));
        const bool unstored = (fused_down && hi == M) || (rebuild && hi == t);
        const bool deep = (hi == t) && (deep_stored || deep_sr);
        down_launch(hi, d, src_kind, src, rhs_of(hi), unstored ? nullptr : U_of(hi), deep);
        hi -= d;
      }
      // coarse core: V-cycle bottom from level C
      if (sr && !fused_down && C == top) {
        core_launch(1, kSrcDirect, H(C), rhs_of(C), Vout(C));
      } else {
        const double* uf = U_of(C + 1);
        if (P.literal) tau_launch(uf, rhs_of(C + 1), C, lv(Q, C));
        core_launch(1, kSrcRestrict, uf, rhs_of(C), Vout(C));
      }
      // One SR level, split tau, b >= 2 nu2, no functionals: the SR up pass
      // (Pi + compatible relaxation) equals the unsegmented one on the cores
      // bit for bit, so it is the top level of the last vertical up kernel,
      // which then never writes V^{M-1}.
      const bool fused_up = fused_down && P.fuse_up;
      const int dsr = std::min(P.d_srup, M - C);       // levels of the SR-topped up kernel
      const int utop = fused_up ? M - dsr : top;       // last ordinary up level
      // post-smoothing leg: stored levels C+1..utop, split from the top down
      // (full kernels on top, a partial one at the bottom), run bottom-up
      int his[64], nup = 0;
      for (int hi = utop; hi >= C + 1; hi -= std::min(P.d_up, hi - C)) his[nup++] = hi;
      for (int k = nup - 1; k >= 0; --k) {
        const int hi = his[k];
        const int d = std::min(P.d_up, hi - C);
        const int lo = hi - d + 1;
        double* out = (hi == top && !sr) ? ((t == M) ? u_out : lv(V, t)) : Vout(hi);
        const double* rsrc = (rebuild && hi == t) ? lv(V, t - 1) : nullptr;
        up_launch(hi, d, rhs_of(hi), lv(V, lo - 1), U_of(hi), out, rsrc, false,
                  deep_stored && hi == t);
      }
      if (fused_up) {
        up_launch(M, dsr, f, lv(V, M - dsr), nullptr, u_out, deep_sr ? lv(V, M - 1) : nullptr,
                  true, deep_sr);
        if (functionals) {
          const int64_t tiles = (p->n + tile_core(kVertThreads) - 1) / tile_core(kVertThreads);
          ProfScope ps("k_functionals", (double)tiles * 16.0 + 16.0, st);
          hipLaunchKernelGGL(k_functionals, dim3(1), dim3(1024), 0, st, this->P, tiles,
                             1.0 / (double)p->n, functionals);
          check();
        }
      } else if (sr) {
        // full update and compatible relaxation on each SR level, upwards
        for (int l = sr_lo; l <= t; ++l) {
          if (two && l == M - 1) continue;  // rebuilt by the finest passes
          // compression only: the kept level-(M-1) solution is the result
          if (l == M && !u_out && !functionals) continue;
          if (two && l == M) seg2_launch(true);
          else seg_launch(l, true, Vout(l - 1), nullptr, l == M ? u_out : lv(V, l), nullptr);
        }
        if (functionals && t == M) {
          ProfScope ps("k_functionals", (double)P.S * 16.0 + 16.0, st);
          hipLaunchKernelGGL(k_functionals, dim3(1), dim3(1024), 0, st, Uh, (int64_t)P.S,
                             1.0 / (double)P.n, functionals);
          check();
        }
      }
    }
  }
};

}  // namespace
}  // namespace fmgsr

using namespace fmgsr;

extern "C" {

void fmgsr_default_options(fmgsr_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->nu1 = 2;
  opt->nu2 = 1;
  opt->sr_levels = 1;
  opt->tau_mode = FMGSR_TAU_SPLIT;
}

size_t fmgsr_workspace_bytes(int64_t n, int32_t levels, const fmgsr_options* opt) {
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  Plan p;
  if (make_plan(n, levels, o, &p) != FMGSR_OK) return 0;
  return p.total;
}

size_t fmgsr_workspace_bytes_for(int64_t n, int32_t levels, int64_t n_segments, int32_t buffer,
                                 const fmgsr_options* opt) {
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  Plan p;
  if (make_plan(n, levels, o, &p) != FMGSR_OK) return 0;
  if (plan_segments(n_segments, buffer, &p) != FMGSR_OK) return 0;
  return plan_bytes(p);
}

size_t fmgsr_launch_lds_bytes(int64_t n, int32_t levels, int64_t n_segments, int32_t buffer,
                              const fmgsr_options* opt) {
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  Plan p;
  if (make_plan(n, levels, o, &p) != FMGSR_OK) return 0;
  if (plan_segments(n_segments, buffer, &p) != FMGSR_OK) return 0;
  return plan_lds(p);
}

}  // extern "C"

namespace fmgsr {
namespace {

// NaN / Inf scan of device arrays for check_finite: clears the workspace
// flag, scans each array, copies the flag back and synchronises the stream.
fmgsr_status scan_finite(const std::vector<std::pair<const double*, int64_t>>& arrays, int* flag,
                         hipStream_t stream) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, stream, flag);
  for (const auto& arr : arrays) {
    const int64_t blocks = std::min<int64_t>((arr.second + 255) / 256, 4096);
    hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0,
                       stream, arr.first, arr.second, flag);
  }
  int h = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  return h ? FMGSR_ENONFINITE : FMGSR_OK;
}

// fmgsr_solve for the Poisson operator.  static_ws: the library's static
// scratch (static_bytes bytes, fmgsr_solve_noalloc), used instead of the
// caller's workspace or a stream-ordered allocation.
fmgsr_status solve_poisson(const double* f, double g_left, double g_right, int64_t n,
                           int32_t levels, int64_t n_segments, int32_t buffer,
                           const fmgsr_options& o, double* u_out, void* hip_stream,
                           char* static_ws, size_t static_bytes) {
  Plan p;
  fmgsr_status st = make_plan(n, levels, o, &p);
  if (st == FMGSR_OK) st = plan_segments(n_segments, buffer, &p);
  if (st != FMGSR_OK) return st;
  // on-the-fly functionals (SR level only); u_out may then be NULL: the fine
  // solution never reaches HBM
  if (o.functionals) {
    if (p.nsr < 1 || p.s < 4 || !is_device_ptr(o.functionals)) return FMGSR_EINVAL;
  }
  if (o.coarse_out) {
    if (!is_device_ptr(o.coarse_out) || (const void*)o.coarse_out == (const void*)f ||
        o.coarse_out == u_out)
      return FMGSR_EINVAL;
  }
  if (!is_device_ptr(f) || (u_out ? !is_device_ptr(u_out) : !(o.functionals || o.coarse_out)))
    return FMGSR_EINVAL;
  if ((const void*)f == (const void*)u_out) return FMGSR_EINVAL;
  if (const fmgsr_status lst = check_lds(p); lst != FMGSR_OK) return lst;
  hipStream_t stream = (hipStream_t)hip_stream;
  char* ws = (char*)o.workspace;
  bool own = false;
  if (static_ws) {
    if (plan_bytes(p) > static_bytes) return FMGSR_ENOMEM;
    ws = static_ws;
  } else if (ws) {
    if (o.workspace_bytes < plan_bytes(p) || !is_device_ptr(ws)) return FMGSR_ENOMEM;
  } else {
    if (hipMallocAsync((void**)&ws, plan_bytes(p), stream) != hipSuccess) {
      (void)hipGetLastError();
      return FMGSR_ENOMEM;
    }
    own = true;
  }
  // check_finite: scan f before solving (nothing is solved if it fails)
  int* flag = (int*)(ws + p.off_flag);
  if (o.check_finite) {
    const fmgsr_status fst = scan_finite({{f, n}}, flag, stream);
    if (fst != FMGSR_OK) {
      if (own && hipFreeAsync(ws, stream) != hipSuccess) (void)hipGetLastError();
      return fst;
    }
  }
  Ctx c;
  c.p = &p;
  c.st = stream;
  c.gL = g_left;
  c.gR = g_right;
  c.f = f;
  c.u_out = u_out;
  c.functionals = o.functionals;
  c.coarse_out = o.coarse_out;
  c.F = (double*)(ws + p.off_F);
  c.U = (double*)(ws + p.off_U);
  c.V = (double*)(ws + p.off_V);
  c.Uh = (double*)(ws + p.off_Uh);
  c.Q = (double*)(ws + p.off_Q);
  c.Utop = (double*)(ws + p.off_Utop);
  c.P = (double*)(ws + p.off_P);
  c.run();
  // check_finite: scan the results
  if (c.err == FMGSR_OK && o.check_finite) {
    std::vector<std::pair<const double*, int64_t>> outs;
    if (u_out) outs.push_back({u_out, n});
    if (o.coarse_out) outs.push_back({o.coarse_out, n / 2});
    if (o.functionals) outs.push_back({o.functionals, 2});
    c.err = scan_finite(outs, flag, stream);
  }
  if (own && hipFreeAsync(ws, stream) != hipSuccess) {
    (void)hipGetLastError();
    if (c.err == FMGSR_OK) c.err = FMGSR_EDEVICE;
  }
  return c.err;
}

// ---------------------------------------------------------------------------
// Static scratch of fmgsr_solve_noalloc: one array per device (each GPU the
// library runs on holds it until the process ends).  In host code the
// symbol's name is only a stand-in; its device address is looked up once per
// device with that device current and kept.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[FMGSR_NOALLOC_SCRATCH_BYTES];

fmgsr_status scratch_address(char** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static char* addr[kMaxDev] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) {
    (void)hipGetLastError();
    return FMGSR_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      return FMGSR_EDEVICE;
    }
    addr[dev] = (char*)ptr;
  }
  *out = addr[dev];
  return FMGSR_OK;
}

}  // namespace
}  // namespace fmgsr

extern "C" {

fmgsr_status fmgsr_solve(const fmgsr_operator* op, const double* f, double g_left,
                         double g_right, int64_t n, int32_t levels, int64_t n_segments,
                         int32_t buffer, const fmgsr_options* opt, double* u_out,
                         void* hip_stream) {
  if (op && (op->kind < FMGSR_OP_POISSON || op->kind > FMGSR_OP_LINEAR_REACTION)) return FMGSR_EINVAL;
  if (op && op->kind != FMGSR_OP_POISSON) {
    // reaction operators: a batch of one problem (synchronous)
    if (!is_device_ptr(op->kappa)) return FMGSR_EINVAL;
    if (opt && opt->functionals) return FMGSR_ENOTSUP;
    const double g[2] = {g_left, g_right};
    return fmgsr_solve_batched(1, &n, nullptr, &levels, n_segments > 0 ? &n_segments : nullptr,
                               buffer, op, f, g, opt, u_out, hip_stream);
  }
  if (op && op->kappa != nullptr) return FMGSR_EINVAL;
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  return solve_poisson(f, g_left, g_right, n, levels, n_segments, buffer, o, u_out, hip_stream,
                       nullptr, 0);
}

fmgsr_status fmgsr_solve_noalloc(const fmgsr_operator* op, const double* f, double g_left,
                                 double g_right, int64_t n, int32_t levels, int64_t n_segments,
                                 int32_t buffer, const fmgsr_options* opt, double* u_out,
                                 void* hip_stream) {
  if (op && (op->kind < FMGSR_OP_POISSON || op->kind > FMGSR_OP_LINEAR_REACTION)) return FMGSR_EINVAL;
  // the reaction operators run through the batched engine, whose plan allocates
  if (op && op->kind != FMGSR_OP_POISSON) return FMGSR_ENOTSUP;
  if (op && op->kappa != nullptr) return FMGSR_EINVAL;
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  if (o.workspace != nullptr || o.workspace_bytes != 0) return FMGSR_EINVAL;
  char* ws = nullptr;
  if (const fmgsr_status st = scratch_address(&ws); st != FMGSR_OK) return st;
  return solve_poisson(f, g_left, g_right, n, levels, n_segments, buffer, o, u_out, hip_stream,
                       ws, FMGSR_NOALLOC_SCRATCH_BYTES);
}

fmgsr_status fmgsr_decompress(const double* coarse, const double* f, double g_left,
                              double g_right, int64_t n, int64_t n_segments, int32_t buffer,
                              const fmgsr_options* opt, int64_t lo, int64_t hi, double* u_out,
                              void* hip_stream) {
  fmgsr_options o;
  if (opt) o = *opt;
  else fmgsr_default_options(&o);
  if (n < 2 || (n & 1) || o.nu2 < 0 || o.nu2 > 16) return FMGSR_EINVAL;
  if (o.precision != FMGSR_FP64 && o.precision != FMGSR_FP32_RELAX) return FMGSR_EINVAL;
  if (lo < 0 || hi > n || lo > hi) return FMGSR_EINVAL;
  // the finest level as the one SR level of a hierarchy: its segment
  // geometry (core, window, threads) exactly as in the solve.  No coarse
  // core runs here, so the plan's core is a single cell (its LDS request
  // must not count).
  Plan p;
  p.n = n;
  p.n0 = 1;
  p.M = 1;
  p.C = 0;
  p.nu1 = 0;
  p.nu2 = o.nu2;
  p.nsr = 1;
  p.f32 = (o.precision == FMGSR_FP32_RELAX);
  if (const fmgsr_status st = plan_segments(n_segments, buffer, &p); st != FMGSR_OK) return st;
  if (!is_device_ptr(coarse) || !is_device_ptr(f) || !is_device_ptr(u_out)) return FMGSR_EINVAL;
  if ((const void*)u_out == (const void*)f || (const void*)u_out == (const void*)coarse)
    return FMGSR_EINVAL;
  if (lo == hi) return FMGSR_OK;
  if (const fmgsr_status lst = check_lds(p); lst != FMGSR_OK) return lst;
  SegArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.gL = g_left;
  a.gR = g_right;
  a.nu = o.nu2;
  a.s = p.s;
  a.buffer = p.b;
  a.pad = p.pad;
  a.win = (int)(p.s + 2 * p.pad);
  a.coarse = coarse;
  a.f = f;
  a.out = u_out;
  a.seg0 = lo / p.s;
  a.out_lo = lo;
  a.out_hi = hi;
  const int64_t segs = (hi - 1) / p.s - a.seg0 + 1;
  hipStream_t stream = (hipStream_t)hip_stream;
  const size_t lds = seg_lds(p.seg_threads);
  // covering patches of f, their coarse image (Pi's reach included), u_out
  const double bytes = 8.0 * ((double)segs * (double)(p.s + 2 * p.b) +
                              (double)segs * (double)(p.s / 2 + p.b / 2 + 4) + (double)(hi - lo));
  ProfScope ps("k_sr_up", bytes, stream);
  const dim3 g((unsigned)segs), b(p.seg_threads);
  if (p.f32) hipLaunchKernelGGL((k_sr_up<kSegRun, true>), g, b, lds, stream, a);
  else hipLaunchKernelGGL((k_sr_up<kSegRun, false>), g, b, lds, stream, a);
  return hipGetLastError() == hipSuccess ? FMGSR_OK : FMGSR_EDEVICE;
}

fmgsr_status fmgsr_profile_enable(const char* filter) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_prof.clear();
  g_prof_filter = filter ? filter : "";
  g_prof_on = true;
  return FMGSR_OK;
}

int32_t fmgsr_profile_collect(fmgsr_kernel_stat* stats, int32_t max_stats) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = false;
  std::vector<fmgsr_kernel_stat> agg;
  int32_t status = 0;
  for (auto& r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
      (void)hipGetLastError();
      status = FMGSR_EDEVICE;
    }
    size_t k = 0;
    while (k < agg.size() && std::strcmp(agg[k].name, r.name) != 0) ++k;
    if (k == agg.size()) {
      fmgsr_kernel_stat z;
      std::memset(&z, 0, sizeof(z));
      std::strncpy(z.name, r.name, sizeof(z.name) - 1);
      agg.push_back(z);
    }
    agg[k].launches += 1;
    agg[k].total_ms += ms;
    agg[k].algo_bytes += r.bytes;
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_prof.clear();
  if (status != 0) return status;
  for (size_t k = 0; k < agg.size() && (int32_t)k < max_stats; ++k)
    if (stats) stats[k] = agg[k];
  return (int32_t)agg.size();
}

const char* fmgsr_status_string(int32_t status) {
  switch (status) {
    case FMGSR_OK: return "FMGSR_OK";
    case FMGSR_EINVAL: return "FMGSR_EINVAL: invalid argument";
    case FMGSR_ENOMEM: return "FMGSR_ENOMEM: workspace allocation failed or too small";
    case FMGSR_EDEVICE: return "FMGSR_EDEVICE: HIP runtime or launch failure";
    case FMGSR_ENOTSUP: return "FMGSR_ENOTSUP: not implemented by this library";
    case FMGSR_ENONFINITE: return "FMGSR_ENONFINITE: NaN or Inf in the input or the result";
    default: return "unknown fmgsr status";
  }
}

const char* fmgsr_version(void) { return "fmgsr 0.2 gfx950"; }

}  // extern "C"
