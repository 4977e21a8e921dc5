"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Both sides receive the same input bits.  The bar is the FP64 tolerance of
1e-12 relative, held twice: over the whole solution (2-norm) and cell by
cell (max |u_gpu - u_ref| <= 1e-12 max |u_ref|), so an error confined to a
few cells cannot hide in the norm.  Where the coarsest grid is a single cell
the two implementations evaluate identical expression trees (no FMA
contraction on either side), so the results are also required to be bitwise
equal; with N0 > 1 the coarsest solve differs (parallel cyclic reduction vs
Thomas) and only the tolerance applies.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1207_6720_amd import fmgsr, workloads as W  # noqa: E402
from tests.parity_bars import literal_noise_bar  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_solve(dev, f_host, **kw):
    f = torch.from_numpy(np.ascontiguousarray(f_host)).to(dev)
    u = fmgsr.solve(f, **kw)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def oracle_solve(f_host, g=(0.0, 0.0), levels=None, segments=1, buffer=0, nu=(2, 1),
                 sr_levels=1, tau="split"):
    return oracle.fmgsr_solve(f_host, g[0], g[1], levels=levels, segments=segments, buffer=buffer,
                              nu1=nu[0], nu2=nu[1], nsr=sr_levels, tau=tau)


def rhs(n, seed, law="inv_k2", nm=16):
    k, c = W.modes(law, nm, seed, n)
    return W.rhs_numpy(n, k, c)


def compare(u_gpu, u_ref, bitwise):
    denom = max(np.linalg.norm(u_ref), 1e-300)
    err = np.linalg.norm(u_gpu - u_ref) / denom
    assert np.all(np.isfinite(u_gpu))
    assert err <= TOL, f"relative difference {err:.3e}"
    cell = np.abs(u_gpu - u_ref).max() / max(np.abs(u_ref).max(), 1e-300)
    assert cell <= TOL, f"largest cell difference {cell:.3e} of max |u|"
    if bitwise:
        nbad = int(np.count_nonzero(u_gpu != u_ref))
        assert nbad == 0, f"{nbad} cells differ (max |d| = {np.abs(u_gpu - u_ref).max():.3e})"
    return err


# (n, levels, segments, buffer, nu, sr_levels, tau, g, seed)
CASES = [
    # the small workload and its seeds
    (1 << 10, 11, 4, 4, (2, 1), 1, "split", (0.0, 0.0), 0),
    (1 << 10, 11, 4, 4, (2, 1), 1, "split", (0.0, 0.0), 1),
    (1 << 10, 11, 4, 4, (2, 1), 1, "split", (0.0, 0.0), 2),
    # tiny hierarchies (coarse core only, one-cell levels, nc = 1 interpolation)
    (1, 1, 1, 0, (2, 1), 0, "split", (0.3, -0.2), 3),
    (2, 2, 1, 0, (2, 1), 1, "split", (0.3, -0.2), 3),
    (2, 2, 1, 0, (2, 1), 0, "split", (0.3, -0.2), 3),
    (4, 3, 2, 1, (2, 1), 1, "split", (0.0, 1.0), 4),
    (8, 4, 2, 3, (1, 1), 1, "literal", (0.5, 0.5), 5),
    (64, 7, 8, 2, (2, 1), 1, "split", (0.0, 0.0), 6),
    # several tiles per stored level, coarse core boundary, ragged tiles
    (1 << 14, 15, 16, 8, (2, 1), 1, "split", (0.0, 0.0), 7),
    (1 << 16, 17, 16, 8, (2, 1), 1, "split", (0.25, -1.5), 8),
    (5 << 12, 13, 5, 8, (2, 1), 1, "split", (0.0, 0.0), 9),     # N0 = 5
    (7 << 12, 12, 28, 3, (2, 1), 1, "split", (0.1, 0.2), 10),   # N0 = 14
    (3 << 9, 10, 3, 4, (2, 1), 1, "split", (0.0, 0.0), 11),     # N0 = 3
    # plain FMG-FAS (every level stored)
    (1 << 12, 13, 1, 0, (2, 1), 0, "split", (0.0, 0.0), 12),
    (1 << 16, 17, 1, 0, (2, 1), 0, "split", (0.0, 0.0), 13),
    # literal tau (Eq. 7 as written), stored and per-patch
    (1 << 12, 13, 8, 8, (2, 1), 1, "literal", (0.0, 0.0), 14),
    (1 << 12, 13, 8, 1, (2, 1), 1, "literal", (0.4, 0.1), 15),
    (1 << 15, 16, 8, 8, (2, 1), 0, "literal", (0.0, 0.0), 16),
    # sweep counts and thin buffers (segments genuinely change the result)
    (1 << 12, 13, 64, 0, (2, 1), 1, "split", (0.0, 0.0), 17),
    (1 << 12, 13, 64, 1, (1, 1), 1, "split", (0.0, 0.0), 18),
    (1 << 12, 13, 32, 2, (3, 2), 1, "split", (0.0, 0.0), 19),
    (1 << 12, 13, 16, 5, (0, 1), 1, "split", (0.0, 0.0), 20),
    (1 << 12, 13, 16, 5, (1, 0), 1, "split", (0.0, 0.0), 21),
    (1 << 12, 13, 2048, 4, (2, 1), 1, "split", (0.0, 0.0), 22),  # two-cell cores
    (1 << 13, 14, 2, 9, (4, 4), 1, "split", (0.0, 0.0), 23),
    # levels = 1 with N0 > 1 (one exact solve)
    (1000, 1, 1, 0, (2, 1), 0, "split", (0.2, 0.7), 24),
    # the top up kernel of each stored step rebuilds the pre-smoothed top
    # level: many down sweeps (two-level down kernels), no post-sweeps,
    # uneven up kernel splits
    (1 << 14, 15, 1, 0, (10, 0), 0, "split", (0.3, -0.2), 25),
    (1 << 15, 16, 1, 0, (10, 1), 0, "split", (0.0, 0.0), 26),
    (1 << 14, 15, 16, 8, (8, 3), 1, "split", (0.0, 0.0), 27),
    (1 << 13, 14, 8, 9, (5, 2), 1, "split", (-0.4, 0.2), 28),
    # top levels of more than 768 tiles: interior tiles on the
    # three-workgroup kernels, edge tiles on the general ones (deep pairs
    # with four and with three levels, one SR level and none, N0 = 5)
    (1 << 22, 23, 1024, 8, (1, 1), 1, "split", (0.0, 0.0), 44),
    (1 << 22, 23, 1, 0, (3, 2), 0, "split", (0.2, -0.3), 45),
    (5 << 20, 21, 1280, 8, (2, 1), 1, "split", (0.0, 0.0), 46),
    # coarse core on one wavefront: N0 a power of two, one to five levels
    # above the level of 64 cells (N0 = 64: the exact solve is one
    # wavefront's cyclic reduction)
    (1 << 12, 11, 8, 4, (2, 1), 1, "split", (0.1, -0.3), 60),   # N0 = 4
    (1 << 13, 8, 4, 4, (2, 1), 1, "split", (0.0, 0.0), 61),     # N0 = 64
    (1 << 8, 4, 2, 2, (2, 1), 1, "split", (0.0, 0.0), 62),      # N0 = 32, one run level
    (1 << 11, 11, 4, 4, (3, 2), 0, "split", (0.2, 0.1), 63),    # N0 = 2
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_L{c[1]}_S{c[2]}_b{c[3]}_nu{c[4][0]}{c[4][1]}_sr{c[5]}_{c[6]}")
def test_parity_vs_oracle(dev, case):
    n, levels, S, b, nu, sr, tau, g, seed = case
    print(f"case n={n} levels={levels} S={S} b={b} nu={nu} sr={sr} tau={tau}", flush=True)
    f = rhs(n, seed)
    kw = dict(g=g, levels=levels, segments=S, buffer=b, nu=nu, sr_levels=sr, tau=tau)
    u_gpu = gpu_solve(dev, f, **kw)
    u_ref = oracle_solve(f, **kw)
    n0 = n >> (levels - 1)
    compare(u_gpu, u_ref, bitwise=(n0 == 1))


# several SR levels (Sec. 4 studies 0-3): block pre-smoothing from I^ of the
# SR level above and full update + CR on every SR level, split tau
# (n, levels, segments, buffer, nu, sr_levels, g, seed)
MULTI_SR_CASES = [
    (1 << 10, 11, 4, 4, (2, 1), 2, (0.0, 0.0), 30),
    (1 << 10, 11, 4, 2, (1, 1), 3, (0.2, -0.1), 31),     # thin buffer: blocks matter
    (16, 5, 1, 1, (2, 1), 4, (0.3, -0.2), 32),           # every level above the coarsest
    (64, 7, 8, 2, (2, 1), 2, (0.0, 0.0), 33),            # core directly below the SR levels
    (1 << 12, 13, 8, 0, (2, 1), 2, (0.0, 0.0), 34),      # no buffer
    (1 << 14, 15, 16, 8, (2, 1), 2, (0.0, 0.0), 35),     # stored level between core and SR
    (1 << 16, 17, 64, 1, (2, 1), 3, (0.25, -1.5), 36),
    (5 << 12, 13, 5, 8, (2, 1), 2, (0.0, 0.0), 37),      # N0 = 5
    (7 << 12, 12, 28, 3, (3, 2), 2, (0.1, 0.2), 38),     # N0 = 14
    # the unstored level M-1 is rebuilt per finest segment from the
    # relaxation of the level-(M-1) segments its window reaches
    (1 << 12, 13, 512, 5, (2, 3), 2, (0.0, 0.0), 39),    # 4-cell cores, b < 2 nu2: two segments per side
    (1 << 12, 13, 512, 8, (2, 1), 2, (0.0, 0.0), 40),    # b >= 2 nu2: one run per window
    (1 << 12, 13, 16, 20, (1, 4), 2, (0.3, 0.0), 41),    # four CR iterations
    (1 << 12, 13, 256, 3, (2, 3), 3, (0.0, -0.5), 42),
    (1 << 13, 14, 4, 64, (2, 1), 2, (0.0, 0.0), 43),     # widest buffer
]


@pytest.mark.parametrize("case", MULTI_SR_CASES,
                         ids=lambda c: f"n{c[0]}_L{c[1]}_S{c[2]}_b{c[3]}_nu{c[4][0]}{c[4][1]}_sr{c[5]}")
def test_parity_several_sr_levels(dev, case):
    n, levels, S, b, nu, sr, g, seed = case
    print(f"case n={n} levels={levels} S={S} b={b} nu={nu} sr={sr}", flush=True)
    f = rhs(n, seed)
    kw = dict(g=g, levels=levels, segments=S, buffer=b, nu=nu, sr_levels=sr)
    u_gpu = gpu_solve(dev, f, **kw)
    u_ref = oracle_solve(f, **kw)
    compare(u_gpu, u_ref, bitwise=(n >> (levels - 1)) == 1)
    # the extra SR levels are a different smoother: the result moves, within
    # the method's accuracy
    one = oracle_solve(f, **dict(kw, sr_levels=1))
    assert not np.array_equal(u_ref, one)


def test_several_sr_levels_fp32_and_functionals(dev):
    n, levels, S, b = 1 << 14, 15, 16, 8
    k, c = W.modes("inv_k2", 16, 40)
    f_host = W.rhs_numpy(n, k, c)
    kw = dict(levels=levels, segments=S, buffer=b, sr_levels=2)
    ref = oracle_solve(f_host, **kw)
    ustar, uex = closed_form_pair(n, k, c)
    disc = np.linalg.norm(ustar - uex) / np.linalg.norm(uex)
    u32 = gpu_solve(dev, f_host, precision="fp32relax", **kw)
    d32 = np.linalg.norm(u32 - ref) / np.linalg.norm(ref)
    print(f"sr_levels=2 fp32 relaxation vs oracle {d32:.2e}, disc {disc:.2e}", flush=True)
    assert d32 <= 0.1 * disc
    f = torch.from_numpy(f_host).to(dev)
    fun = torch.zeros(2, dtype=torch.float64, device=dev)
    fmgsr.solve(f, functionals=fun, write_u=False, **kw)
    torch.cuda.synchronize()
    want = fsum_functionals(ref)
    got = fun.cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-13 * np.abs(want)), (got, want)


def test_several_sr_levels_rejections(dev):
    f = torch.zeros(1 << 10, dtype=torch.float64, device=dev)
    with pytest.raises(fmgsr.FmgsrError):      # odd core on the third SR level
        fmgsr.solve(f, levels=11, segments=256, buffer=4, sr_levels=3)
    with pytest.raises(fmgsr.FmgsrError):      # literal tau
        fmgsr.solve(f, levels=11, segments=4, buffer=4, sr_levels=2, tau="literal")
    with pytest.raises(fmgsr.FmgsrError):      # as many SR levels as grids
        fmgsr.solve(f, levels=11, segments=1, buffer=4, sr_levels=11)


LITERAL_MULTICELL = [
    # n, levels, segments, buffer, sr_levels, g
    (5 << 12, 13, 5, 8, 1, (0.0, 0.0)),
    (3 << 12, 13, 3, 4, 1, (0.5, -0.25)),
    (5 << 10, 11, 1, 0, 0, (0.0, 0.0)),
]


@pytest.mark.parametrize("case", LITERAL_MULTICELL, ids=lambda c: f"n{c[0]}_L{c[1]}_sr{c[4]}")
def test_literal_tau_multicell_coarsest(dev, case):
    """Literal tau with a multi-cell coarsest grid: the two sides' coarsest
    solvers round differently and literal tau turns that into noise of its
    own size, so the bar is that noise as the oracle itself responds to a
    rounding-level perturbation of f (tests/parity_bars.py), per cell and in
    norm."""
    n, levels, S, b, sr, g = case
    print(f"literal multicell n={n} levels={levels} S={S} b={b} sr={sr}", flush=True)
    f_host = rhs(n, 40)
    kw = dict(g=g, levels=levels, segments=S, buffer=b, sr_levels=sr, tau="literal")
    u = gpu_solve(dev, f_host, **kw)
    ref = oracle_solve(f_host, **kw)
    bar_norm, bar_cell = literal_noise_bar(f_host, levels, S, b, nsr=sr, g=g)
    assert bar_norm < 1e-8 and bar_cell < 1e-8
    assert np.all(np.isfinite(u))
    assert np.linalg.norm(u - ref) <= bar_norm * np.linalg.norm(ref)
    assert np.abs(u - ref).max() <= bar_cell * np.abs(ref).max()
    print(f"  rel {np.linalg.norm(u - ref) / np.linalg.norm(ref):.2e} (bar {bar_norm:.2e})")


def test_repeatable_and_workspace_reuse(dev):
    n, levels = 1 << 14, 15
    f = torch.from_numpy(rhs(n, 30)).to(dev)
    ws = fmgsr.alloc_workspace(n, levels, dev)
    a = fmgsr.solve(f, levels=levels, segments=4, buffer=8, workspace=ws).clone()
    ws.fill_(255)                          # garbage in the workspace must not matter
    b = fmgsr.solve(f, levels=levels, segments=4, buffer=8, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # the exact size for these segments (no restricted fine iterate) suffices
    exact = fmgsr.alloc_workspace(n, levels, dev, segments=4, buffer=8)
    assert exact.numel() == ws.numel() - (n // 2) * 8
    exact.fill_(255)
    c = fmgsr.solve(f, levels=levels, segments=4, buffer=8, workspace=exact)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    with pytest.raises(fmgsr.FmgsrError):  # a smaller one is refused
        fmgsr.solve(f, levels=levels, segments=4, buffer=8, workspace=exact[:-256])


def test_side_stream(dev):
    n, levels = 1 << 12, 13
    f_host = rhs(n, 31)
    f = torch.from_numpy(f_host).to(dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u = fmgsr.solve(f, levels=levels, segments=4, buffer=4)
    s.synchronize()
    compare(u.cpu().numpy(), oracle_solve(f_host, levels=levels, segments=4, buffer=4), True)


def test_rejects_host_tensors_and_bad_sizes(dev):
    with pytest.raises(ValueError):
        fmgsr.solve(torch.zeros(16, dtype=torch.float64))
    f = torch.zeros(1000, dtype=torch.float64, device=dev)
    with pytest.raises(fmgsr.FmgsrError):
        fmgsr.solve(f, levels=11)
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(fmgsr.FmgsrError):
        fmgsr.solve(torch.zeros(1024, dtype=torch.float64, device=dev), levels=11,
                    segments=4, buffer=4, workspace=ws)


def test_workload_c2_full_size_parity(dev):
    """N = 2^24, 25 levels, 2^12 segments of 4096 + 8 buffer cells."""
    wl = W.WORKLOADS["c2"]
    k, c = W.modes(wl.law, wl.n_modes, 0)
    f = W.rhs_torch(wl.n, k, c, dev)
    print("c2: GPU solve", flush=True)
    u = fmgsr.solve(f, levels=wl.levels, segments=wl.segments, buffer=wl.buffer)
    torch.cuda.synchronize()
    f_host = f.cpu().numpy()
    print("c2: oracle solve", flush=True)
    u_ref = oracle_solve(f_host, levels=wl.levels, segments=wl.segments, buffer=wl.buffer)
    err = compare(u.cpu().numpy(), u_ref, bitwise=True)
    print(f"c2 parity rel = {err:.3e}", flush=True)


def test_workload_c2_two_sr_levels(dev):
    """N = 2^24 with the two finest levels as SR levels (2^12 segments of
    4096 and of 2048 cells, 8 buffer cells)."""
    wl = W.WORKLOADS["c2"]
    k, c = W.modes(wl.law, wl.n_modes, 1)
    f = W.rhs_torch(wl.n, k, c, dev)
    kw = dict(levels=wl.levels, segments=wl.segments, buffer=wl.buffer, sr_levels=2)
    print("c2, 2 SR levels: GPU solve", flush=True)
    u = fmgsr.solve(f, **kw)
    torch.cuda.synchronize()
    print("c2, 2 SR levels: oracle solve", flush=True)
    u_ref = oracle_solve(f.cpu().numpy(), **kw)
    err = compare(u.cpu().numpy(), u_ref, bitwise=True)
    print(f"c2 (2 SR levels) parity rel = {err:.3e}", flush=True)


@pytest.mark.timeout(900)
def test_workload_c5_full_size_parity(dev):
    """N = 2^28, 29 levels, 2^16 segments of 4096 + 8 buffer cells: the
    benchmark's workload and launch configuration, bitwise against the
    oracle over every cell (N0 = 1).  The oracle holds about 20 GB of host
    memory and runs for a few tens of seconds."""
    wl = W.WORKLOADS["c5"]
    k, c = W.modes(wl.law, wl.n_modes, 0)
    f = W.rhs_torch(wl.n, k, c, dev)
    print("c5: GPU solve", flush=True)
    u = fmgsr.solve(f, levels=wl.levels, segments=wl.segments, buffer=wl.buffer)
    torch.cuda.synchronize()
    f_host = f.cpu().numpy()
    u_gpu = u.cpu().numpy()
    del f, u
    torch.cuda.empty_cache()
    print("c5: oracle solve", flush=True)
    u_ref = oracle_solve(f_host, levels=wl.levels, segments=wl.segments, buffer=wl.buffer)
    del f_host
    err = compare(u_gpu, u_ref, bitwise=True)
    print(f"c5 parity rel = {err:.3e}", flush=True)


def closed_form_pair(n, k, c):
    """Discrete solution (sines are eigenvectors of the cell-centred
    Laplacian, eigenvalue 4 n^2 sin^2(k pi / 2n)) and the continuous one."""
    x = (np.arange(n) + 0.5) / n
    ustar = np.zeros(n)
    uex = np.zeros(n)
    for kk, cc in zip(k, c):
        s_ = np.sin(kk * np.pi * x)
        ustar += cc * (kk * np.pi) ** 2 / (4.0 * n * n * np.sin(kk * np.pi / (2 * n)) ** 2) * s_
        uex += cc * s_
    return ustar, uex


FP32_CASES = [
    (1 << 10, 11, 4, 4, "split", 0),
    (5 << 12, 13, 5, 8, "split", 1),      # N0 = 5
    (1 << 16, 17, 16, 8, "split", 2),
    (1 << 14, 15, 1, 0, "split", 3),      # plain FMG-FAS (sr_levels = 0 below)
]


@pytest.mark.parametrize("case", FP32_CASES, ids=lambda c: f"n{c[0]}_L{c[1]}_S{c[2]}_{c[4]}")
def test_fp32_relaxation_poisson_below_discretisation_error(dev, case):
    n, levels, S, b, tau, seed = case
    sr = 0 if S == 1 else 1
    k, c = W.modes("inv_k2", 16, seed)
    f = W.rhs_numpy(n, k, c)
    kw = dict(levels=levels, segments=S, buffer=b, sr_levels=sr, tau=tau)
    u32 = gpu_solve(dev, f, precision="fp32relax", **kw)
    u64 = gpu_solve(dev, f, **kw)
    ref = oracle_solve(f, **kw)
    ustar, uex = closed_form_pair(n, k, c)
    disc = np.linalg.norm(ustar - uex) / np.linalg.norm(uex)
    d32 = np.linalg.norm(u32 - ref) / np.linalg.norm(ref)
    print(f"n={n} disc={disc:.2e} fp32-vs-oracle={d32:.2e}", flush=True)
    compare(u64, ref, bitwise=(n >> (levels - 1)) == 1)
    assert d32 <= 0.1 * disc


def test_fp32_relaxation_c2_full_size(dev):
    wl = W.WORKLOADS["c2"]
    k, c = W.modes(wl.law, wl.n_modes, 0)
    f = W.rhs_torch(wl.n, k, c, dev)
    kw = dict(levels=wl.levels, segments=wl.segments, buffer=wl.buffer)
    u32 = fmgsr.solve(f, precision="fp32relax", **kw)
    u64 = fmgsr.solve(f, **kw)
    torch.cuda.synchronize()
    d = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    print(f"c2 fp32 vs fp64 relaxation: {d:.2e}", flush=True)
    assert d <= 7e-15   # a tenth of this workload's discretisation error (6.9e-14)


def fsum_functionals(u):
    import math
    n = u.size
    return np.array([math.fsum(u) / n, math.fsum(u * u) / n])


FUNC_CASES = [
    (1 << 10, 11, 4, 4, (0.0, 0.0), 0),
    (5 << 12, 13, 5, 8, (0.3, -0.4), 1),
    (1 << 14, 15, 4096, 2, (0.0, 0.0), 2),   # 4-cell segment cores
]


@pytest.mark.parametrize("case", FUNC_CASES, ids=lambda c: f"n{c[0]}_S{c[2]}")
def test_functionals_on_the_fly(dev, case):
    """h sum u and h sum u^2 accumulated by the SR up pass (fixed order)
    against the oracle's solution summed exactly; the functional-only solve
    (u_out = NULL) gives the same bits."""
    n, levels, S, b, g, seed = case
    f_host = rhs(n, seed)
    f = torch.from_numpy(f_host).to(dev)
    fun = torch.zeros(2, dtype=torch.float64, device=dev)
    u = fmgsr.solve(f, g=g, levels=levels, segments=S, buffer=b, functionals=fun)
    fun_only = torch.zeros(2, dtype=torch.float64, device=dev)
    fmgsr.solve(f, g=g, levels=levels, segments=S, buffer=b, functionals=fun_only, write_u=False)
    torch.cuda.synchronize()
    ref = fsum_functionals(oracle_solve(f_host, g=g, levels=levels, segments=S, buffer=b))
    got = fun.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref)), (got, ref)
    assert torch.equal(fun, fun_only)
    assert np.allclose(fsum_functionals(u.cpu().numpy()), got, rtol=1e-14, atol=0)


def test_functionals_rejections(dev):
    f = torch.zeros(1 << 10, dtype=torch.float64, device=dev)
    fun = torch.zeros(2, dtype=torch.float64, device=dev)
    with pytest.raises(fmgsr.FmgsrError):      # no SR level
        fmgsr.solve(f, levels=11, sr_levels=0, functionals=fun)
    with pytest.raises(fmgsr.FmgsrError):      # 2-cell segment cores
        fmgsr.solve(f, levels=11, segments=512, buffer=2, functionals=fun)


def test_functionals_c2_functional_only(dev):
    """N = 2^24 with the fine solution never written."""
    wl = W.WORKLOADS["c2"]
    k, c = W.modes(wl.law, wl.n_modes, 0)
    f = W.rhs_torch(wl.n, k, c, dev)
    fun = torch.zeros(2, dtype=torch.float64, device=dev)
    fmgsr.solve(f, levels=wl.levels, segments=wl.segments, buffer=wl.buffer, functionals=fun,
                write_u=False)
    torch.cuda.synchronize()
    ref = fsum_functionals(oracle_solve(f.cpu().numpy(), levels=wl.levels, segments=wl.segments,
                                        buffer=wl.buffer))
    got = fun.cpu().numpy()
    print("c2 functionals", got, ref, flush=True)
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref))


def test_binding_checks_extents_before_calling_the_library(dev):
    """Short, float32 or misplaced arrays never reach the C ABI (which cannot
    see extents): each raises ValueError in the binding."""
    n = 1 << 10
    f = torch.zeros(n, dtype=torch.float64, device=dev)
    short = torch.zeros(n - 1, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        fmgsr.solve(f, levels=11, segments=4, buffer=4, out=short)
    with pytest.raises(ValueError):
        fmgsr.solve(f, levels=11, segments=4, buffer=4, op="cubic", kappa=short)
    with pytest.raises(ValueError):
        fmgsr.solve(f, levels=11, segments=4, buffer=4, op="cubic",
                    kappa=torch.ones(n, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        fmgsr.solve(f, levels=11, segments=4, buffer=4, op="cubic")    # kappa missing
    with pytest.raises(ValueError):
        fmgsr.solve(f, levels=11, kappa=f)                             # kappa for poisson
    with pytest.raises(ValueError):
        fmgsr.adjoint(f, f, short, levels=11, segments=4)
    with pytest.raises(ValueError):
        fmgsr.adjoint(f, f, f, levels=11, segments=4, u_fwd=short)
    plan = fmgsr.Batch((n, n), (6, 6), buffer=8, op="cubic")
    both = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        plan.solve(both[:-1], both)                                    # f short
    with pytest.raises(ValueError):
        plan.solve(both, both[: n])                                    # kappa short
    with pytest.raises(ValueError):
        plan.solve(both, None)                                         # kappa missing
    with pytest.raises(ValueError):
        plan.adjoint(both, both[:-1], both)                            # u_fwd short
    with pytest.raises(ValueError):
        plan.adjoint(both, both, both, grad_kappa=both.float())        # float32 gradient
    with pytest.raises(ValueError):
        plan.autotune(both, both, scratch=both[:-1])
    pois = fmgsr.Batch((n,), (6,), buffer=8, op="poisson")
    with pytest.raises(ValueError):
        pois.adjoint(f, f, f)                                          # adjoint of poisson
