"""Pins of the oracle's PDE decompression (Sec. 3.2, method 2): the fine
solution expanded on demand from the stored level-(M-1) solution and f.

- A dense-matrix transcription (tests/dense_reference.py, built from the
  appendix's printed operator entries) gives the same level-(M-1) solution
  and the same expansion.
- Expanding any range reproduces the solve's finest level on it bit for
  bit: the expansion is the final step of the cycle (Eq. 5, Fig. 5), so a
  dropped segment, a shifted range or a wrong Kaczmarz target shows.
- The expansion is local: coarse cells beyond the covering segments' patches
  (plus the interpolation stencil) do not affect it; cells inside do.
- Without compatible relaxation (nu2 = 0) it is the FMG interpolation.
"""
import numpy as np
import pytest

import oracle
from paper_1207_6720_amd import workloads as W
from tests import dense_reference as D

RNG = np.random.default_rng(7)


def _f(n, seed):
    k, c = W.modes("inv_k2", 16, seed, n)
    return W.rhs_numpy(n, k, c)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("tau", ["split", "literal"])
@pytest.mark.parametrize("S,b", [(4, 3), (8, 1)])
def test_keep_and_decompress_match_dense_brute_force(tau, S, b):
    n, levels = 64, 5
    f = _f(n, 1)
    u, c = oracle.fmgsr_solve_keep(f, levels=levels, segments=S, buffer=b, tau=tau,
                                   tau_assembled=True)
    ref_u, ref_c = D.fmgsr(f, levels, S, b, tau=tau, keep_coarse=True)
    assert rel(u, ref_u) < 1e-11
    assert rel(c, ref_c) < 1e-11
    for lo, hi in ((0, n), (5, 29), (16, 17), (63, 64)):
        d = oracle.fmgsr_decompress(ref_c, f, lo, hi, segments=S, buffer=b)
        assert rel(d, D.decompress(ref_c, f, lo, hi, S, b)) < 1e-13


CONFIGS = [
    # n, levels, S, b, nu, nsr, tau, g
    (1 << 10, 11, 4, 4, (2, 1), 1, "split", (0.0, 0.0)),
    (1 << 12, 13, 16, 8, (2, 1), 1, "split", (0.3, -0.7)),
    (1 << 12, 13, 16, 1, (2, 1), 1, "split", (0.0, 0.0)),     # b < 2 nu2: edges reach cores
    (1 << 12, 13, 8, 5, (3, 2), 1, "literal", (0.0, 1.0)),
    (5 << 10, 11, 5, 8, (2, 1), 1, "split", (0.0, 0.0)),      # N0 = 5
    (1 << 12, 13, 8, 4, (2, 1), 2, "split", (0.0, 0.0)),      # two SR levels
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: f"n{c[0]}_S{c[2]}_b{c[3]}_nsr{c[5]}_{c[6]}")
def test_decompression_reproduces_the_solve(cfg):
    n, levels, S, b, nu, nsr, tau, g = cfg
    f = _f(n, 3)
    kw = dict(levels=levels, segments=S, buffer=b, nu1=nu[0], nu2=nu[1], nsr=nsr, tau=tau)
    u, c = oracle.fmgsr_solve_keep(f, g[0], g[1], **kw)
    assert np.array_equal(u, oracle.fmgsr_solve(f, g[0], g[1], **kw))
    dk = dict(gL=g[0], gR=g[1], segments=S, buffer=b, nu1=nu[0], nu2=nu[1])
    s = n // S
    ranges = [(0, n), (0, 1), (n - 1, n), (0, s), (s, 2 * s), (s - 3, s + 3), (7, 7)]
    for _ in range(6):
        lo = int(RNG.integers(0, n))
        ranges.append((lo, int(RNG.integers(lo, n + 1))))
    for lo, hi in ranges:
        d = oracle.fmgsr_decompress(c, f, lo, hi, **dk)
        assert d.shape == (hi - lo,)
        assert np.array_equal(d, u[lo:hi]), (lo, hi)


def test_decompression_is_local():
    n, S, b = 1 << 12, 16, 8
    s = n // S
    f = _f(n, 4)
    _, c = oracle.fmgsr_solve_keep(f, levels=13, segments=S, buffer=b)
    lo, hi = 5 * s + 10, 7 * s - 10          # cores of segments 5 and 6
    base = oracle.fmgsr_decompress(c, f, lo, hi, segments=S, buffer=b)
    # the covering patches span fine cells [5 s - b, 7 s + b); with the
    # interpolation's two coarse cells of reach, coarse cells outside
    # [(5 s - b) / 2 - 2, (7 s + b) / 2 + 2) cannot matter
    reach_lo, reach_hi = (5 * s - b) // 2 - 2, (7 * s + b) // 2 + 2
    for J in (0, reach_lo - 1, reach_hi, n // 2 - 1):
        c2 = c.copy()
        c2[J] += 1.0
        assert np.array_equal(oracle.fmgsr_decompress(c2, f, lo, hi, segments=S, buffer=b), base)
    for J in (lo // 2 + 1, (lo + hi) // 4, hi // 2 - 2):   # coarse cells under the range
        c2 = c.copy()
        c2[J] += 1.0
        assert not np.array_equal(oracle.fmgsr_decompress(c2, f, lo, hi, segments=S, buffer=b),
                                  base), J


def test_decompression_without_relaxation_is_fmg_interpolation():
    n = 1 << 10
    c = RNG.standard_normal(n // 2)
    f = RNG.standard_normal(n)
    d = oracle.fmgsr_decompress(c, f, 0, n, 0.2, -0.4, segments=4, buffer=4, nu2=0)
    assert np.array_equal(d, oracle.interp_fmg(c, 0.2, -0.4))
    # cubic data on the coarse cell centres is interpolated exactly
    xc = (np.arange(n // 2) + 0.5) / (n // 2)
    xf = (np.arange(n) + 0.5) / n
    cub = lambda x: 1.0 + x - 3 * x ** 2 + 2 * x ** 3  # noqa: E731
    d = oracle.fmgsr_decompress(cub(xc), f, 100, 900, 1.0, 1.0, segments=8, buffer=2, nu2=0)
    assert np.abs(d - cub(xf[100:900])).max() < 1e-13


def test_decompress_rejects_bad_ranges():
    c, f = np.zeros(32), np.zeros(64)
    for lo, hi in ((-1, 4), (4, 65), (10, 9)):
        with pytest.raises(ValueError):
            oracle.fmgsr_decompress(c, f, lo, hi, segments=4, buffer=2)
    with pytest.raises(ValueError):
        oracle.fmgsr_decompress(c, f, 0, 8, segments=3, buffer=2)   # 3 does not divide 64
