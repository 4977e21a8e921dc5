"""Pins of the reaction-operator oracle (-u'' + kappa u^3 = f, -u'' + c u = f)
and of its adjoint, against facts that do not come from the oracle itself:

* the discrete equations N(u) = f, evaluated here from their definition;
* the manufactured continuous solution (second-order convergence);
* the real root of the one-cell cubic;
* the closed-form discrete solution of the constant-coefficient linear
  reaction problem (sines are eigenvectors of L);
* the fixed point of the FAS V-cycle (a wrong tau moves it);
* the Poisson oracle (kappa = 0 must reproduce it bit for bit);
* central finite differences of the least-squares functional.
"""
import numpy as np
import pytest

import oracle
from paper_1207_6720_amd import workloads as W


def n_apply(kind, a, u, gL=0.0, gR=0.0):
    """N(u) from the definition: cell-centred Laplacian with odd-reflection
    ghosts plus the reaction term."""
    n = u.size
    ue = np.concatenate([[2 * gL - u[0]], u, [2 * gR - u[-1]]])
    lap = (2 * u - ue[:-2] - ue[2:]) * n * n
    if kind == "cubic":
        return lap + a * u ** 3
    if kind == "linear":
        return lap + a * u
    return lap


def problem(n, j=3, seed=0):
    return W.reaction_problem_numpy(n, seed, j)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --------------------------------------------------------------------------
# Newton and the discrete problem
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 63 * 8])
def test_newton_solves_the_discrete_equations(n):
    f, k, _, _ = problem(max(n, 1))
    for g in [(0.0, 0.0), (0.3, -0.7)]:
        u, it = oracle.rx_newton("cubic", k, f, *g)
        r = n_apply("cubic", k, u, *g) - f
        scale = np.abs(f).max() + n * n * np.abs(u).max()
        assert np.abs(r).max() <= 1e-13 * scale
        assert it <= 30


def test_newton_one_cell_is_the_cubic_root():
    # one cell, h = 1: 4 u + kappa u^3 = F + 2 gL + 2 gR
    for kap, F, gL, gR in [(1.0, 3.0, 0.0, 0.0), (0.5, -7.0, 0.2, 0.4), (1.5, 40.0, -1.0, 2.0)]:
        u, _ = oracle.rx_newton("cubic", np.array([kap]), np.array([F]), gL, gR)
        roots = np.roots([kap, 0.0, 4.0, -(F + 2 * gL + 2 * gR)])
        real = roots[np.abs(roots.imag) < 1e-12].real
        assert real.size == 1
        assert abs(u[0] - real[0]) <= 1e-14 * max(1.0, abs(real[0]))


def test_discretisation_is_second_order():
    errs = []
    for n in [64, 128, 256, 512]:
        f, k, uex, _ = problem(n)
        u, _ = oracle.rx_newton("cubic", k, f)
        errs.append(np.sqrt(np.mean((u - uex) ** 2)))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < q < 4.4 for q in ratios), ratios


@pytest.mark.parametrize("kind", ["cubic", "linear"])
def test_ngs_fixed_point_is_the_discrete_solution(kind):
    n = 16
    f, k, _, _ = problem(n)
    u = np.zeros(n)
    for _ in range(3000):
        u = oracle.rx_ngs_sweep(kind, k, u, f, gL=0.1, gR=-0.2)
    r = n_apply(kind, k, u, 0.1, -0.2) - f
    assert np.abs(r).max() <= 1e-10 * np.abs(f).max()


def test_ngs_respects_the_cell_range():
    n = 32
    f, k, _, _ = problem(n)
    u0 = np.linspace(-1, 1, n)
    u = oracle.rx_ngs_sweep("cubic", k, u0, f, lo=5, hi=20)
    assert np.array_equal(u[:5], u0[:5]) and np.array_equal(u[20:], u0[20:])
    assert not np.array_equal(u[5:20], u0[5:20])


def test_linear_kind_constant_coefficient_closed_form():
    n, c, kk = 256, 7.5, 3
    x = (np.arange(n) + 0.5) / n
    f = np.sin(kk * np.pi * x)
    lam = 4.0 * n * n * np.sin(kk * np.pi / (2 * n)) ** 2
    ustar = f / (lam + c)
    u, _ = oracle.rx_newton("linear", np.full(n, c), f)
    assert rel(u, ustar) <= 1e-12
    v = oracle.rx_fmgsr_solve("linear", f, np.full(n, c), levels=9, segments=4, buffer=4)
    for _ in range(12):
        v = oracle.rx_fas_vcycle("linear", v, f, np.full(n, c), levels=9)
    assert rel(v, ustar) <= 1e-12


# --------------------------------------------------------------------------
# FMG-FAS-SR
# --------------------------------------------------------------------------

def test_kappa_zero_reproduces_the_poisson_oracle_bitwise():
    n = 1024
    f = W.rhs_numpy(n, *W.modes("inv_k2", 8, 1))
    for S, b, nsr, tau in [(4, 4, 1, "split"), (1, 0, 0, "split"), (16, 2, 1, "literal")]:
        ref = oracle.fmgsr_solve(f, 0.1, -0.3, levels=11, segments=S, buffer=b, nsr=nsr, tau=tau)
        a = oracle.rx_fmgsr_solve("cubic", f, np.zeros(n), 0.1, -0.3, levels=11, segments=S,
                                  buffer=b, nsr=nsr, tau=tau)
        p = oracle.rx_fmgsr_solve("poisson", f, None, 0.1, -0.3, levels=11, segments=S,
                                  buffer=b, nsr=nsr, tau=tau)
        assert np.array_equal(a, ref) and np.array_equal(p, ref)


CASES = [(1, 10), (39, 7), (63, 6), (32, 9), (45, 8)]


@pytest.mark.parametrize("n0,L", CASES)
def test_one_fmgsr_iteration_reaches_discretisation_error(n0, L):
    n = n0 << L
    f, k, uex, _ = problem(n)
    ustar, _ = oracle.rx_newton("cubic", k, f)
    s = n0 << max(L - 4, 1)
    u = oracle.rx_fmgsr_solve("cubic", f, k, levels=L + 1, segments=n // s, buffer=8)
    alg, disc = rel(u, ustar), rel(ustar, uex)
    assert alg < 0.2 * disc, (alg, disc)


@pytest.mark.parametrize("n0,L", [(1, 10), (39, 6), (63, 5)])
def test_vcycle_fixed_point_is_the_newton_solution(n0, L):
    """FAS keeps the fine solution fixed only if tau is right."""
    n = n0 << L
    f, k, _, _ = problem(n)
    ustar, _ = oracle.rx_newton("cubic", k, f)
    u = np.zeros(n)
    for _ in range(25):
        u = oracle.rx_fas_vcycle("cubic", u, f, k, levels=L + 1)
    assert rel(u, ustar) <= 1e-11
    # literal tau has the same fixed point
    v = np.zeros(n)
    for _ in range(25):
        v = oracle.rx_fas_vcycle("cubic", v, f, k, levels=L + 1, tau="literal")
    assert rel(v, ustar) <= 1e-11


def test_literal_tau_agrees_with_split():
    for n0, L in [(1, 8), (39, 5), (1, 11)]:
        n = n0 << L
        f, k, _, _ = problem(n)
        a = oracle.rx_fmgsr_solve("cubic", f, k, levels=L + 1, segments=4, buffer=8)
        b = oracle.rx_fmgsr_solve("cubic", f, k, levels=L + 1, segments=4, buffer=8, tau="literal")
        assert rel(b, a) <= 1e-13 * n


@pytest.mark.parametrize("nu1", [1, 2, 3])
def test_per_patch_tau_equals_assembled_when_the_buffer_covers_its_reach(nu1):
    """Per-patch tau on the SR level (Fig. 3 step 4, from each segment's
    extended iterate) against tau assembled from the global iterate.  The
    split reaction tau I(kappa u^3) reads one fine cell beyond the core's
    pairs, and the block smoother's patch equals the global red-black
    iterate up to 2 nu1 - 1 cells in from the patch edge, so the two agree
    bit for bit exactly when b >= 2 nu1; one cell less and they differ.
    Literal tau (Eq. 7) also applies L_h there, reaching two cells beyond
    the core: bitwise from b = 2 nu1 + 1.  The forcing is rough (seeded
    normal values) so that a one-ulp difference in a patch cell is not
    absorbed by the rounding of the restriction, as it can be for a smooth
    one."""
    n0, L = 39, 6
    n = n0 << L
    _, k, _, _ = problem(n, j=4)
    f = np.random.default_rng(5).normal(size=n) * 1e4
    kw = dict(levels=L + 1, segments=8, nu1=nu1, nu2=1)
    for tau, need in (("split", 2 * nu1), ("literal", 2 * nu1 + 1)):
        for b, equal in ((need, True), (need + 3, True), (need - 1, False), (0, False)):
            patch = oracle.rx_fmgsr_solve("cubic", f, k, buffer=b, tau=tau, **kw)
            glob = oracle.rx_fmgsr_solve("cubic", f, k, buffer=b, tau=tau, tau_assembled=True,
                                         **kw)
            assert np.array_equal(patch, glob) == equal, (tau, b)
            assert rel(patch, glob) <= 1e-6


def test_segment_order_does_not_matter():
    n = 39 << 6
    f, k, _, _ = problem(n)
    kw = dict(levels=7, segments=6, buffer=3)
    a = oracle.rx_fmgsr_solve("cubic", f, k, order=0, **kw)
    b = oracle.rx_fmgsr_solve("cubic", f, k, order=1, **kw)
    assert np.array_equal(a, b)


def test_segments_change_the_result_only_slightly():
    n = 1 << 11
    f, k, _, _ = problem(n)
    ustar, _ = oracle.rx_newton("cubic", k, f)
    plain = oracle.rx_fmgsr_solve("cubic", f, k, levels=12, nsr=0)
    sr = oracle.rx_fmgsr_solve("cubic", f, k, levels=12, segments=64, buffer=2)
    assert not np.array_equal(plain, sr)
    assert rel(sr, ustar) < 3 * rel(plain, ustar) + 1e-12


# --------------------------------------------------------------------------
# Kept level-(M-1) solution (PDE compression, Sec. 2.4)
# --------------------------------------------------------------------------

def test_kept_level_with_kappa_zero_is_the_poisson_oracles():
    n = 1024
    f = W.rhs_numpy(n, *W.modes("inv_k2", 8, 2))
    kw = dict(levels=11, segments=8, buffer=4)
    u_ref, c_ref = oracle.fmgsr_solve_keep(f, 0.2, -0.1, **kw)
    u, c = oracle.rx_fmgsr_solve_keep("cubic", f, np.zeros(n), 0.2, -0.1, **kw)
    assert np.array_equal(u, u_ref) and np.array_equal(c, c_ref)
    assert np.array_equal(u, oracle.rx_fmgsr_solve("cubic", f, np.zeros(n), 0.2, -0.1, **kw))


@pytest.mark.parametrize("n0,L,S,b", [(1, 9, 8, 4), (39, 6, 6, 3), (5, 8, 4, 1), (3, 2, 1, 2)])
def test_kept_level_regenerates_the_solution(n0, L, S, b):
    """Sec. 2.4: the finest level follows from the kept level and f alone.
    Rebuilt here from the oracle's primitives (Pi of the kept level, then
    per extended patch nu2 x [Kaczmarz onto the kept level, one nonlinear
    sweep], Eq. 5 and Fig. 5), it must equal the iteration's own result."""
    n = n0 << (L - 1)
    f, k, _, _ = problem(n, seed=n0)
    gL, gR = 0.3, -0.2
    u, c = oracle.rx_fmgsr_solve_keep("cubic", f, k, gL, gR, levels=L, segments=S, buffer=b)
    assert c.size == n // 2
    v = oracle.interp_fmg(c, gL, gR)
    s = n // S
    out = np.empty(n)
    for i in range(S):
        lo, hi = max(i * s - b, 0), min((i + 1) * s + b, n)
        w = v.copy()
        for _ in range(1):  # nu2 = 1
            w = oracle.kaczmarz(w, c, lo, hi)
            w = oracle.rx_ngs_sweep("cubic", k, w, f, lo, hi, gL, gR)
        out[i * s:(i + 1) * s] = w[i * s:(i + 1) * s]
    assert np.array_equal(out, u)
    # a different kept level gives a different fine level (the check is live)
    v2 = oracle.interp_fmg(c * (1 + 1e-9), gL, gR)
    w = oracle.rx_ngs_sweep("cubic", k, oracle.kaczmarz(v2, c, 0, min(s + b, n)), f, 0,
                            min(s + b, n), gL, gR)
    assert not np.array_equal(w[:s], u[:s])


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------

def loss_and_target(n, j=5):
    f, k, _, ut = problem(n, j)
    h = 1.0 / n

    def J(ff, kk):
        u, _ = oracle.rx_newton("cubic", kk, ff)
        return h * np.sum((u - ut) ** 2)
    u, _ = oracle.rx_newton("cubic", k, f)
    return f, k, u, ut, h, J


def test_direct_adjoint_solves_the_transposed_linearised_system():
    n = 200
    f, k, u, ut, h, _ = loss_and_target(n)
    g = 2 * h * (u - ut)
    gf, gk = oracle.rx_adjoint_direct(k, u, g)
    c = 3 * k * u ** 2
    r = n_apply("linear", c, gf) - g
    assert np.abs(r).max() <= 1e-12 * (np.abs(g).max() + n * n * np.abs(gf).max())
    assert np.allclose(gk, -(u ** 3) * gf, rtol=4e-16, atol=0)


def test_direct_adjoint_matches_central_differences():
    """eps = 1e-6 relative to each field's size (directions scaled by max|f|,
    max|kappa|), so the differences stay above the solves' rounding floor."""
    n = 256
    f, k, u, ut, h, J = loss_and_target(n)
    gf, gk = oracle.rx_adjoint_direct(k, u, 2 * h * (u - ut))
    rng = np.random.default_rng(11)
    eps = 1e-6
    for _ in range(6):
        df = rng.normal(size=n) * np.abs(f).max()
        dk = rng.normal(size=n) * np.abs(k).max()
        fd_f = (J(f + eps * df, k) - J(f - eps * df, k)) / (2 * eps)
        fd_k = (J(f, k + eps * dk) - J(f, k - eps * dk)) / (2 * eps)
        assert abs(fd_f - gf @ df) <= 1e-4 * abs(fd_f)
        assert abs(fd_k - gk @ dk) <= 1e-4 * abs(fd_k)


def test_fmgsr_adjoint_converges_to_the_direct_adjoint():
    errs = []
    for L in [7, 8, 9, 10]:
        n = 1 << L
        f, k, u, ut, h, _ = loss_and_target(n)
        g = 2 * h * (u - ut)
        gf, gk = oracle.rx_adjoint_direct(k, u, g)
        af, ak = oracle.rx_fmgsr_adjoint(k, u, g, levels=L + 1, segments=4, buffer=8)
        errs.append(rel(af, gf))
        assert rel(ak, gk) <= 1e-3
    assert errs[-1] <= 1e-5
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(len(errs) - 1)), errs
