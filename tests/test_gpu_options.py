"""GPU tests of two options of fmgsr_solve, through the C ABI:

- the paper's own rhs restriction (two-cell average, the appendix's choice;
  literal tau), against the oracle run with the same transfer pair: bitwise
  with a single-cell coarsest grid; otherwise within the literal-tau noise
  bar of tests/parity_bars.py (per cell and in norm);
- check_finite: a NaN or Inf in f is refused with FMGSR_ENONFINITE before
  anything is solved, a non-finite result is reported after the solve, and
  a finite problem gives the same bits with and without the check.
"""
import ctypes

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


def rhs(n, seed):
    k, c = W.modes("inv_k2", 16, seed, n)
    return W.rhs_numpy(n, k, c)


def compare(a, ref, bitwise, bars=(TOL, TOL)):
    assert np.all(np.isfinite(a))
    assert np.linalg.norm(a - ref) <= bars[0] * np.linalg.norm(ref)
    assert np.abs(a - ref).max() <= bars[1] * np.abs(ref).max()
    if bitwise:
        nbad = int(np.count_nonzero(a != ref))
        assert nbad == 0, f"{nbad} cells differ"


# n, levels, segments, buffer, nu, sr_levels, g, seed
AVG_CASES = [
    (1 << 10, 11, 4, 4, (2, 1), 1, (0.0, 0.0), 0),
    (1 << 14, 15, 16, 8, (2, 1), 1, (0.25, -0.5), 1),     # several tiles per level
    (1 << 12, 13, 8, 1, (2, 1), 1, (0.0, 0.0), 2),        # thin buffer, per-patch tau
    (1 << 16, 17, 1, 0, (2, 1), 0, (0.0, 1.0), 3),        # plain FMG-FAS
    (1 << 12, 13, 16, 6, (1, 1), 1, (0.0, 0.0), 4),       # V(1,1) as in the paper's runs
    (5 << 10, 11, 5, 8, (2, 1), 1, (0.0, 0.0), 5),        # N0 = 5
]


@pytest.mark.parametrize("case", AVG_CASES, ids=lambda c: f"n{c[0]}_S{c[2]}_b{c[3]}_sr{c[5]}")
def test_average_rhs_restriction_matches_oracle(dev, case):
    n, levels, S, b, nu, sr, g, seed = case
    print(f"avg case n={n} levels={levels} S={S} b={b} nu={nu} sr={sr}", flush=True)
    f_host = rhs(n, seed)
    f = torch.from_numpy(f_host).to(dev)
    u = fmgsr.solve(f, g=g, levels=levels, segments=S, buffer=b, nu=nu, sr_levels=sr,
                    tau="literal", rhs_restrict="avg")
    torch.cuda.synchronize()
    ref = oracle.fmgsr_solve(f_host, g[0], g[1], levels=levels, segments=S, buffer=b,
                             nu1=nu[0], nu2=nu[1], nsr=sr, tau="literal", rhs_restrict="avg")
    single = (n >> (levels - 1)) == 1
    # a multi-cell coarsest grid is solved differently on the two sides, and
    # literal tau turns that rounding into noise of its own size
    bars = (TOL, TOL) if single else literal_noise_bar(f_host, levels, S, b, nu, sr, "avg", g)
    compare(u.cpu().numpy(), ref, bitwise=single, bars=bars)
    # the transfer pair matters: full weighting gives another iterate
    u_fw = fmgsr.solve(f, g=g, levels=levels, segments=S, buffer=b, nu=nu, sr_levels=sr,
                       tau="literal")
    torch.cuda.synchronize()
    assert not torch.equal(u, u_fw)


def test_average_rhs_restriction_needs_literal_tau(dev):
    f = torch.zeros(1024, dtype=torch.float64, device=dev)
    with pytest.raises(fmgsr.FmgsrError) as e:
        fmgsr.solve(f, levels=11, segments=4, buffer=4, rhs_restrict="avg")
    assert e.value.status == fmgsr.FMGSR_EINVAL


def test_check_finite(dev):
    n, levels, S, b = 1 << 14, 15, 16, 8
    f_host = rhs(n, 7)
    f = torch.from_numpy(f_host).to(dev)
    kw = dict(levels=levels, segments=S, buffer=b)
    ref = fmgsr.solve(f, **kw)
    out = torch.full_like(f, 3.0)
    fmgsr.solve(f, out=out, check_finite=True, **kw)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    c = torch.empty(n // 2, dtype=torch.float64, device=dev)
    fmgsr.solve(f, coarse_out=c, write_u=False, check_finite=True, **kw)
    for bad in (float("nan"), float("inf"), float("-inf")):
        fb = f.clone()
        fb[n // 3] = bad
        out.fill_(3.0)
        with pytest.raises(fmgsr.FmgsrError) as e:
            fmgsr.solve(fb, out=out, check_finite=True, **kw)
        assert e.value.status == fmgsr.FMGSR_ENONFINITE
        torch.cuda.synchronize()
        assert bool((out == 3.0).all())  # nothing was solved
    # finite input whose result overflows: boundary values near the largest double
    with pytest.raises(fmgsr.FmgsrError) as e:
        fmgsr.solve(f, g=(1e308, 1e308), out=out, check_finite=True, **kw)
    assert e.value.status == fmgsr.FMGSR_ENONFINITE
    torch.cuda.synchronize()


def test_check_finite_rejects_other_values_on_host(dev):
    f = torch.zeros(1024, dtype=torch.float64, device=dev)
    u = torch.empty_like(f)
    o = fmgsr.make_options()
    o.check_finite = 2
    st = fmgsr.lib().fmgsr_solve(None, f.data_ptr(), 0.0, 0.0, 1024, 11, 4, 4, ctypes.byref(o),
                                 u.data_ptr(), None)
    assert st == fmgsr.FMGSR_EINVAL
