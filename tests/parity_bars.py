"""Parity bars that the arithmetic sets, computed with the oracle alone.

Literal tau (Eq. 7 evaluated as written) forms I(L_h u) and L_H(I^ u), two
O(n^2 |u|) terms that cancel exactly; its value is rounding noise whose bits
depend on every bit of the iterate.  Two correct implementations that round
anything differently (with a multi-cell coarsest grid the GPU's parallel
cyclic reduction and the oracle's Thomas sweep do) therefore agree only to
the size of that noise mapped through the cycle, not to 1e-12.  The bar is
measured, per case, as the oracle's own response to a perturbation of f at
the rounding level (4e-16 relative per cell, below anything the method
resolves), times a safety factor of 10, and never below the FP64 bar of
1e-12.  With split tau the same response is ~1e-16 and the bar stays 1e-12
(tests/test_oracle_pins.py::test_literal_tau_results_carry_rounding_noise).
"""
import numpy as np

import oracle

FP64_BAR = 1e-12


def literal_noise_bar(f, levels, segments, buffer, nu=(2, 1), nsr=1, rhs_restrict="fw",
                      g=(0.0, 0.0), factor=10.0):
    """(norm bar, per-cell bar), both relative, for a literal-tau solve of f."""
    rng = np.random.default_rng(3)
    f2 = f * (1.0 + 4e-16 * rng.standard_normal(f.size))
    kw = dict(levels=levels, segments=segments, buffer=buffer, nu1=nu[0], nu2=nu[1], nsr=nsr,
              tau="literal", rhs_restrict=rhs_restrict)
    a = oracle.fmgsr_solve(f, g[0], g[1], **kw)
    b = oracle.fmgsr_solve(f2, g[0], g[1], **kw)
    norm = np.linalg.norm(a - b) / np.linalg.norm(a)
    cell = np.abs(a - b).max() / np.abs(a).max()
    return max(FP64_BAR, factor * norm), max(FP64_BAR, factor * cell)
