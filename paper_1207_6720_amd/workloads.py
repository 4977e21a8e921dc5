"""Seeded synthetic inputs for the 1D model problem -u'' = f on [0,1].

This module only *generates data*: manufactured sine-series solutions and
their exact forcing at cell centres.  It contains none of the solver's
arithmetic and is shared by the tests, the benchmark and the smoke check so
that the HIP path and the CPU oracle receive the same bits.

Workloads (all FP64, Dirichlet data u(0) = u(1) = 0 unless stated):

* ``c1``  N = 2^10, 11 levels, 4 segments, buffer 4;
  u = sin(pi x) + sum_{k=1..8} a_k sin(k pi x), a_k ~ Normal(0, sd 0.1).
* ``c2``  N = 2^24, 25 levels, 2^12 segments of 4096 cells, buffer 8;
  16 modes, a_k ~ Normal(0, sd 1/k^2).
* ``c5``  N = 2^28, 29 levels, 2^16 segments of 4096 cells, buffer 8;
  32 modes, a_k ~ Normal(0, sd 1/k^2).
* ``paper`` the convergence-study forcing of the paper's numerical section:
  f = sum over odd j <= N/16 of sin(j pi x) / j.

For u = sum_k c_k sin(k pi x) the forcing is f = sum_k c_k (k pi)^2 sin(k pi x),
point-sampled at the cell centres x_i = (i + 1/2)/N.
"""
from dataclasses import dataclass

import numpy as np

__all__ = ["Workload", "WORKLOADS", "modes", "rhs_numpy", "exact_numpy",
           "rhs_torch", "exact_torch", "cell_centres"]


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    levels: int
    segments: int
    buffer: int
    n_modes: int
    law: str  # "c1" | "inv_k2" | "paper"

    @property
    def description(self) -> str:
        return (f"1D Poisson N=2^{int(np.log2(self.n))}, {self.levels} levels, "
                f"SR {self.segments} segments x {self.n // self.segments} cells + "
                f"{self.buffer} buffer, V(2,1) red-black, FP64")


WORKLOADS = {
    "c1": Workload("c1", 1 << 10, 11, 4, 4, 8, "c1"),
    "c2": Workload("c2", 1 << 24, 25, 1 << 12, 8, 16, "inv_k2"),
    "c5": Workload("c5", 1 << 28, 29, 1 << 16, 8, 32, "inv_k2"),
}


def modes(law: str, n_modes: int, seed: int, n: int = 0):
    """Return (k, c_k) of the manufactured solution u = sum c_k sin(k pi x)."""
    if law == "paper":
        k = np.arange(1, max(n // 16, 1) + 1, 2, dtype=np.float64)
        # u'' = -f with f = sin(j pi x)/j  =>  c_j = 1 / (j (j pi)^2)
        return k, 1.0 / (k * (k * np.pi) ** 2)
    rng = np.random.default_rng(seed)
    k = np.arange(1, n_modes + 1, dtype=np.float64)
    if law == "c1":
        c = rng.normal(0.0, 0.1, size=n_modes)
        c[0] += 1.0
    elif law == "inv_k2":
        c = rng.normal(0.0, 1.0, size=n_modes) / k ** 2
    else:
        raise ValueError(law)
    return k, c


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def rhs_numpy(n: int, k, c) -> np.ndarray:
    x = cell_centres(n)
    f = np.zeros(n)
    for kk, cc in zip(k, c):
        f += cc * (kk * np.pi) ** 2 * np.sin(kk * np.pi * x)
    return f


def exact_numpy(n: int, k, c) -> np.ndarray:
    x = cell_centres(n)
    u = np.zeros(n)
    for kk, cc in zip(k, c):
        u += cc * np.sin(kk * np.pi * x)
    return u


def rhs_torch(n: int, k, c, device):
    """Forcing generated directly in device memory (FP64)."""
    import torch
    x = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) / n
    f = torch.zeros(n, dtype=torch.float64, device=device)
    for kk, cc in zip(k, c):
        f.add_(torch.sin(x * (float(kk) * np.pi)), alpha=float(cc * (kk * np.pi) ** 2))
    return f


def exact_torch(n: int, k, c, device):
    import torch
    x = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) / n
    u = torch.zeros(n, dtype=torch.float64, device=device)
    for kk, cc in zip(k, c):
        u.add_(torch.sin(x * (float(kk) * np.pi)), alpha=float(cc))
    return u
