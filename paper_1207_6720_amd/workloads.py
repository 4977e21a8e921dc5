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

Reaction problems -u'' + kappa(x) u^3 = f (batched and adjoint workloads):

* kappa(x) = 1 + g(x)/2 with g = sum_{m=1..4} c_m cos(m pi x + phi_m) / sum |c_m|,
  c_m ~ Normal(0, 1), phi_m ~ Uniform[0, 2 pi), so kappa lies in [0.5, 1.5];
* u = sum_{k=1..8} a_k sin(k pi x), a_k ~ Normal(0, sd 1/k), and
  f = sum_k a_k (k pi)^2 sin(k pi x) + kappa u^3 at the cell centres;
* ``c3`` 4096 problems; problem j draws e ~ Uniform[12, 18), L = floor(e) - 5,
  N0 = clamp(round(2^e / 2^L), 32, 63), N = N0 2^L, L + 1 levels, buffer 8;
* ``c4`` 64 problems of N = 2^20 (N0 = 32, 16 levels), buffer 8, with a
  seeded 8-mode target field for the least-squares functional.
"""
from dataclasses import dataclass

import numpy as np

__all__ = ["Workload", "WORKLOADS", "modes", "rhs_numpy", "exact_numpy",
           "rhs_torch", "exact_torch", "cell_centres", "ReactionBatch", "REACTION_WORKLOADS",
           "reaction_batch", "reaction_params"]


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


# ---------------------------------------------------------------------------
# Reaction problems -u'' + kappa u^3 = f
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class ReactionBatch:
    name: str
    sizes: tuple      # fine cells per problem
    levels: tuple     # levels per problem
    buffer: int
    seed: int

    @property
    def batch(self) -> int:
        return len(self.sizes)

    @property
    def total(self) -> int:
        return int(sum(self.sizes))

    @property
    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(np.int64)

    @property
    def description(self) -> str:
        return (f"{self.batch} problems -u''+kappa u^3=f, N in [{min(self.sizes)}, "
                f"{max(self.sizes)}] (total {self.total}), buffer {self.buffer}, V(2,1)")


def reaction_batch(name: str, seed: int = 0, batch: int = None) -> ReactionBatch:
    """Problem sizes of a reaction workload (``c3``: uneven log-uniform sizes,
    ``c4``: equal 2^20 problems; ``small``: a quick uneven batch)."""
    rng = np.random.default_rng([seed, 3])
    if name in ("c3", "small"):
        b = batch or (4096 if name == "c3" else 24)
        lo, hi = (12.0, 18.0) if name == "c3" else (8.0, 12.0)
        e = rng.uniform(lo, hi, size=b)
        L = np.floor(e).astype(np.int64) - 5
        n0 = np.clip(np.rint(2.0 ** e / 2.0 ** L), 32, 63).astype(np.int64)
        sizes = tuple(int(a) << int(c) for a, c in zip(n0, L))
        levels = tuple(int(c) + 1 for c in L)
    elif name == "c4":
        b = batch or 64
        sizes = (1 << 20,) * b
        levels = (16,) * b
    else:
        raise ValueError(name)
    return ReactionBatch(name, sizes, levels, 8, seed)


REACTION_WORKLOADS = ("c3", "c4", "small")


def reaction_params(seed: int, j: int):
    """Per-problem parameters: (a_k for k = 1..8, c_m, phi_m, target a_k)."""
    rng = np.random.default_rng([seed, j, 7])
    k = np.arange(1, 9, dtype=np.float64)
    a = rng.normal(0.0, 1.0, size=8) / k
    cm = rng.normal(0.0, 1.0, size=4)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=4)
    target = rng.normal(0.0, 1.0, size=8) / k
    return a, cm, phi, target


def _reaction_fields(xp, x, a, cm, phi, target, pi):
    """kappa, u_exact, f and u_target at cell centres x (numpy or torch)."""
    g = 0.0 * x
    for m in range(4):
        g = g + float(cm[m]) * xp.cos(x * (float(m + 1) * pi) + float(phi[m]))
    kappa = 1.0 + 0.5 * g / float(np.sum(np.abs(cm)))
    u = 0.0 * x
    lap = 0.0 * x
    ut = 0.0 * x
    for k in range(8):
        s = xp.sin(x * (float(k + 1) * pi))
        u = u + float(a[k]) * s
        lap = lap + float(a[k] * ((k + 1) * pi) ** 2) * s
        ut = ut + float(target[k]) * s
    f = lap + kappa * (u * u * u)
    return kappa, u, f, ut


def reaction_problem_numpy(n: int, seed: int, j: int):
    """(f, kappa, u_exact, u_target) of problem j, host FP64."""
    a, cm, phi, target = reaction_params(seed, j)
    kappa, u, f, ut = _reaction_fields(np, cell_centres(n), a, cm, phi, target, np.pi)
    return f, kappa, u, ut


def reaction_packed_torch(rb: ReactionBatch, device):
    """Packed (f, kappa, u_exact, u_target) of a whole batch, generated in
    device memory for all problems at once (a few dozen whole-batch kernels):
    every cell gathers its problem's parameters."""
    import torch
    B = rb.batch
    params = [reaction_params(rb.seed, j) for j in range(B)]
    tens = lambda rows: torch.tensor(np.array(rows), dtype=torch.float64, device=device)
    a = tens([p[0] for p in params])            # [B, 8]
    cm = tens([p[1] for p in params])           # [B, 4]
    phi = tens([p[2] for p in params])          # [B, 4]
    tg = tens([p[3] for p in params])           # [B, 8]
    csum = cm.abs().sum(dim=1)                  # [B]
    sizes = torch.tensor(rb.sizes, dtype=torch.int64, device=device)
    offs = torch.tensor(rb.offsets, dtype=torch.int64, device=device)
    pid = torch.repeat_interleave(torch.arange(B, device=device), sizes)
    local = torch.arange(rb.total, dtype=torch.int64, device=device) - offs[pid]
    x = (local.to(torch.float64) + 0.5) / sizes[pid].to(torch.float64)
    del local
    pi = np.pi
    g = torch.zeros_like(x)
    for m in range(4):
        g = g + cm[pid, m] * torch.cos(x * (float(m + 1) * pi) + phi[pid, m])
    kappa = 1.0 + 0.5 * g / csum[pid]
    del g
    u = torch.zeros_like(x)
    lap = torch.zeros_like(x)
    ut = torch.zeros_like(x)
    for k in range(8):
        s = torch.sin(x * (float(k + 1) * pi))
        u = u + a[pid, k] * s
        lap = lap + (a[pid, k] * float(((k + 1) * pi) ** 2)) * s
        ut = ut + tg[pid, k] * s
        del s
    f = lap + kappa * (u * u * u)
    return f, kappa, u, ut
