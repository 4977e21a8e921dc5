"""Independent dense-matrix form of FMG-FAS-SR for tiny grids (tests only).

The operators are assembled as dense matrices from the entries the paper's
appendix prints (``tests/golden/appendix_*.txt``) and from the definition of
the cell-centred Laplacian; the cycle is then written with matrix-vector
products, index sets for the segments and a dense Gauss-Seidel splitting.
It shares no code with the C oracle and is used to pin it on grids of up to
a few hundred cells.  Homogeneous Dirichlet data only (the appendix's
operators), coarsest grid of at least 4 cells (so the appendix's boundary
rows of the interpolation matrix do not overlap).
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            kind, a, b, v = line.split()
            rows.append((kind, int(a), int(b), float(v)))
    return rows


def laplacian(n):
    """Dense cell-centred Laplacian, homogeneous Dirichlet (boundary diagonal 3)."""
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    if n == 1:
        A[0, 0] = 4.0
    else:
        A[0, 0] = 3.0
        A[-1, -1] = 3.0
    return A * float(n) ** 2


def fmg_interp(nc):
    """Dense FMG interpolation (nf x nc) from the appendix's printed rows."""
    nf = 2 * nc
    assert nc >= 4
    P = np.zeros((nf, nc))
    ent = _read("appendix_fmg_interp_rows.txt")
    for kind, r, c, v in ent:
        if kind == "boundary":
            P[r - 1, c - 1] = v
            P[nf - r, nc - c] = v          # mirror image for the last rows
    for i in range(5, nf - 4 + 1, 2):     # 1-based odd rows 5..nf-4
        j = (i - 1) // 2 + 1
        for kind, dr, dc, v in ent:
            if kind == "interior_odd":
                P[i - 1 + dr, j - 1 + dc] = v
            elif kind == "interior_even":
                P[i - 1 + dr, j - 1 + dc] = v
    return P / 128.0


def prolongation(nc):
    """Dense linear prolongation (nf x nc) from the appendix's printed entries."""
    nf = 2 * nc
    ent = _read("appendix_transfer_rows.txt")
    P = np.zeros((nf, nc))
    scale = [v for k, _, _, v in ent if k == "prol_scale"][0]
    for kind, r, c, v in ent:
        if kind == "prol_first_col":
            if r <= nf:
                P[r - 1, 0] += v
                P[nf - r, nc - 1] += v     # mirrored last column
    for j in range(2, nc):                 # 1-based interior columns
        for kind, dr, _, v in ent:
            if kind == "prol_interior_col":
                P[2 * j + dr - 1, j - 1] = v
    return P * scale


def restriction_avg(nc):
    nf = 2 * nc
    ent = _read("appendix_transfer_rows.txt")
    R = np.zeros((nc, nf))
    scale = [v for k, _, _, v in ent if k == "restrict_scale"][0]
    for j in range(1, nc + 1):
        for kind, dr, _, v in ent:
            if kind == "restrict_pair":
                R[j - 1, 2 * j - 1 + dr - 1] = v
    return R * scale


def restriction_fw(nc):
    """Full weighting = 1/2 (linear prolongation)^T (the appendix's
    commented-out alternative 0.125 P' with P the unscaled integer matrix)."""
    return 0.5 * prolongation(nc).T


def gs_sweep(A, u, F, E, order):
    """Gauss-Seidel on index set E (exterior frozen), visiting cells in
    ``order`` (a permutation of E)."""
    u = u.copy()
    for i in order:
        u[i] = (F[i] - (A[i] @ u - A[i, i] * u[i])) / A[i, i]
    return u


def rb_order(E):
    E = np.asarray(E)
    return list(E[E % 2 == 0]) + list(E[E % 2 == 1])


def smooth(A, u, F, nu, segments=None, kacz=None, smoother="rb"):
    """nu inner iterations of the point smoother; segments = list of
    (core, ext) index arrays for the additive block-Jacobi form; kacz =
    (R, c) for the Kaczmarz pass of compatible relaxation."""
    n = u.size
    if segments is None:
        segments = [(np.arange(n), np.arange(n))]
    out = np.empty(n)
    for core, ext in segments:
        w = u.copy()
        for it in range(nu):
            if kacz is not None:
                R, c = kacz
                for J in range(R.shape[0]):
                    ch = np.nonzero(R[J])[0]
                    if np.all(np.isin(ch, ext)):
                        rJ = R[J]
                        w = w + rJ * ((c[J] - rJ @ w) / (rJ @ rJ))
            if smoother == "rb":
                w = gs_sweep(A, w, F, ext, rb_order(ext))
            else:
                order = list(ext) if it % 2 == 0 else list(ext)[::-1]
                w = gs_sweep(A, w, F, ext, order)
        out[core] = w[core]
    return out


def make_segments(n, S, b):
    s = n // S
    segs = []
    for i in range(S):
        core = np.arange(i * s, (i + 1) * s)
        ext = np.arange(max(0, i * s - b), min(n, (i + 1) * s + b))
        segs.append((core, ext))
    return segs


def fmgsr(f, levels, segments=1, buffer=0, nu1=2, nu2=1, nsr=1, tau="split",
          rhs_restrict="fw", smoother="rb", block_all=0, keep_coarse=False):
    """Dense FMG-FAS-SR (one iteration), assembled tau on every level.
    keep_coarse: also return the level-(M-1) solution of the final cycle."""
    n = f.size
    M = levels - 1
    ns = [n >> (M - l) for l in range(M + 1)]
    A = [laplacian(m) for m in ns]
    Rs = [None] + [restriction_avg(ns[l - 1]) for l in range(1, M + 1)]     # I^ : l -> l-1
    Rf = [None] + [(restriction_fw(ns[l - 1]) if rhs_restrict == "fw"
                    else restriction_avg(ns[l - 1])) for l in range(1, M + 1)]
    Pl = [None] + [prolongation(ns[l - 1]) for l in range(1, M + 1)]
    Pi = [None] + [fmg_interp(ns[l - 1]) for l in range(1, M + 1)]

    def segs(l):
        if l == 0:
            return None
        if block_all:
            return make_segments(ns[l], ns[l] // block_all, buffer)
        if l > M - nsr:
            return make_segments(ns[l], segments, buffer)
        return None

    F = [None] * (M + 1)
    F[M] = f.copy()
    for l in range(M, 0, -1):
        F[l - 1] = Rf[l] @ F[l]
    Q = [x.copy() for x in F]
    u = [None] * (M + 1)
    uh = [None] * (M + 1)
    u[0] = np.linalg.solve(A[0], Q[0])
    for k in range(M):
        t = k + 1
        u[t] = Pi[t] @ u[k]
        Q[t] = F[t].copy()
        u[t] = smooth(A[t], u[t], Q[t], nu1, segs(t), smoother=smoother)
        for m in range(k, -1, -1):
            uh[m] = Rs[m + 1] @ u[m + 1]
            if tau == "split":
                Q[m] = F[m].copy()
            else:
                Q[m] = Rf[m + 1] @ (Q[m + 1] - A[m + 1] @ u[m + 1]) + A[m] @ uh[m]
            if m == 0:
                u[0] = np.linalg.solve(A[0], Q[0])
            else:
                u[m] = smooth(A[m], uh[m].copy(), Q[m], nu1, segs(m), smoother=smoother)
        for m in range(0, k + 1):
            if m + 1 > M - nsr:
                v = Pi[m + 1] @ u[m]
                u[m + 1] = smooth(A[m + 1], v, Q[m + 1], nu2, segs(m + 1),
                                  kacz=(Rs[m + 1], u[m]), smoother=smoother)
            else:
                u[m + 1] = u[m + 1] + Pl[m + 1] @ (u[m] - uh[m])
                u[m + 1] = smooth(A[m + 1], u[m + 1], Q[m + 1], nu2, segs(m + 1),
                                  smoother=smoother)
    return (u[M], u[M - 1]) if keep_coarse else u[M]


def decompress(c, f, lo, hi, segments, buffer, nu2=1):
    """Fine solution on [lo, hi) from the level-(M-1) solution c: the final
    SR update (FMG interpolation, then nu2 x [Kaczmarz toward c, red-black
    sweep] per extended patch) on the segments whose cores meet [lo, hi)."""
    n = f.size
    nc = n // 2
    s = n // segments
    segs = make_segments(n, segments, buffer)[lo // s:(hi - 1) // s + 1]
    u = smooth(laplacian(n), fmg_interp(nc) @ c, f, nu2, segs, kacz=(restriction_avg(nc), c))
    return u[lo:hi]
