"""fmgsr_solve_noalloc (static device scratch, no allocation) against
fmgsr_solve, both through the C ABI.

With a single-cell coarsest grid both entry points run the same kernels on
the same inputs, so the results must be bitwise equal.  The reference solve
gets a caller workspace filled with NaN bytes, so a workspace cell read
before it is written would show.  Two no-allocation calls run back to back,
the second on a smaller problem, so the second starts from the first one's
scratch contents.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1207_6720_amd import fmgsr, workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 128 << 20


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rhs(n, seed):
    k, c = W.modes("inv_k2", 16, seed, n)
    return W.rhs_numpy(n, k, c)


def reference(f, **kw):
    n, levels = f.numel(), kw["levels"]
    ws = fmgsr.alloc_workspace(n, levels, f.device, nu=kw.get("nu", (2, 1)),
                               sr_levels=kw.get("sr_levels", 1), tau=kw.get("tau", "split"))
    ws.fill_(255)  # NaN bytes
    return fmgsr.solve(f, workspace=ws, **kw)


# (n, levels, segments, buffer, nu, sr_levels, tau, g, seed); calls run in this order
CALLS = [
    (1 << 20, 21, 256, 8, (2, 1), 1, "split", (0.0, 0.0), 0),
    (1 << 12, 13, 4, 4, (2, 1), 1, "split", (0.25, -0.5), 1),
    (3 << 10, 11, 3, 3, (3, 2), 2, "split", (0.0, 0.0), 2),
    (1 << 11, 12, 8, 1, (2, 1), 1, "literal", (0.0, 1.0), 3),
]


def test_noalloc_matches_fmgsr_solve_bitwise(dev):
    outs = []
    for (n, levels, S, b, nu, sr, tau, g, seed) in CALLS:
        print(f"noalloc n={n} levels={levels} S={S} b={b} nu={nu} sr={sr} tau={tau}", flush=True)
        assert fmgsr.workspace_bytes(n, levels, nu=nu, sr_levels=sr, tau=tau) <= SCRATCH_BYTES
        f = torch.from_numpy(rhs(n, seed)).to(dev)
        kw = dict(g=g, levels=levels, segments=S, buffer=b, nu=nu, sr_levels=sr, tau=tau)
        u = torch.empty_like(f)
        fmgsr.solve_noalloc(f, out=u, **kw)
        ref = reference(f, **kw)
        torch.cuda.synchronize()
        assert torch.isfinite(u).all()
        nbad = int((u != ref).sum())
        assert nbad == 0, f"{nbad} cells differ"
        outs.append((f, u.clone(), kw))
    # the first problem again, after smaller ones have used the scratch
    f, u0, kw = outs[0]
    u = fmgsr.solve_noalloc(f, **kw)
    torch.cuda.synchronize()
    assert torch.equal(u, u0)


def test_noalloc_rejections(dev):
    L = fmgsr.lib()
    f = torch.zeros(1 << 24, dtype=torch.float64, device=dev)
    u = torch.empty_like(f)
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    o = fmgsr.make_options()
    # workspace of 2^24 cells is about 400 MiB: larger than the scratch
    st = L.fmgsr_solve_noalloc(None, f.data_ptr(), 0.0, 0.0, f.numel(), 25, 4096, 8,
                               ctypes.byref(o), u.data_ptr(), s)
    assert st == fmgsr.FMGSR_ENOMEM
    # a caller workspace is refused
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    small = f[: 1 << 10]
    o2 = fmgsr.make_options(workspace=ws)
    st = L.fmgsr_solve_noalloc(None, small.data_ptr(), 0.0, 0.0, small.numel(), 11, 4, 4,
                               ctypes.byref(o2), u.data_ptr(), s)
    assert st == fmgsr.FMGSR_EINVAL
    # the reaction operators go through the batched engine, which allocates
    kappa = torch.ones_like(small)
    op = fmgsr.Operator(fmgsr.OPS["cubic"], kappa.data_ptr())
    st = L.fmgsr_solve_noalloc(ctypes.byref(op), small.data_ptr(), 0.0, 0.0, small.numel(), 11,
                               4, 4, ctypes.byref(o), u.data_ptr(), s)
    assert st == fmgsr.FMGSR_ENOTSUP
    torch.cuda.synchronize()
