"""PDE compression in the batched engine (Sec. 2.4) and the adjoint that
rebuilds u_fwd from the kept level instead of reading it, through the C ABI.

* fmgsr_batch_solve_keep: the finest level equals fmgsr_batch_solve's bit for
  bit, and the kept level-(M-1) solution equals the oracle's
  (rx_fmgsr_solve_keep) within 1e-12 per problem (2-norm and per cell),
  bitwise where the coarsest level is one cell.
* fmgsr_batch_adjoint_compressed: u_fwd is rebuilt exactly (each window from
  its own segment's and its neighbours' SR up passes), so the gradients equal
  fmgsr_batch_adjoint's on the same forward's u bit for bit, and through it
  the oracle adjoint's within 1e-12.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1207_6720_amd import fmgsr, workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    if a.size == 0:
        return 0.0
    cell = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
    return max(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300), cell)


def loss_grad(rb, u, ut, dev):
    h = torch.cat([torch.full((int(n),), 1.0 / int(n), dtype=torch.float64, device=dev)
                   for n in rb.sizes])
    return 2.0 * h * (u - ut)


def run_both(rb, plan, f, k, ut, dev):
    """Forward with the kept level, then both adjoints; returns
    (u, coarse, (gf, gk) from u, (gf, gk) compressed)."""
    u_plain = plan.solve(f, k)
    u, coarse = plan.solve_keep(f, k)
    dJ = loss_grad(rb, u, ut, dev)
    gu = plan.adjoint(k, u, dJ)
    gc = plan.adjoint_compressed(k, f, coarse, dJ)
    torch.cuda.synchronize()
    assert torch.equal(u, u_plain)
    return u, coarse, gu, gc


def check_coarse(rb, plan, f, k, coarse, nu=(2, 1), g=None):
    segs = plan.query()["segments"]
    fh, kh, ch = f.cpu().numpy(), k.cpu().numpy(), coarse.cpu().numpy()
    for j in range(rb.batch):
        L = int(rb.levels[j])
        if L < 2:
            continue
        o, n = int(rb.offsets[j]), int(rb.sizes[j])
        gl, gr = (0.0, 0.0) if g is None else g[j]
        _, cref = oracle.rx_fmgsr_solve_keep("cubic", fh[o:o + n], kh[o:o + n], gl, gr,
                                             levels=L, segments=int(segs[j]), buffer=rb.buffer,
                                             nu1=nu[0], nu2=nu[1])
        c = ch[o // 2:o // 2 + n // 2]
        assert rel(c, cref) <= TOL, f"problem {j}: kept level {rel(c, cref):.3e}"
        if (n >> (L - 1)) == 1:
            assert np.array_equal(c, cref), f"problem {j}: kept level not bitwise"


def test_small_batch_groups_and_wide_windows(dev):
    """24 uneven problems: fewer than CUs, so 512 x 8 windows and groups of
    workgroups meeting at barriers, in the forward and in the rebuild."""
    rb = W.reaction_batch("small", seed=21)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    q = plan.query()
    print(f"small: {rb.batch} problems, group {q['group']}, run {q['run']}", flush=True)
    u, coarse, gu, gc = run_both(rb, plan, f, k, ut, dev)
    assert torch.equal(gu[0], gc[0]) and torch.equal(gu[1], gc[1])
    check_coarse(rb, plan, f, k, coarse)
    assert plan.query()["stalled"] == 0


def test_large_batch_one_workgroup_per_problem(dev):
    rb = W.reaction_batch("small", seed=22, batch=600)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    assert plan.query()["group"] == 1
    _, coarse, gu, gc = run_both(rb, plan, f, k, ut, dev)
    assert torch.equal(gu[0], gc[0]) and torch.equal(gu[1], gc[1])
    check_coarse(rb, plan, f, k, coarse)


# sizes, levels, segments, buffer, nu, g
EDGE = [
    ([1 << 9, 3 << 8], [10, 9], None, 4, (2, 1), None),                 # N0 = 1 and 3
    ([5 << 6, 7 << 5, 64], [7, 6, 1], None, 1, (2, 1), [(0.3, -0.2)] * 3),  # one grid, b = 1
    ([48 * 64, 33 * 32], [7, 6], None, 3, (3, 2), [(1.0, 0.5), (-0.4, 0.0)]),
    ([37 * 16, 50 * 32], [5, 6], None, 8, (0, 1), None),
    ([37 * 16, 50 * 32], [5, 6], None, 8, (1, 0), None),
    ([256 * 2, 6], [2, 2], None, 2, (2, 1), None),                     # M = 1: level 0 kept
    ([1 << 12], [13], [256], 8, (2, 1), None),                          # segment core 16
]


@pytest.mark.parametrize("case", EDGE, ids=lambda c: f"n{c[0]}_L{c[1]}_b{c[3]}_nu{c[4][0]}{c[4][1]}")
def test_edge_cases(dev, case):
    sizes, levels, segs, buf, nu, g = case
    print(f"edge case {case}", flush=True)
    rb = W.ReactionBatch("edge", tuple(sizes), tuple(levels), buf, 5)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(sizes, levels, buffer=buf, segments=segs, g=g, op="cubic", nu=nu)
    _, coarse, gu, gc = run_both(rb, plan, f, k, ut, dev)
    assert torch.equal(gu[0], gc[0]) and torch.equal(gu[1], gc[1])
    check_coarse(rb, plan, f, k, coarse, nu=nu, g=g)


def test_compressed_adjoint_matches_the_oracle_adjoint(dev):
    rb = W.reaction_batch("small", seed=23, batch=8)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u, coarse = plan.solve_keep(f, k)
    dJ = loss_grad(rb, u, ut, dev)
    gf, gk = plan.adjoint_compressed(k, f, coarse, dJ)
    torch.cuda.synchronize()
    segs = plan.query()["segments"]
    for j in range(rb.batch):
        o, n = int(rb.offsets[j]), int(rb.sizes[j])
        kj, uj, dj = (t[o:o + n].cpu().numpy() for t in (k, u, dJ))
        rf, rk = oracle.rx_fmgsr_adjoint(kj, uj, dj, levels=int(rb.levels[j]),
                                         segments=int(segs[j]), buffer=rb.buffer)
        assert rel(gf[o:o + n].cpu().numpy(), rf) <= TOL, j
        assert rel(gk[o:o + n].cpu().numpy(), rk) <= TOL, j


def test_fp32_relaxation_rebuild_is_exact(dev):
    """The rebuild runs the forward's own SR up pass in the same precision
    mode, so it reproduces the FP32-relaxed u_fwd bit for bit as well."""
    rb = W.reaction_batch("small", seed=24, batch=12)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic", precision="fp32relax")
    _, _, gu, gc = run_both(rb, plan, f, k, ut, dev)
    assert torch.equal(gu[0], gc[0]) and torch.equal(gu[1], gc[1])


def test_compression_only_and_one_gradient(dev):
    rb = W.reaction_batch("small", seed=25, batch=6)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u, c1 = plan.solve_keep(f, k)
    none, c2 = plan.solve_keep(f, k, write_u=False)
    assert none is None
    dJ = loss_grad(rb, u, ut, dev)
    gf_only = torch.full_like(f, 7.0)
    st = fmgsr.lib().fmgsr_batch_adjoint_compressed(
        plan._h, k.data_ptr(), f.data_ptr(), c2.data_ptr(), dJ.data_ptr(), gf_only.data_ptr(),
        None, torch.cuda.current_stream(dev).cuda_stream)
    assert st == fmgsr.FMGSR_OK
    gf, gk = plan.adjoint(k, u, dJ)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)
    assert torch.equal(gf_only, gf)


def test_one_shot_adjoint_without_u_fwd(dev):
    n, levels = 45 << 7, 8
    f, k, _, ut = W.reaction_problem_numpy(n, 7, 0)
    fd, kd = torch.from_numpy(f).to(dev), torch.from_numpy(k).to(dev)
    u = fmgsr.solve(fd, levels=levels, segments=4, buffer=8, op="cubic", kappa=kd)
    dJ = 2.0 / n * (u - torch.from_numpy(ut).to(dev))
    g_given = fmgsr.adjoint(fd, kd, dJ, levels=levels, segments=4, buffer=8, u_fwd=u)
    g_kept = fmgsr.adjoint(fd, kd, dJ, levels=levels, segments=4, buffer=8)  # kept level path
    assert torch.equal(g_given[0], g_kept[0]) and torch.equal(g_given[1], g_kept[1])


def test_rejections(dev):
    # segment core 2 < pad 6: the window's pad is not covered by the neighbours
    rb = W.ReactionBatch("rej", (1 << 8,), (9,), 4, 5)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=4, segments=[128], op="cubic")
    _, coarse = plan.solve_keep(f, k)
    with pytest.raises(fmgsr.FmgsrError) as e:
        plan.adjoint_compressed(k, f, coarse, f)
    assert e.value.status == fmgsr.FMGSR_ENOTSUP
    pois = fmgsr.Batch(rb.sizes, rb.levels, buffer=4, op="poisson")
    with pytest.raises(ValueError):
        pois.adjoint_compressed(k, f, coarse, f)
    st = fmgsr.lib().fmgsr_batch_solve_keep(plan._h, f.data_ptr(), k.data_ptr(), None,
                                            f.data_ptr(), None)
    assert st == fmgsr.FMGSR_EINVAL  # the kept array aliases f


def test_autograd_keeps_the_coarse_level_by_default(dev):
    rb = W.ReactionBatch("ag", (32 << 4, 17 << 5), (5, 6), 8, 11)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=8, op="cubic")
    grads = {}
    for keep in ("coarse", "u"):
        fr = f.clone().requires_grad_(True)
        kr = k.clone().requires_grad_(True)
        u = fmgsr.CubicSolve.apply(fr, kr, plan, keep)
        ((u - ut) ** 2).sum().backward()
        grads[keep] = (fr.grad.detach(), kr.grad.detach())
    uc = fmgsr.CubicSolve.apply(f, k, plan)
    torch.cuda.synchronize()
    assert torch.equal(grads["coarse"][0], grads["u"][0])
    assert torch.equal(grads["coarse"][1], grads["u"][1])
    assert torch.equal(uc, plan.solve(f, k))


def test_c4_full_size_compressed_adjoint(dev):
    """64 problems of 2^20 cells: the compressed adjoint equals the one that
    reads u_fwd, bit for bit."""
    rb = W.reaction_batch("c4", seed=0)
    f, k, _, ut = W.reaction_packed_torch(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    _, coarse, gu, gc = run_both(rb, plan, f, k, ut, dev)
    print("c4 compressed adjoint done", flush=True)
    assert torch.equal(gu[0], gc[0]) and torch.equal(gu[1], gc[1])
    assert coarse.numel() >= rb.total // 2
