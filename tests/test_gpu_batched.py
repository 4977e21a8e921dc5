"""GPU parity of the batched solver (one persistent launch, reaction operators,
FP32 relaxation, adjoint) against the FP64 CPU oracle, through the C ABI.

Bars: FP64 results within 1e-12 relative of the oracle per problem, both in
the 2-norm and cell by cell (max |d| <= 1e-12 max |u_ref|), bitwise where the coarsest level is one cell (identical expression trees
and Newton steps); FP32 relaxation within a tenth of each problem's
discretisation error (it must stay below it); gradients within 1e-12 of the
oracle's FMG-SR adjoint."""
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


def rel_norm(a, b):
    """2-norm relative difference (accuracy bars: discretisation error,
    finite differences)."""
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rel(a, b):
    """Parity difference: the larger of the 2-norm ratio and the largest cell
    difference over the largest |b| (both must meet the bar)."""
    cell = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300) if a.size else 0.0
    return max(rel_norm(a, b), cell)


def packed(rb, dev):
    f, k, ue, ut = W.reaction_packed_torch(rb, dev)
    torch.cuda.synchronize()
    return f, k, ue, ut


def per_problem(rb, arr):
    a = arr.cpu().numpy() if isinstance(arr, torch.Tensor) else arr
    return [a[o:o + n] for o, n in zip(rb.offsets, rb.sizes)]


def check_against_oracle(rb, plan, f, k, u, kind="cubic", nu=(2, 1), g=None, bitwise_n0_1=True):
    segs = plan.query()["segments"]
    fs, ks, us = per_problem(rb, f), per_problem(rb, k), per_problem(rb, u)
    worst = 0.0
    for j in range(rb.batch):
        gl, gr = (0.0, 0.0) if g is None else g[j]
        ref = oracle.rx_fmgsr_solve(kind, fs[j], None if kind == "poisson" else ks[j], gl, gr,
                                    levels=rb.levels[j], segments=int(segs[j]),
                                    buffer=rb.buffer, nu1=nu[0], nu2=nu[1],
                                    nsr=1 if rb.levels[j] > 1 else 0)
        e = rel(us[j], ref)
        assert np.all(np.isfinite(us[j])), j
        assert e <= TOL, f"problem {j} (n={rb.sizes[j]}, levels={rb.levels[j]}): {e:.3e}"
        n0 = rb.sizes[j] >> (rb.levels[j] - 1)
        if bitwise_n0_1 and n0 == 1:
            assert np.array_equal(us[j], ref), f"problem {j} not bitwise"
        worst = max(worst, e)
    return worst


def test_small_uneven_batch_cubic_fp64(dev):
    rb = W.reaction_batch("small", seed=0)
    print(f"small batch: {rb.batch} problems, total {rb.total}", flush=True)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u = plan.solve(f, k)
    torch.cuda.synchronize()
    print("worst rel", check_against_oracle(rb, plan, f, k, u), flush=True)


def test_repeat_is_deterministic_and_workspace_garbage_free(dev):
    rb = W.reaction_batch("small", seed=1, batch=9)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    a = plan.solve(f, k).clone()
    b = plan.solve(f, k)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("kind", ["poisson", "linear"])
def test_linear_kinds(dev, kind):
    rb = W.reaction_batch("small", seed=2, batch=8)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op=kind)
    u = plan.solve(f, None if kind == "poisson" else k)
    torch.cuda.synchronize()
    check_against_oracle(rb, plan, f, k, u, kind=kind)


# edge cases: one level (direct Newton), two levels, N0 = 1 (bitwise),
# one segment, zero buffer, boundary values, sweep counts
EDGE = [
    # sizes, levels, segments, buffer, nu, g
    ([40, 63, 1, 2], [1, 1, 1, 2], None, 8, (2, 1), None),
    ([64, 96], [2, 2], [1, 2], 0, (2, 1), [(0.3, -0.2), (1.0, 0.5)]),
    ([1024, 2048, 512], [11, 12, 10], [4, 8, 1], 8, (2, 1), [(0.0, 0.0), (0.4, -0.6), (0.1, 0.1)]),
    ([48 * 64, 33 * 32], [7, 6], None, 3, (3, 2), None),
    ([37 * 16, 50 * 32], [5, 6], None, 8, (0, 1), None),
    ([37 * 16, 50 * 32], [5, 6], None, 8, (1, 0), None),
    ([256 * 8], [4], None, 8, (2, 1), None),   # N0 = 256, the largest coarsest level
]


@pytest.mark.parametrize("case", EDGE, ids=lambda c: f"n{c[0]}_L{c[1]}_b{c[3]}_nu{c[4][0]}{c[4][1]}")
def test_edge_cases(dev, case):
    sizes, levels, segs, buf, nu, g = case
    print(f"edge case {case}", flush=True)
    rb = W.ReactionBatch("edge", tuple(sizes), tuple(levels), buf, 5)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(sizes, levels, buffer=buf, segments=segs, g=g, op="cubic", nu=nu)
    u = plan.solve(f, k)
    torch.cuda.synchronize()
    check_against_oracle(rb, plan, f, k, u, nu=nu, g=g)


def test_custom_offsets_leave_gaps_untouched(dev):
    sizes, levels = [39 * 32, 41 * 64], [6, 7]
    rb = W.ReactionBatch("gaps", tuple(sizes), tuple(levels), 8, 6)
    f, k, _, _ = packed(rb, dev)
    offs = [5, 5 + sizes[0] + 7]
    tot = offs[1] + sizes[1] + 3
    F = torch.zeros(tot, dtype=torch.float64, device=dev)
    Kp = torch.ones(tot, dtype=torch.float64, device=dev)
    for o, (a, n) in zip(offs, zip(rb.offsets, rb.sizes)):
        F[o:o + n] = f[a:a + n]
        Kp[o:o + n] = k[a:a + n]
    U = torch.full((tot,), 7.0, dtype=torch.float64, device=dev)
    plan = fmgsr.Batch(sizes, levels, buffer=8, op="cubic", offsets=offs)
    plan.solve(F, Kp, out=U)
    torch.cuda.synchronize()
    Uh = U.cpu().numpy()
    mask = np.ones(tot, dtype=bool)
    for o, n in zip(offs, sizes):
        mask[o:o + n] = False
    assert np.all(Uh[mask] == 7.0)
    u_dense = torch.cat([U[o:o + n] for o, n in zip(offs, sizes)])
    check_against_oracle(rb, plan, f, k, u_dense)


def test_fp32_relaxation_stays_below_discretisation_error(dev):
    rb = W.reaction_batch("small", seed=3, batch=12)
    f, k, ue, _ = packed(rb, dev)
    p64 = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    p32 = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic", precision="fp32relax")
    u64 = p64.solve(f, k)
    u32 = p32.solve(f, k)
    torch.cuda.synchronize()
    fs, ks, es = per_problem(rb, f), per_problem(rb, k), per_problem(rb, ue)
    a64, a32 = per_problem(rb, u64), per_problem(rb, u32)
    segs = p32.query()["segments"]
    for j in range(rb.batch):
        ref = oracle.rx_fmgsr_solve("cubic", fs[j], ks[j], levels=rb.levels[j],
                                    segments=int(segs[j]), buffer=rb.buffer)
        ustar, _ = oracle.rx_newton("cubic", ks[j], fs[j])
        disc = rel_norm(ustar, es[j])
        d32 = rel_norm(a32[j], ref)
        print(f"problem {j}: n={rb.sizes[j]} disc={disc:.2e} fp32-vs-oracle={d32:.2e}", flush=True)
        assert rel(a64[j], ref) <= TOL
        assert d32 <= 0.1 * disc
        assert rel_norm(a32[j], ustar) <= 0.5 * disc


def test_adjoint_matches_oracle(dev):
    rb = W.reaction_batch("small", seed=4, batch=10)
    f, k, _, ut = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u = plan.solve(f, k)
    h = torch.cat([torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev) for n in rb.sizes])
    dJ = 2.0 * h * (u - ut)
    gf, gk = plan.adjoint(k, u, dJ)
    torch.cuda.synchronize()
    segs = plan.query()["segments"]
    ks, us, ds = per_problem(rb, k), per_problem(rb, u), per_problem(rb, dJ)
    gfs, gks = per_problem(rb, gf), per_problem(rb, gk)
    for j in range(rb.batch):
        rf, rk = oracle.rx_fmgsr_adjoint(ks[j], us[j], ds[j], levels=rb.levels[j],
                                         segments=int(segs[j]), buffer=rb.buffer)
        assert rel(gfs[j], rf) <= TOL, j
        assert rel(gks[j], rk) <= TOL, j


def test_single_problem_entry_points(dev):
    n, levels = 45 << 7, 8
    f, k, _, ut = W.reaction_problem_numpy(n, 7, 0)
    fd, kd = torch.from_numpy(f).to(dev), torch.from_numpy(k).to(dev)
    u = fmgsr.solve(fd, levels=levels, segments=4, buffer=8, op="cubic", kappa=kd)
    ref = oracle.rx_fmgsr_solve("cubic", f, k, levels=levels, segments=4, buffer=8)
    assert rel(u.cpu().numpy(), ref) <= TOL
    dJ = torch.from_numpy(2.0 / n * (ref - ut)).to(dev)
    gf, gk = fmgsr.adjoint(fd, kd, dJ, levels=levels, segments=4, buffer=8)  # forward recomputed
    rf, rk = oracle.rx_fmgsr_adjoint(k, u.cpu().numpy(), dJ.cpu().numpy(), levels=levels,
                                     segments=4, buffer=8)
    assert rel(gf.cpu().numpy(), rf) <= TOL
    assert rel(gk.cpu().numpy(), rk) <= TOL


def test_graph_replays_match_eager(dev):
    rb = W.reaction_batch("small", seed=8, batch=10)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    ref = plan.solve(f, k).clone()
    out = torch.zeros_like(f)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
        plan.solve(f, k, out=out)
    torch.cuda.synchronize()
    for r in range(4):
        out.fill_(-1.0)
        plan.solve(f * 1.0, k, out=torch.empty_like(f))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"


def test_autotune_keeps_parity(dev):
    rb = W.reaction_batch("small", seed=9, batch=16)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    ms = plan.autotune(f, k)
    q = plan.query()
    print(f"autotune: {ms:.3f} ms, shape {q['threads']}x{q['run']}, grid {q['grid']}", flush=True)
    assert ms > 0 and q["threads"] in (256, 512)
    u = plan.solve(f, k)
    torch.cuda.synchronize()
    check_against_oracle(rb, plan, f, k, u)


def test_c3_full_size_sampled_parity(dev):
    """4096 problems, N in [2^12, 2^18]: the whole batch in one launch, checked
    problem by problem on a sample (largest, smallest and four others)."""
    rb = W.reaction_batch("c3", seed=0)
    print(f"c3: {rb.batch} problems, total {rb.total}", flush=True)
    f, k, _, _ = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u = plan.solve(f, k)
    torch.cuda.synchronize()
    print("c3: GPU solve done", flush=True)
    assert bool(torch.isfinite(u).all())
    segs = plan.query()["segments"]
    sizes = np.asarray(rb.sizes)
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 1, 1000, 2047, 4095})
    for j in sample:
        o, n = int(rb.offsets[j]), int(rb.sizes[j])
        fj, kj, uj = (t[o:o + n].cpu().numpy() for t in (f, k, u))
        ref = oracle.rx_fmgsr_solve("cubic", fj, kj, levels=rb.levels[j], segments=int(segs[j]),
                                    buffer=rb.buffer)
        e = rel(uj, ref)
        print(f"c3 problem {j}: n={n} rel={e:.2e}", flush=True)
        assert e <= TOL


def test_autograd_and_central_differences(dev):
    """Gradients of J = h sum (u - u_t)^2 through torch.autograd (the library
    adjoint) against central differences of the exact discrete solution map
    (oracle Newton solves), eps = 1e-6 relative to each field, 32 random
    directions per field.  The grids are small on purpose: a Newton solve is
    exact only to about eps_mach times the condition number (~ 0.4 n^2), and
    the differences must stay well above that floor (at n = 2^20 it exceeds
    1e-6 itself)."""
    n0, L = 32, 4
    n = n0 << L
    rb = W.ReactionBatch("fd", (n, n), (L + 1, L + 1), 8, 11)
    f, k, _, ut = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=8, op="cubic")
    fr = f.clone().requires_grad_(True)
    kr = k.clone().requires_grad_(True)
    u = fmgsr.CubicSolve.apply(fr, kr, plan)
    h = 1.0 / n
    loss = h * ((u - ut) ** 2).sum()
    loss.backward()
    gf_auto, gk_auto = fr.grad.detach(), kr.grad.detach()
    # the library adjoint on the same u, directly
    gf_dir, gk_dir = plan.adjoint(k, u.detach(), (2.0 * h * (u - ut)).detach())
    torch.cuda.synchronize()
    assert torch.equal(gf_auto, gf_dir) and torch.equal(gk_auto, gk_dir)
    # FD on the exact discrete map, with the adjoint evaluated at the
    # converged discrete solution
    rng = np.random.default_rng(17)
    eps = 1e-6
    for j in range(rb.batch):
        o = int(rb.offsets[j])
        fj, kj, utj = (t[o:o + n].cpu().numpy() for t in (f, k, ut))
        ustar, _ = oracle.rx_newton("cubic", kj, fj)
        us_d = torch.from_numpy(ustar).to(dev)
        one = fmgsr.Batch((n,), (L + 1,), buffer=8, op="cubic")
        gfj, gkj = one.adjoint(k[o:o + n].contiguous(), us_d,
                               torch.from_numpy(2.0 * h * (ustar - utj)).to(dev))
        gfj, gkj = gfj.cpu().numpy(), gkj.cpu().numpy()

        def J(ff, kk):
            us, _ = oracle.rx_newton("cubic", kk, ff)
            return h * np.sum((us - utj) ** 2)
        fd_f, ad_f, fd_k, ad_k = [], [], [], []
        for _ in range(32):
            df = rng.normal(size=n) * np.abs(fj).max()
            dk = rng.normal(size=n) * np.abs(kj).max()
            fd_f.append((J(fj + eps * df, kj) - J(fj - eps * df, kj)) / (2 * eps))
            fd_k.append((J(fj, kj + eps * dk) - J(fj, kj - eps * dk)) / (2 * eps))
            ad_f.append(gfj @ df)
            ad_k.append(gkj @ dk)
        # agreement of the 32 directional derivatives as vectors (a single
        # direction can make its derivative small by cancellation)
        ef, ek = (rel_norm(np.array(ad_f), np.array(fd_f)),
                  rel_norm(np.array(ad_k), np.array(fd_k)))
        print(f"problem {j}: FD rel f {ef:.2e} kappa {ek:.2e}", flush=True)
        assert ef <= 1e-4 and ek <= 1e-4


def test_c4_full_size_sampled_parity(dev):
    """64 problems of 2^20 cells: forward and adjoint in one launch each,
    checked against the oracle on two problems."""
    rb = W.reaction_batch("c4", seed=0)
    f, k, _, ut = packed(rb, dev)
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic")
    u = plan.solve(f, k)
    n = rb.sizes[0]
    dJ = 2.0 / n * (u - ut)
    gf, gk = plan.adjoint(k, u, dJ)
    torch.cuda.synchronize()
    print("c4: GPU forward + adjoint done", flush=True)
    segs = plan.query()["segments"]
    for j in (0, 63):
        o = int(rb.offsets[j])
        fj, kj, uj, dj, gfj, gkj = (t[o:o + n].cpu().numpy() for t in (f, k, u, dJ, gf, gk))
        ref = oracle.rx_fmgsr_solve("cubic", fj, kj, levels=rb.levels[j], segments=int(segs[j]),
                                    buffer=rb.buffer)
        rf, rk = oracle.rx_fmgsr_adjoint(kj, uj, dj, levels=rb.levels[j], segments=int(segs[j]),
                                         buffer=rb.buffer)
        print(f"c4 problem {j}: u {rel(uj, ref):.2e} grad_f {rel(gfj, rf):.2e} "
              f"grad_kappa {rel(gkj, rk):.2e}", flush=True)
        assert rel(uj, ref) <= TOL and rel(gfj, rf) <= TOL and rel(gkj, rk) <= TOL


def test_group_split_matches_single_workgroup_bitwise(dev):
    """A problem solved alone (its levels split over a group of workgroups
    meeting at barriers, 512 threads x 8 cells) equals the same problem
    inside a large batch (one 256 x 4 workgroup per problem) bit for bit, and
    neither run stalls: the tiles are halo-exact, so neither the tiling nor
    the split changes a value."""
    big = W.reaction_batch("small", seed=12, batch=600)
    f, k, _, _ = packed(big, dev)
    plan_big = fmgsr.Batch(big.sizes, big.levels, buffer=big.buffer, op="cubic")
    u_big = plan_big.solve(f, k)
    torch.cuda.synchronize()
    qb = plan_big.query()
    assert qb["group"] == 1 and (qb["threads"], qb["run"]) == (256, 4)
    for j in (0, 17, 599):
        o, n = int(big.offsets[j]), int(big.sizes[j])
        one = fmgsr.Batch((n,), (big.levels[j],), buffer=big.buffer, op="cubic",
                          segments=(int(qb["segments"][j]),))
        u1 = one.solve(f[o:o + n].contiguous(), k[o:o + n].contiguous())
        torch.cuda.synchronize()
        q1 = one.query()
        print(f"problem {j}: n={n} group={q1['group']} grid={q1['grid']}", flush=True)
        assert q1["group"] > 1 and q1["stalled"] == 0 and q1["run"] == 8
        assert torch.equal(u1, u_big[o:o + n])
    assert plan_big.query()["stalled"] == 0
