#!/usr/bin/env python3
"""Benchmark one FMG-FAS-SR iteration on the GPU (1D Poisson, FP64).

A step is one full solve: forcing hierarchy, FMG cycles on every level, the
SR down and up passes over the finest level, result streamed to u_out.  All
inputs are resident in HBM before the timed region.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload c5|c2|c1|c3|c4] [--gpus 1]

Default workload: N = 2^28 fine cells, 29 levels, 2^16 segments of 4096
cells + 8 buffer cells, V(2,1) red-black Gauss-Seidel, 32-mode seeded
manufactured solution.  Timing: HIP events on the solve's stream around K
back-to-back solves (K = 10 by default).  The dominant kernel (largest share
of a profiled solve) is additionally bracketed by events inside the timed
region to report its achieved algorithmic bandwidth against the 8 TB/s HBM
peak.  The CPU baseline times the FP64 oracle on a bounded sample.

Reaction workloads (batched solver, one persistent launch per step):
  c3  4096 problems -u'' + kappa u^3 = f of 2^12..2^18 cells (--precision
      fp64 | fp32relax); a step is one FMG-FAS-SR iteration of every problem.
  c4  64 problems of 2^20 cells; a step is the forward iteration plus the
      adjoint iteration (gradients w.r.t. f and kappa of h sum (u - u_t)^2).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid unknowns/sec, one FMG-FAS-SR iter to discretization error; % HBM peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def closed_form(n, k, c, dev):
    """Discrete solution of the cell-centred problem (sines are exact
    eigenvectors, eigenvalue 4 n^2 sin^2(k pi / 2n)) and the continuous one."""
    import torch
    x = (torch.arange(n, dtype=torch.float64, device=dev) + 0.5) / n
    ustar = torch.zeros(n, dtype=torch.float64, device=dev)
    uex = torch.zeros(n, dtype=torch.float64, device=dev)
    for kk, cc in zip(k, c):
        s = torch.sin(x * (float(kk) * np.pi))
        lam = 4.0 * n * n * np.sin(kk * np.pi / (2 * n)) ** 2
        ustar.add_(s, alpha=float(cc * (kk * np.pi) ** 2 / lam))
        uex.add_(s, alpha=float(cc))
        del s
    del x
    return ustar, uex


def disc_rel_modes(n, k, c):
    """Relative 2-norm of u* - u_exact at the cell centres, from the mode
    sums: mode k of the discrete solution is c_k rho_k with
    rho_k = theta^2 / sin^2(theta), theta = k pi / 2n, and the sampled sines
    are orthogonal with equal norms, so the error is
    sqrt(sum (c_k (rho_k - 1))^2 / sum c_k^2); rho_k - 1 is evaluated by its
    series for small theta (no cancellation)."""
    num = den = 0.0
    for kk, cc in zip(k, c):
        th = float(kk) * np.pi / (2.0 * n)
        if th < 1e-3:
            t2 = th * th
            rm1 = t2 / 3.0 + t2 * t2 / 15.0 + 2.0 * t2 ** 3 / 189.0
        else:
            rm1 = th * th / np.sin(th) ** 2 - 1.0
        num += (cc * rm1) ** 2
        den += cc * cc
    return float(np.sqrt(num / den))


def traffic_for(workload, kernel, kernel_source_hash):
    """Measured HBM bytes per launch of `kernel` in `workload` from the
    committed counter summary, if it was taken on the current sources of
    that workload's kernels (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    w = t.get("workloads", {}).get(workload, {})
    if w.get("source_sha256") != kernel_source_hash:
        return None
    ent = w.get("kernels", {}).get(kernel)
    return ent.get("hbm_bytes_per_launch") if ent else None


# The HIP sources each family of workloads compiles from.
KERNEL_SOURCES = {
    "poisson": ("fmgsr.hip", "fmgsr_kernels.hpp", "fmgsr_device.hpp", "fmgsr_host.hpp"),
    "batched": ("fmgsr_batched.hip", "fmgsr_device.hpp", "fmgsr_host.hpp"),
}


def kernel_source_hash(family):
    """sha256 over the HIP sources and headers of one family's kernels."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1207_6720_amd", "csrc")
    for name in sorted(KERNEL_SOURCES[family]):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def host_info():
    """Host cores the CPU baseline may use and what they are: the process's
    CPU affinity capped at the per-GPU share of the box (OMP_NUM_THREADS when
    set, else 16), nproc, and the model name from /proc/cpuinfo."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": max(1, min(aff, share)), "nproc": os.cpu_count(), "affinity": aff,
            "model": model}


def _available_host_bytes():
    try:
        import psutil
        return psutil.virtual_memory().available
    except Exception:  # noqa: BLE001
        return 0


def run_threads(jobs, threads):
    """Run the callables in `jobs` on `threads` host threads (the oracle is a
    C library called through ctypes, which releases the GIL); returns the
    wall time."""
    import concurrent.futures
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        for fut in [ex.submit(j) for j in jobs]:
            fut.result()
    return time.perf_counter() - t0


def cpu_baseline(wl, dev, sr_levels=1, tau="split", full_max_log2=28, many_log2=24):
    """The FP64 oracle as written (C, no tuning) on the host, two legs:
    - one thread on the workload itself (the whole N; a 2^25 sample of the
      same law and segment geometry only when the host lacks the memory);
    - all cores: one independent oracle solve per thread (seeds 0..P-1 of
      the same law, N = 2^many_log2, same segment geometry), reported as
      aggregate unknowns/s -- the `value`.
    The oracle holds every level (about 70 bytes per fine cell)."""
    import oracle
    from paper_1207_6720_amd import workloads as W
    info = host_info()
    s_core = wl.n // wl.segments

    def problem(n, seed):
        k, c = W.modes(wl.law, wl.n_modes, seed)
        return W.rhs_torch(n, k, c, dev).cpu().numpy()

    def solve(f):
        n = f.size
        oracle.fmgsr_solve(f, levels=n.bit_length(), segments=max(n // s_core, 1),
                           buffer=wl.buffer, nsr=sr_levels, tau=tau)

    # one thread, the workload's own size when the host holds it
    log2n = wl.n.bit_length() - 1
    if log2n > full_max_log2 or _available_host_bytes() < 100 * wl.n:
        log2n = min(log2n, 25)
    n1 = 1 << log2n
    f1 = problem(n1, 0)
    runs = 1 if n1 >= (1 << 27) else 3
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        solve(f1)
        times.append(time.perf_counter() - t0)
    t1 = float(np.median(times))
    del f1
    log(f"oracle, one thread, N=2^{log2n}: {t1:.2f} s")
    # all cores: P independent solves
    P = info["threads"]
    nm = 1 << min(many_log2, wl.n.bit_length() - 1)
    fs = [problem(nm, seed) for seed in range(P)]
    wall = run_threads([lambda f=f: solve(f) for f in fs], P)
    del fs
    log(f"oracle, {P} threads, {P} x N=2^{nm.bit_length() - 1}: {wall:.2f} s")
    return {"value": P * nm / wall, "unit": "unknowns/s", "cores": P, "kind": "oracle",
            "sample": (f"{P} concurrent single-threaded FMG-FAS-SR iterations of the {wl.name} "
                       f"law (seeds 0..{P - 1}) at N=2^{nm.bit_length() - 1} each, segments of "
                       f"{s_core} cells + {wl.buffer} buffer, {sr_levels} SR level(s), {tau} tau, "
                       f"C oracle as written, one per host thread ({wall:.2f} s wall)"),
            "single_thread": {"value": n1 / t1, "unit": "unknowns/s", "n": n1,
                              "seconds": round(t1, 3), "runs": runs,
                              "note": ("the workload itself" if n1 == wl.n else
                                       f"N=2^{log2n} sample of the workload's law")},
            "host": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c5", "c3", "c4"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32relax"])
    ap.add_argument("--functionals-only", action="store_true",
                    help="Poisson workloads: accumulate h sum u and h sum u^2 on the fly and "
                         "never write the fine solution (u_out = NULL)")
    ap.add_argument("--tau", default="split", choices=["split", "literal"])
    ap.add_argument("--sr-levels", type=int, default=1, choices=[0, 1, 2, 3],
                    help="Poisson workloads: number of SR levels (2 and 3: the finest levels "
                         "below the top are SR levels too, split tau only)")
    ap.add_argument("--adjoint-keep", default="u", choices=["u", "coarse"],
                    help="c4: what the forward keeps for the adjoint: u, or only its "
                         "level-(M-1) solution, with u_fwd rebuilt inside the adjoint")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 2^27 doubles (1 GiB read + 1 GiB "
                         "written) so hardware-counter runs can scale FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: the solver has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1207_6720_amd import fmgsr, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.workload in ("c3", "c4"):
        return run_batched(args, dev)
    wl = W.WORKLOADS[args.workload]
    n = wl.n
    k, c = W.modes(wl.law, wl.n_modes, 0)
    log(f"{fmgsr.version()} workload {wl.name}: {wl.description}")
    f = W.rhs_torch(n, k, c, dev)
    fun = torch.zeros(2, dtype=torch.float64, device=dev)
    if args.functionals_only:
        u = None
        kw_out = dict(functionals=fun, write_u=False)
    else:
        u = torch.empty_like(f)
        kw_out = dict(out=u)
    kw = dict(levels=wl.levels, segments=wl.segments, buffer=wl.buffer, nu=(2, 1),
              sr_levels=args.sr_levels, tau=args.tau, precision=args.precision, **kw_out)
    ws = fmgsr.alloc_workspace(n, wl.levels, dev, nu=(2, 1), sr_levels=args.sr_levels,
                               tau=args.tau, segments=wl.segments, buffer=wl.buffer,
                               functionals=args.functionals_only)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 2^27 doubles copied")
    torch.cuda.synchronize()
    mem_inputs = torch.cuda.memory_allocated(dev)

    # warm-up; the first warm-up solve is profiled kernel by kernel
    fmgsr.profile_enable(None)
    fmgsr.solve(f, workspace=ws, stream=stream, **kw)
    torch.cuda.synchronize()
    prof_all = fmgsr.profile_collect()
    for _ in range(max(args.warmup - 1, 0)):
        fmgsr.solve(f, workspace=ws, stream=stream, **kw)
    torch.cuda.synchronize()
    dominant = max(prof_all, key=lambda kname: prof_all[kname]["total_ms"])
    model_bytes = sum(v["algo_bytes"] for v in prof_all.values())
    log(f"warm-up done; dominant kernel {dominant} "
        f"({prof_all[dominant]['total_ms']:.3f} of {sum(v['total_ms'] for v in prof_all.values()):.3f} ms profiled)")

    # timed region: K solves; the last one carries events around each of
    # the dominant kernel's launches (an event pair per launch adds a few
    # microseconds, so only one solve of the K pays for them)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - 1:
            fmgsr.profile_enable(dominant)
        fmgsr.solve(f, workspace=ws, stream=stream, **kw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom = fmgsr.profile_collect()[dominant]
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f} ms/step)")

    # accuracy of the benchmarked result (closed-form discrete solution)
    ustar, uex = closed_form(n, k, c, dev)
    nrm = lambda t: float(torch.linalg.vector_norm(t))
    if u is None:
        fs = [float(ustar.sum()) / n, float((ustar * ustar).sum()) / n]
        fe = [float(uex.sum()) / n, float((uex * uex).sum()) / n]
        got = fun.cpu().tolist()
        acc = {"functionals": got, "functionals_discrete_closed_form": fs,
               "alg_rel": [abs(a - b) / abs(b) for a, b in zip(got, fs)],
               "disc_rel": [abs(a - b) / abs(b) for a, b in zip(fs, fe)]}
    else:
        acc = {"alg_rel": nrm(u - ustar) / nrm(ustar),
               "disc_rel_measured": nrm(ustar - uex) / nrm(uex),
               "total_rel": nrm(u - uex) / nrm(uex)}
        # the discretisation error from the mode sums (no cancellation): at
        # large N it lies below what FP64 vectors can resolve, and the
        # measured differences above are then the FP64 evaluation floor
        acc["disc_rel"] = disc_rel_modes(n, k, c)
        floor = 16 * np.finfo(np.float64).eps
        acc["at_fp64_floor"] = bool(acc["disc_rel"] < floor)
        if acc["at_fp64_floor"]:
            acc["fp64_floor_rel"] = acc.pop("disc_rel_measured")
            acc["alg_over_disc"] = None
            acc["note"] = ("discretisation error below the FP64 floor: alg_rel and "
                           "fp64_floor_rel are rounding of the FP64 evaluation, not method error")
        else:
            acc["alg_over_disc"] = acc["alg_rel"] / acc["disc_rel"]
    del ustar, uex
    peak_mem = torch.cuda.max_memory_allocated(dev)

    dom_launch_ms = dom["total_ms"] / dom["launches"]
    dom_bytes = dom["algo_bytes"] / dom["launches"]
    achieved = dom_bytes / (dom_launch_ms * 1e-3) / 1e9
    variant = (("" if args.precision == "fp64" else "_" + args.precision)
               + ("" if args.sr_levels == 1 else f"_sr{args.sr_levels}")
               + ("" if args.tau == "split" else "_literal")
               + ("_functionals" if args.functionals_only else ""))
    traffic = traffic_for(wl.name + variant, dominant, kernel_source_hash("poisson"))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dominant,
                "algo_bytes_per_launch": dom_bytes, "avg_launch_ms": round(dom_launch_ms, 4),
                "launches": dom["launches"]}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, dev, args.sr_levels, args.tau)

    value = n / (ms * 1e-3)
    out = {
        "metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32relax", "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}"
                               + ("" if args.precision == "fp64" else ", FP32 relaxation")
                               + ("" if args.sr_levels == 1 else f", {args.sr_levels} SR levels"),
                   "n": n, "levels": wl.levels, "precision": args.precision,
                   "segments": wl.segments, "buffer": wl.buffer, "nu": [2, 1],
                   "smoother": "red-black GS", "tau": args.tau, "sr_levels": args.sr_levels,
                   "functionals_only": args.functionals_only,
                   "seed": 0, "modes": wl.n_modes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "solve_model": {"algo_bytes_per_step": model_bytes,
                        "algo_bytes_per_unknown": round(model_bytes / n, 2),
                        "effective_GBps": round(model_bytes / (ms * 1e-3) / 1e9, 1),
                        "frac_of_hbm_peak": round(model_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "accuracy": acc,
        "memory": {"inputs_and_workspace_bytes": mem_inputs, "peak_allocated_bytes": peak_mem,
                   "workspace_bytes": ws.numel(),
                   "workspace_bytes_full_grid_fmg": fmgsr.workspace_bytes(n, wl.levels, sr_levels=0,
                                                                          tau=args.tau, segments=1,
                                                                          buffer=0),
                   "workspace_bytes_sr": fmgsr.workspace_bytes(n, wl.levels, sr_levels=1,
                                                               tau=args.tau, segments=wl.segments,
                                                               buffer=wl.buffer),
                   "workspace_bytes_two_sr_levels": fmgsr.workspace_bytes(
                       n, wl.levels, sr_levels=2, tau=args.tau, segments=wl.segments,
                       buffer=wl.buffer)},
        "kernels": {kname: {"launches": v["launches"], "ms": round(v["total_ms"], 4),
                            "GBps": round(v["algo_bytes"] / max(v["total_ms"], 1e-9) / 1e6, 1)}
                    for kname, v in sorted(prof_all.items(), key=lambda kv: -kv[1]["total_ms"])},
    }
    print(json.dumps(out), flush=True)


def oracle_sample(rb, f_host, k_host, segs, budget_unknowns):
    """Indices of a bounded oracle sample: problems in batch order until the
    sample holds about budget_unknowns cells."""
    idx, tot = [], 0
    for j in range(rb.batch):
        if tot >= budget_unknowns:
            break
        idx.append(j)
        tot += rb.sizes[j]
    return idx, tot


def run_batched(args, dev):
    import torch
    from paper_1207_6720_amd import fmgsr, workloads as W
    rb = W.reaction_batch(args.workload)
    adjoint = args.workload == "c4"
    log(f"{fmgsr.version()} workload {rb.name}: {rb.description}")
    f, k, ue, ut = W.reaction_packed_torch(rb, dev)
    u = torch.empty_like(f)
    gf, gk, dJ = None, None, None
    plan = fmgsr.Batch(rb.sizes, rb.levels, buffer=rb.buffer, op="cubic",
                       precision=args.precision)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 2^27 doubles copied")
    keep_coarse = adjoint and args.adjoint_keep == "coarse"
    coarse = None
    if adjoint:
        hvec = torch.cat([torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
                          for n in rb.sizes])
        gf, gk, dJ = torch.empty_like(f), torch.empty_like(f), torch.empty_like(f)
        if keep_coarse:
            coarse = torch.empty(plan.coarse_total, dtype=torch.float64, device=dev)

    tuned_ms = plan.autotune(f, k, u, stream=stream)
    log(f"autotuned: {tuned_ms:.3f} ms per solve, {plan.query()['threads']} threads, "
        f"group {plan.query()['group']}")

    def step():
        if keep_coarse:
            plan.solve_keep(f, k, coarse=coarse, out=u, stream=stream)
        else:
            plan.solve(f, k, out=u, stream=stream)
        if adjoint:
            torch.sub(u, ut, out=dJ)
            dJ.mul_(hvec).mul_(2.0)
            if keep_coarse:
                plan.adjoint_compressed(k, f, coarse, dJ, gf, gk, stream=stream)
            else:
                plan.adjoint(k, u, dJ, gf, gk, stream=stream)

    torch.cuda.synchronize()
    mem_inputs = torch.cuda.memory_allocated(dev)
    fmgsr.profile_enable(None)
    step()
    torch.cuda.synchronize()
    prof_all = fmgsr.profile_collect()
    for _ in range(max(args.warmup - 1, 0)):
        step()
    torch.cuda.synchronize()
    dominant = max(prof_all, key=lambda kname: prof_all[kname]["total_ms"])
    log(f"warm-up done; dominant kernel {dominant}")
    fmgsr.profile_enable(dominant)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    dom = fmgsr.profile_collect()[dominant]
    ms = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step")
    q = plan.query()
    segs = q["segments"]

    # accuracy on a sample of problems, on the device: error against the
    # manufactured solution and the residual of the discrete equations
    acc = {"total_rel_max": 0.0, "residual_rel_max": 0.0, "problems": []}
    for j in sorted({0, rb.batch // 2, rb.batch - 1}):
        o, n = int(rb.offsets[j]), int(rb.sizes[j])
        fj, kj, uj, ej = (t[o:o + n] for t in (f, k, u, ue))
        g = torch.cat([-uj[:1], uj, -uj[-1:]])          # homogeneous Dirichlet ghosts
        Nu = (2.0 * uj - (g[:-2] + g[2:])) * float(n * n) + kj * (uj * uj * uj)
        nrm = lambda t_: float(torch.linalg.vector_norm(t_))
        tot, res = nrm(uj - ej) / nrm(ej), nrm(Nu - fj) / nrm(fj)
        acc["problems"].append({"j": j, "n": n, "total_rel": tot, "residual_rel": res})
        acc["total_rel_max"] = max(acc["total_rel_max"], tot)
        acc["residual_rel_max"] = max(acc["residual_rel_max"], res)

    dom_launch_ms = dom["total_ms"] / dom["launches"]
    dom_bytes = dom["algo_bytes"] / dom["launches"]
    achieved = dom_bytes / (dom_launch_ms * 1e-3) / 1e9
    traffic = traffic_for(rb.name + ("" if args.precision == "fp64" else "_" + args.precision),
                          dominant, kernel_source_hash("batched"))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dominant, "algo_bytes_per_launch": dom_bytes,
                "avg_launch_ms": round(dom_launch_ms, 4), "launches": dom["launches"]}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle  # CPU baseline only
        # bounded sample of about ten seconds of oracle work: problems in
        # batch order up to ~2e8 cells (c3), or the 64 problems (c4),
        # forward (+ adjoint) by the oracle, single thread
        budget = (3 << 26) if not adjoint else 64 * int(rb.sizes[0])
        idx, tot = oracle_sample(rb, None, None, segs, budget)
        f_h, k_h = f.cpu().numpy(), k.cpu().numpy()
        ut_h = ut.cpu().numpy() if adjoint else None

        def job(j):
            o, n = int(rb.offsets[j]), int(rb.sizes[j])
            fj, kj = f_h[o:o + n], k_h[o:o + n]
            uj = oracle.rx_fmgsr_solve("cubic", fj, kj, levels=rb.levels[j],
                                       segments=int(segs[j]), buffer=rb.buffer)
            if adjoint:
                oracle.rx_fmgsr_adjoint(kj, uj, 2.0 / n * (uj - ut_h[o:o + n]),
                                        levels=rb.levels[j], segments=int(segs[j]),
                                        buffer=rb.buffer)

        info = host_info()
        P = info["threads"]
        # one thread over the first quarter of the sample, then the whole
        # sample with one problem per host thread at a time
        q_idx = idx[:max(1, len(idx) // 4)]
        q_tot = sum(int(rb.sizes[j]) for j in q_idx)
        t1 = run_threads([lambda j=j: job(j) for j in q_idx], 1)
        t = run_threads([lambda j=j: job(j) for j in idx], P)
        # the sample's oracle results against the GPU's (first problems)
        worst = 0.0
        for j in idx[:4]:
            o, n = int(rb.offsets[j]), int(rb.sizes[j])
            fj, kj = f[o:o + n].cpu().numpy(), k[o:o + n].cpu().numpy()
            ref = oracle.rx_fmgsr_solve("cubic", fj, kj, levels=rb.levels[j],
                                        segments=int(segs[j]), buffer=rb.buffer)
            uj = u[o:o + n].cpu().numpy()
            worst = max(worst, float(np.linalg.norm(uj - ref) / np.linalg.norm(ref)))
        cpu = {"value": tot / t, "unit": "unknowns/s", "cores": P, "kind": "oracle",
               "gpu_vs_oracle_rel_max": worst,
               "sample": (f"{len(idx)} problem(s) of the {rb.name} batch ({tot} cells), "
                          f"{'forward + adjoint' if adjoint else 'one FMG-FAS-SR iteration'} "
                          f"by the C oracle as written, one problem per host thread on {P} "
                          f"threads ({t:.2f} s wall)"),
               "single_thread": {"value": q_tot / t1, "unit": "unknowns/s", "cells": q_tot,
                                 "seconds": round(t1, 3),
                                 "note": f"first {len(q_idx)} problem(s) of the sample"},
               "host": info}
        log(f"oracle sample: {cpu['sample']}")

    out = {
        "metric": METRIC, "value": rb.total / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32relax", "data": "synthetic",
        "config": {"workload": f"{rb.name}: {rb.description}"
                               + (", forward + adjoint per step" if adjoint else ""),
                   "batch": rb.batch, "total_unknowns": rb.total, "buffer": rb.buffer,
                   "nu": [2, 1], "smoother": "red-black nonlinear GS", "precision": args.precision,
                   "seed": rb.seed, "threads": q["threads"], "run": q["run"], "grid": q["grid"],
                   "group": q["group"], "autotuned": True}
                  | ({"adjoint_keep": args.adjoint_keep} if adjoint else {}),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "solve_model": {"algo_bytes_per_step": sum(v["algo_bytes"] for v in prof_all.values()),
                        "algo_bytes_per_unknown": round(sum(v["algo_bytes"] for v in prof_all.values()) / rb.total, 2)},
        "accuracy": acc,
        "memory": {"inputs_and_workspace_bytes": mem_inputs,
                   "workspace_bytes": q["workspace_bytes"],
                   "peak_allocated_bytes": torch.cuda.max_memory_allocated(dev)}
                  | ({"adjoint_state_bytes": 8 * (plan.coarse_total if keep_coarse else rb.total),
                      "adjoint_state": ("the forward's level-(M-1) solution (u_fwd rebuilt "
                                        "inside the adjoint)" if keep_coarse else "u_fwd")}
                     if adjoint else {}),
        "kernels": {kname: {"launches": v["launches"], "ms": round(v["total_ms"], 4),
                            "GBps": round(v["algo_bytes"] / max(v["total_ms"], 1e-9) / 1e6, 1)}
                    for kname, v in prof_all.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
