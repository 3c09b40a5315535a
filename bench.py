"""Throughput of the full time step on one MI355X.

Default workload: the 500x300 2D cavity (Sn-10%Pb-type alloy, west wall
cooled by h = 400 W/m^2K to 298 K, PCG / BiCGSTAB tolerance 1e-10), FP64,
pressure CG preconditioned by a multigrid V-cycle (--precond jacobi for the
inverse diagonal).
A step is one pass of Algorithm 1 (momentum predictor, pressure
correction, projection, solute, energy, phase update) through the HIP
library; value = cells x steps / wall time of the timed steps, with the
state resident on the device.

Also printed in the same JSON line:
  roofline      achieved algorithmic GB/s of the dominant kernel (HIP events
                on the library's stream: windows of 16 launches for the
                single-kernel CG, single launches otherwise) against 8 TB/s,
                and the counter-measured HBM bytes per launch;
  cpu_baseline  the FP64 oracle on the host for a bounded number of steps;
  variants      the same step in mixed precision, with graphs and with
                Jacobi-PCG, the 128x128x64 box (FP64, mixed, Jacobi-PCG), 64
                uneven cavities in one batch (mixed and FP64,
                graph-replayed chunks, tuned tiles) and the served request
                stream (continuous batching, p50/p99 latency).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per full time step (1 GPU), mixed vs FP64; p50/p99 case latency"
HBM_PEAK_GBS = 8000.0


def roofline(g, nsteps, cg_launches_per_step):
    """Dominant kernel class by GPU time per step.  Every launch of a class is
    timed (dispatch-stamped events), so its time per step is the timed total
    over the timing steps; the single-kernel Jacobi CG is timed in windows of
    16 launches, its time per step is the window average x iterations.  The
    multigrid coarse-level class spans several kernels and carries no byte
    count; it is not a candidate."""
    best = None
    classes = {}
    for cls in ("cg", "bicg_a", "bicg_b", "bicg_c", "asm_mom", "asm_trn", "phase", "mg_pq", "mg_down0", "mg_up0"):
        t = g.timing(cls)
        if t["launches"] == 0 or t["bytes"] == 0:
            continue
        t["avg_ms"] = t["ms"] / t["launches"]
        t["bytes_per_launch"] = t["bytes"] / t["launches"]
        t["gbs"] = t["bytes"] / (t["ms"] * 1e-3) / 1e9
        t["cls"] = cls
        t["est_ms_per_step"] = t["avg_ms"] * cg_launches_per_step if cls == "cg" else t["ms"] / nsteps
        classes[cls] = dict(avg_us=round(t["avg_ms"] * 1e3, 2), mb_per_launch=round(t["bytes_per_launch"] / 1e6, 2),
                            gbs=round(t["gbs"], 1), frac=round(t["gbs"] / HBM_PEAK_GBS, 4),
                            ms_per_step=round(t["est_ms_per_step"], 4))
        if best is None or t["est_ms_per_step"] > best["est_ms_per_step"]:
            best = t
    if best is not None:
        best["classes"] = classes
    return best


def kernel_sources_sha():
    """sha256 over the kernel sources (the counters are void once they change)."""
    h = hashlib.sha256()
    for f in ("kcommon.hpp", "sol_dev.hpp", "kernels.hip", "mg.hip"):
        h.update(open(os.path.join(ROOT, "paper_2303_10783_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def counter_traffic(workload, kernel_cls, precond):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the copy reference),
    or None when that summary does not cover this workload and kernel or the
    kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    doc = json.load(open(path))
    key = f"{workload}:{precond}:{kernel_cls}"
    if doc.get("kernel_sources_sha256") != kernel_sources_sha() or key not in doc:
        return None
    return doc[key]["traffic_bytes_per_launch"]


def run_single(sol, W, key, precision, steps, warmup, dev, graph=False, precond="mg", tprecond=None):
    import torch
    case = W.workload_case(key)
    if precision == "mixed":
        case["numerics"]["precision"] = W.PRECISION_MIXED
    g = case["grid"]
    ncell = g["nx"] * g["ny"] * (g["nz"] if g["dim"] == 3 else 1)
    h = sol.Case(case, device=dev)
    if precond != "mg":
        h.set_precond(precond)
    if tprecond:
        h.set_tprecond(tprecond)
    if graph:
        h.set_graph(True)
    if warmup:
        h.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    h.close()
    return dict(value=ncell * steps / secs, ms_per_step=1e3 * secs / steps, steps=steps,
                krylov_iters_per_step={n: round(st["iters_total"][i] / steps, 1) for i, n in enumerate("uvwpCT")},
                steps_redone=st["redone"])


def run_batched(sol, W, precision, steps, warmup, dev, n_cases=64, graph=True, tune=True):
    """64 cavities of uneven size (aspect 0.5-4, 6e3-9.6e4 cells, h and C0
    drawn per case), every kernel launched once for all of them."""
    import torch
    cases = W.batch_cases(n_cases, seed=0, precision=W.PRECISION_MIXED if precision == "mixed" else W.PRECISION_FP64)
    cells = [c["grid"]["nx"] * c["grid"]["ny"] for c in cases]
    tuned = {}
    if tune:
        # one tuning run per size class, on the largest case of the class
        by_cls = {}
        for c, n in zip(cases, cells):
            k = int(n).bit_length()
            if k not in by_cls or n > by_cls[k][1]:
                by_cls[k] = (c, n)
        for k, (c, n) in sorted(by_cls.items()):
            h = sol.Case(c, device=dev)
            tuned[n] = h.autotune()
            h.close()
    hs = [sol.Case(c, device=dev) for c in cases]
    if graph:
        hs[0].set_graph(True)
    b = sol.Batch(hs)
    if warmup:
        b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    b.close()
    for h in hs:
        h.close()
    return dict(value=sum(cells) * steps / secs, ms_per_step=1e3 * secs / steps, steps=steps,
                cases=n_cases, cells=sum(cells), min_cells=min(cells), max_cells=max(cells),
                graph=graph, tuned_rows_per_tile={str(k): v for k, v in sorted(tuned.items())})


def run_served(sol, W, dev, n_requests=40, scale=0.1, steps=200, rate=20.0):
    """Poisson arrivals at `rate`/s of 2D and 3D cases (sizes log-uniform in
    the served ranges times `scale`), 200 steps each, mixed precision."""
    from paper_2303_10783_amd.serve import Request, Server
    reqs = W.served_arrivals(n_requests, seed=0, rate=rate, scale=scale)
    requests = [Request(case=c, steps=steps, arrival=c["arrival_s"], rid=i) for i, c in enumerate(reqs)]
    srv = Server(device=dev, max_active=64, graph=True, keep_results=False)
    out = srv.run(requests)
    out.pop("done")
    out.update(n_requests=n_requests, size_scale=scale, steps_per_request=steps, arrival_rate_per_s=rate)
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}


def cpu_baseline(case, budget_s=12.0, max_steps=20):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    o = oracle.Oracle(case, threads=threads)
    n = case["grid"]["nx"] * case["grid"]["ny"] * (case["grid"]["nz"] if case["grid"]["dim"] == 3 else 1)
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=n * steps / dt, unit="cell-updates/s", cores=threads, kind="oracle",
                sample=f"first {steps} steps of the same workload from its initial state, "
                       f"FP64 C oracle, {threads} OpenMP threads, {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay Krylov chunks as HIP graphs")
    ap.add_argument("--precond", default="mg", choices=["mg", "jacobi"],
                    help="pressure-CG preconditioner (multigrid V-cycle or Jacobi)")
    ap.add_argument("--tprecond", default=None, choices=["jacobi", "jacobi2", "auto"],
                    help="BiCGSTAB preconditioner: one or two Jacobi sweeps, or the library's default "
                         "(auto: two in 2D, one in 3D)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent cases shard across GPUs without communication; not built here)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_10783_amd as sol
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    case = W.workload_case(args.workload)
    if args.precision == "mixed":
        case["numerics"]["precision"] = W.PRECISION_MIXED
    grid = case["grid"]
    ncell = grid["nx"] * grid["ny"] * (grid["nz"] if grid["dim"] == 3 else 1)
    dev = sol.TorchDevice(0)
    g = sol.Case(case, device=dev)
    if args.precond != "mg":
        g.set_precond(args.precond)
    if args.tprecond:
        g.set_tprecond(args.tprecond)
    if args.graph:
        g.set_graph(True)
    if args.warmup:
        g.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    value = ncell * args.steps / secs
    iters = st["iters_total"]

    roof = None
    step_roof = None
    if not args.no_roofline:
        g.set_timing(True)
        st2 = g.step(2)
        best = roofline(g, 2, st2["iters_total"][3] / 2)
        # whole step: algorithmic bytes of every timed class over the two
        # timing steps, per cell-update, at the throughput measured above
        tot = sum(g.timing(c)["bytes"] for c in ("cg", "bicg_a", "bicg_b", "asm_mom", "asm_trn", "phase",
                                                 "mg_pq", "mg_down0", "mg_up0"))
        bpc = tot / (2 * ncell)
        step_roof = dict(bytes_per_cell_update=round(bpc, 1), achieved_gbs=round(bpc * value / 1e9, 1),
                         peak=HBM_PEAK_GBS, frac=round(bpc * value / 1e9 / HBM_PEAK_GBS, 4),
                         note="algorithmic bytes of the Krylov, multigrid level-0, assembly and phase kernels; "
                              "start, finish, coarse-level, divergence and projection launches count as time only")
        g.set_timing(False)
        if best:
            tr = counter_traffic(args.workload, best["cls"], args.precond) if args.precision == "fp64" else None
            roof = dict(bound="hbm", achieved=round(best["gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(best["gbs"] / HBM_PEAK_GBS, 4), traffic=tr,
                        kernel=best["cls"], avg_us=round(best["avg_ms"] * 1e3, 2),
                        bytes_per_launch=int(best["bytes_per_launch"]),
                        timed_launches=int(best["launches"]),
                        all_classes=best["classes"])
    g.close()
    variants = None
    if not args.no_variants:
        variants = {}
        if args.workload == "C2" and args.precision == "fp64":
            variants["C2_mixed"] = run_single(sol, W, "C2", "mixed", args.steps, args.warmup, dev)
            variants["C2_fp64_graph"] = run_single(sol, W, "C2", "fp64", args.steps, args.warmup, dev, graph=True)
            variants["C2_fp64_jacobi"] = run_single(sol, W, "C2", "fp64", args.steps, args.warmup, dev,
                                                    precond="jacobi")
        variants["C3_fp64"] = run_single(sol, W, "C3", "fp64", 5, 1, dev)
        variants["C3_mixed"] = run_single(sol, W, "C3", "mixed", 5, 1, dev)
        variants["C3_fp64_jacobi"] = run_single(sol, W, "C3", "fp64", 5, 1, dev, precond="jacobi")
        variants["C4_batched_mixed"] = run_batched(sol, W, "mixed", 5, 1, dev)
        variants["C4_batched_fp64"] = run_batched(sol, W, "fp64", 5, 1, dev, tune=False)
        variants["C5_served_mixed"] = run_served(sol, W, dev)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(case)
    out = dict(
        metric=METRIC, value=value, unit="cell-updates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=1e3 * secs / args.steps, higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64" if args.precision == "fp64" else "f32+f64", data="synthetic",
        config=dict(workload=f"{args.workload}: 2D cavity {grid['nx']}x{grid['ny']}" if grid["dim"] == 2
                    else f"{args.workload}: 3D box {grid['nx']}x{grid['ny']}x{grid['nz']}",
                    cells=ncell, dt=case["numerics"]["dt"], tol=case["numerics"]["tol_p"],
                    precision=args.precision, pressure_precond=args.precond,
                    transport_precond=args.tprecond or "auto", krylov_iters_per_step={
                        n: round(iters[i] / args.steps, 1) for i, n in enumerate("uvwpCT")},
                    steps_redone=st["redone"]),
        roofline=roof, step_roofline=step_roof, cpu_baseline=cpu, variants=variants,
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()
