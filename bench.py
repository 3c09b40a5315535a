"""Throughput of the full time step on one MI355X.

Headline workload: the 128x128x64 3D box (Sn-10%Pb-type alloy, west face
cooled by h = 400 W/m^2K to 298 K, other faces adiabatic, PCG / BiCGSTAB
tolerance 1e-10), FP64, 500 steps from the initial state (the workload as
defined); pressure CG preconditioned by a multigrid V-cycle.  A step is one
pass of Algorithm 1 (momentum predictor, pressure correction, projection,
solute, energy, phase update) through the HIP library; value = cells x
steps / wall time of the timed steps, with the state resident on the device.
The warm-up steps run first (one-time set-up, caches), then the initial
fields are written back, so the timed steps are steps 1..K of the workload.

Also printed in the same JSON line:
  roofline      achieved algorithmic GB/s of the dominant kernel: HIP events
                stamped by each launch on the library's stream, over a second
                pass of the same K steps from the same initial state; the
                counter-measured HBM bytes per launch (rocprofv3 FETCH_SIZE /
                WRITE_SIZE scaled by a plain copy of known size) when the
                committed counters match the kernel sources;
  cpu_baseline  the FP64 oracle on the host: the first steps of the same
                workload on all host cores and on one core, the 50x30 cavity
                in full, and the per-field error of the GPU's FP64 and mixed
                runs of those first steps against the oracle's fields;
  variants      the same box in mixed precision (500 steps), with the coarse
                multigrid levels one launch each instead of fused in pairs
                (the box and the 500x300 cavity), with the forward
                (residual-probing) assembly route and its assembly kernels'
                times next to the stencil route's, the box in FP64
                and mixed at the tight tolerances that hold the fields within
                1e-8 of the oracle (errors in cpu_baseline), the 500x300
                cavity (1000 steps, FP64 and mixed), the 50x30 cavity (200
                steps, FP64 and mixed), 64 uneven cavities in one batch (300
                steps, mixed and FP64, workload and tight tolerances) and the
                served request stream (Poisson
                arrivals at 20/s of 2D and 3D cases at their stated sizes, 200
                steps each, continuous batching, p50/p99 latency, offered vs
                served load).

`python bench.py --copy-reference` instead runs the plain device copy of a
known size whose hardware counters calibrate the HBM-traffic figures.
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
# solver tolerances (pressure, transport) at which GPU and oracle fields agree
# to 1e-8 per field after the first steps: the workload's 1e-10 lets each
# solver stop anywhere in its band, and the buoyancy amplifies a T* difference
# of that size ~5e3-fold into the velocity
TIGHT = (1e-12, 1e-13)
TIGHT_BATCH = (3e-13, 1e-13)
KCLASSES = ("cg", "bicg_a", "bicg_b", "asm_mom", "asm_trn", "phase", "mg_pq", "mg_down0", "mg_up0")
FIELDS = ("u", "v", "w", "p", "T", "C", "gl", "Cl", "Cs")


def copy_reference():
    """A plain device-to-device copy of 256 MiB (read) + 256 MiB (written),
    five launches: run under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, to
    get the counter values of a kernel whose HBM bytes are known."""
    import torch
    n = 32 * 1024 * 1024
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_reference_bytes_per_launch=n * 8, launches=5)))


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


def kernel_classes(h, nsteps, cg_launches_per_step):
    """Per timed kernel class: average launch time, algorithmic bytes per
    launch, achieved GB/s; the dominant class is the one with the largest GPU
    time per step.  Every launch of a class is timed (dispatch-stamped
    events); the single-kernel Jacobi CG is timed in windows of 16 launches,
    its time per step is the window average x iterations.  The multigrid
    coarse-level class carries no byte count and is not a candidate."""
    best = None
    classes = {}
    for cls in KCLASSES:
        t = h.timing(cls)
        if t["launches"] == 0 or t["bytes"] == 0:
            continue
        t["avg_ms"] = t["ms"] / t["launches"]
        t["bytes_per_launch"] = t["bytes"] / t["launches"]
        t["gbs"] = t["bytes"] / (t["ms"] * 1e-3) / 1e9
        t["cls"] = cls
        t["est_ms_per_step"] = t["avg_ms"] * cg_launches_per_step if cls == "cg" else t["ms"] / nsteps
        classes[cls] = dict(avg_us=round(t["avg_ms"] * 1e3, 2), mb_per_launch=round(t["bytes_per_launch"] / 1e6, 2),
                            gbs=round(t["gbs"], 1), frac=round(t["gbs"] / HBM_PEAK_GBS, 4),
                            ms_per_step=round(t["est_ms_per_step"], 4), launches=int(t["launches"]))
        if best is None or t["est_ms_per_step"] > best["est_ms_per_step"]:
            best = t
    return best, classes


def _cells(case):
    g = case["grid"]
    return g["nx"] * g["ny"] * (g["nz"] if g["dim"] == 3 else 1)


def _describe(key, case):
    g = case["grid"]
    shape = f"2D cavity {g['nx']}x{g['ny']}" if g["dim"] == 2 else f"3D box {g['nx']}x{g['ny']}x{g['nz']}"
    return f"{key}: {shape}"


def run_single(sol, W, key, precision, steps, warmup, dev, *, precond="mg", tprecond=None, graph=False,
               timing=False, keep_fields=None, tols=None, assembly=None, mg_fuse=None):
    """K steps of a named workload from its initial state (after W warm-up
    steps and a rewrite of the initial fields).  With timing, a second pass
    over the same K steps with every solver launch timed by HIP events gives
    the per-kernel roofline.  keep_fields=k also returns the fields after the
    first k steps (a third, short pass)."""
    import torch
    case = W.workload_case(key)
    if precision == "mixed":
        case["numerics"]["precision"] = W.PRECISION_MIXED
    if tols:
        case["numerics"]["tol_p"], case["numerics"]["tol_t"] = tols
    ncell = _cells(case)
    h = sol.Case(case, device=dev)
    if precond != "mg":
        h.set_precond(precond)
    if tprecond:
        h.set_tprecond(tprecond)
    if graph:
        h.set_graph(True)
    if assembly:
        h.set_assembly(assembly)
    if mg_fuse is not None:
        h.set_mg_fuse(mg_fuse)
    if warmup:
        h.step(warmup)
        h.write_fields(case["init"])
    torch.cuda.synchronize()
    d0 = sol.binding.dispatch_count()
    t0 = time.perf_counter()
    st = h.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    launches = (sol.binding.dispatch_count() - d0) / steps
    out = dict(workload=_describe(key, case), cells=ncell, precision=precision, value=ncell * steps / secs,
               ms_per_step=1e3 * secs / steps, launches_per_step=round(launches, 1),
               steps=steps, warmup=warmup, tol=case["numerics"]["tol_p"],
               tol_transport=case["numerics"]["tol_t"],
               krylov_iters_per_step={n: round(st["iters_total"][i] / steps, 1) for i, n in enumerate("uvwpCT")},
               steps_redone=st["redone"])
    if precond != "mg":
        out["pressure_precond"] = precond
    if assembly:
        out["assembly"] = assembly
    if graph:
        out["graph"] = True
    if mg_fuse is not None:
        out["coarse_levels_fused"] = bool(mg_fuse)
    if timing:
        h.write_fields(case["init"])
        h.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2 = h.step(steps)
        torch.cuda.synchronize()
        secs2 = time.perf_counter() - t0
        best, classes = kernel_classes(h, steps, st2["iters_total"][3] / steps)
        # whole step: algorithmic bytes of every timed class per cell-update,
        # at the throughput of the untimed pass
        tot = sum(h.timing(c)["bytes"] for c in KCLASSES)
        bpc = tot / (steps * ncell)
        out["timing_pass_ms_per_step"] = 1e3 * secs2 / steps
        out["step_roofline"] = dict(
            bytes_per_cell_update=round(bpc, 1), achieved_gbs=round(bpc * out["value"] / 1e9, 1),
            peak=HBM_PEAK_GBS, frac=round(bpc * out["value"] / 1e9 / HBM_PEAK_GBS, 4),
            note="algorithmic bytes of the Krylov, multigrid level-0, assembly and phase kernels; start, finish, "
                 "coarse-level, divergence and projection launches count as time only")
        out["_best"] = best
        out["_classes"] = classes
        h.set_timing(False)
    if keep_fields:
        h.write_fields(case["init"])
        h.step(keep_fields)
        out["_fields"] = h.read_fields()
        out["_fields_steps"] = keep_fields
    h.close()
    return out


def run_batched(sol, W, precision, steps, warmup, dev, n_cases=64, graph=True, tune=True, tols=None):
    """64 cavities of uneven size (aspect 0.5-4, 6e3-9.6e4 cells, h and C0
    drawn per case), every kernel launched once for all of them; timed steps
    1..K from the initial state after W warm-up steps."""
    import torch
    cases = W.batch_cases(n_cases, seed=0, precision=W.PRECISION_MIXED if precision == "mixed" else W.PRECISION_FP64)
    if tols:
        for c in cases:
            c["numerics"]["tol_p"], c["numerics"]["tol_t"] = tols
    cells = [_cells(c) for c in cases]
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
        b.close()
        for h, c in zip(hs, cases):
            h.write_fields(c["init"])
        b = sol.Batch(hs)
    torch.cuda.synchronize()
    d0 = sol.binding.dispatch_count()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    launches = (sol.binding.dispatch_count() - d0) / steps
    b.close()
    for h in hs:
        h.close()
    return dict(workload=f"C4: {n_cases} 2D cavities in one batch", precision=precision,
                value=sum(cells) * steps / secs, ms_per_step=1e3 * secs / steps,
                launches_per_step=round(launches, 1), steps=steps, warmup=warmup,
                cases=n_cases, cells=sum(cells), min_cells=min(cells), max_cells=max(cells),
                tol=cases[0]["numerics"]["tol_p"], tol_transport=cases[0]["numerics"]["tol_t"],
                graph=graph, tuned_rows_per_tile={str(k): v for k, v in sorted(tuned.items())})


def run_served(sol, W, dev, n_requests=40, scale=1.0, steps=200, rate=20.0):
    """Poisson arrivals at `rate`/s of 2D and 3D cases (sizes log-uniform in
    the served ranges, 2D 6e3-3.8e5 and 3D 3.3e4-3.5e6 cells at scale 1),
    200 steps each, mixed precision, continuous batching."""
    from paper_2303_10783_amd.serve import Request, Server
    reqs = W.served_arrivals(n_requests, seed=0, rate=rate, scale=scale)
    requests = [Request(case=c, steps=steps, arrival=c["arrival_s"], rid=i) for i, c in enumerate(reqs)]
    srv = Server(device=dev, max_active=64, graph=True, keep_results=False)
    out = srv.run(requests)
    out.pop("done")
    out["rejected"] = len(out["rejected"])
    cells = [_cells(c) for c in reqs]
    out.update(workload="C5: served stream", precision="mixed", n_requests=n_requests, size_scale=scale,
               steps_per_request=steps, arrival_rate_per_s=rate, min_cells=min(cells), max_cells=max(cells),
               total_cell_updates=sum(cells) * steps,
               load_note="offered = cell-updates of the requests over their arrival span; above the served "
                         "rate the queue grows through the run and the latencies include that wait"
               if out["offered_cell_updates_per_s"] > out["cell_updates_per_s"] else "offered below served rate")
    out["value"] = out.pop("cell_updates_per_s")
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()}


def _field_errors(got, ref):
    import numpy as np
    out = {}
    for k in FIELDS:
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        if b.size == 0 or a.size == 0:
            continue
        if k == "p":
            a, b = a - a.mean(), b - b.mean()
        den = np.linalg.norm(b)
        out[k] = float(f"{(np.linalg.norm(a - b) / den if den > 0 else np.linalg.norm(a - b)):.2e}")
    return out


def cpu_baseline(W, key, steps_all, steps_one, gpu_fields=None, c1_gpu_fields=None, tight=None):
    """The FP64 oracle on the host (never tuned for this): the first
    `steps_all` steps of the workload on all host cores (<= 16 threads) and
    the first `steps_one` on one core; the 50x30 cavity in full (200 steps);
    the GPU runs' fields after the same first steps against the oracle's."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    case = W.workload_case(key)
    n = _cells(case)
    o = oracle.Oracle(case, threads=threads)
    t0 = time.perf_counter()
    o.step(steps_all)
    dt = time.perf_counter() - t0
    ref = o.fields()
    o1 = oracle.Oracle(case, threads=1)
    t0 = time.perf_counter()
    o1.step(steps_one)
    dt1 = time.perf_counter() - t0
    out = dict(value=n * steps_all / dt, unit="cell-updates/s", cores=threads, kind="oracle",
               sample=f"first {steps_all} steps of {_describe(key, case)} from its initial state, FP64 C oracle, "
                      f"{threads} OpenMP threads, {dt:.1f} s",
               one_core=dict(value=n * steps_one / dt1, cores=1,
                             sample=f"first {steps_one} step(s) of the same workload on one thread, {dt1:.1f} s"))
    if gpu_fields:
        out["gpu_field_error_vs_oracle"] = {
            "steps": steps_all, "tol": case["numerics"]["tol_p"],
            **{prec: _field_errors(f, ref) for prec, f in gpu_fields.items()}}
    if tight:
        tols, fields = tight
        ct = W.workload_case(key)
        ct["numerics"]["tol_p"], ct["numerics"]["tol_t"] = tols
        ot = oracle.Oracle(ct, threads=threads)
        t0 = time.perf_counter()
        ot.step(steps_all)
        dtt = time.perf_counter() - t0
        out["gpu_field_error_vs_oracle_tight"] = {
            "steps": steps_all, "tol": tols[0], "tol_transport": tols[1], "oracle_seconds": round(dtt, 1),
            **{prec: _field_errors(f, ot.fields()) for prec, f in fields.items()}}
    c1 = W.workload_case("C1")
    n1 = _cells(c1)
    for th, tag in ((threads, "all_cores"), (1, "one_core")):
        oc = oracle.Oracle(c1, threads=th)
        t0 = time.perf_counter()
        oc.step(200)
        d = time.perf_counter() - t0
        out.setdefault("C1", {})[tag] = dict(value=round(n1 * 200 / d, 1), cores=th, seconds=round(d, 2))
    out["C1"]["sample"] = "C1: 2D cavity 50x30, all 200 steps"
    if c1_gpu_fields:
        out["C1"]["gpu_field_error_vs_oracle"] = {prec: _field_errors(f, oc.fields())
                                                  for prec, f in c1_gpu_fields.items()}
    return out


def _public(d):
    return {k: v for k, v in d.items() if not k.startswith("_")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's own count)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="C3", choices=["C1", "C2", "C3"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--jacobi-variants", action="store_true", help="also time Jacobi-PCG pressure solves")
    ap.add_argument("--graph", action="store_true", help="replay Krylov chunks as HIP graphs")
    ap.add_argument("--mg-per-level", action="store_true",
                    help="coarse multigrid levels one launch each (default: fused in pairs)")
    ap.add_argument("--precond", default="mg", choices=["mg", "jacobi"],
                    help="pressure-CG preconditioner (multigrid V-cycle or Jacobi)")
    ap.add_argument("--tprecond", default=None, choices=["jacobi", "jacobi2", "auto"],
                    help="BiCGSTAB preconditioner: one or two Jacobi sweeps, or the library's default "
                         "(auto: two in 2D, one in 3D)")
    ap.add_argument("--batch-only", choices=["mixed", "fp64"], default=None,
                    help="run only the 64-cavity batch (300 steps) in this precision and print its line")
    ap.add_argument("--copy-reference", action="store_true",
                    help="run only the plain 256 MiB device copy used to calibrate the traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent cases shard across GPUs without communication; not built here)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_reference:
        copy_reference()
        return

    import torch
    import paper_2303_10783_amd as sol
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = sol.TorchDevice(0)
    if args.batch_only:
        v = run_batched(sol, W, args.batch_only, args.steps or 300, args.warmup, dev, tune=args.batch_only == "mixed")
        print(json.dumps(v))
        return
    steps = args.steps or W.WORKLOADS[args.workload]["steps"]
    acc_steps = 2 if args.workload == "C3" else 5
    keep = acc_steps if not args.no_cpu_baseline else None
    head = run_single(sol, W, args.workload, args.precision, steps, args.warmup, dev, precond=args.precond,
                      tprecond=args.tprecond, graph=args.graph, timing=not args.no_roofline, keep_fields=keep,
                      mg_fuse=False if args.mg_per_level else None)
    print(f"[bench] headline {head['workload']} {args.precision}: {head['value'] / 1e6:.1f} M cell-updates/s",
          file=sys.stderr, flush=True)
    roof = None
    if head.get("_best"):
        best = head["_best"]
        tr = counter_traffic(args.workload, best["cls"], args.precond) if args.precision == "fp64" else None
        roof = dict(bound="hbm", achieved=round(best["gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(best["gbs"] / HBM_PEAK_GBS, 4), traffic=tr,
                    kernel=best["cls"], avg_us=round(best["avg_ms"] * 1e3, 2),
                    bytes_per_launch=int(best["bytes_per_launch"]), timed_launches=int(best["launches"]),
                    all_classes=head["_classes"])
    variants = None
    gpu_fields = {args.precision: head["_fields"]} if keep else None
    c1_fields = None
    tight_fields = {}
    if not args.no_variants:
        variants = {}
        other = "mixed" if args.precision == "fp64" else "fp64"
        v = run_single(sol, W, args.workload, other, steps, args.warmup, dev, precond=args.precond,
                       tprecond=args.tprecond, graph=args.graph, keep_fields=keep)
        if keep:
            gpu_fields[other] = v["_fields"]
        variants[f"{args.workload}_{other}"] = _public(v)
        for key in ("C2", "C1"):
            if key == args.workload:
                continue
            nst = W.WORKLOADS[key]["steps"]
            for prec in ("fp64", "mixed"):
                v = run_single(sol, W, key, prec, nst, args.warmup, dev,
                               keep_fields=200 if key == "C1" and keep else None)
                if key == "C1" and keep:
                    c1_fields = c1_fields or {}
                    c1_fields[prec] = v["_fields"]
                variants[f"{key}_{prec}"] = _public(v)
                print(f"[bench] {v['workload']} {prec}: {v['value'] / 1e6:.1f} M", file=sys.stderr, flush=True)
        if args.jacobi_variants:
            variants["C3_fp64_jacobi"] = _public(run_single(sol, W, "C3", "fp64", 20, 1, dev, precond="jacobi"))
            variants["C2_fp64_jacobi"] = _public(run_single(sol, W, "C2", "fp64", 50, 1, dev, precond="jacobi"))
        # coarse multigrid levels one launch each (fused in pairs by
        # default): the same steps, the time the fusion saves
        for key in dict.fromkeys((args.workload, "C2")):
            nst = steps if key == args.workload else W.WORKLOADS[key]["steps"]
            v = run_single(sol, W, key, args.precision, nst, args.warmup, dev, mg_fuse=False)
            variants[f"{key}_{args.precision}_mg_per_level"] = _public(v)
            print(f"[bench] {key} coarse levels one launch each: {v['value'] / 1e6:.1f} M", file=sys.stderr,
                  flush=True)
        # the forward (residual-probing) assembly route: its assembly
        # kernels against the stencil route's, same steps
        v = run_single(sol, W, args.workload, args.precision, steps, args.warmup, dev, assembly="forward",
                       timing=True)
        fw = {k: v["_classes"][k] for k in ("asm_mom", "asm_trn") if k in v["_classes"]}
        st_cls = head.get("_classes", {})
        variants[f"{args.workload}_{args.precision}_forward_assembly"] = dict(
            _public(v), assembly_kernels=fw,
            stencil_assembly_kernels={k: st_cls[k] for k in ("asm_mom", "asm_trn") if k in st_cls})
        print(f"[bench] forward assembly: {v['value'] / 1e6:.1f} M", file=sys.stderr, flush=True)
        # the same box at the tolerances that hold 1e-8 per field (pressure
        # 1e-12, transport 1e-13): mixed against FP64 at a stated accuracy
        tight_fields = {}
        for prec in ("fp64", "mixed"):
            v = run_single(sol, W, args.workload, prec, steps, args.warmup, dev, tols=TIGHT, keep_fields=keep)
            if keep:
                tight_fields[prec] = v["_fields"]
            variants[f"{args.workload}_{prec}_tight"] = _public(v)
            print(f"[bench] {v['workload']} {prec} tight: {v['value'] / 1e6:.1f} M", file=sys.stderr, flush=True)
        variants["C4_batched_mixed"] = run_batched(sol, W, "mixed", 300, args.warmup, dev)
        variants["C4_batched_fp64"] = run_batched(sol, W, "fp64", 300, args.warmup, dev, tune=False)
        print(f"[bench] batch: {variants['C4_batched_mixed']['value'] / 1e6:.1f} M mixed", file=sys.stderr,
              flush=True)
        variants["C4_batched_mixed_tight"] = run_batched(sol, W, "mixed", 300, args.warmup, dev, tols=TIGHT_BATCH)
        variants["C4_batched_fp64_tight"] = run_batched(sol, W, "fp64", 300, args.warmup, dev, tune=False,
                                                        tols=TIGHT_BATCH)
        variants["C5_served_mixed"] = run_served(sol, W, dev)
        print(f"[bench] served: {variants['C5_served_mixed']['value'] / 1e6:.1f} M", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, args.workload, acc_steps, 1, gpu_fields=gpu_fields, c1_gpu_fields=c1_fields,
                           tight=(TIGHT, tight_fields) if not args.no_variants and keep else None)
    case = W.workload_case(args.workload)
    out = dict(
        metric=METRIC, value=head["value"], unit="cell-updates/s", n_gpus=1, steps=steps,
        warmup=args.warmup, ms_per_step=head["ms_per_step"], launches_per_step=head["launches_per_step"],
        higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f64" if args.precision == "fp64" else "f32+f64", data="synthetic",
        config=dict(workload=head["workload"] + f", {steps} steps from the initial state",
                    cells=head["cells"], dt=case["numerics"]["dt"], tol=case["numerics"]["tol_p"],
                    precision=args.precision, pressure_precond=args.precond,
                    transport_precond=args.tprecond or "auto",
                    krylov_iters_per_step=head["krylov_iters_per_step"], steps_redone=head["steps_redone"]),
        roofline=roof, step_roofline=head.get("step_roofline"),
        timing_pass_ms_per_step=head.get("timing_pass_ms_per_step"),
        cpu_baseline=cpu, variants=variants,
    )
    print(json.dumps(out))


if __name__ == "__main__":
    main()
