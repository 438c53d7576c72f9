"""Throughput of the full SDMD PIC step on one MI355X.

Default workload: the laser-wakefield-shaped 2D3V run -- 2048 x 256 cells,
dx = 0.125, dy = 0.5, vacuum / 256-cell linear ramp / plateau n = 0.005,
16 cold particles per cell (3,932,160 particles), Gaussian laser a0 = 2,
16 x 16-cell patches, 4 regions of 512 x 256, FP32 split-position particles
with FP64 region reduction and Maxwell.  Synthetic seeded input.

Prints one JSON line: particle-pushes/s of the whole step (all phases: patch
field window, interpolation, Boris, Esirkepov deposition, patch -> region
current sum, Yee, region ghosts, re-binning), the roofline of the dominant
kernel (the particle kernel, against HBM bandwidth) from its average launch
time over the timed trajectory -- replayed from the same input with HIP
events around every kernel on the library's stream -- and the FP64 CPU
oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_1912_04064_amd import workloads as WL
    if name == "lwfa":
        return WL.lwfa_2d()
    if name == "lwfa64":
        return WL.lwfa_2d(precision="fp64")
    if name == "lwfa_filter2":
        import dataclasses
        return dataclasses.replace(WL.lwfa_2d(), filter=2, name="lwfa2048x256_filter2")
    if name == "lwfa_psatd":
        import dataclasses
        return dataclasses.replace(WL.lwfa_2d(nreg=(1, 1)), solver="psatd", name="lwfa2048x256_psatd")
    if name == "thermal64":
        return WL.thermal_2d()
    if name == "thermal2k":
        return WL.thermal_2d(n=(2048, 256), ppc=16, vth=0.05, patch=(16, 16), nreg=(4, 1), precision="fp32s",
                             name="thermal2048x256")
    if name == "cyl3d":
        return WL.cylinder_3d()
    if name == "cyl3d_psatd":
        import dataclasses
        return dataclasses.replace(WL.cylinder_3d(), solver="psatd", name="cyl512x128x128_psatd")
    if name == "cyl3d_small":
        return WL.cylinder_3d(n=(128, 32, 32), radius=4.0)
    raise SystemExit(f"unknown workload {name}")


def particle_bytes(wl):
    """Algorithmic HBM bytes per particle per step of the particle kernel:
    read cell (2 B, split form) + position + momentum + weight, write cell +
    position + momentum."""
    r = 4 if wl.precision == "fp32s" else 8
    cell = 2 if wl.precision == "fp32s" else 0
    rd = cell + wl.dims * r + 3 * r + r
    wr = cell + wl.dims * r + 3 * r
    return rd + wr


VALU_PEAK = 256 * 2.4e9   # wavefront VALU instructions per second (no packed FP32)


def copy_bandwidth(torch, gib=1.0, reps=5):
    """HBM bandwidth a plain device-to-device copy reaches on this GPU (read +
    write bytes over the copy's own time, best of `reps`): the practical
    ceiling a streaming kernel is measured against beside the 8 TB/s peak."""
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def valu_line(insts, launch_ms):
    if insts is None:
        return None
    rate = insts / (launch_ms * 1e-3)
    return {"insts_per_launch": insts, "achieved": rate, "peak": VALU_PEAK, "unit": "wave-instr/s",
            "frac": rate / VALU_PEAK}


def push_counters(wl_name, first, last):
    """Counter figures of the particle kernel (HBM bytes from FETCH_SIZE /
    WRITE_SIZE scaled by a plain copy of known size; VALU and LDS
    wavefront-instructions) averaged over its launches of steps
    [first, last) of the workload, from the committed counter runs
    (profiles/traffic.json), or None when no run covers that window or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("push_kernel", {})
    if rec.get("workload") != {"lwfa": "lwfa2048x256"}.get(wl_name):
        return None
    if kernel_source_hash() != rec.get("source_sha"):
        return None
    return rec.get("windows", {}).get(f"{first}-{last}")


def kernel_source_hash():
    """Hash of the particle kernel's sources with comments and whitespace
    removed: a code change invalidates the stored counter figures, an edit
    of a comment does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("k_push.hip", "part.h", "sdmd_dev.h"):
        with open(os.path.join(ROOT, "paper_1912_04064_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl_name, budget_s=10.0):
    """The FP64 oracle's SDMD step on a bounded sample of the same workload
    (a horizontal band of the grid with its particles, full steps), timed
    twice on the host: one thread (the parity build), and the OpenMP timing
    build of the same source with dynamic scheduling over patches (the
    paper's thread model) on the threads OMP_NUM_THREADS allows (all
    cores when unset).  Both legs compute the same result bit for bit."""
    import oracle as O
    from paper_1912_04064_amd import workloads as WL
    if wl_name.startswith("lwfa"):
        # the plasma band of the run: 256 x 256 cells of plateau + ramp
        wl = WL.lwfa_2d(n=(512, 256), vac_end=64, ramp=256, x0=68.0)
        sample = "lwfa band 512x256 cells (ramp+plateau, 16 ppc, 16x16 patches, 4 regions)"
    elif wl_name.startswith("cyl"):
        wl = WL.cylinder_3d(n=(32, 32, 32), radius=8.0)
        sample = "cylinder 32^3 cells (8 ppc + 16x cylinder, 8^3 patches)"
    else:
        wl = workload(wl_name)
        sample = wl.name
    from tests.helpers import oracle_state
    nproc = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or nproc

    def leg(step):
        g, F, P = oracle_state(wl)
        step(g, F, P)                      # first step: page-in, not timed
        steps = 0
        t0 = time.perf_counter()
        while True:
            step(g, F, P)
            steps += 1
            if time.perf_counter() - t0 > budget_s or steps >= 50:
                break
        dt = time.perf_counter() - t0
        return P.n * steps / dt, steps, dt, P.n

    v1, s1, d1, n = leg(lambda g, F, P: O.step_sdmd(g, F, P))
    vn, sn, dn, _ = leg(lambda g, F, P: O.step_sdmd_threads(g, F, P, threads))
    return {"value": vn, "unit": "particle-pushes/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample}: {n} particles x {sn} steps in {dn:.1f} s on {threads} threads",
            "single_core": {"value": v1, "cores": 1, "sample": f"{n} particles x {s1} steps in {d1:.1f} s"},
            "nproc": nproc, "cpu_model": cpu_model(),
            "schedule": "OpenMP dynamic over patches (SDMD step of the oracle)"}


def _family_rel(a, b):
    """relative L2 difference of a from b per field family (E, Bm, J)"""
    out = {}
    for k, sl in (("E", slice(0, 3)), ("Bm", slice(3, 6)), ("J", slice(6, 9))):
        nb = float(np.linalg.norm(b[sl]))
        out[k] = float(np.linalg.norm(a[sl] - b[sl]) / nb) if nb > 0 else float(np.abs(a[sl]).max())
    return out


def bench_scan(args):
    """Batched parameter scan: independent 2D3V runs stepped together (one
    launch per phase for all runs, two-step hipGraph replay); patch edge,
    segment capacity and field tile width from the autotuner.  Value =
    particle pushes/s summed over the runs.  The roofline object prices the
    particle phase (its algorithmic bytes over its time, from per-phase HIP
    events over the steps that follow the timed ones) and the whole step
    against HBM.  --compare-precision runs the same scan in FP64 as well and
    reports both throughputs and the FP32 split form's difference from the
    FP64 form on a sample of runs."""
    import torch
    from paper_1912_04064_amd import binding as B
    from paper_1912_04064_amd import workloads as WL

    def one(prec, sample):
        wls = WL.scan_batch(n_runs=args.runs, steps=args.steps, precision=prec)
        N = sum(w.n_particles for w in wls)
        cells = sum(w.n_cells for w in wls)
        print(f"[bench] scan {prec}: {len(wls)} runs, {N} particles", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        ctx = B.Context(wls)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        ctx.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F = {i: ctx.fields(i, B.F_E | B.F_B | B.F_J) for i in sample}
        nph = max(1, args.phase_samples or 10)
        ctx.time_phases(nph)
        ph = ctx.diag(0)["t_ms"]
        pk = ctx.diag(0)["t_push_kernel_ms"]   # the particle kernels' own time, events on their launches
        choices = {}
        for i in range(len(wls)):
            dd = ctx.diag(i)
            k = f"patch{dd['patch'][0]}/seg{dd['seg_cap']}/tile{dd['kernel_path'][2]}"
            choices[k] = choices.get(k, 0) + 1
        ctx.close()
        pb = particle_bytes(wls[0])
        push_bytes = N * pb + cells * 48
        step_bytes = N * (52.0 if prec == "fp32s" else 88.0) + cells * 216.0
        rec = {"value": N * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps, "particles": N, "cells": cells,
               "init_s": t_init, "tuned": choices,
               "phase_ms": {"particles": ph[0], "reduce_maxwell": ph[1], "sync_rebin": ph[2], "relayout": ph[3],
                            "steps": [args.warmup + args.steps, args.warmup + args.steps + nph]},
               "roofline": {"bound": "hbm", "kernel": "push_kernel (all runs)",
                            "achieved": push_bytes / (pk * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": push_bytes / (pk * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                            "bytes_per_launch": push_bytes, "launch_ms": pk},
               "step_roofline": {"bytes_per_step": step_bytes, "roofline": HBM_PEAK_GBS * 1e9 * N / step_bytes,
                                 "frac": (N * args.steps / dt) / (HBM_PEAK_GBS * 1e9 * N / step_bytes)}}
        return rec, F

    prec = args.precision
    sample = list(range(min(8, args.runs)))
    rec, F = one(prec, sample)
    out = {"metric": "particle-pushes/s (batched scan)", "value": rec["value"], "unit": "particle-pushes/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "timed_steps": [args.warmup, args.warmup + args.steps], "ms_per_step": rec["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64" if prec == "fp32s" else "f64", "data": "synthetic",
           "config": {"workload": f"scan{args.runs}", "runs": args.runs, "particles": rec["particles"],
                      "cells": rec["cells"], "precision": prec, "tuned": rec["tuned"], "init_s": rec["init_s"]},
           "phase_ms": rec["phase_ms"], "roofline": rec["roofline"], "step_roofline": rec["step_roofline"]}
    if args.compare_precision:
        other = "fp64" if prec == "fp32s" else "fp32s"
        rec2, F2 = one(other, sample)
        F32, F64 = (F, F2) if prec == "fp32s" else (F2, F)
        diffs = {i: _family_rel(F32[i], F64[i]) for i in sample}
        out["forms"] = {prec: {"value": rec["value"], "ms_per_step": rec["ms_per_step"]},
                        other: {"value": rec2["value"], "ms_per_step": rec2["ms_per_step"]}}
        out["fp32s_vs_fp64"] = {"runs": sample, "max": {k: max(d[k] for d in diffs.values()) for k in ("E", "Bm", "J")},
                                "per_run": diffs}
    return out


def bench_serve(args):
    """Served request stream: Poisson arrivals, admission by HBM budget and
    free slots, continuous batching; p50/p99 latency and throughput.  With
    --compare-precision the same stream is served in FP64 as well, and the
    final fields of a sample of runs are compared between the two forms."""
    from paper_1912_04064_amd import serving as S
    from paper_1912_04064_amd import workloads as WL
    reqs = WL.request_stream(args.serve, window_s=args.window)
    sample = [r.rid for r in reqs[:8]]

    def one(prec):
        # A request arrives with its input: the seeded synthetic inputs are
        # made before the stream starts, so the clock sees admission and
        # stepping only.
        t0 = time.perf_counter()
        pre = {r.rid: WL.request_workload(r, precision=prec) for r in reqs}
        print(f"[bench] serve {prec}: {len(reqs)} requests at {args.serve}/s over {args.window} s "
              f"(inputs made in {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
        budget = int(args.budget_gb * 2 ** 30)
        be = S.GpuBackend(max_runs=args.slots, hbm_budget=budget, capture=sample)
        srv = S.Server(be, hbm_budget=budget, max_runs=args.slots, steps_per_call=20)
        recs = srv.serve(reqs, lambda r: pre[r.rid])
        admit_ms = be.admit_s * 1e3 / max(be.admits, 1)
        be.close()
        summ = S.summarize(recs)
        return {"runs_per_s": summ["runs_per_s"], "p50_latency_s": summ["p50_latency_s"],
                "p99_latency_s": summ["p99_latency_s"], "particle_pushes_per_s": summ["particle_pushes_per_s"],
                "max_concurrent": srv.max_active, "admit_ms_mean": admit_ms,
                "device_bytes_peak": be.peak_bytes}, be.captured

    prec = args.precision
    res, cap = one(prec)
    out = {"metric": "runs/s + p99 latency (served)", "value": res["runs_per_s"], "unit": "runs/s", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f32+f64" if prec == "fp32s" else "f64",
           "data": "synthetic", **{k: v for k, v in res.items() if k != "runs_per_s"},
           "config": {"workload": f"poisson{args.serve:g}", "requests": len(reqs), "window_s": args.window,
                      "slots": args.slots, "budget_gb": args.budget_gb, "precision": prec}}
    if args.compare_precision:
        other = "fp64" if prec == "fp32s" else "fp32s"
        res2, cap2 = one(other)
        c32, c64 = (cap, cap2) if prec == "fp32s" else (cap2, cap)
        diffs = {i: _family_rel(c32[i], c64[i]) for i in sample if i in c32 and i in c64}
        out["forms"] = {prec: res, other: res2}
        out["fp32s_vs_fp64"] = {"runs": sorted(diffs), "max": {k: max(d[k] for d in diffs.values())
                                                               for k in ("E", "Bm", "J")} if diffs else None,
                                "per_run": diffs}
    return out


def bench_precision(args):
    """The precision forms side by side on the same GPU: the LWFA input run
    in FP64 and in the FP32 split form from the same particles and fields;
    throughput of each and the FP32 form's relative L2 difference from the
    FP64 run (fields per family, particle momenta) after the same steps."""
    import dataclasses
    import torch
    from paper_1912_04064_amd import binding as B
    base = workload(args.workload)
    res, state = {}, {}
    for prec in ("fp64", "fp32s"):
        wl = dataclasses.replace(base, precision=prec)
        ctx = B.Context([wl], track_ids=True, graph=not args.no_graph)
        d0 = ctx.diag(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F = ctx.fields(0, B.F_E | B.F_B | B.F_J)
        parts = B.sort_by_id(ctx.particles(0))
        d = ctx.diag(0)
        ctx.close()
        u0 = d0["U_E"] + d0["U_B"] + d0["K"]
        res[prec] = {"pushes_per_s": wl.n_particles * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
                     "energy_rel_change": (d["U_E"] + d["U_B"] + d["K"]) / u0 - 1.0,
                     "gauss_residual": d["gauss_residual"]}
        state[prec] = (F, parts)
        print(f"[bench] {prec}: {res[prec]}", file=sys.stderr, flush=True)
    (F64, p64), (F32, p32) = state["fp64"], state["fp32s"]
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    diff = {"E": rel(F32[0:3], F64[0:3]), "B": rel(F32[3:6], F64[3:6]), "J": rel(F32[6:9], F64[6:9]),
            "u": rel(np.stack([p32["ux"], p32["uy"], p32["uz"]]), np.stack([p64["ux"], p64["uy"], p64["uz"]]))}
    return {"metric": "FP32 split vs FP64 on the same GPU", "unit": "relative L2 difference", "n_gpus": 1,
            "steps": args.steps, "higher_is_better": False, "vs_baseline": None, "data": "synthetic",
            "config": {"workload": base.name}, "forms": res, "fp32s_vs_fp64": diff}


def bench_sdsd(args):
    """The paper's central comparison on one GPU: the LWFA input with fields
    on regions (SDMD, 4 regions of 512 x 256) against fields on the patches
    themselves (SDSD: one region per patch, so every patch runs its own Yee
    update and exchanges ghosts with its neighbours), for several patch
    sizes.  Same particle kernel, same input; ms/step and phase split."""
    import dataclasses
    import torch
    from paper_1912_04064_amd import binding as B
    from paper_1912_04064_amd import workloads as WL
    base = WL.lwfa_2d()
    rows = []
    for P in (8, 16, 32):
        for mode in ("sdmd", "sdsd"):
            nreg = (4, 1) if mode == "sdmd" else (base.n[0] // P, base.n[1] // P)
            wl = dataclasses.replace(base, patch=(P, P), nreg=nreg)
            ctx = B.Context([wl], graph=not args.no_graph, deterministic=args.deterministic)
            ctx.step(args.warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.step(args.steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ctx.time_phases(max(1, args.phase_samples))
            ph = np.array(ctx.diag(0)["t_ms"][:3])
            ctx.close()
            row = {"patch": P, "mode": mode, "regions": nreg[0] * nreg[1], "ms_per_step": dt * 1e3 / args.steps,
                   "pushes_per_s": wl.n_particles * args.steps / dt, "particles_ms": float(ph[0]),
                   "fields_ms": float(ph[1]), "sync_ms": float(ph[2])}
            print(f"[bench] {row}", file=sys.stderr, flush=True)
            rows.append(row)
    return {"metric": "ms/step, SDMD regions vs SDSD patches", "unit": "ms/step", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": False, "vs_baseline": None, "dtype": "f32+f64",
            "data": "synthetic", "config": {"workload": base.name, "precision": base.precision}, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="lwfa")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="deterministic mode (fixed-point current sums, bitwise reproducible)")
    ap.add_argument("--phase-samples", type=int, default=0,
                    help="steps of the timed trajectory replayed with per-kernel events (0 = all)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the workload's whole trajectory (its configured step count)")
    ap.add_argument("--runs", type=int, default=256, help="runs of the batched scan (--workload scan)")
    ap.add_argument("--precision", default="fp32s", choices=["fp32s", "fp64"],
                    help="precision form of the batched scan and the served stream")
    ap.add_argument("--serve", type=float, default=0.0, help="served stream: arrival rate in runs/s")
    ap.add_argument("--window", type=float, default=10.0, help="served stream: arrival window in s")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--compare-sdsd", action="store_true",
                    help="fields on regions (SDMD) vs on patches (SDSD) for patch sizes 8, 16, 32")
    ap.add_argument("--compare-precision", action="store_true",
                    help="the workload in FP64 and in the FP32 split form: throughput and their difference")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 512 MiB device copy first (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding "
              "(one region per GPU) is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_04064_amd import binding as B
    if not torch.cuda.is_available():
        raise SystemExit("no GPU")
    if args.serve > 0:
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.compare_sdsd:
        print(json.dumps(bench_sdsd(args)), flush=True)
        return
    if args.workload == "scan":
        print(json.dumps(bench_scan(args)), flush=True)
        return
    if args.compare_precision:
        print(json.dumps(bench_precision(args)), flush=True)
        return
    if args.calib_copy:
        x = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    wl = workload(args.workload)
    N = wl.n_particles
    ncell = wl.n_cells
    print(f"[bench] workload {wl.name}: {N} particles, {ncell} cells, {wl.precision}", file=sys.stderr, flush=True)
    ctx = B.Context([wl], graph=not args.no_graph, deterministic=args.deterministic)
    ctx.step(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)
    d0 = ctx.diag(0)   # energies before the timed steps (synchronising, outside the timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = N * args.steps / (t1 - t0)
    print(f"[bench] timed {args.steps} steps: {ms:.4f} ms/step", file=sys.stderr, flush=True)

    d = ctx.diag(0)
    ctx.close()
    first, last = args.warmup, args.warmup + args.steps
    pb = particle_bytes(wl)
    alg_push = N * pb + ncell * 48          # particles + the FP64 E, Bm window (transfer ii)

    def replay(warm, n):
        """Per-phase kernel times over steps [warm, warm + n) of the same
        trajectory, replayed from the same input with HIP events between the
        phases on the library's stream (kernels back to back)."""
        c = B.Context([wl], graph=not args.no_graph, deterministic=args.deterministic)
        c.step(warm)
        c.time_phases(n)
        dd = c.diag(0)
        t = dd["t_ms"]
        c.close()
        return float(t[0]), float(t[1]), float(t[2]), float(t[3]), float(dd["t_push_kernel_ms"])

    # the dominant kernel over the timed window (the same steps): its own
    # duration per launch, from events attached to its launches
    nph = args.steps if args.phase_samples <= 0 else min(args.steps, args.phase_samples)
    push_ph, yee_avg, post_avg, rel_avg, push_avg = replay(args.warmup, nph)
    achieved = alg_push / (push_avg * 1e-3) / 1e9
    step_bytes = N * pb + ncell * 216
    # (the counters were taken on the plain kernels, not the fixed-point ones)
    ctr = push_counters(args.workload, first, last) if nph == args.steps and not args.deterministic else None

    # the whole step against HBM: the survey's per-push bytes (52 B of
    # split-form particle traffic with a 4-byte cell index + 216 B of FP64
    # field traffic per cell, shared by the particles per cell)
    ppc = N / ncell
    bpp_step = (52.0 if wl.precision == "fp32s" else 88.0) + 216.0 / ppc
    step_roof = HBM_PEAK_GBS * 1e9 / bpp_step

    out = {
        "metric": "particle-pushes/s (full SDMD step)",
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "timed_steps": [first, last],
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if wl.precision == "fp32s" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": list(wl.n), "particles": N, "patch": list(d["patch"][:wl.dims]),
                   "regions": list(wl.nreg), "precision": wl.precision, "solver": wl.solver, "filter": wl.filter,
                   "graph": not args.no_graph, "run_steps": wl.steps, "deterministic": args.deterministic},
        "step_hbm_GBps_algorithmic": step_bytes / (ms * 1e-3) / 1e9,
        "step_roofline": {"bytes_per_push": bpp_step, "roofline": step_roof, "unit": "particle-pushes/s",
                          "frac": value / step_roof},
        "phase_ms": {"particles": push_ph, "reduce_maxwell": yee_avg, "sync_rebin": post_avg,
                     "relayout": rel_avg, "steps": [first, first + nph]},
        "roofline": {"bound": "hbm", "kernel": "push_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": ctr["bytes_per_launch"] if ctr else None, "bytes_per_launch": alg_push,
                     "launch_ms": push_avg, "steps": [first, first + nph],
                     "timing": "HIP events attached to the kernel's launches (start to end), per launch"},
        # the particle kernel's VALU issue rate over the same window: one
        # wavefront VALU instruction per CU per clock when packed FP32 is not
        # used (256 CUs x 2.4 GHz); counts from the committed counter run of
        # this window, null when there is none
        "valu": valu_line(ctr["valu_insts_per_launch"] if ctr else None, push_avg),
        "relayouts": d["n_relayout"],
        # total energy (fields + electrons) over the timed steps, and the
        # Gauss-law residual div_h E - rho against the initial state
        "energy": {"start": d0["U_E"] + d0["U_B"] + d0["K"], "end": d["U_E"] + d["U_B"] + d["K"],
                   "rel_change": (d["U_E"] + d["U_B"] + d["K"]) / (d0["U_E"] + d0["U_B"] + d0["K"]) - 1.0,
                   "gauss_residual": d["gauss_residual"]},
    }
    # the same kernel against what a plain copy reaches on this GPU (not in
    # counter runs, whose calibration copy must stay the largest copy)
    if not args.calib_copy:
        cbw = copy_bandwidth(torch)
        out["roofline"]["achievable_copy_GBps"] = cbw
        out["roofline"]["frac_of_copy"] = achieved / cbw
    if not args.no_full_run and wl.steps > 0:
        # the workload's whole trajectory (its configured step count, the
        # laser entering the plasma and the wake forming): the same figures
        # over every step, timed the same way
        # set-up from host memory (pic_init: the particles and fields are
        # handed over in host arrays, copied to HBM and binned) timed apart
        torch.cuda.synchronize()
        ts = time.perf_counter()
        c = B.Context([wl], graph=not args.no_graph, deterministic=args.deterministic)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - ts
        t0 = time.perf_counter()
        c.step(wl.steps)
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t0
        df = c.diag(0)
        c.close()
        fph, fy, fq, fr, fp = replay(0, wl.steps)
        fv = N * wl.steps / dtf
        fctr = None if args.deterministic else push_counters(args.workload, 0, wl.steps)
        out["full_run"] = {
            "steps": [0, wl.steps], "value": fv, "ms_per_step": dtf * 1e3 / wl.steps,
            # the same run with its set-up from host buffers (PCIe copies,
            # binning, graph capture on the first step) counted in
            "setup_s": setup_s, "value_with_setup": N * wl.steps / (dtf + setup_s),
            "step_roofline_frac": fv / step_roof,
            "phase_ms": {"particles": fph, "reduce_maxwell": fy, "sync_rebin": fq, "relayout": fr},
            "push_kernel": {"launch_ms": fp, "achieved": alg_push / (fp * 1e-3) / 1e9,
                            "frac": alg_push / (fp * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "traffic": fctr["bytes_per_launch"] if fctr else None,
                            "valu": valu_line(fctr["valu_insts_per_launch"] if fctr else None, fp)},
            "relayouts": df["n_relayout"], "gauss_residual": df["gauss_residual"]}
        print(f"[bench] full run {wl.steps} steps: {dtf * 1e3 / wl.steps:.4f} ms/step", file=sys.stderr, flush=True)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
