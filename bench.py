#!/usr/bin/env python3
"""Benchmark of the shifted SPAI-preconditioned CG hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input, inputs
already resident in HBM:
  pencil setup (sliced-ELL copy, float32 mirrors, transpose map)
  -> SPAI build at every expansion point
  -> batched mixed-precision PCG for all (shift, column) systems
  -> SPAI update of every preconditioner to the next outer iteration's
     (drifted) expansion points (one batched call)
  -> batched mixed-precision PCG again, with the update chains.
``value`` = systems solved to 1e-8 relative error (checked against the
oracle's double-double reference) per second of step time.  Beside it: the
plain float64 one-system-at-a-time GPU PCG on the same systems, SPAI
build/update milliseconds, the roofline of the dominant kernel and the CPU
oracle's rate.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4s]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import gc
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synthetic import beam  # noqa: E402

METRIC = "PCG solves/s @1e-8 rel err, batched-mixed vs plain FP64; SPAI build/update ms"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X dense float64 (vector and matrix)
ERR_TOL = 1e-8

# Workloads (seeded, synthetic).  "s" = the surrogate with every EI scaled by
# h^4 (same n, pattern, loads, shifts, seeds and heterogeneity).
WORKLOADS = {
    "c4s": dict(base="c3", surrogate=True, desc="Hermite cantilever n=1,000,000 (EI=1 scaled by h^4), "
                "m=4 seeded unit loads, 16 shifts logspace(0,4,16) then 16 drifted (x(1+1e-3 U(-1,1)))"),
    "c5s": dict(base="c5", surrogate=True, desc="Hermite cantilever n=10,000,000 (EI log-uniform "
                "[0.1,10], scaled by h^4), m=4, 32 shifts logspace(0,5,32) then 32 drifted"),
    "c2s": dict(base="c2", surrogate=True, desc="Hermite cantilever n=100,000 (EI log-uniform "
                "[0.5,2], scaled by h^4), tip load, 8 shifts logspace(0,4,8) then 8 drifted"),
    "c1": dict(base="c1", surrogate=False, desc="Hermite cantilever n=1000, EI=1 (literal), tip "
               "load, s=100"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_inputs(name, seed=0):
    w = WORKLOADS[name]
    pen, f, shifts, rng = beam.make_workload(w["base"], surrogate=w["surrogate"], seed=seed)
    drifted = beam.drift_shifts(shifts, 1e-3, rng)
    return pen, f, np.asarray(shifts, float), np.asarray(drifted, float)


# ---------------------------------------------------------------- profiles
#
# HBM traffic of the row kernels comes from two rocprofv3 counter passes
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) over one quick step with a
# forced tile, each scaled by what the same counter reads for a plain 1 GiB
# device copy in the same run.  The table is keyed by the hash of the row
# kernels' source and of the solve that drives them (its options set how many
# systems an average launch sweeps): after any change to either it no longer
# applies.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1606_01216_amd", "csrc", f)
                  for f in ("pcg_kernels.hpp", "pcg.hip")]
PROFILES = os.path.join(ROOT, "profiles")
PMC_KERNELS = {"update_prec": "k_update_prec<float, {w}, {r}, {u}, false",
               "dir_spmv": "k_dir_spmv<float, {w}, {r}, {u}, false"}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(workload):
    return os.path.join(PROFILES, f"row_kernels_{workload}_hbm_traffic.json")


def measured_traffic(workload, tile, kernel):
    """HBM bytes per launch of `kernel` from the committed counter table, or
    None when there is none for this tile or the kernels changed since."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        tab = json.load(fh)
    if tab.get("source_hash") != kernel_source_hash():
        return None
    ent = tab.get("tiles", {}).get(f"{tile[0]}x{tile[1]}", {}).get(kernel)
    return None if ent is None else ent["hbm_bytes_per_launch"]


def _read_counters(path):
    import csv
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def summarize_pmc(args):
    import glob
    root = args.summarize_pmc
    out = {"workload": args.workload, "source_hash": kernel_source_hash(),
           "counters": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch), one rocprofv3 pass each",
           "scaling": "each counter times (copied bytes / counter reading) of a 1 GiB device "
                      "copy (__amd_rocclr_copyBuffer) in the same run",
           "launches": "the second mixed-precision solve of the step (after its k_clear_active)",
           "command": args.command, "tiles": {}}
    for fdir in sorted(glob.glob(os.path.join(root, "*_fetch"))):
        tile = os.path.basename(fdir)[:-len("_fetch")]
        r, u = (int(v) for v in tile.split("x"))
        per = {}
        for counter, d in (("FETCH_SIZE", fdir), ("WRITE_SIZE", fdir[:-len("fetch")] + "write")):
            rows = _read_counters(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])
            rows = [x for x in rows if x["Counter_Name"] == counter]
            copies = [float(x["Counter_Value"]) for x in rows
                      if "copyBuffer" in x["Kernel_Name"] and int(x["Grid_Size"]) >= 1 << 17]
            factor = 1024.0 * 1024.0 / (sum(copies) / len(copies))
            last = max(int(x["Dispatch_Id"]) for x in rows if "k_clear_active" in x["Kernel_Name"])
            for kname, pat in PMC_KERNELS.items():
                pat = pat.format(w=6, r=r // 64, u=u)
                vals = [float(x["Counter_Value"]) * 1024.0 * factor for x in rows
                        if pat in x["Kernel_Name"] and int(x["Dispatch_Id"]) > last]
                ent = per.setdefault(kname, {"launches": len(vals)})
                ent[counter.lower() + "_bytes_per_launch"] = int(sum(vals) / len(vals))
                ent[counter.lower() + "_scale"] = round(factor, 4)
        for ent in per.values():
            ent["hbm_bytes_per_launch"] = ent["fetch_size_bytes_per_launch"] + \
                ent["write_size_bytes_per_launch"]
        out["tiles"][tile] = per
    path = args.out or traffic_file(args.workload)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


def summarize_trace(args):
    import csv
    with open(args.summarize_trace) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", args.command, "```", "",
             "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:20]:
        name = r["Name"].replace("|", "/")
        lines.append(f"| `{name[:110]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    if args.bench_json:
        with open(args.bench_json) as fh:
            b = json.loads(fh.read().strip().splitlines()[-1])
        rf = b["roofline"]
        r, u = b["config"]["tile"]["rows_per_wave"] // 64, b["config"]["tile"]["systems_per_group"]
        pat = PMC_KERNELS[rf["kernel"]].format(w=6, r=r, u=u)
        hit = [x for x in rows if pat in x["Name"]]
        lines += ["", f"Dominant kernel `{rf['kernel']}` (tile {r * 64} rows x {u} systems): bench.py "
                  f"events {rf['avg_launch_us']} us per launch over the profiled solve; rocprofv3 "
                  f"average over all its launches in the run: "
                  + (f"{float(hit[0]['AverageNs']) / 1e3:.1f} us" if hit else "not found"),
                  f"bench line: value {b['value']} {b['unit']}, {b['ms_per_step']} ms/step, "
                  f"achieved {rf['achieved']} GB/s ({rf['frac']} of {rf['peak']})."]
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(text)


def measure_moments(ctx, stream, dev, n, m, nblocks, nb=4, reps=5):
    """The block operations of one pass of the moment sequence (Algorithm 1)
    at the workload's size, outside the timed step: the right-hand side
    M V_j, the orthogonalisation of the nblocks solution blocks (n x m)
    against nb earlier basis blocks with normalisation, the thin QR of the
    nblocks * m collected columns, and the projection onto them.  Seeded
    random blocks stand in for the solutions (timing does not depend on the
    values).  Also the A^T B kernel alone for 64 x 64 columns, timed with
    HIP events on the context stream."""
    import torch
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    k = nblocks * m
    with torch.cuda.stream(stream):
        v = torch.randn((nb * m, n), dtype=torch.float64, device=dev, generator=gen)
        ctx.block_qr(v)                       # orthonormal columns
        ctx.global_orth(None, v, m, normalize=True)   # blocks of unit Frobenius norm
        x0 = torch.randn((k, n), dtype=torch.float64, device=dev, generator=gen)
        y = torch.randn((k, n), dtype=torch.float64, device=dev, generator=gen)
        torch.cuda.synchronize()

        def wall(fn, setup):
            ts = []
            for _ in range(reps):
                arg = setup()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn(arg)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return statistics.median(ts)

        def events(fn):
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            return statistics.median(ts)

        t_rhs = events(lambda: ctx.pencil_apply(1.0, 0.0, v[:m]))
        t_orth = wall(lambda xx: ctx.global_orth(v, xx, m, normalize=True), lambda: x0.clone())
        xo = x0.clone()
        ctx.global_orth(v, xo, m, normalize=True)
        t_qr = wall(lambda w: ctx.block_qr(w), lambda: xo.clone())
        w = xo.clone()
        ctx.block_qr(w)
        t_proj = wall(lambda w_: ctx.project(w_), lambda: w)
        t_gram = events(lambda: ctx.gram(w, y))
    gb = 2 * k * n * 8 / 1e9
    tf = 2.0 * k * k * n / 1e12
    return {"n": n, "m": m, "blocks": nblocks, "basis_blocks": nb,
            "rhs_apply_ms": round(t_rhs, 4), "orth_ms": round(t_orth, 3),
            "qr_ms": round(t_qr, 3), "project_ms": round(t_proj, 3),
            "gram": {"columns": [k, k], "ms": round(t_gram, 4),
                     "gbs": round(gb / (t_gram * 1e-3), 1),
                     "tflops": round(tf / (t_gram * 1e-3), 2),
                     "frac_hbm": round(gb / (t_gram * 1e-3) / HBM_PEAK_GBS, 4),
                     "frac_fp64": round(tf / (t_gram * 1e-3) / FP64_PEAK_TFLOPS, 4)}}


def measure_copy(stream, dev, mib=1024, reps=5):
    """A plain device copy of `mib` MiB (float32) on the context stream: read
    plus written bytes over the median of `reps` event-timed copies, the
    practical streaming ceiling the row kernels are compared with."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    times = []
    with torch.cuda.stream(stream):
        dst.copy_(src)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            dst.copy_(src)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
    del src, dst
    return 2.0 * (mib << 20) / (statistics.median(times) * 1e-3) / 1e9


def measure_airga_iteration(ctx, stream, F, n, shifts=(1.0, 30.0, 500.0), rmax=24,
                            solve_kw=None, max_outer=1):
    """AIRGA's outer loop at full size through airga_reduce (Algorithm 1 with
    SPAI-preconditioned solves): SPAI builds and solves at the l expansion
    points, thin QR of each block, the moment loop (sigma_j by the moment
    error, moment solves, trace orthogonalisation, intermediate models and
    their H2 changes), the final basis and model, and the next expansion
    points.  Output: tip deflection.  Wall time of the call."""
    import torch
    from paper_1606_01216_amd import airga
    kw = dict(solve_kw or {})
    m = F.shape[0]
    l = len(shifts)
    cp = torch.zeros((1, n), dtype=torch.float64, device=F.device)
    cp[0, n - 2] = 1.0
    out = {"n": n, "m": m, "l": l, "rmax": rmax, "shifts": list(shifts), "max_outer": max_outer}
    try:
        with torch.cuda.stream(stream):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.reduce(F, cp, list(shifts), r_max=rmax, max_outer=max_outer,
                             mode=kw.get("mode", airga.MODE_FP64), tol=kw.get("tol", 1e-10),
                             max_iter=kw.get("max_iter", 20000),
                             poll_every=kw.get("poll_every", 8))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
        h = res["history"][-1]
        out.update({"ms": round((t1 - t0) * 1e3, 2), "iterations": res["iterations"],
                    "J": h["J"], "sigmas": h["sigmas"], "moment_steps": h["moment_steps"],
                    "max_iters": h["max_iters"], "all_converged": h["all_converged"],
                    "last_inner_h2_change": h["last_inner_change"],
                    "next_shifts": [float(f"{v:.6g}") for v in res["next_shifts"]]})
    except airga.AirgaError as e:
        out["error"] = str(e)
    return out


def measure_outer(r=64, m=4, p=1, l=16, reps=20, seed=0):
    """The decisions of AIRGA's outer iteration (host code of the library) at
    the largest reduced order the block operations take: poles of an order-r
    reduced pencil, the next l expansion points, and the H2 distance of two
    order-r models.  Random symmetric positive definite reduced matrices
    with Rayleigh damping; mean wall time of `reps` calls."""
    from paper_1606_01216_amd import airga
    rng = np.random.default_rng(seed)

    def model():
        g = rng.standard_normal((r, r))
        mh = g @ g.T + r * np.eye(r)
        g = rng.standard_normal((r, r))
        kh = g @ g.T + np.eye(r)
        return (mh, kh, rng.standard_normal((r, m)), rng.standard_normal((p, r)), None)
    a, b = model(), model()
    alpha, beta = 0.05, 0.02
    t0 = time.perf_counter()
    for _ in range(reps):
        poles = airga.qep_poles(a[0], a[1], alpha, beta)
    t1 = time.perf_counter()
    for _ in range(reps):
        airga.next_shifts(poles, l)
    t2 = time.perf_counter()
    for _ in range(reps):
        airga.h2_distance(a, b, alpha, beta)
    t3 = time.perf_counter()
    ms = lambda dt: round(dt * 1e3 / reps, 4)  # noqa: E731
    return {"r": r, "m": m, "p": p, "l": l, "qep_poles_ms": ms(t1 - t0),
            "next_shifts_ms": ms(t2 - t1), "h2_distance_ms": ms(t3 - t2)}


def measure_spai_mr(ctx, stream, shifts, precs, F, X, solve_kw, mr_iters=20, tol=0.01):
    """The paper's minimal-residual SPAI loop (Algorithm 2, option mr_iters)
    against the exact column solves, outside the timed step: build time per
    shift (HIP events on the context stream), mean column residual
    ||e_j - K p_j|| of both, and the mixed solve of the same systems with the
    minimal-residual preconditioners."""
    import torch
    from paper_1606_01216_amd import airga
    with torch.cuda.stream(stream):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        mr = [ctx.spai_build(s, mr_iters=mr_iters, tol=tol) for s in shifts]
        e1.record(stream)
        e1.synchronize()
        build_ms = e0.elapsed_time(e1) / len(shifts)
        obj_mr = statistics.mean(p.export()[1].mean().item() for p in mr)
        obj_ex = statistics.mean(p.export()[1].mean().item() for p in precs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.pcg_solve(shifts, mr, F, X, **solve_kw)
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t0) * 1e3
    its = [e["iters"] for e in st]
    out = {"mr_iters": mr_iters, "tol": tol, "build_ms_per_shift": round(build_ms, 4),
           "mean_column_residual": {"mr": round(obj_mr, 5), "exact": round(obj_ex, 5)},
           "pcg_mixed_ms": round(solve_ms, 3), "iters_median": statistics.median(its),
           "iters_max": max(its),
           "converged": sum(e["status"] == airga.SYS_CONVERGED for e in st), "systems": len(st)}
    for p in mr:
        p.release()
    return out


# ------------------------------------------------------- algorithmic bytes
#
# Bytes each kernel of a solve must move (DESIGN's kernel table), from the
# work the library counted in a profiled solve: launches, (system, launch)
# passes and (shift, launch) passes.  w = bytes per vector value, fw = per
# preconditioner value, ib = column information per stored entry.
def kernel_bytes(name, launches, sysp, shp, *, stored, n, ib, w, fw, m, first_passes=0,
                 mixed=True, gp=0, red_sys=0, assign_sys=0, zs_launches=0, zs_sys=0):
    if name == "dir_spmv":
        return launches * stored * (ib + 2 * w) + sysp * 4 * w * n
    if name == "update_prec":
        return launches * stored * ib + shp * stored * fw + (sysp * 7 - first_passes) * w * n
    if name == "init_prec":
        return launches * stored * ib + shp * stored * fw + sysp * 2 * w * n
    if name == "chain":
        # int32 columns once per launch, each (shift, factor) pair's values,
        # and per (system, factor): read t, write z
        return launches * stored * 4 + shp * stored * fw + sysp * 2 * w * n
    if name == "ir_residual":
        # float64 M and K with their columns, F once per launch and column,
        # per system: read X, write r; the first residual of a solve from
        # X = 0 (zs_launches launches) reads no pencil, and in mixed mode no
        # X either (zs_sys systems; float64 solves write the zero X instead)
        return ((launches - zs_launches) * stored * (ib + 16) + launches * m * 8 * n +
                sysp * (8 + w) * n - zs_sys * 8 * n)
    if name == "ir_update":
        # mixed: read X and the correction, write X (the first sweep of a
        # solve without a starting guess assigns X: no read, assign_sys
        # systems); float64: copy out
        return (sysp * (16 + w) - assign_sys * 8) * n if mixed else sysp * 16 * n
    if name == "reduce":
        # one block per active system reads its partials: about 8 B per
        # row-kernel block and slot (gp blocks, red_sys (system, slot) reads)
        return red_sys * gp * 8
    return None


def row_blocks(n, rows_per_wave):
    """Blocks of a row-kernel launch (4 wavefronts of rows_per_wave rows over
    the 64-row padded matrix), one partial per block and system and slot."""
    n_pad = -(-n // 64) * 64
    waves = -(-n_pad // rows_per_wave)
    return -(-waves // 4)


def kernel_rows(kt, kwk, **kw):
    """Per-kernel launches, time, algorithmic bytes and GB/s of a profiled solve."""
    sysp_of = {k: v[0] for k, v in kwk.items()}
    # slots the reductions read: 1 per direction pass, 3 per update pass, 2 per restart
    red_sys = (sysp_of.get("dir_spmv", 0) + 3 * sysp_of.get("update_prec", 0) +
               2 * sysp_of.get("init_prec", 0))
    rows = []
    for name in ("dir_spmv", "update_prec", "init_prec", "chain", "ir_residual", "ir_update",
                 "reduce"):
        la, ms = kt.get(name, (0, 0.0))
        sysp, shp = kwk.get(name, (0, 0))
        if la:
            b = kernel_bytes(name, la, sysp, shp, red_sys=red_sys, **kw)
            rows.append(dict(kernel=name, launches=la, total_ms=round(ms, 4),
                             avg_us=round(1e3 * ms / la, 2),
                             gbs=round(b / (ms * 1e-3) / 1e9, 1) if b and ms > 0 else None,
                             bytes=int(b) if b is not None else None))
    return rows


# ------------------------------------------------------------ CPU baseline
#
# The oracle's reference solves on this host's cores: one thread, and all
# the cores this process may use (up to CPU_WORKERS, the host-core share of
# one GPU on the benchmark machine), independent shifts on threads (the C
# part of the oracle releases the interpreter lock).
CPU_WORKERS = 16


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    return model, visible


def oracle_refs(pen, shift_list, f, precision, workers):
    """Oracle X(s) (m, n) for every shift in shift_list."""
    from oracle import _native, direct
    _native.lib()
    job = lambda s: direct.reference_solve(pen, s, f, precision)  # noqa: E731
    if workers <= 1:
        return [job(s) for s in shift_list]
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(job, shift_list))


def median_time(fn, reps=3, label=None):
    """(median seconds over reps runs, result of the last run); with a label,
    one progress line per run."""
    ts, res = [], None
    for i in range(reps):
        t0 = time.perf_counter()
        res = fn()
        ts.append(time.perf_counter() - t0)
        if label:
            log(f"[bench] {label}: run {i + 1} of {reps}, {ts[-1]:.2f} s")
    return statistics.median(ts), res


def measure_cpu_baseline(pen, f, shift_sets, sample_shifts=4, reps=3):
    """Oracle timings (double-double and binary64 banded Cholesky) on one
    thread for a sample of shifts and on all cores for every shift of the
    step, medians of `reps`; returns the timings and both references."""
    model, visible = cpu_info()
    workers = max(1, min(CPU_WORKERS, visible))
    allsh = [s for ss in shift_sets for s in ss]
    m = f.shape[0]
    sample = list(shift_sets[0][:sample_shifts])
    t_dd1, _ = median_time(lambda: oracle_refs(pen, sample, f, "dd", 1), reps,
                           "oracle double-double, one thread")
    t_ddw, refs_dd = median_time(lambda: oracle_refs(pen, allsh, f, "dd", workers), reps,
                                 f"oracle double-double, {workers} threads")
    t_641, _ = median_time(lambda: oracle_refs(pen, sample, f, "f64", 1), reps,
                           "oracle binary64, one thread")
    t_64w, refs_64 = median_time(lambda: oracle_refs(pen, allsh, f, "f64", workers), reps,
                                 f"oracle binary64, {workers} threads")
    ns, na = len(sample) * m, len(allsh) * m
    return dict(cpu_model=model, cores_visible=visible, cores_all=workers,
                dd_1=ns / t_dd1, dd_all=na / t_ddw, f64_1=ns / t_641, f64_all=na / t_64w,
                sample_systems=ns, all_systems=na, t_dd1=t_dd1, t_ddw=t_ddw, t_641=t_641,
                t_64w=t_64w), refs_dd, refs_64


def rel_errors(X, refs, S, m):
    """Per-system ||X - ref|| / ||ref|| for X (S, m, n) and refs[k] (m, n)."""
    out = []
    for k in range(S):
        for c in range(m):
            nr = np.linalg.norm(refs[k][c])
            out.append(float(np.linalg.norm(X[k, c] - refs[k][c]) / nr))
    return out


# ------------------------------------------ update-chain sequence (1e5 DOF)
def measure_c2_sequence(dev, stream, tol=1e-8, seed=0, reps=2):
    """The plain float64 solve sequence of the 100,000-DOF beam: the SPAI
    (equilibrated, without the symmetric average, whose factor at s = 1 is
    indefinite and breaks every chain built on it) is built at the first of
    8 log-spaced shifts and updated along them (the
    horizontal chain Q_8 ... Q_2 P_1), then updated again at three seeded
    vertical drifts of every shift (epsilon 1e-2, 1e-3, 1e-3), each new
    expansion point solved once with its chain (float64, one system per
    solve, relative residual tol).  Every solve is checked against the
    oracle's double-double reference.  The sequence runs `reps` times; the
    last run is reported (the first also autotunes)."""
    import torch
    from paper_1606_01216_amd import airga
    pen, f, shifts, rng = beam.make_workload("c2", surrogate=True, seed=seed)
    levels = [np.asarray(shifts, float)]
    for eps in (1e-2, 1e-3, 1e-3):
        levels.append(beam.drift_shifts(levels[-1], eps, rng))
    n = pen.n
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = airga.Context(0, stream)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    F = t(f, torch.float64)
    X = torch.zeros((len(levels), len(shifts), 1, n), dtype=torch.float64, device=dev)
    kw = dict(tol=tol, mode=airga.MODE_FP64, max_iter=20000, poll_every=8, use_graph=False)
    with torch.cuda.stream(stream):
        ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                       t(pen.m_val, torch.float64), t(pen.k_val, torch.float64),
                       pen.alpha, pen.beta)
        for _ in range(reps):
            recs, handles = [], []
            torch.cuda.synchronize()
            t_all0 = time.perf_counter()
            prev_level = None
            for z, lev in enumerate(levels):
                cur = []
                for i, s in enumerate(lev):
                    e0, e1 = ev(), ev()
                    e0.record(stream)
                    if z == 0:
                        p = (ctx.spai_build(float(s), symmetrize=False) if i == 0
                             else ctx.spai_update(cur[-1], float(s)))
                    else:
                        p = ctx.spai_update(prev_level[i], float(s))
                    e1.record(stream)
                    cur.append(p)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, st = ctx.pcg_solve([float(s)], [p], F, X[z, i:i + 1], **kw)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    info = p.info()
                    recs.append(dict(z=z + 1, i=i + 1, shift=float(s), chain_len=info.chain_len,
                                     skipped_frac=round(info.skipped_cols / n, 4),
                                     kind="build" if (z == 0 and i == 0) else
                                     ("horizontal" if z == 0 else "vertical"),
                                     prec_ms=round(e0.elapsed_time(e1), 4),
                                     solve_ms=round((t1 - t0) * 1e3, 3), iters=st[0]["iters"],
                                     status=airga.STATUS_NAMES[st[0]["status"]]))
                handles.extend(cur)
                prev_level = cur
            torch.cuda.synchronize()
            t_all = time.perf_counter() - t_all0
            for p in handles:
                p.release()
    Xh = X.cpu().numpy()
    refs = oracle_refs(pen, [s for lev in levels for s in lev], f, "dd",
                       max(1, min(CPU_WORKERS, cpu_info()[1])))
    for r, ref in zip(recs, refs):
        x = Xh[r["z"] - 1, r["i"] - 1, 0]
        r["rel_err"] = float(f"{np.linalg.norm(x - ref[0]) / np.linalg.norm(ref[0]):.3e}")
    ctx.close()
    by_len = {}
    for r in recs:
        by_len.setdefault(r["chain_len"], []).append(r)
    upd = [r for r in recs if r["kind"] != "build"]
    solved_upd = [r for r in upd if r["skipped_frac"] < 1.0]
    return {
        "workload": "Hermite cantilever n=100,000 (EI log-uniform [0.5,2], scaled by h^4), tip "
                    "load, 8 shifts logspace(0,4,8), 3 vertical drifts (1e-2, 1e-3, 1e-3)",
        "n": n, "tol_relres": tol, "solves": len(recs), "sequence_ms": round(t_all * 1e3, 2),
        "solved_to_1e-8": sum(r["rel_err"] <= ERR_TOL for r in recs),
        "max_rel_err": max(r["rel_err"] for r in recs),
        "build_ms": recs[0]["prec_ms"],
        "update_ms_mean": round(statistics.mean(r["prec_ms"] for r in upd), 4),
        "update_ms_mean_with_solved_columns": round(statistics.mean(
            r["prec_ms"] for r in solved_upd), 4) if solved_upd else None,
        "update_skipped_frac_mean": {
            "horizontal": round(statistics.mean(r["skipped_frac"] for r in upd
                                                if r["kind"] == "horizontal"), 4),
            "vertical": round(statistics.mean(r["skipped_frac"] for r in upd
                                              if r["kind"] == "vertical"), 4)},
        "by_chain_len": {str(k): {"solves": len(v),
                                  "iters_mean": round(statistics.mean(r["iters"] for r in v), 1),
                                  "solve_ms_mean": round(statistics.mean(r["solve_ms"] for r in v), 3)}
                         for k, v in sorted(by_len.items())},
        "solves_detail": recs}


def measure_complex(ctx, stream, pen, f, F, sigmas, tol, reps=3, angle=np.pi / 6):
    """Complex expansion points s_k = sigma_k e^{i angle} (the workload's real
    points turned off the real axis; K(s) complex symmetric): the complex
    SPAI at every point and one batched COCG of all (point, column) systems
    in float64, warmed by one untimed run, wall time median of `reps`;
    every system against the oracle's complex double-double reference.
    Algorithmic bytes per iteration and system: 64 n (direction kernel: read
    z and p, write p and w) + 112 n (update kernel: read r, w, x, p, write
    x, r, z), 16-byte complex values; per launch the pencil (20 B per stored
    entry: column, M, K) and per (point, launch) the factor (16 B)."""
    import torch
    from paper_1606_01216_amd import airga
    n, m = pen.n, F.shape[0]
    cs = [complex(v * np.exp(1j * angle)) for v in sigmas]
    with torch.cuda.stream(stream):
        # the context holds the workload's pencil (set by every step)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # one untimed build first (the first launches of a process load the
        # kernels and grow the factor pool), then the timed one
        for p in ctx.spai_build_complex_many(cs):
            p.release()
        e0.record(stream)
        precs = ctx.spai_build_complex_many(cs)
        e1.record(stream)
        e1.synchronize()
        build_ms = e0.elapsed_time(e1) / len(cs)
        X = torch.empty((len(cs), m, n), dtype=torch.complex128, device=F.device)
        ctx.cocg_solve(cs, precs, F, X, tol=tol)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = ctx.cocg_solve(cs, precs, F, X, tol=tol)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
    t = statistics.median(ts)
    its = [e["iters"] for e in st]
    stored = ctx.pencil_info().nnz_stored
    launches = 2 * max(its)
    byts = sum(its) * 176 * n + launches * 20 * stored + max(its) * len(cs) * 16 * stored
    # the same systems in MIXED mode (float32 COCG inside float64 refinement)
    with torch.cuda.stream(stream):
        Xm = torch.empty_like(X)
        ctx.cocg_solve(cs, precs, F, Xm, tol=tol, mode=airga.MODE_MIXED)
        tsm = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, stm = ctx.cocg_solve(cs, precs, F, Xm, tol=tol, mode=airga.MODE_MIXED)
            torch.cuda.synchronize()
            tsm.append(time.perf_counter() - t0)
    refs = oracle_refs_complex(pen, cs, f, max(1, min(CPU_WORKERS, cpu_info()[1])))
    Xh = X.cpu().numpy()
    errs = [rel_errors_c(Xh[k, c], refs[k][c]) for k in range(len(cs)) for c in range(m)]
    ok = sum(e <= ERR_TOL for e in errs)
    Xmh = Xm.cpu().numpy()
    del Xm
    errsm = [rel_errors_c(Xmh[k, c], refs[k][c]) for k in range(len(cs)) for c in range(m)]
    tm = statistics.median(tsm)
    mixed = {"precision": "float32 COCG inside float64 refinement",
             "cocg_solves_per_s": round(sum(e <= ERR_TOL for e in errsm) / tm, 2),
             "seconds_median_of_3": round(tm, 4),
             "solved_to_1e-8": sum(e <= ERR_TOL for e in errsm), "max_rel_err": max(errsm),
             "iters_median": statistics.median(e["iters"] for e in stm),
             "iters_max": max(e["iters"] for e in stm),
             "sweeps_max": max(e["sweeps"] for e in stm),
             "converged": sum(e["status"] == airga.SYS_CONVERGED for e in stm)}
    # the update to nearby points (each sigma_k moved by a seeded factor
    # 1 + 0.05 U(-1, 1), same angle) and the solves with the chains Q P
    drift = np.random.default_rng(7).uniform(-1.0, 1.0, len(cs))
    cs2 = [complex(z * (1.0 + 0.05 * d)) for z, d in zip(cs, drift)]
    with torch.cuda.stream(stream):
        for p in ctx.spai_update_complex_many(precs, cs2):  # untimed, as for the build
            p.release()
        e0.record(stream)
        upd = ctx.spai_update_complex_many(precs, cs2)
        e1.record(stream)
        e1.synchronize()
        upd_ms = e0.elapsed_time(e1) / len(cs)
        X2 = torch.empty_like(X)
        # capped: a system whose recurrence residual stalls above tol is
        # reported as such (with its error) rather than run to 20000 steps
        ctx.cocg_solve(cs2, upd, F, X2, tol=tol, max_iter=2000)
        ts2 = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st2 = ctx.cocg_solve(cs2, upd, F, X2, tol=tol, max_iter=2000)
            torch.cuda.synchronize()
            ts2.append(time.perf_counter() - t0)
        # and in MIXED mode: every sweep restarts from the float64 residual
        ctx.cocg_solve(cs2, upd, F, X, tol=tol, max_iter=2000, mode=airga.MODE_MIXED)
        ts3 = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st3 = ctx.cocg_solve(cs2, upd, F, X, tol=tol, max_iter=2000, mode=airga.MODE_MIXED)
            torch.cuda.synchronize()
            ts3.append(time.perf_counter() - t0)
    infos = [u.info() for u in upd]
    refs2 = oracle_refs_complex(pen, cs2, f, max(1, min(CPU_WORKERS, cpu_info()[1])))
    X2h = X2.cpu().numpy()
    errs2 = [rel_errors_c(X2h[k, c], refs2[k][c]) for k in range(len(cs2)) for c in range(m)]
    X3h = X.cpu().numpy()
    errs3 = [rel_errors_c(X3h[k, c], refs2[k][c]) for k in range(len(cs2)) for c in range(m)]
    t3 = statistics.median(ts3)
    t2 = statistics.median(ts2)
    its2 = [e["iters"] for e in st2]
    updates = {"drift": "sigma_k (1 + 0.05 U(-1, 1)), seeded",
               "spai_update_ms_per_point": round(upd_ms, 4),
               "skipped_frac_mean": round(statistics.mean(i.skipped_cols / n for i in infos), 4),
               "chain_len_max": max(i.chain_len for i in infos),
               "cocg_solves_per_s": round(sum(e <= ERR_TOL for e in errs2) / t2, 2),
               "seconds_median_of_3": round(t2, 4),
               "solved_to_1e-8": sum(e <= ERR_TOL for e in errs2), "max_rel_err": max(errs2),
               "iters_median": statistics.median(its2), "iters_max": max(its2),
               "converged": sum(e["status"] == airga.SYS_CONVERGED for e in st2),
               "not_converged": [{"sigma": float(f"{abs(cs2[i // m]):.6g}"), "column": i % m,
                                  "status": airga.STATUS_NAMES[e["status"]], "iters": e["iters"],
                                  "relres": float(f"{e['relres']:.3e}"),
                                  "rel_err": float(f"{errs2[i]:.3e}")}
                                 for i, e in enumerate(st2) if e["status"] != airga.SYS_CONVERGED],
               "mixed": {"cocg_solves_per_s": round(sum(e <= ERR_TOL for e in errs3) / t3, 2),
                         "seconds_median_of_3": round(t3, 4),
                         "solved_to_1e-8": sum(e <= ERR_TOL for e in errs3),
                         "max_rel_err": max(errs3),
                         "iters_median": statistics.median(e["iters"] for e in st3),
                         "iters_max": max(e["iters"] for e in st3),
                         "sweeps_max": max(e["sweeps"] for e in st3),
                         "converged": sum(e["status"] == airga.SYS_CONVERGED for e in st3)}}
    for p in upd + precs:
        p.release()
    return {"workload": f"{len(cs)} complex points sigma_k e^(i pi/6), sigma_k = the real "
                        f"workload's points; {m} loads; {len(cs) * m} systems",
            "updates": updates, "mixed": mixed,
            "precision": "complex float64", "spai_build_ms_per_shift": round(build_ms, 4),
            "cocg_solves_per_s": round(ok / t, 2), "seconds_median_of_3": round(t, 4),
            "solved_to_1e-8": ok, "systems": len(errs), "max_rel_err": max(errs),
            "iters_median": statistics.median(its), "iters_max": max(its),
            "converged": sum(e["status"] == airga.SYS_CONVERGED for e in st),
            "algorithmic_gbs": round(byts / t / 1e9, 1),
            "frac_hbm": round(byts / t / 1e9 / HBM_PEAK_GBS, 4)}


def oracle_refs_complex(pen, shifts, f, workers):
    from oracle import _native, direct
    _native.lib()
    with cf.ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda s: direct.reference_solve_complex(pen, s, f, "dd"), shifts))


def rel_errors_c(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def measure_c1_literal(dev, stream):
    """The literal 1000-DOF cantilever (EI = 1, s = 100, tip load, SPAI on
    the pattern of K(s), CG to 1e-10): float64 and mixed solves, their
    errors against the oracle's double-double and binary64 references, and
    the binary64 floor (the oracle's binary64 Cholesky against double-double;
    no float64 solver gets much below it at cond(K(s)) ~ 3e10)."""
    import torch
    from oracle import direct
    from paper_1606_01216_amd import airga
    pen, f, shifts, _ = beam.make_workload("c1")
    s = float(shifts[0])
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = airga.Context(0, stream)
    out = {"workload": "Hermite cantilever n=1000, EI=1 (literal), tip load, s=100", "n": pen.n}
    ref = direct.reference_solve(pen, s, f, "dd")[0]
    r64 = direct.reference_solve(pen, s, f, "f64")[0]
    nr = np.linalg.norm(ref)
    out["f64_cholesky_vs_dd"] = float(f"{np.linalg.norm(r64 - ref) / nr:.3e}")
    with torch.cuda.stream(stream):
        ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                       t(pen.m_val, torch.float64), t(pen.k_val, torch.float64), pen.alpha,
                       pen.beta)
        p = ctx.spai_build(s)
        F = t(f, torch.float64)
        for name, mode in (("fp64", airga.MODE_FP64), ("mixed", airga.MODE_MIXED)):
            ctx.pcg_solve([s], [p], F, tol=1e-10, max_iter=40000, mode=mode)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X, st = ctx.pcg_solve([s], [p], F, tol=1e-10, max_iter=40000, mode=mode)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            x = X[0, 0].cpu().numpy()
            out[name] = {"status": airga.STATUS_NAMES[st[0]["status"]], "iters": st[0]["iters"],
                         "ms": round(ms, 3),
                         "rel_err_vs_dd": float(f"{np.linalg.norm(x - ref) / nr:.3e}"),
                         "rel_err_vs_f64": float(f"{np.linalg.norm(x - r64) / np.linalg.norm(r64):.3e}"),
                         "finished_fp64": bool(st[0]["finished_fp64"])}
        p.release()
    ctx.close()
    return out


def measure_airga_updates(dev, stream, max_outer=4, update_from=3):
    """AIRGA's loop with the cheap update across outer iterations (Algorithm
    5) where the expansion points settle: the literal 60-DOF cantilever (EI =
    1, alpha = 0.01, beta = 0.001), points 1, 30, 500, tip input and output,
    r_max = 12; from outer iteration update_from on each point's
    preconditioner is the update of the previous one.  Per iteration: the
    points, J, whether the factors were updated, the longest chain, the
    largest CG iteration count and the relative H2 change."""
    import torch
    from paper_1606_01216_amd import airga
    pen = beam.make_beam(30, seed=3, alpha=0.01, beta=0.001)
    n = pen.n
    f = np.zeros((1, n))
    f[0, n - 2] = 1.0
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = airga.Context(0, stream)
    with torch.cuda.stream(stream):
        ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                       t(pen.m_val, torch.float64), t(pen.k_val, torch.float64), pen.alpha,
                       pen.beta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.reduce(t(f, torch.float64), t(f, torch.float64), [1.0, 30.0, 500.0], r_max=12,
                         max_outer=max_outer, update_from=update_from, tol=1e-12)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    return {"workload": "literal Hermite cantilever n=60, EI=1, alpha=0.01, beta=0.001, points "
                        "1, 30, 500, tip input and output, r_max=12",
            "update_from": update_from, "ms": round(ms, 2), "iterations": res["iterations"],
            "history": [{"shifts": [float(f"{v:.6g}") for v in h["shifts"]], "J": h["J"],
                         "updated": h["updated"], "chain_len_max": h["chain_len_max"],
                         "max_iters": h["max_iters"], "all_converged": h["all_converged"],
                         "change": None if h["change"] is None else float(f"{h['change']:.3e}")}
                        for h in res["history"]]}


# ------------------------------------------------------------ literal shapes
#
# The unscaled beams (EI as stated, h = 1 / n_el) have equilibrated condition
# numbers of about 3e11 (n / 1e3)^4 at s = 1: from n = 1e5 on, no float64 CG
# reaches 1e-8 and float32 refinement cannot contract.  Their solves are
# timed at a fixed iteration count instead (tolerance 1e-30, so every system
# runs exactly `cap` iterations, the same for batched and one-at-a-time
# solves); the statuses at the cap and the errors against the oracle's
# double-double reference are reported as observed.
LITERAL_TOL = 1e-30


def literal_refs(pen, shift_list, f, workers):
    """The oracle's double-double reference per shift, or None where the
    stored K(s) is not positive definite even in double-double: the binary64
    rounding of the unscaled beam's entries (relative 1e-16 of entries near
    12 EI / h^3) exceeds the smallest eigenvalue once cond(K(s)) passes about
    1e16, so the matrix that was stored may have no Cholesky factor at all.
    Returns (refs, notes)."""
    from oracle import _native, direct
    _native.lib()

    def job(s):
        try:
            return direct.reference_solve(pen, s, f, "dd"), "dd"
        except np.linalg.LinAlgError as e:
            return None, f"none: {e}"
    with cf.ThreadPoolExecutor(max(1, workers)) as ex:
        out = list(ex.map(job, shift_list))
    return [o[0] for o in out], [o[1] for o in out]


def _literal_solve(ctx, stream, shifts, precs, F, X, kw, rows_kw, reps=3):
    """Median wall time of `reps` capped solves (after one untimed run),
    then one profiled run: (seconds, stats, kernel rows, solve-level GB/s)."""
    import torch
    with torch.cuda.stream(stream):
        ctx.pcg_solve(shifts, precs, F, X, **kw)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = ctx.pcg_solve(shifts, precs, F, X, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ctx.pcg_solve(shifts, precs, F, X, profile=True, **kw)
        kt, kwk = ctx.kernel_times(), ctx.kernel_work()
        tile = ctx.tile_config()
    n = F.shape[1]
    rows = kernel_rows(kt, kwk, gp=row_blocks(n, tile[0]), **rows_kw)
    sec = statistics.median(ts)
    tot = sum(r["bytes"] for r in rows if r["bytes"])
    return sec, st, rows, round(tot / sec / 1e9, 1), tile


def _status_counts(st):
    from paper_1606_01216_amd import airga
    out = {}
    for e in st:
        k = airga.STATUS_NAMES[e["status"]]
        out[k] = out.get(k, 0) + 1
    return out


def _err_summary(errs):
    if not errs:
        return {"systems": 0}
    return {"systems": len(errs), "min": float(f"{min(errs):.3e}"),
            "median": float(f"{statistics.median(errs):.3e}"), "max": float(f"{max(errs):.3e}"),
            "within_1e-8": sum(e <= ERR_TOL for e in errs)}


def measure_literal_batched(dev, stream, base, cap, err_idx, fp64=True, plain=2, reps=3):
    """One literal workload (c3 or c5): the batched SPAI build of all its
    shifts (median of 3), then the batched solves of every system at `cap`
    iterations: float64 (config 3) if `fp64`, mixed (config 4: one float32
    sweep of `cap` iterations, then the float64 residual), and `plain`
    systems one at a time in float64.  Errors against the double-double
    reference for the shifts `err_idx` (all their loads)."""
    import torch
    from paper_1606_01216_amd import airga
    pen, f, shifts, _ = beam.make_workload(base)
    n, m, S = pen.n, f.shape[0], len(shifts)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = airga.Context(0, stream)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    out = {"n": n, "m": m, "shifts": S, "systems": S * m, "cap_iters": cap}
    with torch.cuda.stream(stream):
        ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                       t(pen.m_val, torch.float64), t(pen.k_val, torch.float64), pen.alpha,
                       pen.beta)
        info = ctx.pencil_info()
        F = t(f, torch.float64)
        bms = []
        for _ in range(3):
            e0, e1 = ev(), ev()
            e0.record(stream)
            precs = ctx.spai_build_many(list(shifts))
            e1.record(stream)
            torch.cuda.synchronize()
            bms.append(e0.elapsed_time(e1))
            if len(bms) < 3:
                for p in precs:
                    p.release()
        out["spai_build_ms_per_shift"] = round(statistics.median(bms) / S, 4)
    stored = info.nnz_stored
    ib = 1 if info.bandwidth <= 64 else 4
    base_kw = dict(shifts=list(shifts), precs=precs, F=F)
    X = torch.zeros((S, m, n), dtype=torch.float64, device=dev)
    refs, notes = literal_refs(pen, [shifts[i] for i in err_idx], f,
                               min(CPU_WORKERS, cpu_info()[1], len(err_idx)))
    out["reference"] = {f"{shifts[i]:.6g}": note for i, note in zip(err_idx, notes)}

    def errors(Xd):
        xs = Xd[list(err_idx)].cpu().numpy()
        return [float(np.linalg.norm(xs[a, c] - refs[a][c]) / np.linalg.norm(refs[a][c]))
                for a in range(len(err_idx)) if refs[a] is not None for c in range(m)]

    legs = []
    if fp64:
        legs.append(("batched_fp64", dict(tol=LITERAL_TOL, mode=airga.MODE_FP64, max_iter=cap,
                                          poll_every=8),
                     dict(w=8, fw=8, first_passes=0, mixed=False, zs_launches=1)))
    legs.append(("batched_mixed", dict(tol=LITERAL_TOL, mode=airga.MODE_MIXED, max_iter=cap,
                                       inner_max=cap, inner_tol=LITERAL_TOL, max_sweeps=1,
                                       poll_every=8),
                 dict(w=4, fw=4, first_passes=S * m, mixed=True, assign_sys=S * m, zs_launches=1,
                      zs_sys=S * m)))
    for name, kw, rkw in legs:
        log(f"[bench] literal {base}: {name} at {cap} iterations")
        sec, st, rows, gbs, tile = _literal_solve(
            ctx, stream, base_kw["shifts"], precs, F, X, kw,
            dict(stored=stored, n=n, ib=ib, m=m, **rkw), reps)
        iters = [e["iters"] for e in st]
        out[name] = {"seconds_median_of_3": round(sec, 4),
                     "ms_per_iteration": round(sec * 1e3 / max(iters), 4),
                     "system_iterations_per_s": round(sum(iters) / sec, 1),
                     "iters_min": min(iters), "iters_max": max(iters),
                     "status": _status_counts(st), "algorithmic_gbs": gbs,
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "tile": list(tile),
                     "kernels": rows, "rel_err_vs_dd": _err_summary(errors(X))}
    if plain:
        log(f"[bench] literal {base}: plain float64 one system at a time")
        kw = dict(tol=LITERAL_TOL, mode=airga.MODE_FP64, max_iter=cap, poll_every=8)
        Xp = torch.zeros((1, 1, n), dtype=torch.float64, device=dev)
        with torch.cuda.stream(stream):
            ctx.pcg_solve([float(shifts[0])], [precs[0]], F[0:1], Xp, **kw)
            ts, sts = [], []
            for k in range(plain):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = ctx.pcg_solve([float(shifts[k])], [precs[k]], F[0:1], Xp, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                sts += st
        sec = statistics.mean(ts)
        out["plain_fp64"] = {"systems_timed": plain, "seconds_per_system": round(sec, 4),
                             "ms_per_iteration": round(sec * 1e3 / cap, 4),
                             "system_iterations_per_s": round(cap / sec, 1),
                             "status": _status_counts(sts)}
        if fp64:
            out["batched_fp64_vs_plain_per_iteration"] = round(
                out["batched_fp64"]["system_iterations_per_s"] /
                out["plain_fp64"]["system_iterations_per_s"], 2)
    out["batched_mixed_vs_plain_per_iteration"] = round(
        out["batched_mixed"]["system_iterations_per_s"] /
        out["plain_fp64"]["system_iterations_per_s"], 2) if plain else None
    out["err_shifts"] = [float(f"{shifts[i]:.6g}") for i in err_idx]
    for p in precs:
        p.release()
    ctx.close()
    del X, F
    torch.cuda.empty_cache()
    return out


def measure_literal_c2(dev, stream, cap):
    """Config 2 literal: the 100,000-DOF beam (EI log-uniform [0.5, 2]),
    tip load; SPAI built at s_1 and updated along the 8 log-spaced shifts
    (the horizontal chain), each solved once in float64 at `cap`
    iterations; per shift the build or update ms, the chain length, the
    skipped fraction, the status and the error against double-double."""
    import torch
    from paper_1606_01216_amd import airga
    pen, f, shifts, _ = beam.make_workload("c2")
    n = pen.n
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    ctx = airga.Context(0, stream)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    F = t(f, torch.float64)
    X = torch.zeros((len(shifts), 1, n), dtype=torch.float64, device=dev)
    kw = dict(tol=LITERAL_TOL, mode=airga.MODE_FP64, max_iter=cap, poll_every=8, use_graph=False)
    recs, handles = [], []
    with torch.cuda.stream(stream):
        ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                       t(pen.m_val, torch.float64), t(pen.k_val, torch.float64), pen.alpha,
                       pen.beta)
        for i, s in enumerate(shifts):
            e0, e1 = ev(), ev()
            e0.record(stream)
            p = (ctx.spai_build(float(s), symmetrize=False) if i == 0
                 else ctx.spai_update(handles[-1], float(s)))
            e1.record(stream)
            handles.append(p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = ctx.pcg_solve([float(s)], [p], F, X[i:i + 1], **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = p.info()
            recs.append(dict(shift=float(f"{s:.6g}"), kind="build" if i == 0 else "update",
                             chain_len=info.chain_len,
                             skipped_frac=round(info.skipped_cols / n, 4),
                             prec_ms=round(e0.elapsed_time(e1), 4),
                             solve_ms=round((t1 - t0) * 1e3, 3), iters=st[0]["iters"],
                             status=airga.STATUS_NAMES[st[0]["status"]],
                             relres=float(f"{st[0]['relres']:.3e}")))
        for p in handles:
            p.release()
    refs, notes = literal_refs(pen, list(shifts), f, min(CPU_WORKERS, cpu_info()[1]))
    Xh = X.cpu().numpy()
    for r, x, ref, note in zip(recs, Xh, refs, notes):
        r["reference"] = note
        r["rel_err_vs_dd"] = (None if ref is None else
                              float(f"{np.linalg.norm(x[0] - ref[0]) / np.linalg.norm(ref[0]):.3e}"))
    ctx.close()
    return {"n": n, "cap_iters": cap, "solves": recs}


def measure_literal(dev, stream, cap=200, c5_cap=100):
    return {
        "note": "unscaled beams, every system run to a fixed iteration count (tolerance 1e-30); "
                "statuses and errors as observed",
        "c2": dict(workload="Hermite cantilever n=100,000, EI log-uniform [0.5,2] (literal), tip "
                            "load, 8 shifts logspace(0,4,8): build at s_1, horizontal update chain",
                   **measure_literal_c2(dev, stream, cap)),
        "c3_c4": dict(workload="Hermite cantilever n=1,000,000, EI=1 (literal), m=4 seeded unit "
                               "loads, 16 shifts logspace(0,4,16)",
                      **measure_literal_batched(dev, stream, "c3", cap, err_idx=(0, 5, 10, 15))),
        "c5": dict(workload="Hermite cantilever n=10,000,000, EI log-uniform [0.1,10] (literal), "
                            "m=4, 32 shifts logspace(0,5,32)",
                   **measure_literal_batched(dev, stream, "c5", c5_cap, err_idx=(0, 10, 21, 31),
                                             fp64=False, plain=1)),
    }


def measure_batched_fp64(ctx, stream, sets, F, tol, poll_every, reps=5):
    """Config 3: batched float64 PCG of every system of a step (one call per
    shift set, all its systems in one set of kernels), warmed by one untimed
    run; wall time median of `reps`, then one profiled run (kernel table)."""
    import torch
    from paper_1606_01216_amd import airga
    kw = dict(tol=tol, mode=airga.MODE_FP64, max_iter=20000, poll_every=poll_every)
    with torch.cuda.stream(stream):
        def run(profile=False):
            sts = []
            for ss, pp, XX in sets:
                _, st = ctx.pcg_solve(ss, pp, F, XX, profile=profile, **kw)
                sts += st
            return sts
        run()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        # profiled: the second set only (kernel table of one solve)
        ss, pp, XX = sets[-1]
        _, stp = ctx.pcg_solve(ss, pp, F, XX, profile=True, **kw)
        kt, kwk = ctx.kernel_times(), ctx.kernel_work()
        tile = ctx.tile_config()
    return statistics.median(ts), sts, kt, kwk, tile


def measure_plain_fp64(ctx, stream, sets, F, tol, poll_every, reps=5):
    """Plain float64 PCG one system at a time on the same systems and
    preconditioners, into preallocated outputs; warmed by one untimed pass,
    wall time median of `reps` passes."""
    import torch
    from paper_1606_01216_amd import airga
    n = F.shape[1]
    kw = dict(tol=tol, mode=airga.MODE_FP64, max_iter=20000, poll_every=poll_every)
    with torch.cuda.stream(stream):
        def run():
            sts = []
            for ss, pp, XX in sets:
                for k in range(len(ss)):
                    for c in range(F.shape[0]):
                        _, st = ctx.pcg_solve([ss[k]], [pp[k]], F[c:c + 1],
                                              XX[k, c].view(1, 1, n), **kw)
                        sts.append(st[0])
            return sts
        run()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
    return statistics.median(ts), sts


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--workload", default="c4s", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain float64 comparator")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the 100,000-DOF update-chain sequence")
    ap.add_argument("--no-complex", action="store_true",
                    help="skip the complex-expansion-point leg")
    ap.add_argument("--complex-only", action="store_true",
                    help="run only the complex-expansion-point leg and print its JSON")
    ap.add_argument("--c2-only", action="store_true",
                    help="run only the update-chain sequence and print its JSON (for profilers)")
    ap.add_argument("--no-airga-iteration", action="store_true",
                    help="skip the full-size AIRGA iteration (its small solves would enter a "
                         "profiler's per-kernel averages)")
    ap.add_argument("--no-literal", action="store_true",
                    help="skip the literal shapes at a fixed iteration count")
    ap.add_argument("--literal-only", action="store_true",
                    help="run only the literal shapes, the literal 1000-DOF beam and the "
                         "AIRGA loop with updates, and print their JSON")
    ap.add_argument("--quick", action="store_true", help="timed steps only (for profilers)")
    ap.add_argument("--tile", default=None,
                    help="force the tile 'ROWS,SYSTEMS' (matrix rows per wavefront, systems per "
                         "group) instead of the autotuner's choice")
    ap.add_argument("--summarize-pmc", metavar="DIR", default=None,
                    help="CPU only: turn DIR/<tile>_{fetch,write}/*counter_collection.csv into "
                         "the traffic table (written to --out)")
    ap.add_argument("--summarize-trace", metavar="CSV", default=None,
                    help="CPU only: turn a rocprofv3 kernel_stats.csv into a text summary "
                         "(written to --out), checked against --bench-json")
    ap.add_argument("--bench-json", default=None)
    ap.add_argument("--command", default="", help="the profiling command, recorded in the summary")
    ap.add_argument("--out", default=None)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="with --quick: afterwards copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.summarize_pmc:
        return summarize_pmc(args)
    if args.summarize_trace:
        return summarize_trace(args)
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs the path on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1606_01216_amd import airga

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.c2_only:
        stream = torch.cuda.Stream(device=dev)
        print(json.dumps(measure_c2_sequence(dev, stream)))
        return
    if args.literal_only:
        stream = torch.cuda.Stream(device=dev)
        print(json.dumps({"literal": measure_literal(dev, stream),
                          "c1_literal": measure_c1_literal(dev, stream),
                          "airga_updates": measure_airga_updates(dev, stream)}))
        return
    if args.complex_only:
        pen, f, shifts, _ = build_inputs(args.workload)
        stream = torch.cuda.Stream(device=dev)
        ctx = airga.Context(0, stream)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
        with torch.cuda.stream(stream):
            ctx.set_pencil(t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32),
                           t(pen.m_val, torch.float64), t(pen.k_val, torch.float64),
                           pen.alpha, pen.beta)
        print(json.dumps(measure_complex(ctx, stream, pen, f, t(f, torch.float64), shifts,
                                         args.tol)))
        ctx.close()
        return
    log(f"[bench] building inputs {args.workload}")
    pen, f, shifts, drifted = build_inputs(args.workload)
    n, m, S = pen.n, f.shape[0], len(shifts)
    B = S * m

    def t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt)

    rp, ci = t(pen.row_ptr, torch.int32), t(pen.col_idx, torch.int32)
    mv, kv = t(pen.m_val, torch.float64), t(pen.k_val, torch.float64)
    F = t(f, torch.float64)
    X1 = torch.zeros((S, m, n), dtype=torch.float64, device=dev)
    X2 = torch.zeros((S, m, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    ctx = airga.Context(0, stream)
    # The active count is read back every 16 iterations: the refinement sweeps
    # of these workloads end within about 16 inner iterations, so one read per
    # sweep replaces two (the library's default is 8).
    solve_kw = dict(tol=args.tol, mode=airga.MODE_MIXED, max_sweeps=12,
                    max_iter=20000, poll_every=16)
    if args.tile:
        solve_kw["tile"] = tuple(int(v) for v in args.tile.split(","))
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(record=None, profile=False):
        """One pass of the hot path; optional per-phase events on ctx.stream."""
        marks = [ev() for _ in range(6)] if record is not None else None

        def mark(i):
            if marks is not None:
                marks[i].record(stream)

        with torch.cuda.stream(stream):
            mark(0)
            ctx.set_pencil(rp, ci, mv, kv, pen.alpha, pen.beta)
            mark(1)
            precs = ctx.spai_build_many(list(shifts))
            mark(2)
            _, st1 = ctx.pcg_solve(shifts, precs, F, X1, profile=profile, **solve_kw)
            mark(3)
            upd = ctx.spai_update_many(precs, list(drifted))
            mark(4)
            _, st2 = ctx.pcg_solve(drifted, upd, F, X2, profile=profile, **solve_kw)
            mark(5)
        if record is not None:
            torch.cuda.synchronize()
            record.append([marks[i].elapsed_time(marks[i + 1]) for i in range(5)])
        return precs, upd, st1, st2

    # The objects alive now (torch's import alone leaves ~170k) are moved out
    # of the cyclic garbage collector's reach: a full pass over them stalls
    # the host for ~50 ms, and one falls at an unpredictable step every ~100
    # steps.  Later passes only scan objects created after this point.
    gc.collect()
    gc.freeze()
    log(f"[bench] n={n} m={m} shifts={S} systems/step={2 * B}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        precs, upd, st1, st2 = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] {ms_per_step:.2f} ms/step")
    iters = [e["iters"] for e in st1 + st2]
    conv = sum(e["status"] == airga.SYS_CONVERGED for e in st1 + st2)
    if args.quick:
        if args.copy_mib > 0:
            src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            log(f"[bench] copied {args.copy_mib} MiB three times")
        print(json.dumps({"metric": METRIC, "ms_per_step": ms_per_step, "converged": conv,
                          "systems": 2 * B}))
        return

    # phase breakdown (one extra step with events on the context stream)
    phases = []
    step(record=phases)
    ph = phases[0]
    # profiled step: per-launch kernel timing with HIP events on ctx.stream
    # (the handles of this last step stay valid for the comparator below: every
    # step re-sets the pencil, which invalidates earlier handles)
    precs, upd, _, st2p = step(profile=True)
    # the first update of each inner solve writes x = alpha p without reading
    # x (the iterate starts at zero): one pass per (system, sweep)
    first_passes = sum(e["sweeps"] for e in st2p)
    kt2 = ctx.kernel_times()
    kw2 = ctx.kernel_work()
    tile = ctx.tile_config()
    info = ctx.pencil_info()

    stored = info.nnz_stored
    # column information per stored entry: a 1-byte offset for banded
    # pencils (bandwidth <= 64, the LDS-window kernels), else a 4-byte index
    ib = 1 if info.bandwidth <= 64 else 4
    gp = row_blocks(n, tile[0])
    sets_mixed = ((list(shifts), precs, X1), (list(drifted), upd, X2))

    # config 3: batched float64 PCG of the same systems and preconditioners
    batched64 = None
    X3a = X3b = None
    if not args.no_plain:
        log("[bench] batched float64 PCG (same systems, all in one set of kernels)")
        X3a, X3b = torch.zeros_like(X1), torch.zeros_like(X2)
        t64, st64, kt64, kw64, tile64 = measure_batched_fp64(
            ctx, stream, ((list(shifts), precs, X3a), (list(drifted), upd, X3b)), F, args.tol,
            solve_kw["poll_every"])
        gp64 = row_blocks(n, tile64[0])
        rows64 = kernel_rows(kt64, kw64, stored=stored, n=n, ib=ib, w=8, fw=8, m=m,
                             first_passes=0, mixed=False, gp=gp64, zs_launches=1)
        batched64 = dict(seconds=t64, stats=st64, rows=rows64, tile=tile64)

    # plain float64, one system at a time, same systems and preconditioners
    plain = None
    Xp1 = Xp2 = None
    if not args.no_plain:
        log("[bench] plain float64 one-system-at-a-time comparator")
        Xp1, Xp2 = torch.zeros_like(X1), torch.zeros_like(X2)
        tp, pst = measure_plain_fp64(ctx, stream, ((list(shifts), precs, Xp1),
                                                   (list(drifted), upd, Xp2)), F, args.tol,
                                     solve_kw["poll_every"])
        plain = dict(seconds=tp, stats=pst)

    # ---- CPU baseline leg: the oracle's reference solves (double-double and
    # binary64 banded Cholesky) for every system of the step, timed on this
    # host, and the accuracy of the GPU results against both.
    errs = {}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import spai as ospai, pencil as opencil
        log("[bench] oracle reference solves (CPU)")
        cpu, refs_dd, refs_64 = measure_cpu_baseline(pen, f, (list(shifts), list(drifted)))
        rd = (refs_dd[:S], refs_dd[S:])
        r6 = (refs_64[:S], refs_64[S:])
        for key, pair in (("mixed", (X1, X2)), ("plain", (Xp1, Xp2)), ("batched64", (X3a, X3b))):
            if pair[0] is None:
                continue
            xa, xb = pair[0].cpu().numpy(), pair[1].cpu().numpy()
            errs[key] = (rel_errors(xa, rd[0], S, m) + rel_errors(xb, rd[1], S, m),
                         rel_errors(xa, r6[0], S, m) + rel_errors(xb, r6[1], S, m))
        # oracle SPAI on a column sample of the first shift, scaled to n columns
        rng = np.random.default_rng(0)
        cols = np.sort(rng.choice(n, size=min(n, 4000), replace=False))
        a0 = opencil.shifted_operator(pen, shifts[0])
        ts0 = time.perf_counter()
        ospai.spai_build(a0, cols=cols)
        cpu["spai_sample_s"] = time.perf_counter() - ts0
        cpu["spai_cols"] = len(cols)
        # the oracle's own trust metric: binary64 against double-double
        cpu["f64_vs_dd_max"] = max(
            float(np.linalg.norm(a - b) / np.linalg.norm(b))
            for A, Bm in zip(refs_64, refs_dd) for a, b in zip(A, Bm))

    errs_mixed = errs.get("mixed", ([], []))[0]
    n_ok = sum(e <= ERR_TOL for e in errs_mixed) if errs_mixed else conv
    value = n_ok / (ms_per_step / 1e3)

    # ---- roofline of the dominant row kernel (algorithmic bytes / duration)
    rows = kernel_rows(kt2, kw2, stored=stored, n=n, ib=ib, w=4, fw=4, m=m,
                       first_passes=first_passes, mixed=True, gp=gp, assign_sys=B, zs_launches=1,
                       zs_sys=B)
    dom = max((r for r in rows if r["bytes"] and r["kernel"] != "reduce"),
              key=lambda r: r["total_ms"])
    traffic = measured_traffic(args.workload, tile, dom["kernel"])
    roofline = {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom["gbs"] / HBM_PEAK_GBS, 4),
                "traffic": traffic, "avg_launch_us": dom["avg_us"],
                "bytes_per_launch": int(dom["bytes"] / dom["launches"])}
    copy_gbs = measure_copy(stream, dev)
    roofline["copy_gbs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(dom["gbs"] / copy_gbs, 4)
    # the whole profiled solve: every kernel's algorithmic bytes over the
    # same solve's wall time in the (graph-replayed) phase step
    solve_bytes = sum(r["bytes"] or 0 for r in rows)
    solve_level = {"bytes": int(solve_bytes), "ms": round(ph[4], 3),
                   "gbs": round(solve_bytes / (ph[4] * 1e-3) / 1e9, 1),
                   "frac_hbm": round(solve_bytes / (ph[4] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['desc']}", "n": n,
                   "systems_per_step": 2 * B, "tol_relres": args.tol, "err_tol": ERR_TOL,
                   "precision": "float32 matrix, SPAI and vectors in the inner PCG, float64 "
                                "refinement",
                   "tile": {"rows_per_wave": tile[0], "systems_per_group": tile[1]}},
        "solved_to_1e-8": n_ok, "max_rel_err": max(errs_mixed) if errs_mixed else None,
        "max_rel_err_vs_f64_oracle": max(errs["mixed"][1]) if "mixed" in errs else None,
        "iters_median": statistics.median(iters), "iters_max": max(iters),
        "phases_ms": {"pencil_setup": round(ph[0], 3), "spai_build_total": round(ph[1], 3),
                      "pcg_mixed_1": round(ph[2], 3), "spai_update_total": round(ph[3], 3),
                      "pcg_mixed_2": round(ph[4], 3)},
        "spai_build_ms_per_shift": round(ph[1] / S, 4),
        "spai_update_ms_per_shift": round(ph[3] / S, 4),
        "update_skipped_frac": round(float(np.mean([u.info().skipped_cols for u in upd])) / n, 4),
        "batched_mixed_pcg_solves_per_s": round(2 * B / ((ph[2] + ph[4]) / 1e3), 2),
        "kernels": rows,
        "solve_level": solve_level,
        "roofline": roofline,
    }

    def accuracy(key, stats):
        if key in errs:
            e_dd, e_64 = errs[key]
            return (sum(e <= ERR_TOL for e in e_dd), max(e_dd), max(e_64))
        return (sum(s["status"] == airga.SYS_CONVERGED for s in stats), None, None)

    if batched64 is not None:
        ok, edd, e64 = accuracy("batched64", batched64["stats"])
        r64 = batched64["rows"]
        d64 = max((r for r in r64 if r["bytes"] and r["kernel"] != "reduce"),
                  key=lambda r: r["total_ms"])
        its = [e["iters"] for e in batched64["stats"]]
        out["batched_fp64"] = {
            "pcg_solves_per_s": round(ok / batched64["seconds"], 2),
            "seconds_median_of_5": round(batched64["seconds"], 4), "solved_to_1e-8": ok,
            "max_rel_err": edd, "max_rel_err_vs_f64_oracle": e64,
            "iters_median": statistics.median(its), "iters_max": max(its),
            "tile": {"rows_per_wave": batched64["tile"][0],
                     "systems_per_group": batched64["tile"][1]},
            "kernels": r64,
            "roofline": {"bound": "hbm", "kernel": d64["kernel"], "achieved": d64["gbs"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(d64["gbs"] / HBM_PEAK_GBS, 4),
                         "avg_launch_us": d64["avg_us"],
                         "bytes_per_launch": int(d64["bytes"] / d64["launches"])}}
        out["speedup_mixed_vs_batched_fp64"] = round(
            out["batched_mixed_pcg_solves_per_s"] / max(out["batched_fp64"]["pcg_solves_per_s"],
                                                        1e-30), 2)
    if plain is not None:
        ok, edd, e64 = accuracy("plain", plain["stats"])
        pst = plain["stats"]
        out["plain_fp64"] = {"pcg_solves_per_s": round(ok / plain["seconds"], 2),
                             "seconds_median_of_5": round(plain["seconds"], 4),
                             "solved_to_1e-8": ok, "max_rel_err": edd,
                             "max_rel_err_vs_f64_oracle": e64,
                             "iters_median": statistics.median(s["iters"] for s in pst)}
        out["speedup_pcg_vs_plain_fp64"] = round(out["batched_mixed_pcg_solves_per_s"] /
                                                 max(out["plain_fp64"]["pcg_solves_per_s"], 1e-30), 2)
    log("[bench] moment-sequence block operations")
    # the collected blocks of one pass, up to the 64 columns the thin QR takes
    out["moments"] = measure_moments(ctx, stream, dev, n, m, min(S, 64 // m))
    log("[bench] minimal-residual SPAI mode")
    out["spai_mr"] = measure_spai_mr(ctx, stream, list(shifts), precs, F, X1, solve_kw)
    log("[bench] outer-iteration decisions")
    out["outer_decisions"] = measure_outer(l=min(S, 64 // m) if m else S)
    if not args.no_airga_iteration:
        log("[bench] one AIRGA outer iteration")
        # the first run also tunes and captures the solves of the new batch
        # sizes (l m and m systems): reported apart, the second run is `ms`
        first = measure_airga_iteration(ctx, stream, F, n, solve_kw=solve_kw)
        out["airga_iteration"] = measure_airga_iteration(ctx, stream, F, n, solve_kw=solve_kw)
        out["airga_iteration"]["first_ms"] = first.get("ms")
    if not args.no_c2:
        log("[bench] update-chain sequence (100,000 DOFs, float64, one system per solve)")
        out["c2_update_chain"] = measure_c2_sequence(dev, stream)
    if not args.no_complex:
        log("[bench] complex expansion points (COCG)")
        out["complex_shifts"] = measure_complex(ctx, stream, pen, f, F, shifts, args.tol)
    if not args.no_literal:
        log("[bench] literal shapes at a fixed iteration count")
        out["literal"] = measure_literal(dev, stream)
    if not args.no_airga_iteration:
        log("[bench] literal 1000-DOF beam; AIRGA loop with updates")
        out["c1_literal"] = measure_c1_literal(dev, stream)
        out["airga_updates"] = measure_airga_updates(dev, stream)
    if cpu is not None:
        out["cpu_baseline"] = {
            "value": round(cpu["dd_1"], 3), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"double-double banded Cholesky reference solves: {cpu['sample_systems']} "
                      f"systems (the first {cpu['sample_systems'] // m} shifts) on one thread, "
                      f"median of 3 ({cpu['t_dd1']:.2f} s); all {cpu['all_systems']} systems of "
                      f"a step on {cpu['cores_all']} threads, median of 3 ({cpu['t_ddw']:.2f} s); "
                      f"the same in binary64; oracle SPAI on {cpu['spai_cols']} sampled columns "
                      f"took {cpu['spai_sample_s']:.2f} s "
                      f"(~{cpu['spai_sample_s'] * n / cpu['spai_cols']:.0f} s per full build)",
            "cpu_model": cpu["cpu_model"], "cores_visible": cpu["cores_visible"],
            "cores_all": cpu["cores_all"], "value_all_cores": round(cpu["dd_all"], 3),
            "fp64_value": round(cpu["f64_1"], 3), "fp64_value_all_cores": round(cpu["f64_all"], 3),
            "f64_vs_dd_max_rel_diff": float(f"{cpu['f64_vs_dd_max']:.3e}")}
    print(json.dumps(out))
    for p in precs + upd:
        p.release()
    ctx.close()


if __name__ == "__main__":
    main()
