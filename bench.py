"""Throughput benchmark: DoF/s to FP64 true rel-res 1e-8 on one MI355X.

Workload: random metasurface on a 1024 x 1024 interior with a 20-cell PML
(1064 x 1064 = 1,132,096 DoF), lambda = 30 cells, 64 pillars (eps 12.25) on an
eps 2.13 substrate, current-sheet source, 8 x 8 overlapping subdomains
(overlap 8 + 16-cell local PML), seed 2.  Inputs are synthetic and resident in
HBM before timing starts.

One step = the whole hot path on one problem: node permittivity assembly,
numeric multifrontal factorisation of all 64 subdomains, and the FGMRES solve
(FP64 outer iteration, one source-transfer round per preconditioner
application) until the FP64 true relative residual is <= 1e-8.  The timed
form uses complex64 fronts ("mixed"); the plain complex128 form is timed too
and reported beside it.

Prints one JSON line: the throughput, the roofline of the dominant kernel class
(algorithmic bytes or flops per launch over its measured launch time, against the
published MI355X peak, with the HBM bytes per launch from the committed PMC
summary) and the oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF/s to rel-res 1e-8: mixed+batched+learned vs plain FP64 DDM, 1 GPU"
PEAK = {"hbm": 8000.0, "fp32_mfma": 157.3, "fp64": 78.6}   # GB/s, TFLOP/s


def workload():
    import workloads
    return workloads.configs.metasurface_sheet()


def workloads_batched():
    import workloads
    return workloads.configs.metasurface_sheet(nrhs=4)


def params_of(w, prec, leaf=0):
    p = w.params()
    return dict(nx=p["nx"], ny=p["ny"], k0=p["k0"], pml=p["pml"], pml_order=p["pml_order"],
                pml_R=p["pml_R"], px=p["px"], py=p["py"], overlap=p["overlap"],
                local_pml=p["local_pml"], local_pml_order=p["local_pml_order"],
                local_pml_R=p["local_pml_R"], front_prec=prec, leaf_size=leaf)


def run_form(stf, torch, ctx, w, prec, steps, warmup, tol, restart, max_iter, timing, leaf=0,
             rounds=1, nrhs=1):
    eps = torch.from_numpy(w.eps_cells).cuda()
    b = torch.from_numpy(w.b[0] if nrhs == 1 else w.b[:nrhs]).cuda()
    x = torch.empty_like(b)
    pb = stf.Problem(ctx, params_of(w, prec, leaf), eps)
    infos = []

    def step():
        pb.assemble(eps)
        pb.factor()
        _, inf = pb.solve(b, x=x, tol=tol, restart=restart, max_iter=max_iter, rounds=rounds)
        infos.append(inf[0] if nrhs == 1 else inf)

    for _ in range(warmup):
        step()
    profile, dom = {}, None
    if timing:
        # One extra step with every kernel class timed gives the per-class
        # breakdown and the dominant class.
        ctx.set_timing(True)
        step()
        for k, name in enumerate(stf.KERNEL_CLASSES):
            profile[name] = ctx.kernel_stats(k)
        ctx.set_timing(False)
        dom = max(profile, key=lambda k: profile[k][0])
    # The timed steps run with no event timing at all.
    infos.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {}
    if timing:
        # The same number of steps again with the dominant class's launches
        # bracketed by HIP events on the library's stream: its per-launch time.
        timed_infos = list(infos)
        ctx.set_timing(True, classes=[dom])
        for _ in range(steps):
            step()
        stats[dom] = ctx.kernel_stats(dom)
        ctx.set_timing(False)
        infos[:] = timed_infos
    info = pb.info()
    if nrhs == 1:
        # Power of the last solution through two horizontal lines ten cells
        # inside the global PML: towards +y near the top, towards -y near the
        # bottom (the source sheet lies between them).
        pml_lo, pml_hi = w.params()["pml"][2], w.params()["pml"][3]
        lo, hi = w.params()["pml"][0], w.nx - w.params()["pml"][1]
        up = pb.line_flux(x, 1, w.ny - pml_hi - 11, lo, hi)
        down = -pb.line_flux(x, 1, pml_lo + 10, lo, hi)
        info["power"] = {"up": up, "down": down}
    pb.close()
    return (t1 - t0) / steps, infos, stats, info, profile


def stationary_form(stf, torch, ctx, w, prec, tol, max_rounds):
    """Algorithm 1 as the paper runs it, a stationary iteration of
    source-transfer rounds, on the same problem (factored once, not part of the
    timed step): rounds to the FP64 true rel-res tol and their wall time."""
    eps = torch.from_numpy(w.eps_cells).cuda()
    b = torch.from_numpy(w.b[0]).cuda()
    pb = stf.Problem(ctx, params_of(w, prec), eps)
    pb.factor()
    x = torch.empty_like(b)
    pb.stationary_solve(b, x=x, tol=tol, max_rounds=max_rounds)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, inf = pb.stationary_solve(b, x=x, tol=tol, max_rounds=max_rounds)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    pb.close()
    return {"rounds": inf["rounds"], "relres_true": inf["relres_true"],
            "converged": inf["status"] == 0, "solve_ms": round(t * 1e3, 3),
            "form": "complex64 fronts" if prec == stf.STF_C64 else "complex128 fronts"}


# Kernel classes of the library's kernels (by kernel name) and the source file
# that holds them (a PMC summary is valid only for the source it was taken on).
CLASS_OF = [("k_fwd_", "sweep_fwd"), ("k_bwd_", "sweep_bwd"), ("k_factor_", "front_lu"),
            ("k_stencil", "stencil"), ("k_scatter", "scatter"), ("k_mdot", "arnoldi"),
            ("k_mupdate", "arnoldi"), ("k_norm_reduce", "arnoldi"), ("k_hacc", "arnoldi"),
            ("k_gs", "arnoldi")]
SOURCE_OF = {"sweep_fwd": "kernels_front.hip", "sweep_bwd": "kernels_front.hip",
             "front_lu": "kernels_front.hip", "scatter": "kernels_front.hip",
             "stencil": "kernels_stencil.hip", "arnoldi": "kernels_krylov.hip"}
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_traffic_metasurface_1064.md")
COPY_BYTES = 1 << 29          # the calibration copy: 512 MiB read and 512 MiB written


def source_sha(cls):
    import hashlib
    path = os.path.join(ROOT, "paper_2509_20801_amd", "csrc", SOURCE_OF[cls])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(cls):
    """HBM bytes per launch of class `cls` from the committed PMC summary, or
    None when there is none or its kernels have changed since."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    for line in open(PMC_SUMMARY):
        if line.startswith("traffic_json: "):
            d = json.loads(line[len("traffic_json: "):])
            c = d.get("classes", {}).get(cls)
            if c and c.get("source_sha") == source_sha(cls):
                return c["bytes_per_launch"]
    return None


def copy_probe():
    """Calibration kernel for the PMC byte counters: a plain device copy of
    COPY_BYTES (run under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)."""
    import torch
    a = torch.ones(COPY_BYTES // 8, dtype=torch.complex64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d bytes per call" % COPY_BYTES)


def pmc_summary(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir):
    """Markdown summary of two PMC passes (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) over a bench run, each scaled so that the calibration copy reads
    COPY_BYTES; per kernel class: launches and HBM bytes per launch."""
    import csv
    import collections
    import glob

    def rows(d):
        return list(csv.DictReader(open(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])))

    def copy_kib(d):
        v = [float(r["Counter_Value"]) for r in rows(d) if "opy" in r["Kernel_Name"]]
        return max(v)                            # the 512 MiB copy dispatches

    scale = {"fetch": COPY_BYTES / (copy_kib(copy_fetch_dir) * 1024.0),
             "write": COPY_BYTES / (copy_kib(copy_write_dir) * 1024.0)}
    agg = collections.defaultdict(lambda: {"n": 0, "fetch": 0.0, "write": 0.0})
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        for r in rows(d):
            name = r["Kernel_Name"]
            cls = next((c for pfx, c in CLASS_OF if pfx in name), None)
            if cls is None:
                continue
            if key == "fetch":
                agg[cls]["n"] += 1
            agg[cls][key] += float(r["Counter_Value"]) * 1024.0 * scale[key]
    out = {"calibration": {k: round(v, 4) for k, v in scale.items()}, "classes": {}}
    lines = ["| class | launches | fetch MB/launch | write MB/launch | HBM bytes/launch |",
             "|---|---|---|---|---|"]
    for cls, a in sorted(agg.items(), key=lambda kv: -(kv[1]["fetch"] + kv[1]["write"])):
        n = max(a["n"], 1)
        per = (a["fetch"] + a["write"]) / n
        out["classes"][cls] = {"launches": a["n"], "bytes_per_launch": round(per, 1),
                               "fetch_per_launch": round(a["fetch"] / n, 1),
                               "write_per_launch": round(a["write"] / n, 1),
                               "source_sha": source_sha(cls)}
        lines.append("| %s | %d | %.3f | %.3f | %.4g |" % (cls, a["n"], a["fetch"] / n / 1e6,
                                                          a["write"] / n / 1e6, per))
    print("\n".join(lines))
    print()
    print("traffic_json: " + json.dumps(out))


def roofline(stf, w, prec, infos, stats, steps):
    """Roofline of the kernel class with the largest summed time: its algorithmic
    work per launch (fine nested-dissection reference counts) over its measured
    per-launch time, against the published peak of the bound it is priced on."""
    ref = stf.plan_query(params_of(w, prec, leaf=4))     # fine nested dissection reference
    es = 8 if prec == stf.STF_C64 else 16
    N = w.nx * w.ny
    iters = sum(i["iters"] for i in infos)
    cycles = sum(i["restarts"] for i in infos)
    units = {
        # algorithmic work per step summed over the timed steps
        "front_lu": ("mfma", ref["lu_flops"] * steps / 1e12),                # TFLOP
        "sweep_fwd": ("hbm", ref["factor_entries"] / 2 * es * iters / 1e9),  # GB
        "sweep_bwd": ("hbm", ref["factor_entries"] / 2 * es * iters / 1e9),
        "stencil": ("hbm", N * (48 * iters + 64 * (cycles + steps)) / 1e9),
    }
    dom = next(iter(stats))
    ms, launches = stats[dom]
    if dom not in units:
        return dom, None
    bound, work = units[dom]
    per_launch = work / launches
    avg_s = ms / launches / 1e3
    achieved = per_launch / avg_s
    if bound == "mfma":
        peak = PEAK["fp32_mfma"] if prec == stf.STF_C64 else PEAK["fp64"]
        unit = "TFLOP/s"
    else:
        peak, unit = PEAK["hbm"], "GB/s"
    traffic = measured_traffic(dom)
    return dom, {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                 "frac": round(achieved / peak, 4),
                 "traffic": None if traffic is None else round(traffic, 1),
                 "traffic_unit": "HBM bytes per launch (PMC)",
                 "algorithmic_per_launch": round(per_launch * (1e9 if bound == "hbm" else 1e12), 1),
                 "kernel": dom, "avg_launch_ms": round(ms / launches, 4), "launches": launches}


def cpu_baseline(w, gpu_iters, restart):
    """Oracle (NumPy/SciPy, one thread) on a bounded sample of the same workload:
    SuperLU factorisations of 16 of the 64 subdomains (all four shapes) and
    3 full-size FGMRES iterations, extrapolated to 64 subdomains and to the GPU
    run's iteration count."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    from oracle import ddm, fdfd, krylov
    with threadpool_limits(limits=1):
        p = w.params()
        t0 = time.perf_counter()
        A = fdfd.global_matrix(p, w.eps_cells)
        subs = ddm.partition(p)
        gax = fdfd.global_axes(p)
        t_asm = time.perf_counter() - t0
        pick = [s for s in subs if (s.kx in (0, 3, 4, 7) and s.ky in (0, 3, 4, 7))]
        t0 = time.perf_counter()
        for s in pick:
            spla.splu(ddm.local_matrix(p, w.eps_cells, s, gax).tocsc())
        t_fac = (time.perf_counter() - t0) * len(subs) / len(pick)
        B = ddm.SourceTransfer(p, w.eps_cells)          # full factors for the iteration sample
        b = w.b[0].ravel()
        k = 3
        t0 = time.perf_counter()
        krylov.fgmres(lambda v: A @ v, b, B.apply, tol=0.0, restart=max(restart, k), max_iter=k)
        t_it = (time.perf_counter() - t0) / k
    total = t_asm + t_fac + gpu_iters * t_it
    return {"value": round(w.nx * w.ny / total, 1), "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": "SuperLU factors of 16/64 subdomains + 3 full-size FGMRES iterations, "
                      "extrapolated to 64 subdomains and %d iterations (%.1f s est.)" % (gpu_iters, total)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=10)
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel HIP event timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the complex128 reference form")
    ap.add_argument("--no-batched", action="store_true", help="skip the four-RHS batched form")
    ap.add_argument("--no-stationary", action="store_true",
                    help="skip the stationary source-transfer iteration (the paper's own scheme)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only the PMC calibration copy (512 MiB)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="summarise rocprofv3 --pmc output directories and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs on a single MI355X "
              "(sharding over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2509_20801_amd as stf

    w = workload()
    ctx = stf.Context(0)
    t_mixed, inf_mixed, stats, info, profile = run_form(stf, torch, ctx, w, stf.STF_C64,
                                                       args.steps, args.warmup, args.tol,
                                                       args.restart, args.max_iter,
                                                       not args.no_timing)
    ok = all(i["status"] == 0 and i["relres_true"] <= args.tol for i in inf_mixed)
    N = w.nx * w.ny
    out = {"metric": METRIC, "value": round(N / t_mixed, 1), "unit": "DoF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_mixed * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64 fronts + f64 Krylov", "data": "synthetic",
           "config": {"workload": "metasurface 1064x1064 (1024^2 + 20-cell PML), 64 pillars, "
                                  "current sheet, 8x8 subdomains, overlap 8 + local PML 16",
                      "ndof": N, "form": "mixed (complex64 fronts, FP64 FGMRES)",
                      "restart": args.restart, "tol": args.tol, "parallelism": "1 GPU"},
           "iters": inf_mixed[0]["iters"], "relres_true": inf_mixed[0]["relres_true"],
           "converged": ok, "power": {k: round(v, 6) for k, v in info["power"].items()}}
    if stats:
        dom, rl = roofline(stf, w, stf.STF_C64, inf_mixed, stats, args.steps)
        out["roofline"] = rl
        out["kernel_ms_per_step"] = {k: round(v[0], 3) for k, v in profile.items()}
    if not args.no_plain:
        t_plain, inf_plain, _, _, _ = run_form(stf, torch, ctx, w, stf.STF_C128, 1, 1, args.tol,
                                               args.restart, args.max_iter, False)
        out["plain_fp64"] = {"value": round(N / t_plain, 1), "ms_per_step": round(t_plain * 1e3, 3),
                             "iters": inf_plain[0]["iters"]}
        out["speedup_vs_plain"] = round(t_plain / t_mixed, 3)
    if not args.no_batched:
        # Batched form: four current sheets (rows 64, 128, 192, 224 of the
        # substrate) solved together; every preconditioner application sweeps
        # the four right-hand sides with one read of the factors.
        wb = workloads_batched()
        t_b, inf_b, _, _, _ = run_form(stf, torch, ctx, wb, stf.STF_C64, 1, 1, args.tol,
                                       args.restart, args.max_iter, False, nrhs=4)
        out["batched_4rhs"] = {"value": round(4 * N / t_b, 1), "unit": "DoF*RHS/s",
                               "ms_per_step": round(t_b * 1e3, 3),
                               "iters": [i["iters"] for i in inf_b[0]],
                               "converged": all(i["status"] == 0 and i["relres_true"] <= args.tol
                                                for i in inf_b[0])}
    if not args.no_stationary:
        out["stationary"] = stationary_form(stf, torch, ctx, w, stf.STF_C64, args.tol, 200)
    out["device_bytes"] = info["device_bytes"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, inf_mixed[0]["iters"], args.restart)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
