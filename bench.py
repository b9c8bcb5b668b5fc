#!/usr/bin/env python3
"""Benchmark: Darcy + transport solves per second on one MI355X.

One step = one full pass of the hot path over the resident 64^3 workload
(four clipped fractures, contrast 1e4): per-cell VAG matrices, cell
elimination and assembly, preconditioned CG to rtol 1e-8, cell recovery and
fluxes, porous volumes, CFL step and 200 explicit upwind steps.  The mesh's
symbolic phase (topology only) is done once before timing and reported apart.

Prints one JSON line (see the field list at the end of main()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(h, sinfo, tinfo, levels=None, precision="fp64", sweeps=2, kcycle=0):
    n, nnz = sinfo["n_unknowns"], sinfo["nnz"]
    spmv = 12 * nnz + 4 * (n + 1) + 16 * n                       # CSR FP64: val+col, row_ptr, x, y
    step = 12 * tinfo["t_nnz"] + 24 * tinfo["n_rows"]            # upwind sweep: entries, diag, c in/out
    out = dict(spmv=spmv, transport_step=step)
    if levels:
        # one preconditioner application: on each visit of a level, two matrix
        # passes on the finest (residual, smoothing sweep) and 2 * sweeps on the
        # coarser ones (sweeps - 1 pre-sweeps after the first iterate, residual,
        # sweeps post-sweeps), about 13 vector passes plus the aggregate maps,
        # the coarse vector; the coarsest level is a dense product.  A K-cycle
        # on level m (1 <= m <= kcycle, not the coarsest) visits it twice per
        # visit of level m - 1 and adds two products with A_m and about 15
        # vector passes.
        v = 4 if precision in ("mixed", "mixed_ir") else 8      # matrix value bytes
        w = 4 if precision == "mixed_ir" else 8                  # vector value bytes
        nlev = len(levels)
        visits, b = 1, 0
        for i, (rows, nz, _) in enumerate(levels[:-1]):
            dg = 8 * rows if v == 4 else 0  # FP32 levels keep their diagonal in FP64
            if 1 <= i <= kcycle:
                b += visits * (2 * ((v + 4) * nz + dg) + 15 * rows * w)
                visits *= 2
            nc = levels[i + 1][0]
            passes = 2 if i == 0 else 2 * max(1, sweeps)
            b += visits * (passes * ((v + 4) * nz + dg) + 13 * rows * w + 8 * rows + nc * w)
        rows = levels[-1][0]
        b += visits * (rows * rows * w + 2 * rows * w)
        out["vcycle"] = b
        out["level_visits"] = visits
    return out


def kcycle_levels(vag, opts, args, levels):
    """Coarse levels that run K-cycles: 1..amg_kcycle below the coarsest, with
    CG outside and no FP32 inner solve (the library's rule)."""
    if not levels or args.krylov != "cg" or args.precision == "mixed_ir" or args.amg_kind == "classical":
        return 0
    k = opts.get("amg_kcycle", vag.default_options().amg_kcycle)
    return max(0, min(k, len(levels) - 2))


def cpu_baseline(prob, budget_s=30.0):
    """The oracle, as it stands, on one full solve of the same workload;
    returns the baseline record and the oracle's result."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    res = oracle.run(prob, rtol=prob.rtol)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one full solve of {prob.name} (Jacobi-PCG to rtol {prob.rtol:g} + {prob.n_steps} steps), "
                      f"{dt:.2f} s"}, res


def results(vag, h):
    """Pressures and concentrations of a handle, on the host."""
    return vag.to_numpy(h.pressure()) | vag.to_numpy(h.concentration())


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def differences(r, ref):
    """Relative L2 pressure and max-abs concentration differences."""
    return {"u_node_rel_l2": rel_l2(r["u_node"], ref["u_node"]),
            "u_frac_rel_l2": rel_l2(r["u_frac"], ref["u_frac"]) if len(ref["u_frac"]) else 0.0,
            "c_cell_max_abs": float(np.abs(r["c_cell"] - ref["c_cell"]).max()),
            "c_node_max_abs": float(np.abs(r["c_node"] - ref["c_node"]).max())}


def copy_bandwidth(torch, mib=512, reps=20):
    """Achievable device copy rate (read + write bytes per second), GB/s."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 16.0 * n / (ms * 1e-3) / 1e9


def serving_bench(vag, synth, n_jobs, workers, budget, seed=4):
    """Config-4 serving stream: n_jobs jittered n^3 jobs (n in [16, 96], 1-20
    patches, one ratio per job, 100 steps).  Saturation runs (all jobs at t=0)
    give the throughput of each mode; Poisson arrivals at 0.7 x the FP64
    saturation rate give p50/p99 latency (scheduled arrival -> outputs on the
    host), the same arrival times for both modes."""
    import time as _t
    t0 = _t.perf_counter()
    jobs = [synth.config4_job(j) for j in range(n_jobs)]
    gen_s = _t.perf_counter() - t0
    modes = {"fp64": dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_FP64, rtol=1e-8, max_iter=20000),
             "mixed": dict(precond=vag.VAG_PC_AMG, precision=vag.VAG_MIXED, rtol=1e-8, max_iter=20000)}

    def run(mode, arrivals):
        srv = vag.Server(hbm_budget=budget, n_workers=workers)
        try:
            base = srv.clock()
            ids = []
            for p, ta in zip(jobs, arrivals):
                while srv.clock() - base < ta:
                    _t.sleep(min(1e-3, max(0.0, ta - (srv.clock() - base))))
                ids.append(srv.submit(p, n_steps=p.n_steps, **modes[mode]))
            res = []
            for i in ids:
                res.append(srv.wait(i))
                if len(res) % 16 == 0:
                    log(f"serving {mode}: {len(res)}/{len(ids)} jobs done")
            st = srv.stats()
        finally:
            srv.close()
        bad = [r["message"] for r in res if r["status"] != 0]
        if bad:
            raise RuntimeError(f"serving job failed: {bad[0]}")
        lat = np.array([r["t_end"] - (base + ta) for r, ta in zip(res, arrivals)])
        span = max(r["t_end"] for r in res) - base
        return dict(jobs_per_s=round(len(res) / span, 3), makespan_s=round(span, 3),
                    p50_ms=round(1e3 * float(np.percentile(lat, 50)), 2),
                    p99_ms=round(1e3 * float(np.percentile(lat, 99)), 2),
                    mean_create_ms=round(float(np.mean([r["ms_create"] for r in res])), 2),
                    mean_gpu_solve_ms=round(float(np.mean([r["solve"]["ms_assembly"] + r["solve"]["ms_setup"] +
                                                           r["solve"]["ms_solve"] + r["solve"]["ms_fluxes"]
                                                           for r in res])), 2),
                    mean_iterations=round(float(np.mean([r["solve"]["iterations"] for r in res])), 1),
                    peak_GB=round(st["peak_bytes_in_use"] / 1e9, 2), budget_GB=round(st["budget"] / 1e9, 2))

    log(f"serving: {n_jobs} jobs generated in {gen_s:.1f} s")
    zero = [0.0] * n_jobs
    out = {"jobs": n_jobs, "workers": workers, "job_generation_s": round(gen_s, 1)}
    out["saturation"] = {m: run(m, zero) for m in modes}
    lam = 0.7 * out["saturation"]["fp64"]["jobs_per_s"]
    rng = np.random.default_rng(seed)
    arrivals = list(np.cumsum(rng.exponential(1.0 / lam, n_jobs)))
    out["poisson_rate_jobs_per_s"] = round(lam, 3)
    out["poisson"] = {m: run(m, arrivals) for m in modes}
    return out


def pmc_traffic(kernel, workload):
    """Counter-measured HBM bytes per dispatch of `kernel` (FETCH_SIZE and
    WRITE_SIZE, calibrated by a copy of known size), from the committed
    rocprofv3 summary of this workload; None where none was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) > 5 and cells[1] == f"vag::{kernel}":
            return int(cells[-2])  # the last column: calibrated bytes per dispatch
    return None


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def describe(args, prob):
    n = args.n
    if args.workload == "config2":
        return (f"config2: cartesian {n}^3 hexahedra, 4 clipped face fractures, contrast 1e4, "
                f"{args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")
    if args.workload == "config3":
        return (f"config3: jittered {n}^3 hexahedra, lognormal anisotropic tensors, 40 face patches "
                f"(contrasts 1e2/1e4/1e6), {args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")
    return (f"config5: jittered {n}^3 hexahedra, lognormal anisotropic tensors, 200 face patches at 1e6, "
            f"{args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precond", choices=["jacobi", "amg", "bjilu0"], default=os.environ.get("VAG_BENCH_PRECOND", "amg"))
    ap.add_argument("--workload", choices=["config2", "config3", "config5"], default="config2",
                    help="config2: 64^3, 4 clipped fractures (the headline); config3: jittered anisotropic 128^3, "
                         "40 patches, FP32-AMG GMRES with FP64 refinement; config5: 192^3, 200 patches at 1e6, "
                         "FP32-AMG CG with FP64 refinement")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed_ir"], default=None)
    ap.add_argument("--krylov", choices=["cg", "gmres", "bicgstab"], default=None)
    ap.add_argument("--n", type=int, default=None, help="cells per side (default: the workload's)")
    ap.add_argument("--keep-faces", action="store_true", help="fracture faces stay unknowns (no group elimination)")
    ap.add_argument("--amg-sweeps", type=int, default=0, help="l1-Jacobi sweeps on the coarse levels (0: default)")
    ap.add_argument("--amg-coarse-size", type=int, default=0, help="stop coarsening below this many rows (0: default)")
    ap.add_argument("--amg-hops", type=int, default=0, help="aggregate radius: 2 (default) or 1")
    ap.add_argument("--wells", type=int, default=0,
                    help="perforate this many fracture faces (one rate injector, the rest at a fixed pressure)")
    ap.add_argument("--amg-kind", choices=["aggregation", "classical"], default="aggregation")
    ap.add_argument("--ilu-block-rows", type=int, default=0, help="block-Jacobi ILU(0) block size (0: default)")
    ap.add_argument("--amg-kcycle", type=int, default=-1, help="coarse levels with K-cycles (-1: library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=int(os.environ.get("VAG_BENCH_SERVING_JOBS", "256")),
                    help="config-4 serving stream of this many jobs after the timed steps (0: skip)")
    ap.add_argument("--serving-workers", type=int, default=8)
    ap.add_argument("--serving-budget-gb", type=float, default=0.0, help="0: 80%% of free device memory")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only copy a buffer of this many MiB 5 times (calibrates the HBM byte counters), then exit")
    args = ap.parse_args()
    if args.copy_probe_mb > 0:
        import torch
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n, "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is a design note, "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1602_03641_amd import vag

    defaults = {"config2": (64, "fp64", "cg"), "config3": (128, "mixed", "cg"), "config5": (192, "mixed", "cg")}
    n_def, prec_def, kry_def = defaults[args.workload]
    args.n = args.n or n_def
    args.precision = args.precision or (prec_def if args.precond == "amg" else "fp64")
    args.krylov = args.krylov or ("bicgstab" if args.precond == "bjilu0" else kry_def)
    log(f"generating {args.workload} n={args.n}")
    prob = getattr(synth, args.workload)(n=args.n)
    if args.wells > 0:
        synth.add_wells(prob, args.n, n_inj=1, n_prod=args.wells - 1)
    log(f"{len(prob.hex8)} cells, {prob.n_frac} fracture faces; creating the handle")
    opts = dict(rtol=prob.rtol, cfl=prob.cfl, max_iter=50000, inner_rtol=1e-2, gmres_restart=100,
                precond={"amg": vag.VAG_PC_AMG, "jacobi": vag.VAG_PC_JACOBI, "bjilu0": vag.VAG_PC_BJILU0}[args.precond],
                precision={"fp64": vag.VAG_FP64, "mixed": vag.VAG_MIXED, "mixed_ir": vag.VAG_MIXED_IR}[args.precision],
                krylov={"cg": vag.VAG_CG, "gmres": vag.VAG_GMRES, "bicgstab": vag.VAG_BICGSTAB}[args.krylov],
                eliminate_frac_faces=0 if args.keep_faces else 1)
    if args.amg_sweeps > 0:
        opts["amg_sweeps"] = args.amg_sweeps
    if args.amg_hops > 0:
        opts["amg_aggregate_hops"] = args.amg_hops
    if args.amg_coarse_size > 0:
        opts["amg_coarse_size"] = args.amg_coarse_size
    if args.amg_kcycle >= 0:
        opts["amg_kcycle"] = args.amg_kcycle
    if args.amg_kind == "classical":
        opts["amg_kind"] = 1
    if args.ilu_block_rows > 0:
        opts["ilu_block_rows"] = args.ilu_block_rows
    t0 = time.perf_counter()
    h = vag.Handle(prob, **opts)
    torch.cuda.synchronize()
    symbolic_s = time.perf_counter() - t0

    def step():
        s = h.solve_pressure()
        t = h.transport(n_steps=prob.n_steps)
        return s, t

    log(f"symbolic phase and uploads {symbolic_s:.2f} s; warmup")
    for _ in range(args.warmup):
        sinfo, tinfo = step()
        log(f"warmup step: {sinfo['iterations']} iterations, residual {sinfo['rel_residual']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sinfo, tinfo = step()
        if args.steps <= 5 or k % 5 == 4:
            log(f"timed step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    # roofline of the dominant kernel: per-launch time from HIP events on the handle's stream
    levels = h.amg_levels() if args.precond == "amg" else None
    ab = algorithmic_bytes(h, sinfo, tinfo, levels, args.precision, args.amg_sweeps if args.amg_sweeps > 0 else vag.default_options().amg_sweeps,
                           kcycle_levels(vag, opts, args, levels))
    ms_spmv = h.benchmark_kernel(vag.VAG_KERNEL_SPMV, 100)
    ms_step = h.benchmark_kernel(vag.VAG_KERNEL_TRANSPORT_STEP, 100)
    ms_prec = h.benchmark_kernel(vag.VAG_KERNEL_PRECOND, 50)
    n_spmv = sinfo["iterations"] + 1
    share = {"spmv": ms_spmv * n_spmv, "transport_step": ms_step * tinfo["n_steps"]}
    dom = max(share, key=share.get)
    ms_dom = ms_spmv if dom == "spmv" else ms_step
    achieved = ab[dom] / (ms_dom * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "pcg_spmv_kernel" if dom == "spmv" else "transport_step_kernel",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": pmc_traffic("pcg_spmv_kernel<double, double>" if dom == "spmv" else "transport_step_kernel",
                                       {"config2": "config2_64cubed", "config3": "config3_128cubed"}.get(args.workload, "") if args.n == n_def else ""),
                "bytes_per_launch": ab[dom], "ms_per_launch": ms_dom,
                "other": {"spmv_GBs": round(ab["spmv"] / (ms_spmv * 1e-3) / 1e9, 1),
                          "transport_step_GBs": round(ab["transport_step"] / (ms_step * 1e-3) / 1e9, 1),
                          "precond_ms": round(ms_prec, 4)}}
    if "vcycle" in ab:
        roofline["other"]["vcycle_GBs"] = round(ab["vcycle"] / (ms_prec * 1e-3) / 1e9, 1)
        roofline["other"]["vcycle_bytes"] = ab["vcycle"]

    copy_gbs = copy_bandwidth(torch)
    roofline["other"]["copy_GBs"] = round(copy_gbs, 1)
    roofline["other"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    log("kernel timings done")
    gpu_res = results(vag, h)

    # the same workload in the other precision (FP64 <-> FP32 hierarchy), timed the same way
    other, other_res = None, None
    if args.precond == "amg" and args.workload == "config2" and args.precision in ("fp64", "mixed"):
        alt = "mixed" if args.precision == "fp64" else "fp64"
        h2 = vag.Handle(prob, **(opts | {"precision": vag.VAG_MIXED if alt == "mixed" else vag.VAG_FP64}))
        for _ in range(args.warmup):
            h2.solve_pressure()
            h2.transport(n_steps=prob.n_steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            s2 = h2.solve_pressure()
            h2.transport(n_steps=prob.n_steps)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        ms_prec2 = h2.benchmark_kernel(vag.VAG_KERNEL_PRECOND, 50)
        lv2 = h2.amg_levels()
        ab2 = algorithmic_bytes(h2, s2, tinfo, lv2, alt, args.amg_sweeps if args.amg_sweeps > 0 else vag.default_options().amg_sweeps,
                                kcycle_levels(vag, opts, args, lv2))
        other = {"precision": alt, "value": round(args.steps / el2, 4), "iterations": s2["iterations"],
                 "rel_residual": s2["rel_residual"], "ms_solve": round(s2["ms_solve"], 3),
                 "vcycle_GBs": round(ab2["vcycle"] / (ms_prec2 * 1e-3) / 1e9, 1),
                 "difference_to_headline": None}
        other_res = results(vag, h2)
        other["difference_to_headline"] = differences(other_res, gpu_res)
        del h2
        log(f"{alt}: {other['value']} solves/s")
    serving = None
    if args.serving_jobs > 0 and args.workload == "config2":
        log(f"serving stream of {args.serving_jobs} jobs")
        serving = serving_bench(vag, synth, args.serving_jobs, args.serving_workers,
                                int(args.serving_budget_gb * 1e9))

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline and args.workload == "config2":
        log("oracle baseline")
        cpu, ores = cpu_baseline(prob)
        oref = {"u_node": ores["darcy"]["u_node"], "u_frac": ores["darcy"]["u_frac"],
                "c_cell": ores["c_cell"], "c_node": ores["c_node"]}
        vs_oracle = {"note": f"both sides solved to rtol {prob.rtol:g}", args.precision: differences(gpu_res, oref)}
        if other is not None:
            vs_oracle[other["precision"]] = differences(other_res, oref)

    out = {
        "metric": "Darcy+transport solves/sec", "value": round(args.steps / elapsed, 4), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": describe(args, prob),
                   "precond": args.precond, "precision": args.precision, "krylov": args.krylov,
                   "amg_kcycle_levels": kcycle_levels(vag, opts, args, levels),
                   "amg_kind": args.amg_kind if args.precond == "amg" else None,
                   "wells": args.wells,
                   "fracture_faces": "kept" if args.keep_faces else "eliminated",
                   "n_unknowns": sinfo["n_unknowns"], "nnz": sinfo["nnz"], "n_frac": prob.n_frac},
        "iterations": sinfo["iterations"], "rel_residual": sinfo["rel_residual"],
        "phase_ms": {k: round(sinfo[k], 3) for k in ("ms_assembly", "ms_setup", "ms_solve", "ms_fluxes")}
        | {"transport_setup": round(tinfo["ms_setup"], 3), "transport_steps": round(tinfo["ms_steps"], 3)},
        "symbolic_s": round(symbolic_s, 3),
        "amg_levels": levels,
        "outer_iterations": sinfo["outer_iterations"],
        "system": {"rows": sinfo["n_unknowns"], "nnz": sinfo["nnz"],
                   "stored": levels[0][2] if levels else None},
        "upwind_operator": {"rows": tinfo["n_rows"], "nnz": tinfo["t_nnz"], "stored": tinfo["t_stored"]},
        "roofline": roofline, "cpu_baseline": cpu, "other_precision": other, "vs_oracle": vs_oracle,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
