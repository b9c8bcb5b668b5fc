#!/usr/bin/env python3
"""Benchmark: Darcy + transport solves per second on one MI355X.

One step = one full pass of the hot path over the resident workload:
per-cell VAG matrices, cell elimination and assembly, AMG setup,
preconditioned CG to rtol 1e-8, cell recovery and fluxes, porous volumes,
CFL step and the workload's explicit upwind steps.  The mesh's symbolic phase
(topology only) is done once before timing and reported apart.

The headline workload is the largest single-GPU instance: 192^3 jittered
hexahedra (7.1 M cells), lognormal anisotropic permeability, 200 face patches
at contrast 1e6, FP32 AMG hierarchy inside FP64 CG to rtol 1e-8, then 1000
upwind steps.  The 64^3 four-fracture workload (both precisions, difference
to the oracle) and the serving stream follow as extra keys.

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
    CG or GMRES outside and no FP32 inner solve (the library's rule)."""
    if not levels or args.krylov not in ("cg", "gmres") or args.precision == "mixed_ir" or args.amg_kind == "classical":
        return 0
    k = opts.get("amg_kcycle", vag.default_options().amg_kcycle)
    return max(0, min(k, len(levels) - 2))


def cpu_baseline(prob, budget_s=30.0):
    """The oracle, as it stands, on one full solve of the same workload (a
    size it finishes in seconds); returns the baseline record and the
    oracle's result."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    res = oracle.run(prob, rtol=prob.rtol)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one full solve of {prob.name} (Jacobi-PCG to rtol {prob.rtol:g} + {prob.n_steps} steps), "
                      f"{dt:.2f} s"}, res


def cpu_baseline_sampled(prob, vag, h, dt, n_steps_sample=20, cell_stride=64):
    """The oracle, as it stands, on a bounded sample of a workload too large
    for it to solve in minutes (its global assembly sorts one triplet per
    local-matrix entry, and Jacobi-PCG needs thousands of iterations there):

    * n_steps_sample of the workload's upwind steps on the full mesh, fed the
      GPU's fluxes and porous volumes (orc_transport, one thread), scaled to
      the workload's step count;
    * the local VAG matrices and porous volumes of every cell_stride-th cell
      (orc_porous_volumes on those cells, one thread), scaled to all cells.

    The value is one solve's worth of these phases; the global assembly and
    the Jacobi-PCG solve are left out, so it bounds the oracle's rate from
    above."""
    import oracle
    import synth
    flux = {k: v.cpu().numpy() for k, v in h.fluxes().items()}
    phi = {k: v.cpu().numpy() for k, v in h.porous_volumes().items()}
    if prob.wells:
        flux["well_rate"] = h.well_rates()
    op = oracle.OracleProblem(prob)
    log(f"oracle baseline: {n_steps_sample} upwind steps on the full mesh")
    t0 = time.perf_counter()
    oracle.transport(op, flux, phi, dt, n_steps_sample)
    t_steps = time.perf_counter() - t0
    log(f"oracle baseline: {t_steps:.2f} s; local matrices of every {cell_stride}th cell")
    cells = np.arange(0, prob.n_cells, cell_stride)
    used, inv = np.unique(prob.hex8[cells], return_inverse=True)
    sub = synth.Problem(
        name=f"{prob.name}-cells/{cell_stride}", dims=prob.dims, xyz=prob.xyz[used],
        hex8=inv.reshape(-1, 8).astype(np.int32), frac_nodes=np.zeros((0, 4), np.int32),
        frac_width=np.zeros(0), frac_perm=np.zeros(0), frac_poro=np.zeros(0), perm=prob.perm[cells],
        poro=prob.poro[cells], mu=prob.mu, dirichlet=prob.dirichlet[used], p_bar=prob.p_bar[used],
        c_bar=prob.c_bar[used])
    t0 = time.perf_counter()
    oracle.porous_volumes(sub)
    t_cells = time.perf_counter() - t0
    per_solve = t_steps * prob.n_steps / n_steps_sample + t_cells * prob.n_cells / len(cells)
    log(f"oracle baseline: {t_cells:.2f} s; {per_solve:.1f} s per solve")
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{prob.name}: {n_steps_sample} of its {prob.n_steps} upwind steps on the full mesh with the "
                       f"GPU's fluxes ({t_steps:.2f} s) and the local matrices + porous volumes of "
                       f"{len(cells)} of its {prob.n_cells} cells ({t_cells:.2f} s), scaled to one solve "
                       f"({per_solve:.1f} s); the oracle's global assembly and Jacobi-PCG solve are left out, "
                       "so the value is an upper bound of its rate; one thread (these oracle loops are serial)")}


def cpu_baseline_general(prob, synth, kind, cell_stride=2000, small=(8, 8, 8), steps=3):
    """The general-cell oracle (numpy, loops per cell and per flux) on a
    bounded sample of a general-cell workload: the local matrices of every
    cell_stride-th cell of the real mesh, scaled to all cells, and transport
    steps of the same generator on a small grid, scaled per flux to the
    workload's fluxes and step count.  The global assembly and solve are left
    out, so the value bounds the oracle's rate from above."""
    from oracle import general_cells as gc
    cells = np.asarray(prob.cells)[::cell_stride]
    used, inv = np.unique(cells, return_inverse=True)
    sub = gc.Mesh(prob.xyz[used], inv.reshape(cells.shape), prob.perm[::cell_stride], prob.poro[::cell_stride])
    t0 = time.perf_counter()
    for K in range(len(cells)):
        gc.cell_matrix(sub, K)
    t_cells = time.perf_counter() - t0
    q = synth.general_workload(kind, small, 2, n_patches=2)
    m = gc.Mesh(q.xyz, q.cells, q.perm, q.poro, q.frac_faces(), q.frac_width, q.frac_perm, q.frac_poro, q.dirichlet,
                q.p_bar, q.c_bar, q.mu)
    sol = gc.solve_darcy(m)
    phi = gc.porous_volumes(m, sol)
    dt = gc.cfl_dt(m, sol, phi, 0.9)
    t0 = time.perf_counter()
    gc.transport(m, sol, phi, dt, steps)
    t_steps = time.perf_counter() - t0
    n_edges_small = sum(len(c) for c in q.cells) + 2 * q.n_frac + len(np.concatenate(q.frac_faces() or [[]]))
    n_edges = int(np.asarray(prob.cells).size) + 2 * prob.n_frac + int(sum(len(f) for f in prob.frac_faces()))
    per_solve = t_cells * prob.n_cells / len(cells) + t_steps / steps / n_edges_small * n_edges * prob.n_steps
    log(f"general-cell oracle baseline: {per_solve:.1f} s per solve")
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"{prob.name}: the general-cell oracle's local matrices of {len(cells)} of its {prob.n_cells} "
                       f"cells ({t_cells:.2f} s) and {steps} transport steps of the same generator on a "
                       f"{small[0]}x{small[1]}x{small[2]} grid ({t_steps:.2f} s, {n_edges_small} fluxes), scaled to "
                       f"all cells and to {n_edges} fluxes x {prob.n_steps} steps ({per_solve:.1f} s); its global "
                       "assembly and solve are left out, so the value is an upper bound of its rate; one thread "
                       "(numpy loops)")}


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
    give the throughput of each mode (after an untimed pass of each);
    Poisson arrivals at 0.7 x the FP64 saturation rate give p50/p99 latency
    (scheduled arrival -> outputs on the host), the same arrival times for
    both modes.  The transport steps of the jobs below 2^18 control volumes
    run batched; batched_job_steps / batched_step_launches is how many jobs
    a launch took on average."""
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
                    peak_GB=round(st["peak_bytes_in_use"] / 1e9, 2), budget_GB=round(st["budget"] / 1e9, 2),
                    batched_job_steps=st["job_steps"], batched_step_launches=st["step_launches"])

    log(f"serving: {n_jobs} jobs generated in {gen_s:.1f} s")
    zero = [0.0] * n_jobs
    out = {"jobs": n_jobs, "workers": workers, "job_generation_s": round(gen_s, 1)}
    # an untimed pass of each mode first: the first pass of a process pays for
    # growing the device block cache and for first-use host paths, which
    # would otherwise favour whichever mode runs second
    for m in modes:
        run(m, zero)
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


PROFILE_NAME = {"config2": "config2_64cubed", "config3": "config3_128cubed", "config5": "config5_192cubed",
                "tet": "tet_96x96x112", "prism": "prism_128cubed"}
DEFAULTS = {"config2": (64, "fp64", "cg"), "config3": (128, "mixed", "gmres"), "config5": (192, "mixed", "cg"),
            "tet": (96, "mixed", "cg"), "prism": (128, "mixed", "cg")}
# general-cell workloads: the grid each is split from (tetrahedra: the size of the paper's tetrahedral
# mesh, 6.2 M cells and 1.06 M nodes; prisms: 4.2 M cells)
GENERAL_DIMS = {"tet": lambda n: (n, n, n * 7 // 6), "prism": lambda n: (n, n, n)}


def make_problem(synth, workload, n):
    if workload in GENERAL_DIMS:
        return synth.general_workload(workload, GENERAL_DIMS[workload](n), 1, n_patches=40, n_steps=200,
                                      name=f"{workload}{GENERAL_DIMS[workload](n)}")
    return getattr(synth, workload)(n=n)


def profiled_mean_us(kernel, workload):
    """Mean duration of `kernel` in the committed rocprofv3 kernel statistics
    of this workload (None where none was taken)."""
    path = os.path.join(ROOT, "profiles", f"{workload}_kernel_stats.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        cells = [c.strip().strip("`") for c in line.split("|")]
        if len(cells) > 5 and cells[1] == f"vag::{kernel}":
            return float(cells[4])
    return None


def describe(args, prob):
    n = args.n
    if args.workload == "config2":
        return (f"config2: cartesian {n}^3 hexahedra, 4 clipped face fractures, contrast 1e4, "
                f"{args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")
    if args.workload == "config3":
        return (f"config3: jittered {n}^3 hexahedra, lognormal anisotropic tensors, 40 face patches "
                f"(contrasts 1e2/1e4/1e6), {args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")
    if args.workload in GENERAL_DIMS:
        d = GENERAL_DIMS[args.workload](n)
        what = {"tet": "tetrahedra (6 per grid hexahedron)", "prism": "prisms (2 per grid hexahedron)"}[args.workload]
        return (f"{args.workload}: jittered {d[0]}x{d[1]}x{d[2]} grid split into {what}, {prob.n_cells} cells and "
                f"{prob.n_nodes} nodes given by their faces, lognormal anisotropic tensors, 40 face patches "
                f"(contrasts 1e2/1e4/1e6, {prob.n_frac} fracture faces), {args.krylov.upper()} rtol {prob.rtol:g}, "
                f"{prob.n_steps} upwind steps")
    return (f"config5: jittered {n}^3 hexahedra, lognormal anisotropic tensors, 200 face patches at 1e6, "
            f"{args.krylov.upper()} rtol {prob.rtol:g}, {prob.n_steps} upwind steps")


def dtype_of(precision):
    """The arithmetic the path computes in."""
    return {"fp64": "f64",
            "mixed": "f64 (f32 AMG hierarchy values)",
            "mixed_ir": "f64 refinement around f32 inner Krylov and f32 AMG hierarchy"}[precision]


def solver_options(vag, args, prob):
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
    return opts


def timed_steps(torch, h, prob, steps, warmup, label):
    """warmup untimed steps, then `steps` timed ones, synchronised on both sides."""
    def step():
        return h.solve_pressure(), h.transport(n_steps=prob.n_steps)

    for _ in range(warmup):
        sinfo, tinfo = step()
        log(f"{label} warmup step: {sinfo['iterations']} iterations, residual {sinfo['rel_residual']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        sinfo, tinfo = step()
        if steps <= 5 or k % 5 == 4:
            log(f"{label} timed step {k + 1}/{steps}")
    torch.cuda.synchronize()
    return sinfo, tinfo, time.perf_counter() - t0


def kernel_rates(vag, h, args, opts, sinfo, tinfo, workload, n_is_default):
    """Roofline of the dominant kernel (per-launch HIP-event time on the
    handle's stream) and the SpMV / preconditioner rates."""
    levels = h.amg_levels() if args.precond == "amg" else None
    ab = algorithmic_bytes(h, sinfo, tinfo, levels, args.precision,
                           args.amg_sweeps if args.amg_sweeps > 0 else vag.default_options().amg_sweeps,
                           kcycle_levels(vag, opts, args, levels))
    ms_spmv = h.benchmark_kernel(vag.VAG_KERNEL_SPMV, 100)
    ms_step = h.benchmark_kernel(vag.VAG_KERNEL_TRANSPORT_STEP, 100)
    ms_prec = h.benchmark_kernel(vag.VAG_KERNEL_PRECOND, 50)
    n_spmv = sinfo["iterations"] + 1
    share = {"spmv": ms_spmv * n_spmv, "transport_step": ms_step * tinfo["n_steps"]}
    dom = max(share, key=share.get)
    ms_dom = ms_spmv if dom == "spmv" else ms_step
    kname = "pcg_spmv_kernel<double, double>" if dom == "spmv" else "transport_step_kernel"
    achieved = ab[dom] / (ms_dom * 1e-3) / 1e9
    prof = PROFILE_NAME.get(workload, "") if n_is_default else ""
    roofline = {"bound": "hbm", "kernel": kname.split("<")[0],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": pmc_traffic(kname, prof) if prof else None,
                "bytes_per_launch": ab[dom], "ms_per_launch": ms_dom,
                "other": {"spmv_GBs": round(ab["spmv"] / (ms_spmv * 1e-3) / 1e9, 1),
                          "transport_step_GBs": round(ab["transport_step"] / (ms_step * 1e-3) / 1e9, 1),
                          "precond_ms": round(ms_prec, 4)}}
    us_prof = profiled_mean_us(kname, prof) if prof else None
    if us_prof:
        roofline["profiled_us_per_launch"] = us_prof
        roofline["frac_profiled"] = round(ab[dom] / (us_prof * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    if "vcycle" in ab:
        roofline["other"]["vcycle_GBs"] = round(ab["vcycle"] / (ms_prec * 1e-3) / 1e9, 1)
        roofline["other"]["vcycle_frac"] = round(ab["vcycle"] / (ms_prec * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        roofline["other"]["vcycle_bytes"] = ab["vcycle"]
    return roofline, levels


def config2_leg(vag, torch, synth, args):
    """The 64^3 four-fracture workload in both precisions, with the oracle's
    full solve beside it (its system and upwind operator fit in the 256 MB
    last-level cache, so its rates are effective bandwidths, not HBM)."""
    import copy
    a2 = copy.copy(args)
    a2.workload, a2.n = "config2", 64
    a2.precision = "fp64" if args.precond == "amg" else args.precision
    prob = synth.config2(n=64)
    out = {"workload": describe(a2, prob), "rates": "cache-resident: effective bandwidth, not HBM"}
    res = {}
    for prec in (["fp64", "mixed"] if args.precond == "amg" else [a2.precision]):
        a2.precision = prec
        opts = solver_options(vag, a2, prob)
        h = vag.Handle(prob, **opts)
        sinfo, tinfo, el = timed_steps(torch, h, prob, args.steps, min(args.warmup, 3), f"config2 {prec}")
        rl, _ = kernel_rates(vag, h, a2, opts, sinfo, tinfo, "config2", True)
        out[prec] = {"value": round(args.steps / el, 4), "ms_per_step": round(1e3 * el / args.steps, 3),
                     "dtype": dtype_of(prec), "iterations": sinfo["iterations"],
                     "rel_residual": sinfo["rel_residual"],
                     "transport_step_GBs": rl["other"]["transport_step_GBs"],
                     "spmv_GBs": rl["other"]["spmv_GBs"], "vcycle_GBs": rl["other"].get("vcycle_GBs")}
        res[prec] = results(vag, h)
        h.close()
        log(f"config2 {prec}: {out[prec]['value']} solves/s")
    if len(res) == 2:
        out["mixed"]["difference_to_fp64"] = differences(res["mixed"], res["fp64"])
    if not args.no_cpu_baseline:
        log("config2 oracle baseline")
        cpu, ores = cpu_baseline(prob)
        oref = {"u_node": ores["darcy"]["u_node"], "u_frac": ores["darcy"]["u_frac"],
                "c_cell": ores["c_cell"], "c_node": ores["c_node"]}
        out["cpu_baseline"] = cpu
        out["vs_oracle"] = {"note": f"both sides solved to rtol {prob.rtol:g}"} | {
            k: differences(r, oref) for k, r in res.items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precond", choices=["jacobi", "amg", "bjilu0"], default=os.environ.get("VAG_BENCH_PRECOND", "amg"))
    ap.add_argument("--workload", choices=["config2", "config3", "config5", "tet", "prism"], default="config5",
                    help="config5 (the headline): 192^3 jittered anisotropic, 200 patches at 1e6, FP32-AMG CG, "
                         "1000 steps; config3: jittered anisotropic 128^3, 40 patches; config2: 64^3, 4 clipped "
                         "fractures")
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
    ap.add_argument("--log-jsonl", default=None,
                    help="append one JSON record per solve, transport call and served job, and the result line, "
                         "to this file")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the config-2 leg and the serving stream")
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
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library drives one device and does "
              "not shard a solve over several", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_1602_03641_amd import vag

    if args.log_jsonl:
        vag.set_log(args.log_jsonl)
    n_def, prec_def, kry_def = DEFAULTS[args.workload]
    args.n = args.n or n_def
    args.precision = args.precision or (prec_def if args.precond == "amg" else "fp64")
    args.krylov = args.krylov or ("bicgstab" if args.precond == "bjilu0" else kry_def)
    log(f"generating {args.workload} n={args.n}")
    prob = make_problem(synth, args.workload, args.n)
    if args.wells > 0:
        synth.add_wells(prob, args.n, n_inj=1, n_prod=args.wells - 1)
    log(f"{prob.n_cells} cells, {prob.n_frac} fracture faces; creating the handle")
    opts = solver_options(vag, args, prob)
    t0 = time.perf_counter()
    h = vag.Handle(prob, **opts)
    torch.cuda.synchronize()
    symbolic_s = time.perf_counter() - t0
    log(f"symbolic phase and uploads {symbolic_s:.2f} s; warmup")
    sinfo, tinfo, elapsed = timed_steps(torch, h, prob, args.steps, args.warmup, args.workload)
    ms_per_step = 1e3 * elapsed / args.steps
    roofline, levels = kernel_rates(vag, h, args, opts, sinfo, tinfo, args.workload, args.n == n_def)
    copy_gbs = copy_bandwidth(torch)
    roofline["other"]["copy_GBs"] = round(copy_gbs, 1)
    roofline["other"]["frac_of_copy"] = round(roofline["achieved"] / copy_gbs, 4)
    log("kernel timings done")

    cpu = None
    vs_oracle = None
    if not args.no_cpu_baseline:
        if args.workload == "config2":
            log("oracle baseline")
            cpu, ores = cpu_baseline(prob)
            gpu_res = results(vag, h)
            oref = {"u_node": ores["darcy"]["u_node"], "u_frac": ores["darcy"]["u_frac"],
                    "c_cell": ores["c_cell"], "c_node": ores["c_node"]}
            vs_oracle = {"note": f"both sides solved to rtol {prob.rtol:g}", args.precision: differences(gpu_res, oref)}
        elif args.workload in GENERAL_DIMS:
            cpu = cpu_baseline_general(prob, synth, args.workload)
        else:
            cpu = cpu_baseline_sampled(prob, vag, h, tinfo["dt"])
    h.close()
    del h
    vag.trim_memory()

    extra = None
    serving = None
    if not args.no_extras and args.workload != "config2":
        extra = config2_leg(vag, torch, synth, args)
    if not args.no_extras and args.serving_jobs > 0:
        log(f"serving stream of {args.serving_jobs} jobs")
        serving = serving_bench(vag, synth, args.serving_jobs, args.serving_workers,
                                int(args.serving_budget_gb * 1e9))

    out = {
        "metric": "Darcy+transport solves/sec", "value": round(args.steps / elapsed, 4), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype_of(args.precision),
        "data": "synthetic",
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
        "roofline": roofline, "cpu_baseline": cpu, "vs_oracle": vs_oracle,
        "config2": extra, "serving": serving,
    }
    print(json.dumps(out), flush=True)
    if args.log_jsonl:
        vag._log("bench", out)


if __name__ == "__main__":
    main()
