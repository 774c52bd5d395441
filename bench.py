"""Benchmark of the SLR hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form both|fp64] [--no-serve] [--no-large]
                    [--no-cpu-baseline]

Workload: 3-D 7-point Laplacian on a 64^3 grid (n = 262,144), 4x4x4 box
decomposition (64 subdomains), IC(0) factors of the B_i and of C, rank
k = 32 from 160 Lanczos steps, PCG to rtol 1e-8, one right-hand side
b = A x*, x* ~ U[-1, 1] (seeded).

One step = one pass of the whole hot path on the device: the Lanczos build
of (U_k, Lambda_k, theta) on H with the resident factors, then the
preconditioned Krylov solve (every iteration: SpMV, BLAS-1, the SLR apply
with its two batched B solves, interface sweeps and rank-k block).  Host
factorisation is setup and is not timed.  Prints one JSON line.

Beside the step rate the line carries the 64^3 apply and B-kernel
rooflines, the serving comparison, the oracle's rate on a host core and
(large_apply) the apply bandwidth on the shifted 128^3 workload, where the
apply is bound by bytes rather than by dependency chains, (large_solve)
that workload solved in the form that converges, and (multi_rhs_apply) the
32-column apply of the 1024^2 diffusion workload after autotuning.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "PCG solves/s at rtol 1e-8, SLR-apply HBM GB/s; p50/p99 latency mixed vs FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


FORMS = {
    # FP64 factors and U_k, plain PCG
    "fp64": dict(fact_prec="fp64", uk_prec="fp64", method="pcg", c_order="multicolor", dtype="f64"),
    # FP32 factors, BF16 U_k on matrix cores (FP32 accumulation); flexible CG
    # with FP64 recurrences, dot products and residuals
    "mixed": dict(fact_prec="fp32", uk_prec="bf16", method="fcg", c_order="multicolor",
                  dtype="f32/bf16-apply, f64-krylov"),
}


def bsolve_bytes(info, nrhs, bf):
    """Algorithmic bytes of one batched B-solve launch (apply, first half):
    every stored factor entry of the forward and backward sweeps read once
    (value + 4-byte index; a diagonal counts as one entry), E^T entries read
    once, f read once, g read once and g' written once per column."""
    return ((2 * info["nnz_LB"] + info["nnz_E"]) * (bf + 4)
            + nrhs * (info["m"] * 8 + 2 * info["s"] * 8))


def apply_bytes(info, nrhs, bf, bu, k):
    """Algorithmic bytes of one whole apply: four B sweeps, two interface
    sweeps, E and E^T once each, U_k read twice, vectors once each.  With
    the recursive interface solver the two interface sweeps become K^T and
    K: four half solves over C1's blocks, two C2 sweeps, F and F^T once
    each, U2 read four times (FP64) and the inner vectors."""
    if info.get("s1", 0) > 0:
        s1, s2, k2 = info["s1"], info["s"] - info["s1"], info["k2"]
        return ((4 * info["nnz_LB"] + 4 * info["nnz_LC1"] + 2 * info["nnz_LC2"] + 2 * info["nnz_E"]
                 + 2 * info["nnz_F"]) * (bf + 4)
                + 2 * info["s"] * k * bu + 4 * s2 * k2 * 8
                + nrhs * (2 * info["n"] * 8 + 2 * info["m"] * 8 + 4 * info["s"] * 8 + 11 * s1 * 8 + 12 * s2 * 8))
    return ((4 * info["nnz_LB"] + 2 * info["nnz_LC"] + 2 * info["nnz_E"]) * (bf + 4)
            + 2 * info["s"] * k * bu
            + nrhs * (2 * info["n"] * 8 + 2 * info["m"] * 8 + 8 * info["s"] * 8))


def _oracle_step(pr, form):
    """One oracle step on the workload: Lanczos build on the resident
    factors, then the solve of the one right-hand side.  Returns
    (seconds of the Lanczos build, seconds of the solve, result)."""
    import oracle as O
    P = O.setup(pr.csr, pr.part, pr.nparts, 0, b_fact=pr.b_fact, c_fact=pr.c_fact,
                c_order=form["c_order"], fact_prec=form["fact_prec"])
    v0 = pr.v0()[P.perm[P.m:]]
    xs, b = pr.rhs()
    t0 = time.perf_counter()
    O.lanczos_lowrank(P, pr.k, pr.lanczos_steps, v0, "lambda_k1")
    if form["uk_prec"] == "fp32":
        P.U = O.round_fp32(P.U)
    elif form["uk_prec"] == "bf16":
        P.U = O.round_bf16(P.U)
    t1 = time.perf_counter()
    res = O.solve(P, b[:, 0], "fcg" if form["method"] == "fcg" else "pcg")
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1, res


def _oracle_step_1t(args):
    from threadpoolctl import threadpool_limits
    import slr_inputs as si
    name, form = args
    with threadpool_limits(1):
        tl, ts, res = _oracle_step(si.make_config(name), form)
    return tl + ts


def host_cpu():
    """Model name and usable cores of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(pr, form, runs=3, max_procs=15):
    """The oracle as it stands, on the GPU machine's host, on a bounded sample of
    the same workload: one full step (Lanczos build + PCG solve of the one
    right-hand side).  Two legs: one thread (median of `runs` steps), and
    all usable cores as independent oracle processes, one step each, one
    thread each (whole-job throughput; the oracle's loops are serial, so
    cores add throughput over right-hand sides, not speed per solve)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    from threadpoolctl import threadpool_limits
    model, cores = host_cpu()
    times, lan, sol = [], [], []
    res = None
    with threadpool_limits(1):
        for _ in range(runs):
            tl, ts, res = _oracle_step(pr, form)
            times.append(tl + ts)
            lan.append(tl)
            sol.append(ts)
    med = float(np.median(times))
    procs = max(1, min(cores, max_procs))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=procs, mp_context=multiprocessing.get_context("fork")) as ex:
        per = list(ex.map(_oracle_step_1t, [(pr.name, form)] * procs))
    wall = time.perf_counter() - t0
    return {"value": round(1.0 / med, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"one full step on the same workload (oracle Lanczos {pr.lanczos_steps} steps "
                       f"{np.median(lan):.2f} s + PCG {res.iters} its {np.median(sol):.2f} s), 1 thread, "
                       f"median of {runs}"),
            "host_cpu": model, "host_cores": cores, "runs_s": [round(t, 3) for t in times],
            "oracle_iters": res.iters, "oracle_relres": res.true_relres,
            "all_cores": {"value": round(procs / wall, 4), "unit": "solves/s", "cores": procs,
                          "sample": f"{procs} independent oracle steps in {procs} processes (1 thread each), "
                                    f"wall {wall:.2f} s incl. process start and setup; per-step "
                                    f"median {np.median(per):.2f} s"}}


def roofline_block(achieved_gbs, ab, ms, kernel):
    return {"bound": "hbm", "achieved": round(achieved_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved_gbs / HBM_PEAK_GBS, 5), "traffic": None, "kernel": kernel,
            "algorithmic_bytes_per_launch": int(ab), "avg_launch_ms": round(ms, 5)}


def multi_rhs_apply(P, torch, nrhs=32, reps=10):
    """The 2-D diffusion 1024^2 workload (n = 1.05M, 256 uneven subdomains,
    k = 64 from 320 Lanczos steps): one apply of 32 right-hand sides in one
    launch sequence, mixed form (FP32 factors, BF16 U_k on matrix cores) and
    FP64 form; algorithmic bytes as for the 64^3 apply."""
    import slr_inputs as si
    pr = si.make_config("diffusion2d_1024")
    out = {"workload": "2-D diffusion -div(e^g grad u) 1024^2 (n=1048576), 16x16 random cuts (256 subdomains), "
                       f"IC(0) B_i and C (multicolour), k=64 from 320 Lanczos steps, {nrhs} RHS in one apply"}
    for name, fp, up in (("mixed", "fp32", "bf16"), ("fp64", "fp64", "fp64")):
        G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
                  c_fact=pr.c_fact, c_order="multicolor", fact_prec=fp, uk_prec=up, v0=pr.v0())
        torch.cuda.synchronize()
        info = G.query()
        ms0 = G.time_kernel("apply", nrhs, reps)
        tune = G.autotune(nrhs)
        ms = G.time_kernel("apply", nrhs, reps)
        st = {s: round(G.time_kernel(s, nrhs, reps), 5) for s in ("bsolve1", "lowrank", "bsolve2")}
        bf = 8 if fp == "fp64" else 4
        bu = {"fp64": 8, "fp32": 4, "bf16": 2}[up]
        ab = apply_bytes(info, nrhs, bf, bu, info["k"])
        gbs = ab / (ms * 1e-3) / 1e9
        out[name] = {"apply_us": round(ms * 1e3, 2), "apply_us_built_in_plan": round(ms0 * 1e3, 2), "autotune": tune,
                     "algorithmic_bytes": int(ab), "GBs": round(gbs, 1),
                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4), "stage_ms": st,
                     "roofline": roofline_block(gbs, ab, ms, "whole apply (B solves, sweeps, rank-k)")}
        log(f"[bench:multi] {name}: apply {ms * 1e3:.1f} us = {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% "
            f"of peak); stages {st}")
        del G
        torch.cuda.empty_cache()
    return out


def apply_profile(P, torch, name, form, nrhs, reps, autotune=False, threshold=False, recursive=False,
                  solve=False, plan=None):
    """Only set up one workload and time its apply (for profiler runs).
    threshold: ILDLT / ICT local solvers with drop tolerance 1e-4, B_i in
    minimum degree order and C in HID order (the form in which the shifted
    128^3 workload converges) instead of the zero-fill ones in multicolour
    order.  recursive (with threshold): the recursive SLR on C (inner rank
    64) in place of C's ICT factor.  solve: one FGMRES(40) solve of the
    workload's right-hand side afterwards (iterations, seconds, true
    relative residual)."""
    import slr_inputs as si
    pr = si.make_config(name)
    fp, up = {"fp64": ("fp64", "fp64"), "fp32": ("fp32", "fp32"), "mixed": ("fp32", "bf16")}[form]
    if threshold:
        kw = dict(b_fact="ildlt" if pr.b_fact.startswith("ildlt") else "ict", c_fact="ict", droptol=1e-4,
                  c_order="hid", b_order="mindeg")
        if recursive:
            kw.update(c_levels=2, k2=64)
    else:
        kw = dict(b_fact=pr.b_fact, c_fact=pr.c_fact, c_order="multicolor")
    t0 = time.perf_counter()
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, fact_prec=fp, uk_prec=up,
              v0=pr.v0(), **kw)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"{name} set up in {setup_s:.1f} s")
    tune = G.autotune(nrhs) if autotune else None
    if plan:
        # a B launch plan given as threads,lds_div,rmax,persistent (slr_set_bsolve_plan)
        th, dv, rm, pe = (int(v) for v in plan.split(","))
        G.set_bsolve_plan(nrhs > 1, th, dv, rm, pe)
        tune = {"plan": plan}
    info = G.query()
    ms = G.time_kernel("apply", nrhs, reps)
    stages = {s: round(G.time_kernel(s, nrhs, reps), 5) for s in ("bsolve1", "cfwd", "lowrank", "cbwd", "bsolve2")}
    sol = None
    if solve:
        xs, b = pr.rhs()
        bd = torch.tensor(b[:, :1], dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, sinfo = G.solve(bd[:, 0], "fgmres", rtol=1e-8, maxit=3000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rr = float(np.linalg.norm(b[:, 0] - pr.scipy() @ x.cpu().numpy()) / np.linalg.norm(b[:, 0]))
        sol = {"method": "fgmres(40)", "iters": sinfo[0]["iters"], "status": sinfo[0]["status"],
               "solve_s": round(t2 - t1, 3), "true_relres": rr}
    bf = 8 if fp == "fp64" else 4
    bu = {"fp64": 8, "fp32": 4, "bf16": 2}[up]
    ab = apply_bytes(info, nrhs, bf, bu, info["k"])
    bb = bsolve_bytes(info, nrhs, bf)
    rec = {k_: info[k_] for k_ in ("s1", "k2", "theta2", "c1_levels", "c2_levels", "nnz_LC1", "nnz_LC2", "nnz_F")} \
        if recursive else None
    print(json.dumps({"workload": name, "form": form, "nrhs": nrhs, "threshold_hid": threshold,
                      "recursive_c": rec, "setup_s": round(setup_s, 2),
                      "setup_host_s": round(info["setup_host_s"], 2),
                      "setup_lanczos_s": round(info["setup_lanczos_s"], 3), "solve": sol,
                      "c_levels": info["c_levels"], "apply_ms": round(ms, 5),
                      "apply_algorithmic_bytes": int(ab), "apply_GBs": round(ab / (ms * 1e-3) / 1e9, 1),
                      "bsolve1_algorithmic_bytes": int(bb),
                      "bsolve1_GBs": round(bb / (stages["bsolve1"] * 1e-3) / 1e9, 1),
                      "stage_ms": stages, "autotune": tune, "s": info["s"], "m": info["m"], "p": info["p"], "k": info["k"],
                      "nnz_LB": info["nnz_LB"], "nnz_LC": info["nnz_LC"], "nnz_E": info["nnz_E"]}))


def measure_form(P, pr, form, steps, warmup, v0, bd, xs, log_prefix):
    import torch
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
              c_fact=pr.c_fact, c_order=form["c_order"], fact_prec=form["fact_prec"],
              uk_prec=form["uk_prec"], v0=v0)
    torch.cuda.synchronize()
    info = G.query()
    log(f"{log_prefix} setup: host {info['setup_host_s']:.2f} s, Lanczos {info['setup_lanczos_s']:.3f} s; "
        f"s={info['s']} m={info['m']} theta={info['theta']:.5f}")

    def step():
        G.update_lowrank(pr.k, pr.lanczos_steps, v0)
        return G.solve(bd, form["method"], rtol=1e-8, maxit=300)

    for i in range(warmup):
        x, inf = step()
        log(f"{log_prefix} warmup {i}: iters {inf[0]['iters']} relres {inf[0]['relres']:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for i in range(steps):
        x, inf = step()
        iters.append(inf[0]["iters"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    log(f"{log_prefix} {steps} steps in {el:.3f} s; iters {iters}; relres {inf[0]['relres']:.2e}")
    relres = inf[0]["relres"]
    err = float(np.abs(x.cpu().numpy() - xs[:, 0]).max())
    t1 = time.perf_counter()
    ns = max(3, steps)
    for i in range(ns):
        G.solve(bd, form["method"], rtol=1e-8, maxit=300)
    torch.cuda.synchronize()
    solve_only = ns / (time.perf_counter() - t1)
    t2 = time.perf_counter()
    nl = max(2, steps // 2)
    for i in range(nl):
        G.update_lowrank(pr.k, pr.lanczos_steps, v0)
    torch.cuda.synchronize()
    lanczos_ms = 1e3 * (time.perf_counter() - t2) / nl
    stages = {st: G.time_kernel(st, 1, 50) for st in ("bsolve1", "cfwd", "lowrank", "cbwd", "bsolve2",
                                                      "apply", "spmv")}
    log(f"{log_prefix} stage ms: " + ", ".join(f"{k} {v:.4f}" for k, v in stages.items()))
    bf = 8 if form["fact_prec"] == "fp64" else 4
    bu = {"fp64": 8, "fp32": 4, "bf16": 2}[form["uk_prec"]]
    res = {"steps_per_s": round(steps / el, 4), "ms_per_step": round(1e3 * el / steps, 3), "iters": iters[-1],
           "final_relres_fp64": relres, "max_abs_err_vs_xstar": err,
           "solve_only_solves_per_s": round(solve_only, 3), "lanczos_build_ms": round(lanczos_ms, 3),
           "lanczos_reorth_steps": G.query()["lanczos_reorth"],
           "apply_ms": round(stages["apply"], 5),
           "apply_algorithmic_GBs": round(apply_bytes(info, 1, bf, bu, info["k"]) / (stages["apply"] * 1e-3) / 1e9, 2),
           "stage_ms": {k: round(v, 5) for k, v in stages.items()}}
    return G, info, res, stages, bf


def measure_refactor(P, pr, form, v0, reps=5):
    """Device refactorisation (slr_refactor) of the workload's own values
    against the host setup of the same preconditioner (factorisation,
    analysis, packing and upload)."""
    import torch
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
              c_fact=pr.c_fact, c_order=form["c_order"], fact_prec=form["fact_prec"],
              uk_prec=form["uk_prec"], v0=v0, refactor=True)
    host_s = G.query()["setup_host_s"]
    G.refactor(pr.csr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        G.refactor(pr.csr)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    log(f"[bench:refactor] device refactorisation {ms:.3f} ms vs host setup {1e3 * host_s:.1f} ms")
    del G
    return {"refactor_ms": round(ms, 3), "host_setup_ms": round(1e3 * host_s, 3)}


SERVE_MAXIT = 1000


def large_apply(P, torch, reps=20):
    """Apply bandwidth on the shifted 3-D 128^3 workload (n = 2.1M, 512
    subdomains, ILDL^T(0) B_i, IC(0) C, k = 64 from 320 Lanczos steps), one
    right-hand side: the problem where the apply's bytes, not its dependency
    chains, set the time.  Both storage forms; algorithmic bytes as for the
    64^3 apply."""
    import slr_inputs as si
    pr = si.make_config("shifted3d_128")
    out = {"workload": "shifted 3-D 7-point Laplacian 128^3 (n=2097152), 8x8x8 boxes (512 subdomains), "
                       "ILDL^T(0) B_i, IC(0) C (multicolour), k=64 from 320 Lanczos steps, 1 RHS"}
    for name, fp, up in (("fp64", "fp64", "fp64"), ("fp32", "fp32", "fp32")):
        G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact=pr.b_fact,
                  c_fact=pr.c_fact, c_order="multicolor", fact_prec=fp, uk_prec=up, v0=pr.v0())
        torch.cuda.synchronize()
        info = G.query()
        ms = G.time_kernel("apply", 1, reps)
        bf = 8 if fp == "fp64" else 4
        bu = 8 if up == "fp64" else 4
        ab = apply_bytes(info, 1, bf, bu, info["k"])
        gbs = ab / (ms * 1e-3) / 1e9
        bb = bsolve_bytes(info, 1, bf)
        bms = G.time_kernel("bsolve1", 1, reps)
        out[name] = {"apply_us": round(ms * 1e3, 2), "algorithmic_bytes": int(ab), "GBs": round(gbs, 1),
                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "roofline": roofline_block(gbs, ab, ms, "whole apply (B solves, sweeps, rank-k)"),
                     "bsolve_roofline": roofline_block(bb / (bms * 1e-3) / 1e9, bb, bms,
                                                       "k_bsolve (batched B_i solves + E^T epilogue)")}
        log(f"[bench:large] {name}: apply {ms * 1e3:.1f} us = {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of peak)")
        del G
        torch.cuda.empty_cache()
    return out


def large_solve(P, torch):
    """The shifted 3-D 128^3 workload in the form that converges: ILDLT B_i
    in minimum degree order, drop tolerance 1e-4, k = 64 from 320 Lanczos
    steps, and the recursive SLR on C (HID order, ICT C1 / C2, inner rank 64
    from 320 steps); FGMRES(40) to rtol 1e-8 (at most 3000 iterations) on
    the workload's right-hand side.  Setup, apply and solve time, the
    iteration count (the oracle's is 931) and the true FP64 residual."""
    import slr_inputs as si
    pr = si.make_config("shifted3d_128")
    t0 = time.perf_counter()
    G = P.SLR(pr.csr, pr.part, pr.nparts, k=pr.k, lanczos_steps=pr.lanczos_steps, b_fact="ildlt", c_fact="ict",
              droptol=1e-4, c_order="hid", b_order="mindeg", c_levels=2, k2=64, v0=pr.v0())
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = G.query()
    ms = G.time_kernel("apply", 1, 10)
    xs, b = pr.rhs()
    bd = torch.tensor(b[:, 0], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, sinfo = G.solve(bd, "fgmres", rtol=1e-8, maxit=3000)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t1
    rr = float(np.linalg.norm(b[:, 0] - pr.scipy() @ x.cpu().numpy()) / np.linalg.norm(b[:, 0]))
    ab = apply_bytes(info, 1, 8, 8, info["k"])
    out = {"workload": "shifted 3-D 7-point Laplacian 128^3 (n=2097152), 20 negative eigenvalues, 8x8x8 boxes; "
                       "ILDLT B_i (minimum degree order), recursive SLR on C (HID order, ICT C1/C2, inner k=64), "
                       "drop tolerance 1e-4, k=64 from 320 Lanczos steps, FGMRES(40), rtol 1e-8, FP64",
           "setup_s": round(setup_s, 2), "setup_host_s": round(info["setup_host_s"], 2),
           "setup_lanczos_s": round(info["setup_lanczos_s"], 3), "apply_ms": round(ms, 4),
           "apply_GBs": round(ab / (ms * 1e-3) / 1e9, 1), "iters": sinfo[0]["iters"], "status": sinfo[0]["status"],
           "solve_s": round(solve_s, 3), "true_relres": rr, "oracle_iters": 931}
    log(f"[bench:large] recursive FGMRES: {sinfo[0]['iters']} iterations in {solve_s:.2f} s, relres {rr:.2e}")
    del G
    torch.cuda.empty_cache()
    return out


def serving(P, torch, n_req, seed=13):
    """Continuous batching (mixed form, flexible CG) vs one-request-at-a-time
    plain FP64 PCG over four resident preconditioners."""
    import slr_inputs as si
    from paper_1505_04340_amd import serve
    names = ["serve_lap2d_256", "serve_lap2d_512", "serve_lap3d_64", "serve_lap3d_96"]
    prs = [si.make_config(nm) for nm in names]
    mixed, plain = [], []
    for pr in prs:
        kw = dict(k=pr.k, lanczos_steps=pr.lanczos_steps, c_order="multicolor", v0=pr.v0())
        mixed.append(P.SLR(pr.csr, pr.part, pr.nparts, fact_prec="fp32", uk_prec="bf16", **kw))
        plain.append(P.SLR(pr.csr, pr.part, pr.nparts, **kw))
    ns = [pr.n for pr in prs]
    out = {"matrices": [f"{nm} (n={pr.n}, p={pr.nparts}, k={pr.k})" for nm, pr in zip(names, prs)]}

    def run(kind, rate):
        reqs = serve.make_requests(ns, n_req, rate, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "mixed_batched":
            svc = serve.Service(mixed, "fcg", maxit=SERVE_MAXIT)
            svc.run(reqs)
            dev = svc.peak_bytes
            svc.close()
        else:
            serve.serve_plain(plain, reqs, "pcg", maxit=SERVE_MAXIT)
            dev = 0
        wall = time.perf_counter() - t0
        sm = serve.summarize(reqs, wall)
        if dev:
            sm["batch_device_bytes"] = dev
        log(f"[serve] {kind} rate {rate:.1f}/s: {sm}")
        return sm

    sat_p = run("plain_fp64", 0.0)
    sat_m = run("mixed_batched", 0.0)
    rate = 0.8 * sat_p["requests_per_s"]
    out["saturation"] = {"plain_fp64": sat_p, "mixed_batched": sat_m}
    out["poisson_rate_per_s"] = round(rate, 3)
    out["poisson"] = {"plain_fp64": run("plain_fp64", rate), "mixed_batched": run("mixed_batched", rate)}
    out["speedup_solves_per_s"] = round(sat_m["solves_per_s"] / sat_p["solves_per_s"], 3)
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bsolve_lap3d_64_hbm_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1505_04340_amd", "csrc", "slr_kernels.hip")

# The paper's own timings for the nearest problems (Sec. 6, the tables of
# SPD and of indefinite model problems): CPU wall-clock seconds on its stated
# hardware.  Context only: its partitions (METIS), local factors (ICT /
# ILDLT with fill) and shifts differ from the workloads measured here.
PAPER_CONTEXT = {
    "hardware": "2x Intel Xeon X5560 (4 cores each, 2.8 GHz), 24 GB; C/C++ with MKL and OpenMP",
    "spd_64cubed_slr_cg": {"n": 262144, "subdomains": 64, "rank": 32, "fill": 6.3, "setup_s": 1.52,
                           "iters": 38, "iteration_s": 0.633,
                           "note": "7-point Laplacian 64^3, METIS partition, ICT factors; SLR-CG"},
    "indefinite_100cubed_slr_gmres": {"n": 1000000, "subdomains": 128, "rank": 180, "fill": 14.6,
                                      "setup_s": 62.9, "iters": 88, "iteration_s": 13.9,
                                      "note": "7-point Laplacian 100^3 shifted by 0.05, ILDLT factors; "
                                              "SLR-GMRES(40)"},
}


def recorded_traffic():
    """HBM bytes per k_bsolve launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel source has changed since the counters
    were taken (the summary records the source's sha256)."""
    try:
        text = open(TRAFFIC_FILE).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"slr_kernels\.hip sha256: ([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch [^\n]*: (\d+)", text)
    if not m or not t or m.group(1) != sha:
        return None
    return int(t.group(1))


def copy_calibration(nbytes=1 << 30, reps=4):
    """A plain device-to-device copy of nbytes, reps times: the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to HBM bytes."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 128^3 apply-bandwidth measurement")
    ap.add_argument("--serve-requests", type=int, default=96)
    ap.add_argument("--config", default="lap3d_64")
    ap.add_argument("--form", choices=("both", "fp64"), default="both",
                    help="fp64: measure only the FP64 form (the headline), not the mixed one beside it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter calibration)")
    ap.add_argument("--no-multi", action="store_true", help="skip the 1024^2 32-RHS apply measurement")
    ap.add_argument("--apply-profile", default=None,
                    help="only set up this workload and time its apply (for profiler runs)")
    ap.add_argument("--apply-form", choices=("fp64", "fp32", "mixed"), default="fp64")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--autotune", action="store_true", help="with --apply-profile: slr_autotune first")
    ap.add_argument("--threshold", action="store_true",
                    help="with --apply-profile: ILDLT/ICT (1e-4), minimum degree B_i, HID C")
    ap.add_argument("--recursive", action="store_true",
                    help="with --threshold: the recursive SLR on C (inner rank 64)")
    ap.add_argument("--solve", action="store_true", help="with --apply-profile: one FGMRES(40) solve as well")
    ap.add_argument("--plan", default=None,
                    help="with --apply-profile: B launch plan threads,lds_div,rmax,persistent (slr_set_bsolve_plan)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.apply_profile:
        import torch
        import paper_1505_04340_amd as P
        torch.cuda.set_device(0)
        apply_profile(P, torch, args.apply_profile, args.apply_form, args.nrhs, args.reps, args.autotune,
                      args.threshold, args.recursive, args.solve, args.plan)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is a design note, not a built path)", file=sys.stderr)
        sys.exit(2)

    import slr_inputs as si

    pr = si.make_config(args.config)
    cpu = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU: the all-cores leg forks oracle
        # processes, which must not inherit an open device
        log("[bench] CPU baseline (oracle: 1 thread, then all cores) ...")
        cpu = cpu_baseline(pr, FORMS["fp64"])
        log(f"[bench] CPU baseline {cpu['value']:.4f} solves/s (1 thread), "
            f"{cpu['all_cores']['value']:.3f} solves/s ({cpu['all_cores']['cores']} processes)")

    import torch
    import paper_1505_04340_amd as P

    torch.cuda.set_device(0)
    log(f"[bench] {pr.name} n={pr.n} p={pr.nparts} k={pr.k}; device LDS per workgroup "
        f"{P.slr_device_lds_bytes()} bytes")
    xs, b = pr.rhs()
    bd = torch.tensor(b[:, 0], dtype=torch.float64, device="cuda")
    v0 = pr.v0()
    forms = {}
    G = None
    for name in ("fp64", "mixed") if args.form == "both" else ("fp64",):
        Gf, info, res, stages, bf = measure_form(P, pr, FORMS[name], args.steps, args.warmup, v0, bd, xs,
                                                 f"[bench:{name}]")
        forms[name] = res
        if name == "fp64":
            G, info64, stages64, bf64 = Gf, info, stages, bf
        else:
            del Gf
    res = forms["fp64"]
    bb = bsolve_bytes(info64, 1, bf64)
    achieved = bb / (stages64["bsolve1"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": recorded_traffic() if args.config == "lap3d_64" else None,
            "kernel": "k_bsolve (batched B_i solves + E^T epilogue)",
            "algorithmic_bytes_per_launch": int(bb), "avg_launch_ms": round(stages64["bsolve1"], 5)}
    out = {
        "metric": METRIC, "value": res["steps_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": FORMS["fp64"]["dtype"],
        "data": "synthetic",
        "config": {"workload": "3-D 7-point Laplacian 64^3 (n=262144), 4x4x4 boxes (64 subdomains), "
                               "IC(0) B_i and C (multicolour C ordering), k=32 from 160 Lanczos steps, "
                               "PCG rtol 1e-8, 1 RHS; step = device Lanczos build + solve",
                   "form": "fp64", "nrhs": 1},
        "roofline": roof,
        "iters": res["iters"], "final_relres_fp64": res["final_relres_fp64"],
        "solve_only_solves_per_s": res["solve_only_solves_per_s"], "lanczos_build_ms": res["lanczos_build_ms"],
        "apply_ms": res["apply_ms"], "apply_algorithmic_GBs": res["apply_algorithmic_GBs"],
        "forms": forms,
        "refactor": measure_refactor(P, pr, FORMS["fp64"], v0),
    }
    del G
    torch.cuda.empty_cache()
    if not args.no_large:
        out["large_apply"] = large_apply(P, torch)
        out["large_solve"] = large_solve(P, torch)
    if not args.no_multi:
        out["multi_rhs_apply"] = multi_rhs_apply(P, torch)
    if not args.no_serve:
        out["serving"] = serving(P, torch, args.serve_requests)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    out["paper_context"] = PAPER_CONTEXT
    print(json.dumps(out))


if __name__ == "__main__":
    main()
