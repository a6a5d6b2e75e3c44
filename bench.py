#!/usr/bin/env python3
"""Benchmark of the complex additive multilevel cycle on one MI355X.

Headline workload: d = 3, levels 1..6 (729^3 finest cells, 730^3 = 389 M
complex128 vertices), -Lap u - phi u with phi = k^2 (1 + 0.5i), k = 40,
theta = 0, one Gaussian load, BPX, omega 0.6 on every level.  One step = one
pipelined additive cycle over the whole hierarchy (coarse descent, fused
finest sweep, coarse backtracking, residual norm).  Inputs are resident in
HBM before timing starts.

Printed JSON line (last line of stdout): vertex-updates/s per cycle (interior
vertices of all levels per cycle time), the finest sweep's achieved HBM
bandwidth against the 8 TB/s peak, time to relative residual 1e-10 with the
BiCGStab driver in FP64 and with complex64 corrections inside FP64 residual
refinement (and the mixed solution's deviation from the FP64 one), the FP64
CPU oracle's rate on a bounded sample, and extras: the 3D level-5 k = 20
complex-grid workload (BPX and hb cycles, time to 1e-10 from zero and from a
nested start), the 2D level-5 k = 10 workload's 30-cycle latency, the
potential workload's varying-phi cycle and adjoint gradient, the same-grid
multichannel cycle, and the 96-problem batched workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def updates_per_cycle(dim, L, lmin=1):
    return sum((3 ** l - 1) ** dim for l in range(lmin, L + 1))


def fused_bytes(dim, L, variant, word=16):
    """Algorithmic HBM bytes of one finest sweep: read w, b and write w' per
    finest vertex; per coarse vertex read sc (and si for BPX), write R r (and
    I s into sf for add / si for BPX)."""
    NL = (3 ** L + 1) ** dim
    Nc = (3 ** (L - 1) + 1) ** dim
    coarse_words = {"add": 3, "hb": 2, "bpx": 4}[variant]
    return word * (3 * NL + coarse_words * Nc)


def single_touch_bytes(dim, L, lmin=1, word=16):
    """Bytes per cycle of the method's own single-touch form (Section 5's
    pipelined traversal with constant phi): 5 words per finest vertex (read u,
    sc, b; write u, sc) and 14 per coarse vertex (pre, post and the finer
    level's transfers of u, sc, si, sf, b)."""
    NL = (3 ** L + 1) ** dim
    Nc = sum((3 ** l + 1) ** dim for l in range(lmin, L))
    return word * (5 * NL + 14 * Nc)


FUSED_SOURCES = ["mg_fused_ops.h", "mg_fused.hip", "mg_internal.h", "mg_common.h"]


def fused_source_digest():
    """sha256 over the sources the finest-sweep kernel is compiled from."""
    h = hashlib.sha256()
    for name in FUSED_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1508_03954_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(tile, level):
    """HBM traffic of the finest sweep from the committed rocprofv3 counter
    summary of that level, scaled by the copy-kernel calibration; None when
    absent, when the kernel sources changed since the counters were taken or
    when the counters were taken for another tile."""
    path = os.path.join(ROOT, "profiles", f"fused3_l{level}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256") != fused_source_digest():
        return None
    return rec.get("tiles", {}).get(str(tile), {}).get("bytes_per_launch")


def time_cycles(s, steps, warmup, torch, ramp_s=0.3):
    """W untimed warmup cycles, then K timed ones.  Before the warmup the device
    runs untimed cycles for ramp_s seconds, so that the timed cycles run at the
    clocks of a loaded GPU (a cold device ramps its clocks over the first tenths
    of a second)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < ramp_s:
        s.cycle(20, norms=False)
        torch.cuda.synchronize()
    s.cycle(warmup, norms=False)
    torch.cuda.synchronize()
    s.time_sweeps(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(s.stream)
    s.cycle(steps, norms=False)
    stop.record(s.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    sweep_ms, cnt = s.sweep_time()
    s.time_sweeps(False)
    return ms / steps, sweep_ms / max(cnt, 1), cnt


def _oracle_pipeline(level):
    """The FP64 oracle's pipelined cycle state for the 3D k = 40 problem at
    `level` (setup: input, load, helpers)."""
    import oracle as O
    from oracle.cycle import Params
    from paper_1508_03954_amd.inputs import config_3d_large
    prob = config_3d_large(level_max=level)
    p = Params(dim=3, level_max=level, theta=prob.theta, phi=prob.phi, variant="bpx", omega=0.6)
    b = O.lumped_rhs(prob.chi, level, prob.theta)
    return O.Pipelined(p, b)


def _timed_cycle(pipe):
    """Wall time of one oracle cycle with numpy on one BLAS thread."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        pipe.cycle()
        return time.perf_counter() - t0


def _oracle_worker(level, barrier, q):
    pipe = _oracle_pipeline(level)
    barrier.wait()
    q.put(_timed_cycle(pipe))


def host_cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(procs=0, level=5):
    """The FP64 oracle as it stands, on the host: one pipelined cycle of the
    3D k = 40 problem (the headline's problem family) at level 5, 244^3, the
    largest size whose oracle cycle fits a bounded sample (its cost is linear
    in the vertex count; level 6 would need ~30x the memory).  Timed in one
    process, then in `procs` processes that start their cycles together after
    their setup (the oracle's numpy arithmetic is single-threaded, so the
    cores are used by processes): rate = all their vertex updates over the
    slowest process's cycle time."""
    import multiprocessing as mp
    import psutil
    ups = updates_per_cycle(3, level)
    t1 = _timed_cycle(_oracle_pipeline(level))
    ncpu = os.cpu_count() or 1
    if procs <= 0:
        # each process peaks near 12 GB at level 5; use at most 40 % of the
        # free memory, at most 8 processes and the cores there are
        per_proc = 12e9
        procs = max(1, min(8, ncpu, int(0.4 * psutil.virtual_memory().available / per_proc)))
    ctx = mp.get_context("fork")
    barrier, q = ctx.Barrier(procs), ctx.Queue()
    ps = [ctx.Process(target=_oracle_worker, args=(level, barrier, q)) for _ in range(procs)]
    for p in ps:
        p.start()
    times = [q.get() for _ in ps]
    for p in ps:
        p.join()
    return {
        "value": procs * ups / max(times),
        "unit": "vertex-updates/s",
        "cores": procs,
        "kind": "oracle",
        "sample": f"one pipelined FP64 oracle cycle (numpy, one BLAS thread per process) of the 3D k=40, "
                  f"phi=k^2(1+0.5i), BPX problem at level {level} ({3 ** level + 1}^3 vertices, {ups} vertex "
                  f"updates) in each of {procs} processes started together after their setup; rate = their "
                  f"updates over the slowest process's cycle time ({max(times):.2f} s)",
        "single_thread": {"value": ups / t1, "cores": 1, "seconds_per_cycle": t1},
        "host": {"nproc": ncpu, "cpu_model": host_cpu_model()},
    }


def batched_extra(torch, solve=True):
    """96 independent problems (64 2D with finest level 3..6, 32 3D with 3..5,
    k in [5, 60], phi = k^2 (1 + 0.5i), complex64 corrections): one batched
    persistent cycle vs the same cycles launched problem by problem."""
    import numpy as np
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_batched
    probs = config_batched()
    kws = [dict(dim=p.dim, level_max=p.level_max, phi=p.phi, variant="bpx", precision="fp32_refine") for p in probs]
    b = mg.Batch(kws)
    rhs = [s.rhs_from_nodal(torch.from_numpy(p.chi).cuda()) for s, p in zip(b.solvers, probs)]

    def reset():
        for s, r in zip(b.solvers, rhs):
            s.set_rhs(r)
            s.set_solution(torch.zeros_like(r))
        torch.cuda.synchronize()

    reset()
    best, best_us, times = b.autotune(reps=3)
    reset()
    reps = 10
    b.cycle(2, norms=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.cycle(reps, norms=False)
    e1.record(b.stream)
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / reps
    reset()
    for s in b.solvers:
        s.cycle(1, norms=False)
    torch.cuda.synchronize()
    e0.record(b.stream)
    for _ in range(reps):
        for s in b.solvers:
            s.cycle(1, norms=False)
    e1.record(b.stream)
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / reps
    U = sum(updates_per_cycle(p.dim, p.level_max) for p in probs)
    NL = sum((3 ** p.level_max + 1) ** p.dim for p in probs)
    # time to 1e-10 for all 96 problems: the batched Krylov driver (lockstep
    # BiCGStab, complex64 corrections in FP64 refinement) against the same
    # solves run problem by problem
    if not solve:
        b.close()
        return {"workload": "96 problems: 64 2D (finest level 3..6) + 32 3D (3..5), k~U[5,60], phi=k^2(1+0.5i), "
                            "BPX, complex64 corrections, seeds [4, i]",
                "finest_vertices": NL, "vertex_updates_per_cycle": U, "batched_ms_per_cycle": t_batch,
                "sequential_ms_per_cycle": t_seq, "speedup": t_seq / t_batch,
                "autotune": {"config": best, "us_per_config": [round(t, 1) for t in times]}}
    us = [torch.zeros_like(r) for r in rhs]
    b.solve(rhs, us, rtol=1e-2, maxit=50)       # first call sets up the batched Krylov buffers
    us = [torch.zeros_like(r) for r in rhs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, rel, rc = b.solve(rhs, us, rtol=1e-10, maxit=20000)
    torch.cuda.synchronize()
    t_bsolve = time.perf_counter() - t0
    log(f"[bench] batched solve to 1e-10: {t_bsolve:.2f} s (status {rc}, worst relres {max(rel):.2e}, "
        f"inner iterations up to {max(its)})")
    useq = [torch.zeros_like(r) for r in rhs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_its, seq_rc = [], 0
    for s, r, u in zip(b.solvers, rhs, useq):
        _, it, rr, rc1 = s.solve(r, u0=u, rtol=1e-10, maxit=20000)
        seq_its.append(it)
        seq_rc = seq_rc or rc1
    torch.cuda.synchronize()
    t_ssolve = time.perf_counter() - t0
    log(f"[bench] the same solves problem by problem: {t_ssolve:.2f} s")
    solve = {"driver": "batched BiCGStab in lockstep (one persistent launch per preconditioner application), "
                       "complex64 corrections in FP64 refinement", "seconds": t_bsolve, "status": int(rc),
             "max_relres": float(max(rel)), "max_inner_iterations": int(max(its)),
             "hardest_problem": int(np.argmax(its)),
             "sequential_seconds": t_ssolve, "sequential_status": int(seq_rc),
             "sequential_max_inner_iterations": int(max(seq_its)),
             "speedup": t_ssolve / t_bsolve}
    b.close()
    log(f"[bench] batched: {t_batch * 1e3:.0f} us per cycle of all 96 problems vs {t_seq * 1e3:.0f} us "
        f"problem by problem (configuration {best})")
    return {"workload": "96 problems: 64 2D (finest level 3..6) + 32 3D (3..5), k~U[5,60], phi=k^2(1+0.5i), "
                        "BPX, complex64 corrections, seeds [4, i]",
            "finest_vertices": NL, "vertex_updates_per_cycle": U,
            "batched_ms_per_cycle": t_batch, "sequential_ms_per_cycle": t_seq,
            "batched_vertex_updates_per_s": U / (t_batch * 1e-3),
            "sequential_vertex_updates_per_s": U / (t_seq * 1e-3),
            "speedup": t_seq / t_batch, "autotune": {"config": best, "us_per_config": [round(t, 1) for t in times]},
            "time_to_1e-10": solve}


def refine_extra(torch, level):
    """3D k = 40, phi = k^2 (1 + 0.5i): BiCGStab to relative residual 1e-10 with
    complex64 corrections inside FP64 residual refinement vs the plain
    complex128 solve; the mixed result's deviation from the FP64 one."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_3d_large
    prob = config_3d_large(level_max=level)
    res = {"workload": f"{prob.name}: d=3, levels 1..{level} ({3 ** level + 1}^3 vertices), BPX, omega 0.6"}
    chi = torch.from_numpy(prob.chi).cuda()
    del prob
    u64 = None
    for prec in ("fp32_refine", "fp64"):
        s = mg.Solver(3, level, phi=1600.0 * (1 + 0.5j), variant="bpx", precision=prec)
        b = s.rhs_from_nodal(chi)
        u = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, its, rel, rc = s.solve(b, u0=u, rtol=1e-10, maxit=3000, driver="bicgstab")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        true_rel = s.residual_norm(u, b) / s.residual_norm(torch.zeros_like(b), b)
        res[prec] = {"seconds": dt, "iterations": its, "relres": rel, "true_relres": true_rel, "status": rc}
        log(f"[bench] L={level} {prec}: {dt:.2f} s, {its} iterations, relres {true_rel:.2e}")
        if prec == "fp32_refine":
            u_mixed = u
        else:
            u64 = u
        del s, b
        torch.cuda.empty_cache()
    res["mixed_vs_fp64_rel_error"] = (torch.linalg.vector_norm(u_mixed - u64) /
                                      torch.linalg.vector_norm(u64)).item()
    res["speedup"] = res["fp64"]["seconds"] / res["fp32_refine"]["seconds"]
    return res


def cycle_record(s, L, variant, steps, warmup, ramp_s, torch, tune_reps=3, tile=None, autotune=True):
    """Autotuned (or fixed-tile) timing of one hierarchy's pipelined cycle:
    vertex-updates/s, the finest sweep's live duration and its roofline."""
    dim = 3
    tune = None
    if tile is not None:
        s.set_tile(tile)
        tune = {"tile": tile, "fixed": True}
    elif autotune:
        best, best_us, times = s.autotune(reps=tune_reps)
        tune = {"tile": best, "us_per_tile": [round(t, 1) for t in times]}
        log(f"[bench] autotune L={L}: tile {best} ({best_us:.1f} us); all: {', '.join(f'{t:.1f}' for t in times)}")
    ms_step, sweep_ms, nsw = time_cycles(s, steps, warmup, torch, ramp_s)
    ups = updates_per_cycle(dim, L)
    fb = fused_bytes(dim, L, variant)
    achieved = fb / (sweep_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(s.tiles()[0], L)
    log(f"[bench] L={L} {variant}: cycle {ms_step * 1e3:.1f} us, finest sweep {sweep_ms * 1e3:.1f} us ({nsw} timed), "
        f"{achieved:.0f} GB/s algorithmic")
    roof = {
        "kernel": "k_fused3 (finest-level fused sweep)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": fb,
        "avg_launch_us": sweep_ms * 1e3,
        "launches_timed": nsw,
        # the whole cycle priced at the method's single-touch byte count
        "cycle_effective_GBs": single_touch_bytes(dim, L) / (ms_step * 1e-3) / 1e9,
    }
    return ms_step, ups, roof, tune


def time_solve(s, b, torch, driver="bicgstab", maxit=3000):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, its, rel, rc = s.solve(b, rtol=1e-10, maxit=maxit, driver=driver)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return u, {"seconds": dt, "iterations": its, "relres": rel, "status": rc}


def headline(args, torch):
    """The 3D level-6 problem: k = 40, phi = k^2 (1 + 0.5i), theta = 0, BPX,
    omega 0.6 on every level.  Plain complex128 cycle rate and sweep roofline;
    BiCGStab to 1e-10 in FP64 and with complex64 corrections inside FP64
    residual refinement, and the deviation of the mixed solution from the
    FP64 one."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_3d_large
    L = args.level
    prob = config_3d_large(level_max=L)
    chi = torch.from_numpy(prob.chi).cuda()
    theta, phi = prob.theta, prob.phi
    name = prob.name
    del prob
    log(f"[bench] {name}: 3D L={L} ({3 ** L + 1}^3 vertices), steps={args.steps} warmup={args.warmup}")
    s = mg.Solver(3, L, theta=theta, phi=phi, variant="bpx", omega=0.6, sweep=args.sweep)
    b = s.rhs_from_nodal(chi)
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    ms_step, ups, roof, tune = cycle_record(s, L, "bpx", args.steps, args.warmup, args.ramp_s, torch,
                                           tune_reps=2, tile=args.tile,
                                           autotune=args.sweep != "generic" and not args.no_autotune)
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    rh, _ = s.cycle(3)
    log(f"[bench] residual h-norms of the first cycles: {', '.join(f'{v:.3e}' for v in rh)}")
    rec = {"ms_per_step": ms_step, "value": ups / (ms_step * 1e-3), "ups": ups, "roofline": roof, "tune": tune,
           "workload": f"{name}: d=3, levels 1..{L} ({3 ** L + 1}^3 complex128 vertices), k=40, "
                       f"phi=k^2(1+0.5i), theta=0, one Gaussian load (sigma 0.05), bpx, omega=0.6 on every level"}
    if args.no_solve:
        return rec
    b0 = torch.zeros_like(b)
    bnorm = s.residual_norm(b0, b)
    u64, r64 = time_solve(s, b, torch)
    r64["true_relres"] = s.residual_norm(u64, b) / bnorm
    log(f"[bench] FP64 BiCGStab to 1e-10: {r64['seconds']:.2f} s, {r64['iterations']} iterations, "
        f"relres {r64['true_relres']:.2e}")
    del s
    torch.cuda.empty_cache()
    m = mg.Solver(3, L, theta=theta, phi=phi, variant="bpx", omega=0.6, precision="fp32_refine")
    um, rm = time_solve(m, b, torch)
    del m
    torch.cuda.empty_cache()
    # the mixed solution's true residual with an FP64 operator
    chk = mg.Solver(3, L, level_min=L, theta=theta, phi=phi, variant="bpx", omega=0.6, sweep="generic")
    rm["true_relres"] = chk.residual_norm(um, b) / bnorm
    del chk
    err = (torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64)).item()
    log(f"[bench] complex64-in-FP64 refinement to 1e-10: {rm['seconds']:.2f} s, {rm['iterations']} inner "
        f"iterations, relres {rm['true_relres']:.2e}, |u_mixed - u_fp64| / |u_fp64| = {err:.2e}")
    rec["time_to_1e-10"] = {
        "driver": "bicgstab (preconditioner: one zero-start additive cycle)",
        "seconds": r64["seconds"],
        "fp64": r64,
        "fp32_refine": dict(rm, form="complex64 level corrections, FP64 residual and update"),
        "mixed_vs_fp64_rel_error": err,
        "speedup_mixed_over_fp64": r64["seconds"] / rm["seconds"],
    }
    del u64, um, b, chi
    torch.cuda.empty_cache()
    return rec


def csg_extra(args, torch):
    """The 3D level-5 problem: k = 20 on the complex grid h exp(i pi/6), four
    Gaussians plus 1e-3 noise; BPX and hb cycles, BiCGStab to 1e-10 from zero
    and from a nested start."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_3d_csg
    L = 5
    prob = config_3d_csg(level_max=L, variant="bpx")
    chi = torch.from_numpy(prob.chi).cuda()
    out = {"workload": f"{prob.name}: d=3, levels 1..{L} ({3 ** L + 1}^3 complex128 vertices), k=20, "
                       f"theta=pi/6, 4 Gaussians + 1e-3 noise, omega=0.6 on every level"}
    for variant in ("bpx", "hb"):
        s = mg.Solver(3, L, theta=prob.theta, phi=prob.phi, variant=variant, omega=0.6)
        b = s.rhs_from_nodal(chi)
        s.set_rhs(b)
        s.set_solution(torch.zeros_like(b))
        ms, ups, roof, tune = cycle_record(s, L, variant, 200, 10, args.ramp_s, torch, tune_reps=5,
                                           autotune=not args.no_autotune)
        out[variant] = {"value": ups / (ms * 1e-3), "ms_per_step": ms, "vertex_updates_per_cycle": ups,
                        "roofline": roof, "autotune": tune}
        if variant == "bpx":
            b0 = torch.zeros_like(b)
            bnorm = s.residual_norm(b0, b)
            u, rec = time_solve(s, b, torch, maxit=2000)
            rec["true_relres"] = s.residual_norm(u, b) / bnorm
            out["time_to_1e-10"] = dict(rec, driver="bicgstab (preconditioner: one zero-start additive cycle)")
            log(f"[bench] L=5 BiCGStab to 1e-10: {rec['seconds']:.3f} s, {rec['iterations']} iterations")
            # nested start: levels 3 and 4 solved to 1e-2 with the sampled load,
            # each from the prolonged level below (one untimed call makes the
            # coarser levels' contexts)
            s.solve_nested(chi, level_start=L - 2, coarse_rtol=1e-2, rtol=1e-10, maxit=2000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, its, rel, rc = s.solve_nested(chi, level_start=L - 2, coarse_rtol=1e-2, rtol=1e-10, maxit=2000)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            out["time_to_1e-10_nested"] = {
                "driver": "bicgstab from the prolonged solutions of levels L-2 and L-1 (each solved to 1e-2)",
                "seconds": t1 - t0, "finest_iterations": its, "relres": rel,
                "true_relres": s.residual_norm(u, b) / bnorm, "status": rc}
            log(f"[bench] L=5 nested BiCGStab to 1e-10: {t1 - t0:.3f} s, {its} finest iterations")
        del s, b
        torch.cuda.empty_cache()
    return out


def latency_extra(torch):
    """The 2D problem: levels 1..5 (244^2), k = 10, phi = k^2 (1 + 0.5i), one
    Gaussian load, BPX, omega 0.6: its 30 cycles from u = 0 as one call (the
    grid is cache-resident, so this measures per-cycle latency)."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_2d_bpx
    prob = config_2d_bpx(level_max=5)
    s = mg.Solver(2, 5, theta=prob.theta, phi=prob.phi, variant="bpx", omega=0.6)
    b = s.rhs_from_nodal(torch.from_numpy(prob.chi).cuda())
    tile, _, _ = s.autotune(reps=5)
    reps, ms = 20, []
    for _ in range(reps + 2):
        s.set_rhs(b)
        s.set_solution(torch.zeros_like(b))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.cycle(prob.cycles, norms=False)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = sorted(ms[2:])
    med = ms[len(ms) // 2]
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    rh, _ = s.cycle(prob.cycles)
    ups = updates_per_cycle(2, 5)
    log(f"[bench] 2D k=10: {prob.cycles} cycles in {med * 1e3:.0f} us ({med / prob.cycles * 1e3:.1f} us per cycle)")
    return {"workload": f"{prob.name}: d=2, levels 1..5 (244^2 complex128 vertices), k=10, phi=k^2(1+0.5i), "
                        f"one Gaussian load, bpx, omega=0.6, {prob.cycles} cycles from u=0",
            "ms_for_30_cycles": med, "us_per_cycle": med / prob.cycles * 1e3,
            "vertex_updates_per_s": ups * prob.cycles / (med * 1e-3), "tile": tile,
            "residual_reduction_30_cycles": rh[-1] / rh[0], "samples": reps}


def adjoint_extra(torch):
    """The potential problem: 3D levels 1..5, k = 15, V = 8 Gaussians, phi =
    k^2 (1 + 0.3i) - V (nodal phi: the per-cell path with the FAS form).  The
    varying-phi cycle's rate, then J = sum over the shell of |u|^2 and dJ/dV
    through torch.autograd: forward solve, adjoint solve and gradient kernel,
    BiCGStab to 1e-10 each."""
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.adjoint import ShellFunctional
    from paper_1508_03954_amd.inputs import config_potential, shell_mask
    prob = config_potential(level_max=5)
    L = prob.level_max
    phi = torch.from_numpy(prob.phi_field()).cuda()
    s = mg.Solver(3, L, theta=prob.theta, phi=0.0, phi_field=phi, variant="bpx", omega=0.6)
    b = s.rhs_from_nodal(torch.from_numpy(prob.chi).cuda())
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    s.cycle(5, norms=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.cycle(20, norms=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms_cycle = e0.elapsed_time(e1) / 20
    del s
    cfg = {"dim": 3, "level_max": L, "theta": prob.theta, "phi0": prob.phi, "variant": "bpx", "rtol": 1e-10,
           "maxit": 3000}
    shell = torch.from_numpy(shell_mask(L, 3, 0.9, 0.95)).cuda()
    V = torch.from_numpy(prob.potential).cuda().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = ShellFunctional.apply(V, b, shell, cfg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ups = updates_per_cycle(3, L)
    log(f"[bench] potential workload: varying-phi cycle {ms_cycle * 1e3:.0f} us; forward solve {t1 - t0:.3f} s, "
        f"adjoint solve + gradient {t2 - t1:.3f} s")
    return {"workload": f"{prob.name}: d=3, levels 1..5 (244^3 complex128 vertices), k=15, phi=k^2(1+0.3i)-V(x), "
                        "V = 8 Gaussians, shell 0.9<|x|<0.95, bpx, omega=0.6",
            "varying_phi_cycle_ms": ms_cycle, "varying_phi_vertex_updates_per_s": ups / (ms_cycle * 1e-3),
            "forward_solve_s": t1 - t0, "adjoint_and_gradient_s": t2 - t1, "J": J.item(),
            "rtol": 1e-10}


def multichannel_extra(torch, level=5):
    """Same-grid multichannel form on the 3D level-5 grid (244^3): nchan
    channels with k spread over [5, 40] (phi = k^2 (1 + 0.5i)), BPX, omega
    0.6, one AoS cycle for all channels, against the same channels cycled one
    by one by single-channel contexts (fused sweep, and the generic passes the
    multichannel cycle is built from).  Reported per channel and vertex."""
    from paper_1508_03954_amd import mg
    n = 3 ** level + 1
    ups = updates_per_cycle(3, level)
    out = {"workload": f"3D levels 1..{level} ({n}^3 vertices), k in [5, 40], phi=k^2(1+0.5i), bpx, omega=0.6",
           "channels": {}}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for nchan in (1, 2, 4, 8, 16):
        ks = [5.0 + 35.0 * c / max(nchan - 1, 1) for c in range(nchan)]
        phis = [k * k * (1 + 0.5j) for k in ks]
        m = mg.MultiChannel(3, level, phis, variant="bpx", omega=0.6)
        g = torch.Generator(device="cuda").manual_seed(nchan)
        b = torch.randn((n, n, n, nchan), dtype=torch.complex128, device="cuda", generator=g)
        m.set_rhs(b)
        m.set_solution(torch.zeros_like(b))
        ms = timed(lambda: m.cycle(1, norms=False), 5)
        m.close()
        del b
        torch.cuda.empty_cache()
        rec = {"ms_per_cycle": ms, "ns_per_vertex_update_per_channel": ms * 1e6 / (ups * nchan)}
        if nchan in (1, 16):
            # the same channels one by one, single-channel contexts
            for sweep in ("fused", "generic"):
                tot = 0.0
                for ph in phis[: min(nchan, 4)]:
                    s = mg.Solver(3, level, phi=ph, variant="bpx", omega=0.6, sweep=sweep)
                    bb = torch.randn((n, n, n), dtype=torch.complex128, device="cuda")
                    s.set_rhs(bb)
                    s.set_solution(torch.zeros_like(bb))
                    tot += timed(lambda: s.cycle(1, norms=False), 5)
                    del s, bb
                    torch.cuda.empty_cache()
                per = tot / min(nchan, 4)
                rec[f"single_channel_{sweep}_ms_per_channel"] = per
        out["channels"][str(nchan)] = rec
        log(f"[bench] multichannel {nchan}: {ms:.2f} ms per cycle, "
            f"{rec['ns_per_vertex_update_per_channel']:.3f} ns per vertex update and channel")
    return out


def adapt_extra(torch, reps=10):
    """Feature-based adaptivity on the headline envelope (3D levels 1..6,
    730^3 finest): base grid 244^3; level 5 is marked (10 % refine, 2 % erase,
    20 bins, residual veto 1e-2) and adapted, then the partial level 6 is
    marked and its hanging and new vertices interpolated.  Field: four complex
    Gaussian bumps on uniform noise of size 1e-5 (small against the bumps'
    curvature, so that refinement follows the bumps), drawn on the device;
    residual: uniform noise of size 1e-4.  Marking reads u and r of every persistent vertex and the class
    byte of every vertex and writes one mark byte per vertex: 2 B per vertex
    of the envelope + 32 B per candidate is the algorithmic traffic."""
    import numpy as np
    from paper_1508_03954_amd import mg
    dim, lmin, lkeep, lmax = 3, 1, 5, 6
    a = mg.Adapt(dim, lmin, lkeep, lmax)

    def field(level, seed, scale=None):
        n = 3 ** level + 1
        g = torch.Generator(device="cuda").manual_seed(seed)
        if scale is not None:
            return torch.complex(scale * (2 * torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64) - 1),
                                 scale * (2 * torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64) - 1))
        u = torch.complex(1e-5 * torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64),
                          1e-5 * torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64))
        rng = np.random.default_rng(seed)
        x = torch.arange(n, device="cuda", dtype=torch.float64) / 3 ** level
        for _ in range(4):
            c, sig = rng.uniform(0.2, 0.8, 3), rng.uniform(0.03, 0.08)
            amp = complex(rng.uniform(-1, 1), rng.uniform(-1, 1))
            gz, gy, gx = (torch.exp(-(x - c[i]) ** 2 / (2 * sig * sig)) for i in range(3))
            u += amp * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
        return u

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"workload": "3D envelope levels 1..6 (730^3 finest), base grid 244^3, 20 bins, 10 % refine, 2 % erase, "
                       "veto 1e-2; u = 4 complex Gaussian bumps on noise 1e-5, r = noise 1e-4"}
    u5, r5 = field(5, 81), field(5, 82, 1e-4)
    ms5 = timed(lambda: a.mark(5, u5, r5, 1.0, stats=False))
    st5 = a.mark(5, u5, r5, 1.0)
    counts = a.adapt()
    n5, n6 = (3 ** 5 + 1) ** 3, (3 ** 6 + 1) ** 3
    out["level5"] = {"mark_ms": ms5, "candidates": st5["n"], "refined": st5["refined"], "erased": st5["erased"],
                     "k": st5["k"], "e": st5["e"],
                     "mark_GBs": (2 * n5 + 32 * st5["n"]) / (ms5 * 1e-3) / 1e9}
    out["level6_classes"] = dict(zip(("absent", "persistent", "hanging", "boundary"), counts[6]))
    del u5, r5
    u6, r6 = field(6, 83), field(6, 84, 1e-4)
    ms6 = timed(lambda: a.mark(6, u6, r6, 1.0, stats=False))
    st6 = a.mark(6, u6, r6, 1.0)
    out["level6"] = {"mark_ms": ms6, "candidates": st6["n"], "erased": st6["erased"],
                     "mark_GBs": (2 * n6 + 32 * st6["n"]) / (ms6 * 1e-3) / 1e9}
    del r6
    # one adaptation step of every level (cells, then classes; no new marks)
    out["adapt_ms"] = timed(lambda: a.adapt(counts=False))
    uc = field(5, 85, 1.0)
    out["interpolate_level6_ms"] = timed(lambda: a.interpolate(6, uc, u6))
    a.close()
    del u6, uc
    torch.cuda.empty_cache()
    log(f"[bench] adaptivity: mark 244^3 {ms5:.3f} ms ({out['level5']['mark_GBs']:.0f} GB/s), "
        f"mark 730^3 envelope ({st6['n']} candidates) {ms6:.3f} ms ({out['level6']['mark_GBs']:.0f} GB/s), "
        f"adapt {out['adapt_ms']:.3f} ms, interpolate 730^3 {out['interpolate_level6_ms']:.3f} ms")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--level", type=int, default=6, help="finest level of the 3D k=40 workload (default 6: 730^3)")
    ap.add_argument("--sweep", default="auto", choices=["auto", "generic", "fused"])
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle processes of the all-core CPU baseline (0: as many as cores and memory allow, "
                         "at most 8)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the 244^3 and batched workloads")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-1e-10 solves of the headline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--ramp-s", type=float, default=0.3,
                    help="seconds of untimed cycles before the warmup cycles (device clock ramp)")
    ap.add_argument("--tile", type=int, default=None, help="fixed tile variant of the fused sweep (no autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy three times (calibrates hardware byte counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 96-problem batched measurement (and the copy probe if asked) and print "
                         "its record; for counter runs of the batched kernel")
    ap.add_argument("--csg-only", action="store_true",
                    help="run only the 3D level-5 k=20 workload and print its record; for counter runs")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the potential (varying phi, adjoint) workload and print its record")
    ap.add_argument("--adapt-only", action="store_true",
                    help="run only the feature-based adaptivity measurement and print its record")
    ap.add_argument("--multichannel-only", action="store_true",
                    help="run only the same-grid multichannel measurement and print its record")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the workload is a single-GPU "
                                   "kernel; run with --gpus 1"}))
        sys.exit(2)

    # the CPU baseline runs first, before the device is touched: its worker
    # processes are forked from a process without GPU state
    cpu = None
    if not (args.no_cpu_baseline or args.batched_only or args.csg_only or args.adjoint_only or args.multichannel_only or args.adapt_only):
        log("[bench] CPU baseline: FP64 oracle on the host ...")
        cpu = cpu_baseline(args.cpu_procs)
        log(f"[bench] oracle {cpu['value']:.3e} vertex-updates/s on {cpu['cores']} processes, "
            f"{cpu['single_thread']['value']:.3e} on one")

    import torch
    from paper_1508_03954_amd import mg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mg.load_library()
    if args.batched_only or args.csg_only or args.adjoint_only or args.multichannel_only or args.adapt_only:
        if args.batched_only:
            out = {"batched": batched_extra(torch, solve=not args.no_solve)}
        elif args.csg_only:
            out = {"csg_l5": csg_extra(args, torch)}
        elif args.adjoint_only:
            out = {"potential_adjoint": adjoint_extra(torch)}
        elif args.adapt_only:
            out = {"adapt": adapt_extra(torch)}
        else:
            out = {"multichannel": multichannel_extra(torch)}
        if args.copy_probe:
            copy_probe(torch, out)
        print(json.dumps(out))
        return

    h = headline(args, torch)
    L = args.level
    out = {
        "metric": "vertex-updates/s per additive cycle",
        "value": h["value"],
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_ramp_s": args.ramp_s,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": h["workload"],
            "vertex_updates_per_cycle": h["ups"],
            "parallelism": "single GPU",
            "sweep": "fused" if args.sweep != "generic" else "generic",
            "autotune": h["tune"],
        },
        "roofline": h["roofline"],
    }
    if "time_to_1e-10" in h:
        out["time_to_1e-10"] = h["time_to_1e-10"]
    if not args.no_extras:
        out["extra_3d_k20_l5"] = csg_extra(args, torch)
        out["extra_2d_k10_latency"] = latency_extra(torch)
        out["extra_potential_adjoint"] = adjoint_extra(torch)
        out["extra_multichannel"] = multichannel_extra(torch)
        out["extra_adapt"] = adapt_extra(torch)
        out["batched"] = batched_extra(torch, solve=not args.no_solve)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.copy_probe:
        copy_probe(torch, out)
    print(json.dumps(out))


def copy_probe(torch, out):
    """A plain 1 GiB device copy, three times: the reference for the byte counters."""
    src = torch.ones(1 << 26, dtype=torch.complex128, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_probe_bytes"] = 2 * src.numel() * 16


if __name__ == "__main__":
    main()
