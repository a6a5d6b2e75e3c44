#!/usr/bin/env python3
"""Benchmark of the complex additive multilevel cycle on one MI355X.

Workload (default): d = 3, levels 1..5 (243^3 finest cells, 244^3 complex128
vertices), -Lap u - k^2 u with k = 20 on the complex grid h exp(i pi/6), load =
four Gaussians plus 1e-3 complex noise, BPX, omega 0.6 on every level.  One
step = one pipelined additive cycle over the whole hierarchy (coarse descent,
fused finest sweep, coarse backtracking, residual norm).  Inputs are resident
in HBM before timing starts.

Printed JSON line (last line of stdout): vertex-updates/s per cycle (interior
vertices of all levels per cycle time), the finest sweep's achieved HBM
bandwidth against the 8 TB/s peak, the FP64 CPU oracle's rate on a bounded
sample, the hierarchical-basis variant's rate, and time to relative residual
1e-10 with the BiCGStab driver.
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


def traffic_from_profiles(tile):
    """HBM traffic of the finest sweep from the committed rocprofv3 counter
    summary, scaled by the copy-kernel calibration; None when absent, when the
    kernel sources changed since the counters were taken or when the counters
    were taken for another tile."""
    path = os.path.join(ROOT, "profiles", "fused3_traffic.json")
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


def cpu_baseline(prob, variant, cycles):
    """The FP64 oracle as it stands on the host (numpy, one BLAS thread)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    from oracle.cycle import Params
    L, dim = prob.level_max, prob.dim
    p = Params(dim=dim, level_max=L, theta=prob.theta, phi=prob.phi, variant=variant, omega=0.6)
    b = O.lumped_rhs(prob.chi, L, prob.theta)
    with threadpool_limits(1):
        pipe = O.Pipelined(p, b)
        t0 = time.perf_counter()
        for _ in range(cycles):
            pipe.cycle()
        dt = (time.perf_counter() - t0) / cycles
    return {
        "value": updates_per_cycle(dim, L) / dt,
        "unit": "vertex-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{cycles} pipelined FP64 oracle cycle(s) of the same {dim}D L={L} {variant} workload "
                  f"(full size; setup excluded), numpy with one BLAS thread; {dt:.2f} s per cycle",
    }


def batched_extra(torch):
    """96 independent problems (64 2D with finest level 3..6, 32 3D with 3..5,
    k in [5, 60], phi = k^2 (1 + 0.5i), complex64 corrections): one batched
    persistent cycle vs the same cycles launched problem by problem."""
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
    b.close()
    log(f"[bench] batched: {t_batch * 1e3:.0f} us per cycle of all 96 problems vs {t_seq * 1e3:.0f} us "
        f"problem by problem (configuration {best})")
    return {"workload": "96 problems: 64 2D (finest level 3..6) + 32 3D (3..5), k~U[5,60], phi=k^2(1+0.5i), "
                        "BPX, complex64 corrections, seeds [4, i]",
            "finest_vertices": NL, "vertex_updates_per_cycle": U,
            "batched_ms_per_cycle": t_batch, "sequential_ms_per_cycle": t_seq,
            "batched_vertex_updates_per_s": U / (t_batch * 1e-3),
            "sequential_vertex_updates_per_s": U / (t_seq * 1e-3),
            "speedup": t_seq / t_batch, "autotune": {"config": best, "us_per_config": [round(t, 1) for t in times]}}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--variant", default="bpx", choices=["add", "hb", "bpx"])
    ap.add_argument("--sweep", default="auto", choices=["auto", "generic", "fused"])
    ap.add_argument("--cpu-cycles", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the hb-variant and time-to-residual runs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--ramp-s", type=float, default=0.3,
                    help="seconds of untimed cycles before the warmup cycles (device clock ramp)")
    ap.add_argument("--tile", type=int, default=None, help="fixed tile variant of the fused sweep (no autotune)")
    ap.add_argument("--refine-level", type=int, default=0,
                    help="also solve the 3D k=40 problem at this level with complex64 refinement vs FP64 (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy three times (calibrates hardware byte counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 96-problem batched measurement (and the copy probe if asked) and print "
                         "its record; for counter runs of the batched kernel")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the workload is a single-GPU "
                                   "kernel; run with --gpus 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1508_03954_amd import mg
    from paper_1508_03954_amd.inputs import config_3d_csg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mg.load_library()
    if args.batched_only:
        out = {"batched": batched_extra(torch)}
        if args.copy_probe:
            copy_probe(torch, out)
        print(json.dumps(out))
        return
    L, dim = args.level, 3
    prob = config_3d_csg(level_max=L, variant=args.variant)
    chi = torch.from_numpy(prob.chi).cuda()

    def make(variant):
        s = mg.Solver(dim, L, theta=prob.theta, phi=prob.phi, variant=variant, omega=0.6, sweep=args.sweep)
        b = s.rhs_from_nodal(chi)
        s.set_rhs(b)
        s.set_solution(torch.zeros_like(b))
        return s, b

    s, b = make(args.variant)
    log(f"[bench] {prob.name}: {dim}D L={L} ({3 ** L + 1}^3 vertices), steps={args.steps} warmup={args.warmup}")
    tune = None
    if args.tile is not None:
        s.set_tile(args.tile)
        tune = {"tile": args.tile, "fixed": True}
    elif args.sweep != "generic" and not args.no_autotune:
        best, best_us, times = s.autotune(reps=5)
        tune = {"tile": best, "us_per_tile": [round(t, 1) for t in times]}
        log(f"[bench] autotune: tile {best} ({best_us:.1f} us); all: {', '.join(f'{t:.1f}' for t in times)}")
    ms_step, sweep_ms, nsw = time_cycles(s, args.steps, args.warmup, torch, args.ramp_s)
    ups = updates_per_cycle(dim, L)
    value = ups / (ms_step * 1e-3)
    fb = fused_bytes(dim, L, args.variant)
    achieved = fb / (sweep_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(s.tiles()[0])
    log(f"[bench] cycle {ms_step * 1e3:.1f} us, finest sweep {sweep_ms * 1e3:.1f} us ({nsw} timed), "
        f"{achieved:.0f} GB/s algorithmic")
    # residual history sanity (the stationary cycle on this indefinite problem may grow)
    s.set_rhs(b)
    s.set_solution(torch.zeros_like(b))
    rh, _ = s.cycle(3)
    log(f"[bench] residual h-norms of the first cycles: {', '.join(f'{v:.3e}' for v in rh)}")

    out = {
        "metric": "vertex-updates/s per additive cycle",
        "value": value,
        "unit": "vertex-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_ramp_s": args.ramp_s,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{prob.name}: d=3, levels 1..{L} ({3 ** L + 1}^3 complex128 vertices), k=20, "
                        f"theta=pi/6, 4 Gaussians + 1e-3 noise, {args.variant}, omega=0.6 on every level",
            "vertex_updates_per_cycle": ups,
            "parallelism": "single GPU",
            "sweep": "fused" if args.sweep != "generic" else "generic",
            "autotune": tune,
        },
        "roofline": {
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
        },
    }

    if not args.no_extras:
        other = "hb" if args.variant != "hb" else "bpx"
        s2, b2 = make(other)
        if args.sweep != "generic" and not args.no_autotune and args.tile is None:
            s2.autotune(reps=5)
        ms2, sw2, _ = time_cycles(s2, args.steps, args.warmup, torch, args.ramp_s)
        out["extra_variant"] = {"variant": other, "value": ups / (ms2 * 1e-3), "ms_per_step": ms2,
                                "sweep_us": sw2 * 1e3,
                                "sweep_GBs": fused_bytes(dim, L, other) / (sw2 * 1e-3) / 1e9}
        del s2
        # time to relative residual 1e-10: BiCGStab preconditioned by one zero-start cycle
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, its, rel, rc = s.solve(b, rtol=1e-10, maxit=2000, driver="bicgstab")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        true_rel = s.residual_norm(u, b) / s.residual_norm(torch.zeros_like(b), b)
        out["time_to_1e-10"] = {"driver": "bicgstab (preconditioner: one zero-start additive cycle)",
                                "seconds": t1 - t0, "iterations": its, "relres": rel,
                                "true_relres": true_rel, "status": rc}
        log(f"[bench] BiCGStab to 1e-10: {t1 - t0:.3f} s, {its} iterations, relres {true_rel:.2e}")
        # the same from a nested start: levels 3 and 4 solved to 1e-2 with the
        # sampled load, each from the prolonged level below (one untimed call
        # makes the coarser levels' contexts)
        s.solve_nested(chi, level_start=L - 2, coarse_rtol=1e-2, rtol=1e-10, maxit=2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, its, rel, rc = s.solve_nested(chi, level_start=L - 2, coarse_rtol=1e-2, rtol=1e-10, maxit=2000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        true_rel = s.residual_norm(u, b) / s.residual_norm(torch.zeros_like(b), b)
        out["time_to_1e-10_nested"] = {"driver": "bicgstab from the prolonged solutions of levels L-2 and L-1 "
                                                  "(each solved to 1e-2)", "seconds": t1 - t0,
                                       "finest_iterations": its, "relres": rel, "true_relres": true_rel,
                                       "status": rc}
        log(f"[bench] nested BiCGStab to 1e-10: {t1 - t0:.3f} s, {its} finest iterations, relres {true_rel:.2e}")

    if not args.no_extras:
        out["batched"] = batched_extra(torch)
    if args.refine_level:
        out["fp32_refinement"] = refine_extra(torch, args.refine_level)

    if not args.no_cpu_baseline:
        log("[bench] CPU baseline: FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(prob, args.variant, args.cpu_cycles)
        log(f"[bench] oracle {out['cpu_baseline']['value']:.3e} vertex-updates/s")

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
