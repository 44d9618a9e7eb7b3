"""Throughput of the GP-MOOD stage engine on one MI355X.

Workload (the headline configuration): 2D four-quadrant Riemann problem on
[0,1]^2 with 2048 x 2048 cells, outflow boundaries, quadrant states drawn from
PCG64 seed 1 (rho in [0.1, 2], |u|,|v| <= 1.5, p in [0.02, 2]), GP-MOOD7 with the
7->5->3->1 cascade, ell = 12 dx, HLLC, SSP-RK3, CFL 0.8.  Synthetic input.

A step is one full SSP-RK3 step: the FP64 dt max-reduction and three stages, each
with its complete MOOD cascade.  The metric is cell-updates per second per RK
stage: cells * 3 * steps / elapsed, where elapsed is wall time between two
torch.cuda.synchronize() calls around exactly `steps` steps after `warmup` steps.
The value is the FP64 path (the precision the method is stated in); the FP32 bulk
path (FP64 dt and totals) is reported beside it under "fp32".

The roofline object is for the dominant kernel (the first pass at the top order),
whose launches are bracketed by HIP events on the library's stream during the
timed region.  The kernel is bound by vector ALU work, so `achieved` is its
algorithmic flop count per launch (4.4 kflop per cell x 2048^2 cells) divided by
its mean launch time; `traffic` is the HBM bytes per launch measured with
rocprofv3 counters for the current kernel sources (null if they changed).

"configured_run" runs the configuration as specified, 500 steps from the initial
state, in both precisions, and states the FP32 error: against the FP64 run after
500 steps, and against the FP64 oracle after one step.  cpu_baseline times the
plain FP64 oracle (OpenMP over rows, all host cores) on the first two steps of the
2048^2 problem, plus a single-thread sample (512^2, two steps).

Further legs: the batched ensemble (256 four-quadrant problems of sides 128 to
1024, FP32, one HIP-graph replay per step) against the same work one problem at a
time ("batched"); a reverse-mode rollout (512^2 vortex + density bump, 200 steps,
checkpoints every 20, "adjoint"); the 384^3 3D blast (GP-MOOD5, FP32, "blast3d").

Usage: python bench.py [--gpus 1] [--steps 500] [--warmup 20] [--configured-steps 500]
                       [--batch-steps 10] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 2048
SEED = 1
CASCADE = (3, 2, 1, 0)
CFL = 0.8
ORDER_SAMPLE_STEPS = 5   # untimed steps after the timed region that sample the final-order fractions
CPU_STEPS = 2            # full SSP-RK3 steps of the oracle for the CPU baseline
CPU_1T_N = 512           # grid of the single-thread oracle sample
BATCH_N = 256            # problems of the batched ensemble
COPY_PROBE_BYTES = 512 << 20
METRIC = "cell-updates/s per RK stage (GP-MOOD7 2D, incl. cascade), % HBM peak; FP32 vs FP64"

# Algorithmic work of one cell-stage of the first pass at radius 3 (GP-MOOD7 2D),
# the method as stated: 4 faces x 4 Gauss nodes x 4 variables x 25-long dot
# products = 1600 FMA = 3200 flop, 8 HLLC solves (~90 flop + 5 div + 2 sqrt
# each), ~300 flop of Riemann-state checks, detection and update: ~4.4 kflop.
ALGO_FLOPS_PER_CELL = 4400
# What this build executes per cell with the quarter-basis form (FMA = 2 flop,
# a division or square root = 1): reconstruction 4 x (36 adds + 4 x (25 FMA + 8
# adds)) = 1072, HLLC 8 x 98 = 784, quadrature 8 x 4 FMA = 64, update 28,
# RK combination (mean over stages) 8.
EXEC_FLOPS_PER_CELL = 1956


def bytes_per_cell(esz):
    """Minimal HBM bytes per cell-stage of the first pass: read U_s (4 values),
    U^n in stages 1 and 2 (4 values, 2/3 on average), write U_out (4 values) and
    the order byte."""
    return 4 * esz + (2.0 / 3.0) * 4 * esz + 4 * esz + 1


PEAK = {"f32": 157.3e12, "f64": 78.6e12}   # published vector peaks (FP32: packed math)
PEAK_UNPACKED = 78.6e12                     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK = 8.0e12

# HBM bytes per first-pass launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (mean over the launches of 3 steps, so 1/3 stage-0 launches that read no U^n),
# scaled by the counters' reading of a 512 MiB device copy (FETCH x 2.0, WRITE x
# 1.0).  Valid for the kernel sources with this hash only; see profiles/.
TRAFFIC = {"src": "77d0b64a68d63acd", "f32": 371.6e6, "f64": 688.1e6}
KERNEL_SOURCES = ["gpmood_kernels.hip", "gpmood_device.h", "gpmood_tables.h", "gpmood_abi.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2110_08683_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def run_gpu(prec, steps, warmup, U0):
    import torch

    from paper_2110_08683_amd import GPMood
    g = GPMood(N, N, bc=(1, 1), prec=prec, cascade=CASCADE, device="cuda:0")
    g.gpm_init_state(U0)
    g.gpm_step(CFL, warmup)
    torch.cuda.synchronize()
    g.gpm_instrument(1)  # HIP events around every first pass and cascade, no extra kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.gpm_step(CFL, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ins = g.gpm_instrument_read()
    elapsed = t1 - t0
    ncell = N * N
    value = ncell * 3 * steps / elapsed
    fp_ms = ins["first_pass_ms"] / max(1, ins["first_pass_launches"])
    stages = max(1, ins["stages"])
    # final-order statistics from a few more steps, outside the timed region
    g.gpm_instrument(3)
    g.gpm_step(CFL, ORDER_SAMPLE_STEPS)
    lev_ins = g.gpm_instrument_read()
    g.gpm_instrument(0)
    lev = lev_ins["level_cells"]
    out = {
        "value": value,
        "ms_per_step": 1e3 * elapsed / steps,
        "first_pass_ms_mean": fp_ms,
        "cascade_ms_mean": ins["cascade_ms"] / stages,
        "mood_iters_mean": ins["mood_iters"] / stages,
        "final_order_fraction": [l / (ncell * max(1, lev_ins["stages"])) for l in lev[:len(CASCADE)]],
    }
    U = g.gpm_get_state()
    out["finite"] = bool((U == U).all())
    g.close()
    return out


def roofline(prec, res):
    esz = 4 if prec == "f32" else 8
    cells = N * N
    t = res["first_pass_ms_mean"] * 1e-3
    achieved = ALGO_FLOPS_PER_CELL * cells / t
    traffic = TRAFFIC.get(prec) if TRAFFIC["src"] == kernel_source_hash() else None
    return {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK[prec] / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK[prec],
        "traffic": traffic,
        "kernel": "k_first_pass<%s,R=3>" % ("float" if prec == "f32" else "double"),
        "flops_per_cell": ALGO_FLOPS_PER_CELL,
        "cells_per_launch": cells,
        "mean_launch_ms": res["first_pass_ms_mean"],
        "executed_flops_per_cell": EXEC_FLOPS_PER_CELL,
        "executed_TFLOPs": EXEC_FLOPS_PER_CELL * cells / t / 1e12,
        "frac_of_unpacked_peak": achieved / (PEAK_UNPACKED if prec == "f32" else PEAK[prec]),
        "hbm_algorithmic_GBps": bytes_per_cell(esz) * cells / t / 1e9,
        "hbm_measured_GBps": None if traffic is None else traffic / t / 1e9,
        "hbm_frac": bytes_per_cell(esz) * cells / t / HBM_PEAK,
    }


def batch_sizes():
    """256 square problems, side uniform over {128, 192, ..., 1024} (numpy PCG64, seed 1000)."""
    import numpy as np
    rng = np.random.default_rng(1000)
    return [int(x) for x in rng.choice(np.arange(128, 1025, 64), size=BATCH_N)]


def run_batch(steps, warmup):
    """The batched ensemble: every problem a four-quadrant problem with its own seed
    (1000 + k), GP-MOOD7 FP32, one HIP-graph replay per SSP-RK3 step; timed with the
    default first-pass march length and cascade threshold and again, from the same
    initial states, with the library's autotuned march lengths per size class and
    cascade threshold."""
    import torch

    import gpmood_inputs as gi
    from paper_2110_08683_amd import GPMood, GPMoodBatch
    sides = batch_sizes()
    U0s = [gi.quadrants(n, n, seed=1000 + k) for k, n in enumerate(sides)]
    timed = {}
    tune = None
    for mode in ("default", "autotuned"):
        b = GPMoodBatch([(n, n) for n in sides], bc=(1, 1), prec="f32", cascade=CASCADE, device="cuda:0")
        for k in range(len(sides)):
            b.gpm_batch_init_state(k, U0s[k])
        if mode == "autotuned":
            t0 = time.perf_counter()
            rows, gain = b.gpm_batch_autotune(CFL, reps=3)
            tail, tgain = b.gpm_batch_autotune_cascade(CFL, reps=2)
            by_side = {}
            for n, r in zip(sides, rows):
                by_side[n] = r
            tune = {"seconds": time.perf_counter() - t0, "first_pass_gain": gain,
                    "rows_per_wave_by_side": {str(n): by_side[n] for n in sorted(by_side)},
                    "cascade_threshold": tail, "stage_gain_of_threshold": tgain}
        b.gpm_batch_step(CFL, warmup, use_graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.gpm_batch_step(CFL, steps, use_graph=True)
        torch.cuda.synchronize()
        timed[mode] = time.perf_counter() - t0
        iters, _ = b.gpm_batch_status()
        b.close()
    el = timed["autotuned"]
    cells = sum(n * n for n in sides)
    # the same work one problem at a time: one single-problem context per distinct
    # side (its first problem's initial state), weighted by the side's multiplicity
    seq = 0.0
    for n in sorted(set(sides)):
        k = sides.index(n)
        g = GPMood(n, n, bc=(1, 1), prec="f32", cascade=CASCADE, device="cuda:0")
        g.gpm_init_state(U0s[k])
        g.gpm_step(CFL, warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.gpm_step(CFL, steps)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - t1) * sides.count(n)
        g.close()
    return {"value": cells * 3 * steps / el, "unit": "cell-updates/s", "problems": BATCH_N, "cells": cells,
            "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * el / steps,
            "default_tuning_value": cells * 3 * steps / timed["default"],
            "autotuned_over_default": timed["default"] / el, "autotune": tune,
            "mood_iters_last_stage_mean": float(iters.mean()),
            "one_at_a_time_value": cells * 3 * steps / seq, "speedup_vs_one_at_a_time": seq / el,
            "workload": "256 four-quadrant problems (seeds 1000+k), square sides uniform over "
                        "{128,...,1024} step 64 (seed 1000), outflow, GP-MOOD7 7-5-3-1, FP32, CFL 0.8, "
                        "one HIP-graph replay per step"}


def run_adjoint(steps, every):
    """Reverse-mode rollout: 512^2 vortex + Gaussian density bump on [0,10]^2,
    periodic, GP-MOOD7 FP32, loss = sum over the middle quarter of rho^2 dx dy,
    gradient with respect to the initial state and ell; timed with checkpoints
    every `every` steps (the backward recomputes each segment) and with the whole
    tape kept (no recomputation)."""
    import torch

    import gpmood_inputs as gi
    from paper_2110_08683_amd import GPMood
    from paper_2110_08683_amd.adjoint import rollout
    n = 512
    g = GPMood(n, n, hi=(10.0, 10.0), bc=(0, 0), prec="f32", cascade=CASCADE, device="cuda:0")
    U0 = torch.tensor(gi.vortex_bump(n, n, seed=5), dtype=torch.float32, device="cuda:0").requires_grad_(True)
    ell = torch.tensor(g.ell, dtype=torch.float64, requires_grad=True)
    a, b = n // 4, 3 * n // 4
    out = {"workload": "512^2 isentropic vortex + Gaussian density bump (seed 5) on [0,10]^2, periodic, "
                       "GP-MOOD7 FP32, CFL 0.8, loss = sum_box rho^2 dx dy", "steps": steps}
    grads = []
    for mode, ev in (("checkpointed", every), ("taped", 0)):
        # warm-up (library and allocator) on a short rollout
        UT = rollout(g, U0, 2, cfl=CFL, checkpoint_every=ev, ell=ell)
        ((UT[0, a:b, a:b].double() ** 2).sum() * (10.0 / n) ** 2).backward()
        U0.grad = None
        ell.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        UT = rollout(g, U0, steps, cfl=CFL, checkpoint_every=ev, ell=ell)
        loss = (UT[0, a:b, a:b].double() ** 2).sum() * (10.0 / n) ** 2
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        grads.append(U0.grad.detach().clone())
        out[mode] = {"checkpoint_every": ev, "forward_ms_per_step": 1e3 * (t1 - t0) / steps,
                     "backward_ms_per_step": 1e3 * (t2 - t1) / steps, "backward_over_forward": (t2 - t1) / (t1 - t0),
                     "loss": float(loss.detach()), "grad_rho0_norm": float(U0.grad[0].double().norm()),
                     "dL_dell": float(ell.grad)}
        U0.grad = None
        ell.grad = None
    out["taped_equals_checkpointed"] = bool(torch.equal(grads[0], grads[1]))
    g.close()
    return out


def run_3d(steps, warmup, n=384):
    """3D blast (GP-MOOD5, FP32 bulk, FP64 dt and totals): n^3 unit cube, outflow,
    rho = 1 +- 1% (PCG64 seed 3), p = 1e-5, p = 1e4 within 3 dx of the centre, CFL 0.3."""
    import torch

    import gpmood_inputs as gi
    from paper_2110_08683_amd import GPMood3D
    g = GPMood3D((n, n, n), bc=(1, 1, 1), prec="f32", cascade=(2, 1, 0), device="cuda:0")
    g.gpm3_init_state(gi.blast3d(n))
    t0 = g.gpm3_totals()
    g.gpm3_step(0.3, warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g.gpm3_step(0.3, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    counts, iters = g.gpm3_troubled_counts()
    tot = g.gpm3_totals()
    g.close()
    return {"value": n ** 3 * 3 * steps / el, "unit": "cell-updates/s", "cells": n ** 3, "steps": steps,
            "warmup": warmup, "ms_per_step": 1e3 * el / steps, "mood_iters_last_stage": iters,
            "final_order_fraction_last_stage": [float(x) / n ** 3 for x in counts],
            "mass_drift": float(abs(tot[0] - t0[0]) / t0[0]),
            "workload": f"3D blast {n}^3, outflow, rho 1 +- 1% (seed 3), p 1e-5 / 1e4 within 3 dx, "
                        "GP-MOOD5 5-3-1, FP32, CFL 0.3"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(U0):
    """The plain FP64 oracle on the host: the first CPU_STEPS steps of the 2048^2
    problem on all threads (the state after the first step is returned for the
    error statement), then a single-thread sample at 512^2."""
    import oracle
    import gpmood_inputs as gi
    o = oracle.Oracle(N, N, bc=(1, 1), cascade=CASCADE)
    dt1 = o.dt(U0, CFL)
    t0 = time.perf_counter()
    U1, _, _, it1 = o.run(U0, fixed_dt=dt1, nsteps=1)
    U2, _, _, it2 = o.run(U1, cfl=CFL, nsteps=CPU_STEPS - 1)
    el = time.perf_counter() - t0
    threads = oracle.num_threads()
    # single-thread sample
    n1 = CPU_1T_N
    o1 = oracle.Oracle(n1, n1, bc=(1, 1), cascade=CASCADE)
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    _, _, _, it_1t = o1.run(gi.quadrants(n1, n1, seed=SEED), cfl=CFL, nsteps=CPU_STEPS)
    el1 = time.perf_counter() - t1
    oracle.set_num_threads(threads)
    out = {"value": N * N * 3 * CPU_STEPS / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "the first %d SSP-RK3 steps (%d stages, full MOOD loops, %d evaluations in all, dt "
                     "reductions included) of the same 2048^2 four-quadrant problem, FP64, %d threads, %.1f s"
                     % (CPU_STEPS, 3 * CPU_STEPS, int(it1.sum() + it2.sum()), threads, el),
           "single_thread": {"value": n1 * n1 * 3 * CPU_STEPS / el1, "unit": "cell-updates/s", "cores": 1,
                             "sample": "the first %d steps of the %d^2 four-quadrant problem (seed %d), FP64, "
                                       "1 thread, %.1f s" % (CPU_STEPS, n1, SEED, el1)}}
    return out, U1, dt1


def field_errors(U, ref):
    """Per field: relative L1 (sum |U - ref| / sum |ref|) and relative Linf (max |U -
    ref| / max |ref|)."""
    import numpy as np
    d = np.abs(U - ref)
    return {"rel_l1": [float(d[v].sum() / max(np.abs(ref[v]).sum(), 1e-300)) for v in range(4)],
            "rel_linf": [float(d[v].max() / max(np.abs(ref[v]).max(), 1e-300)) for v in range(4)]}


def run_configured(steps, U0):
    """The configuration as specified: `steps` SSP-RK3 steps from the initial state,
    FP64 and FP32 (no warm-up: the run itself is the workload; the library's first
    launches are warmed on a separate 2-step run).  Returns each precision's rate,
    MOOD evaluations per stage and cascade time, and the FP32 error against FP64 at
    the end."""
    import torch

    from paper_2110_08683_amd import GPMood
    out, finals = {}, {}
    for prec in ("f64", "f32"):
        w = GPMood(N, N, bc=(1, 1), prec=prec, cascade=CASCADE, device="cuda:0")
        w.gpm_init_state(U0)
        w.gpm_step(CFL, 2)
        w.close()
        g = GPMood(N, N, bc=(1, 1), prec=prec, cascade=CASCADE, device="cuda:0")
        g.gpm_init_state(U0)
        g.gpm_instrument(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.gpm_step(CFL, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ins = g.gpm_instrument_read()
        stages = max(1, ins["stages"])
        finals[prec] = g.gpm_get_state()
        out[prec] = {"value": N * N * 3 * steps / el, "ms_per_step": 1e3 * el / steps,
                     "mood_iters_per_stage": ins["mood_iters"] / stages,
                     "cascade_ms_per_stage": ins["cascade_ms"] / stages,
                     "first_pass_ms": ins["first_pass_ms"] / max(1, ins["first_pass_launches"]),
                     "finite": bool((finals[prec] == finals[prec]).all())}
        g.close()
    out["fp32_over_fp64"] = out["f32"]["value"] / out["f64"]["value"]
    out["fp32_vs_fp64_after_run"] = field_errors(finals["f32"], finals["f64"])
    out["workload"] = ("2048^2 four-quadrant problem, seed 1, %d SSP-RK3 steps from the initial state, "
                       "GP-MOOD7 7-5-3-1, CFL 0.8" % steps)
    return out


def one_step(prec, U0, dt):
    """One SSP-RK3 step of the 2048^2 problem at a fixed dt on the GPU (host result)."""
    from paper_2110_08683_amd import GPMood
    g = GPMood(N, N, bc=(1, 1), prec=prec, cascade=CASCADE, device="cuda:0")
    g.gpm_init_state(U0)
    g.gpm_set_dt(dt)
    g.gpm_step(0.0, 1)
    U = g.gpm_get_state()
    g.close()
    return U


# The implosion of Sec. "The implosion problem in 2D" as the paper runs it (400^2,
# t = 2.5, SSP-RK3, CFL 0.8, ell = 12 dx), its six method variants: name, stencil,
# cascade, CSD on.
IMPLOSION_VARIANTS = [
    ("POL-MOOD3 without CSD", "poly3", (1, 0), False),
    ("GP-MOOD3 without CSD", "diamond", (1, 0), False),
    ("POL-MOOD3 with CSD", "poly3", (1, 0), True),
    ("GP-MOOD3 with CSD", "diamond", (1, 0), True),
    ("GP-MOOD5 with CSD", "diamond", (2, 1, 0), True),
    ("GP-MOOD7 with CSD", "diamond", (3, 1, 0), True),
]


def run_implosion(name, stencil, cascade, csd, prec, n=400, tend=2.5, cfl=0.8):
    """One implosion run to t = tend (the last step clipped): steps, wall time, the
    largest x <-> y asymmetry seen (max |rho - rho^T| / max rho, checked every 100
    steps and at the end), the largest fraction of cells a step ends below the top
    order, and the densest point on the diagonal (the jet)."""
    import numpy as np
    import gpmood_inputs as gi
    from paper_2110_08683_amd import GPM_CSD, GPM_FLAGS_ALL, GPMood
    flags = GPM_FLAGS_ALL if csd else GPM_FLAGS_ALL & ~GPM_CSD
    g = GPMood(n, n, hi=(0.3, 0.3), bc=(2, 2), prec=prec, cascade=cascade, flags=flags, stencil=stencil)
    g.gpm_init_state(gi.implosion(n))
    t, k, frac, asym = 0.0, 0, 0.0, 0.0
    t0 = time.time()
    while t < tend * (1.0 - 1e-14):
        dt = min(g.gpm_compute_dt(cfl), tend - t)
        g.gpm_set_dt(dt)
        g.gpm_step(0.0, 1)
        t += dt
        k += 1
        c, _ = g.gpm_troubled_counts()
        frac = max(frac, float(c[1:].sum()) / (n * n))
        if k % 100 == 0:
            U = g.gpm_get_state()
            asym = max(asym, float(np.abs(U[0] - U[0].T).max() / U[0].max()))
    wall = time.time() - t0
    U = g.gpm_get_state()
    asym = max(asym, float(np.abs(U[0] - U[0].T).max() / U[0].max()))
    tip, amb = jet_tip(U[0], 0.3 / n)
    return {"variant": name, "prec": prec, "steps": k, "t": t, "wall_s": wall,
            "asymmetry_max": asym, "lowered_fraction_max": frac,
            "rho_min": float(U[0].min()), "jet_tip_xy": tip, "ambient_rho": amb,
            "paper_jet_tip_xy": PAPER_TIP.get(name)}


# The tip of the jet's mushroom head on the diagonal at t = 2.5 as the paper states
# it in words (Sec. "The implosion problem in 2D"): x = y ~ 0.22 for GP-MOOD5 and
# GP-MOOD7, 0.18 for GP-MOOD3, 0.17 for POL-MOOD3, all with CSD.
PAPER_TIP = {"GP-MOOD7 with CSD": 0.22, "GP-MOOD5 with CSD": 0.22, "GP-MOOD3 with CSD": 0.18,
             "POL-MOOD3 with CSD": 0.17}


def jet_tip(rho, h):
    """x = y of the outer edge of the jet's mushroom head: the farthest cell on the
    diagonal, below x = y = 0.19 (the waves crossing the diagonal farther out are
    common to every variant), whose density is 0.1 below the ambient density (the
    median on the diagonal over 0.13 < x = y < 0.19, between the jet and those
    waves); the head is light gas.  Returns (tip, ambient)."""
    import numpy as np
    n = rho.shape[0]
    diag = np.diagonal(rho)
    s = (np.arange(n) + 0.5) * h
    amb = float(np.median(diag[(s > 0.13) & (s < 0.19)]))
    low = np.nonzero((diag < amb - 0.1) & (s < 0.19))[0]
    return (float(s[low.max()] + 0.5 * h) if low.size else None), amb


def implosion_line():
    out = []
    for name, stencil, cascade, csd in IMPLOSION_VARIANTS:
        r = run_implosion(name, stencil, cascade, csd, "f64")
        print(f"[bench] implosion {name} f64: {r['steps']} steps {r['wall_s']:.1f} s, "
              f"asymmetry {r['asymmetry_max']:.1e}, jet tip x=y {r['jet_tip_xy']}", file=sys.stderr, flush=True)
        out.append(r)
    name, stencil, cascade, csd = IMPLOSION_VARIANTS[-1]
    r = run_implosion(name, stencil, cascade, csd, "f32")
    print(f"[bench] implosion {name} f32: {r['steps']} steps {r['wall_s']:.1f} s, "
          f"asymmetry {r['asymmetry_max']:.1e}", file=sys.stderr, flush=True)
    out.append(r)
    return {"workload": "implosion 400^2 on [0,0.3]^2, reflecting walls, t = 2.5, SSP-RK3, CFL 0.8, ell = 12 dx",
            "data": "synthetic", "runs": out}


# The Mach 100 light jet as the paper runs it (600^2, t = 0.04, HLL, SSP-RK3,
# CFL 0.8, ell = 12 dx): GP-MOOD3, 5 and 7.
JET_VARIANTS = [("GP-MOOD3", (1, 0)), ("GP-MOOD5", (2, 1, 0)), ("GP-MOOD7", (3, 1, 0))]


def run_jet(name, cascade, prec, n=600, tend=0.04, cfl=0.8, double=False):
    """One jet run to t = tend (the last step clipped): steps, wall time, the
    largest fraction of cells a step ends below the top order, min density and
    pressure, and the largest mirror asymmetry about x = 0.75 (max |rho - rho
    mirrored| / max rho, checked every 100 steps and at the end)."""
    import numpy as np
    import gpmood_inputs as gi
    from paper_2110_08683_amd import GPMood
    slit = gi.DOUBLE_JET_SLIT if double else gi.MACH_JET_SLIT
    g = GPMood(n, n, hi=(1.5, 1.5), bc=(1, 1), prec=prec, cascade=cascade, solver="hll", slit=slit)
    g.gpm_init_state(gi.double_jet(n) if double else gi.mach_jet(n))
    t, k, frac, asym = 0.0, 0, 0.0, 0.0
    t0 = time.time()
    while t < tend * (1.0 - 1e-14):
        dt = min(g.gpm_compute_dt(cfl), tend - t)
        g.gpm_set_dt(dt)
        g.gpm_step(0.0, 1)
        t += dt
        k += 1
        c, _ = g.gpm_troubled_counts()
        frac = max(frac, float(c[1:].sum()) / (n * n))
        if k % 100 == 0:
            U = g.gpm_get_state()
            asym = max(asym, float(np.abs(U[0] - U[0][:, ::-1]).max() / U[0].max()))
    wall = time.time() - t0
    U = g.gpm_get_state()
    asym = max(asym, float(np.abs(U[0] - U[0][:, ::-1]).max() / U[0].max()))
    p = 0.4 * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0])
    return {"problem": "double Mach 800 jets" if double else "Mach 100 jet", "variant": name, "prec": prec, "steps": k, "t": t, "wall_s": wall, "lowered_fraction_max": frac,
            "rho_min": float(U[0].min()), "p_min": float(p.min()), "mirror_asymmetry_max": asym,
            "jet_head_y": float((np.nonzero((U[0] < 13.0).any(axis=1))[0].max() + 1) * 1.5 / n)}


def jet_line():
    out = []
    for name, cascade in JET_VARIANTS:
        r = run_jet(name, cascade, "f64")
        print(f"[bench] jet {name} f64: {r['steps']} steps {r['wall_s']:.1f} s, lowered <= "
              f"{100 * r['lowered_fraction_max']:.2f}%", file=sys.stderr, flush=True)
        out.append(r)
    for name, cascade in JET_VARIANTS:
        r = run_jet(name, cascade, "f64", tend=0.005, double=True)
        print(f"[bench] double jet {name} f64: {r['steps']} steps {r['wall_s']:.1f} s, lowered <= "
              f"{100 * r['lowered_fraction_max']:.2f}%", file=sys.stderr, flush=True)
        out.append(r)
    return {"workload": "Mach 100 light jet (t = 0.04) and the double Mach 800 jet collision (t = 0.005), 600^2 "
                        "on [0,1.5]^2, slits 0.7 <= x <= 0.8, HLL, SSP-RK3, CFL 0.8, ell = 12 dx",
            "data": "synthetic", "runs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 leg of the timed run")
    ap.add_argument("--configured-steps", type=int, default=500,
                    help="steps of the configured run from the initial state, both precisions (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=10,
                    help="steps of the batched-ensemble leg (0 skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=200,
                    help="steps of the reverse-mode leg (0 skips it)")
    ap.add_argument("--steps-3d", type=int, default=5, help="steps of the 3D blast leg (0 skips it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--implosion", action="store_true",
                    help="instead of the throughput line, run the paper's implosion variants (400^2 to t = 2.5)")
    ap.add_argument("--jet", action="store_true",
                    help="instead of the throughput line, run the paper's Mach 100 jet (600^2 to t = 0.04)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for {a.gpus})", file=sys.stderr)
        sys.exit(2)
    if a.implosion:
        print(json.dumps(implosion_line()), flush=True)
        return
    if a.jet:
        print(json.dumps(jet_line()), flush=True)
        return
    import gpmood_inputs as gi
    if a.copy_probe:
        import torch
        src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: 3 copies of {COPY_PROBE_BYTES} bytes", file=sys.stderr, flush=True)
        del src, dst
    U0 = gi.quadrants(N, N, seed=SEED)
    print(f"[bench] fp64 {a.steps} steps after {a.warmup} warmup", file=sys.stderr, flush=True)
    r64 = run_gpu("f64", a.steps, a.warmup, U0)
    print(f"[bench] fp64 done: {r64['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
    r32 = None
    if not a.no_fp32:
        r32 = run_gpu("f32", a.steps, a.warmup, U0)
        print(f"[bench] fp32 done: {r32['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)

    def mood(r):
        # the cascade is bound by the latency of its dependent passes (one MOOD
        # evaluation each), not by a throughput roof: its figure is the time per
        # evaluation and the share of the stage
        return {"iters_per_stage": r["mood_iters_mean"], "final_order_fraction": r["final_order_fraction"],
                "cascade_ms_per_stage": r["cascade_ms_mean"], "first_pass_ms": r["first_pass_ms_mean"],
                "cascade_us_per_evaluation": 1e3 * r["cascade_ms_mean"] / max(r["mood_iters_mean"] - 1.0, 1.0),
                "cascade_share_of_stage": r["cascade_ms_mean"] / (r["ms_per_step"] / 3.0)}

    line = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D four-quadrant Riemann problem, 2048x2048 on [0,1]^2, outflow, PCG64 seed 1, "
                               "GP-MOOD7 cascade 7-5-3-1, ell=12dx, HLLC, SSP-RK3, CFL 0.8",
                   "cells": N * N, "precision": "f64"},
        "roofline": roofline("f64", r64),
        "mood": mood(r64),
    }
    if r32 is not None:
        line["fp32"] = {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "roofline": roofline("f32", r32),
                        "mood": mood(r32), "precision": "f32 bulk, f64 dt reduction and totals"}
        line["fp32_over_fp64"] = r32["value"] / r64["value"]
    if a.configured_steps > 0:
        print(f"[bench] configured run: {a.configured_steps} steps, fp64 and fp32", file=sys.stderr, flush=True)
        line["configured_run"] = run_configured(a.configured_steps, U0)
        cr = line["configured_run"]
        print(f"[bench] configured run done: fp64 {cr['f64']['value']:.3e}, fp32 {cr['f32']['value']:.3e}",
              file=sys.stderr, flush=True)
    if a.batch_steps > 0:
        print(f"[bench] batched ensemble {a.batch_steps} steps", file=sys.stderr, flush=True)
        line["batched"] = run_batch(a.batch_steps, 2)
        print(f"[bench] batched done: {line['batched']['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
    if a.steps_3d > 0:
        print(f"[bench] 3d blast {a.steps_3d} steps", file=sys.stderr, flush=True)
        line["blast3d"] = run_3d(a.steps_3d, 1)
        print(f"[bench] 3d done: {line['blast3d']['value']:.3e} cell-updates/s", file=sys.stderr, flush=True)
    if a.adjoint_steps > 0:
        print(f"[bench] adjoint rollout {a.adjoint_steps} steps", file=sys.stderr, flush=True)
        line["adjoint"] = run_adjoint(a.adjoint_steps, 20)
        print(f"[bench] adjoint done: backward/forward {line['adjoint']['checkpointed']['backward_over_forward']:.2f} "
              f"checkpointed, {line['adjoint']['taped']['backward_over_forward']:.2f} taped",
              file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cb, U1o, dt1 = cpu_baseline(U0)
        line["cpu_baseline"] = cb
        # the error of each GPU path against the oracle after one step at the oracle's dt
        line["error_vs_oracle_one_step"] = {"f64": field_errors(one_step("f64", U0, dt1), U1o),
                                            "f32": field_errors(one_step("f32", U0, dt1), U1o),
                                            "workload": "2048^2 four-quadrant problem, seed 1, one SSP-RK3 step at "
                                                        "the oracle's CFL 0.8 dt"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
