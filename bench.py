#!/usr/bin/env python3
"""Throughput of adaptive EE2 steps on one MI355X.

Workload: 2-D periodic Cahn-Hilliard on [0,1]^2, 1024 x 1024 grid (h = 1/1024),
eps = 0.01, y0 = 0.1 + iid U(-0.05, 0.05) (seed 1), adaptive EE2 (Fig. 4) with
tol = 1e-4, Krylov dimension 30, tau0 = T = 1e-3, run from y0 to t = T.  A
step is one pass of the whole hot path: the Arnoldi process (DCGS2
orthogonalisation) driven by the fused Jacobian stencil matvec, the
small-matrix phi with the residual-time trace, the solution update and the
error estimate / step controller (whose stencil also yields the next start
vector).  The timed region is the whole run to T: the adaptive controller,
not --steps, fixes how many steps that is (about 15000, nearly all at the
largest Krylov dimension with a trace).

Forms: FP32-mixed (Krylov basis and stencils in FP32; state, reductions, phi,
update and estimate in FP64) and plain FP64.  `value` is the FP32-mixed steps/s;
the FP64 figures, the relative difference of the two states at T, the adaptive
LIM at the same size, the 3-D 256^3 EE2 case and the batched and served forms
are reported beside it.  The roofline figures come from back-to-back launches
of the kernel over the Arnoldi iterations of every REPLAY_EVERY-th step of the
timed run, timed by HIP events on the launching stream.  The CPU baseline is
the FP64 NumPy/SciPy oracle on the first steps of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
        W untimed warm-up steps (a throw-away run from y0), then the timed
        runs to T; K is the window of the adaptive LIM form.
    python bench.py --copy-calibration     (plain copy of known size, for the
                                            hardware-counter scale)
    python bench.py --counters             (FP32-mixed run to T, then the
                                            replay of its dominant kernel, under
                                            a symbol of its own that a profiler's
                                            kernel filter selects)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_SIDE, EPS, TOL, M_MAX, TAU0, T_END, SEED = 1024, 0.01, 1e-4, 30, 1e-3, 1e-3, 1
MAX_STEPS = 60000           # cap of the run to T (records buffer)
REPLAY_EVERY = 10           # replay the Arnoldi iterations of every 10th step
LIM_TAU0 = 2.5e-7
C3_SIDE, C3_EPS, C3_TOL, C3_M, C3_SEED = 256, 0.02, 1e-6, 40, 2
HBM_PEAK_GBPS = 8000.0
METRIC = "CH time steps/s and HBM GB/s at 1024² (EE Krylov), FP32/batched vs FP64 plain"
DOMINANT = "k_matvec_s (2-D row-strip DCGS2 Jacobian matvec with its 2j+2 basis dot products)"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dc_matvec_1024sq_fp32_traffic.md")
KERNEL_SOURCES = ("ch_strip.hip", "ch_common.h", "ch_internal.h")


def ee_step_bytes(j: int, m_max: int, w: int, N: int, fp32: bool) -> float:
    """Algorithmic bytes of one EE2 step of Krylov dimension j with DCGS2
    (each operand vector read or written once; w bytes per basis element).

    Iteration k = 0..j: matvec reads u_k, the state (FP32 copy in the mixed
    form) and q_0..q_{k-1}, and writes w when k < m_max: (k + 2 + [k < m_max]) w.
    Update pass k = 0..j-1: reads q_0..q_{k-1}, u_k, w; writes q_k, u_{k+1}:
    (k + 4) w.  Solution update: reads y and j columns, writes y^{n+1}
    (16 + j w).  Estimate: reads y^{n+1}, y^n, f(y^n); writes f, v_1 (and the
    FP32 copy of y) (32 + w (+4)).
    """
    arn = sum((k + 2 + (1 if k < m_max else 0)) * w for k in range(j + 1))
    arn += sum((k + 4) * w for k in range(j))
    return float(N) * (arn + 16 + j * w + 32 + w + (4 if fp32 else 0))


def dc_iters(recs, m_max: int):
    """Arnoldi iterations whose DCGS2 launches do work over the steps `recs`:
    matvec k = 0..j, update k = 0..j-1, phi tests 1..min(j, m_max - 1)."""
    mv, up, phi = [], [], []
    for r in recs:
        j = r["j"]
        if j == 0:
            continue
        mv += list(range(j + 1))
        up += list(range(j))
        phi += list(range(1, min(j, m_max - 1) + 1))
    return mv, up, phi


def replay(ctx, prob, kernel, m_max, iters=None, count=0):
    """Back-to-back launches of one kernel (under a symbol of its own, so a
    profiler reports them apart) over the given Arnoldi iterations or LIM
    stage count, timed by two HIP events on the launching stream."""
    us, nbytes = ctx.time_kernel(prob, kernel, m_max, iters=iters, count=count)
    n = len(iters) if iters is not None else count
    return {"launches": n, "total_us": us, "bytes": nbytes, "avg_launch_us": us / n,
            "bytes_per_launch": nbytes / n, "achieved_GBps": nbytes / (us * 1e-6) / 1e9 if us > 0 else 0.0}


def run_ee_form(ctx, ch, torch, prob, y0, tau0, T, warmup, m_max, tol, fp32, N, max_steps=MAX_STEPS,
                replay_every=REPLAY_EVERY):
    """W warm-up steps (a throw-away run from y0: allocations, code objects),
    then the timed run from y0 until t = T (or max_steps), then back-to-back
    launches of the DCGS2 kernels over the Arnoldi iterations of every
    replay_every-th step, for the per-kernel figures.  Returns the figures and
    the final state."""
    ctx.run_ee(prob, torch.from_numpy(y0.copy()).to("cuda"), tau0, T=T, max_steps=max(warmup, 1), m_max=m_max,
               tol=tol)
    y = torch.from_numpy(y0.copy()).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, recs = ctx.run_ee(prob, y, tau0, t0=0.0, T=T, max_steps=max_steps, m_max=m_max, tol=tol, records=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    w = 4 if fp32 else 8
    nbytes = sum(ee_step_bytes(r["j"], m_max, w, N, fp32) for r in recs)
    sample = recs[::replay_every]
    mv, up, phi = dc_iters(sample, m_max)
    last_j = recs[-1]["j"] if recs else 0
    kern = {"dc_matvec": replay(ctx, prob, ch.CH_KERNEL_DC_MATVEC, m_max, mv)}
    kern["dc_update"] = replay(ctx, prob, ch.CH_KERNEL_DC_UPDATE, m_max, up)
    phi = [k for k in phi if k <= last_j]
    if phi:
        kern["phi"] = replay(ctx, prob, ch.CH_KERNEL_PHI, m_max, phi)
    js = [r["j"] for r in recs]
    return {
        "steps": st["steps"], "seconds": dt, "steps_per_s": st["steps"] / dt,
        "ms_per_step": 1000.0 * dt / max(st["steps"], 1), "t_end": st["t"],
        "mean_j": sum(js) / max(len(js), 1),
        "frac_at_m_max": sum(1 for j in js if j == m_max) / max(len(js), 1),
        "traced_frac": sum(r["traced"] for r in recs) / max(len(recs), 1),
        "matvecs_per_s": st["matvecs"] / dt, "sim_time_per_s": st["t"] / dt,
        "effective_GBps": nbytes / dt / 1e9, "kernels": kern,
        "replayed_steps": f"every {replay_every}th step of the timed run ({len(sample)} steps)",
        "replay_plan": {"dc_matvec": mv},
    }, y


def lim_form(ctx, ch, torch, y0, steps, warmup):
    """Adaptive LIM (Fig. 2) on the same 1024^2 workload, FP64, tol 1e-4,
    tau0 = 2.5e-7 (= 2.5e-4 T)."""
    prob = ch.Problem(2, N_SIDE, EPS, False, ch.CH_FP64)
    y = torch.from_numpy(y0.copy()).to("cuda")
    st_w, _ = ctx.run_lim(prob, y, LIM_TAU0, T=T_END, max_steps=warmup, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, recs = ctx.run_lim(prob, y, st_w["tau_next"], t0=st_w["t"], T=T_END, max_steps=steps, tol=TOL,
                           records=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # the 2p - 1 stages of order p run as stage 0 alone, then p - 1 launches
    # of two stages each: the pair launches of the timed steps, replayed
    stage = replay(ctx, prob, ch.CH_KERNEL_LIM_STAGE2, 1, count=sum(r["j"] - 1 for r in recs))
    mean_p = sum(r["j"] for r in recs) / max(len(recs), 1)
    return {"workload": "adaptive LIM (Fig. 2), same 1024^2 field, FP64, tol 1e-4, tau0 = 2.5e-7",
            "steps_per_s": round(st["steps"] / dt, 3), "ms_per_step": round(1000.0 * dt / max(st["steps"], 1), 4),
            "mean_p": round(mean_p, 2), "matvecs_per_s": round(st["matvecs"] / dt, 1),
            "sim_time_per_s": (st["t"] - st_w["t"]) / dt,
            "stage_roofline": {"kernel": "two LIM stages per launch (read y^n and z, write the second stage)",
                               "bound": "hbm", "achieved": round(stage["achieved_GBps"], 1), "peak": HBM_PEAK_GBPS,
                               "unit": "GB/s", "frac": round(stage["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                               "avg_launch_us": round(stage["avg_launch_us"], 3),
                               "bytes_per_launch": stage["bytes_per_launch"], "launches": stage["launches"]},
            # the stage rate in the terms of the one-stage form (24 bytes per
            # point per stage): the bandwidth that form would need to match it
            "per_stage_us": round(stage["avg_launch_us"] / 2.0, 3),
            "single_stage_equivalent_GBps": round(2.0 * stage["achieved_GBps"], 1),
            "single_stage_equivalent_frac": round(2.0 * stage["achieved_GBps"] / HBM_PEAK_GBPS, 4)}


def c3_form(ctx, ch, torch, steps: int = 20, warmup: int = 1):
    """3-D periodic 256^3, eps = 0.02, y0 = U(-0.05, 0.05) (seed 2), adaptive
    EE2 with Krylov dimension 40 and tol 1e-6, tau0 = 1e-3, the 20-step
    horizon from y0: FP32-mixed and FP64.  The FP64 basis (41 x 128 MiB) is far
    larger than the 256 MB last-level cache, so its kernel figures are
    HBM-bound.  Also the roofline of one FP64 LIM stage (Fig. 1) on that field."""
    from paper_2502_14589_amd.inputs import cube_3d_field

    y0 = cube_3d_field(C3_SEED, C3_SIDE)
    N = C3_SIDE ** 3
    out = {"workload": "3-D periodic 256^3, eps 0.02, y0 = U(-0.05,0.05) seed 2, adaptive EE2, Krylov dim 40, "
                       "tol 1e-6, tau0 1e-3, 20 steps from y0"}
    for name, prec in (("fp32_mixed", ch.CH_FP32_MIXED), ("fp64", ch.CH_FP64)):
        f, _ = run_ee_form(ctx, ch, torch, ch.Problem(3, C3_SIDE, C3_EPS, False, prec), y0, 1e-3, math.inf,
                           warmup, C3_M, C3_TOL, prec == ch.CH_FP32_MIXED, N, max_steps=steps, replay_every=1)
        mv = f["kernels"]["dc_matvec"]
        up = f["kernels"]["dc_update"]
        out[name] = {"steps_per_s": round(f["steps_per_s"], 3), "ms_per_step": round(f["ms_per_step"], 3),
                     "mean_j": f["mean_j"], "traced_frac": f["traced_frac"],
                     "effective_GBps": round(f["effective_GBps"], 1),
                     "dc_matvec_GBps": round(mv["achieved_GBps"], 1), "dc_update_GBps": round(up["achieved_GBps"], 1),
                     "dc_matvec_frac": round(mv["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                     "dc_update_frac": round(up["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                     "dc_matvec_avg_launch_us": round(mv["avg_launch_us"], 3),
                     "dc_matvec_bytes_per_launch": mv["bytes_per_launch"], "dc_matvec_launches": mv["launches"]}
    # the LIM stage (Fig. 1) on the same field, FP64: a short adaptive run sets
    # up the workspace, then back-to-back stage launches are timed
    prob = ch.Problem(3, C3_SIDE, C3_EPS, False, ch.CH_FP64)
    y = torch.from_numpy(y0.copy()).to("cuda")
    ctx.run_lim(prob, y, 1e-6, max_steps=3, tol=1e-4)
    count = 40
    us, by = ctx.time_kernel(prob, ch.CH_KERNEL_LIM_STAGE, 1, count=count)
    gbps = by / us / 1e3
    out["lim_stage_fp64"] = {"kernel": "one LIM stage (read y^n and the previous stage, write the next)",
                             "bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": round(gbps / HBM_PEAK_GBPS, 4), "avg_launch_us": round(us / count, 3),
                             "bytes_per_launch": by / count, "launches": count}
    return out


def batched(ctx, ch, torch, steps: int = 50, sequential_sample: int = 8):
    """64 ragged 2-D instances (sides 128..512, eps log-uniform in [0.01, 0.05],
    mean U(-0.3, 0.3) + U(-0.05, 0.05), seed 3), each advanced `steps` adaptive
    EE2 steps (tol 1e-4, Krylov dimension 30, tau0 1e-3) in FP32-mixed, all in
    one batched run; compared with the same instances run one at a time."""
    from paper_2502_14589_amd.inputs import batch_instances

    inst = batch_instances()
    ns, eps = [it.n for it in inst], [it.eps for it in inst]
    fields = [torch.from_numpy(it.y0.copy()).to("cuda") for it in inst]
    ctx.run_ee_batch(fields[:2], ns[:2], eps[:2], precision=ch.CH_FP32_MIXED, tau0=TAU0, max_steps=2,
                     m_max=M_MAX, tol=TOL)    # warm-up (allocations, code objects)
    fields = [torch.from_numpy(it.y0.copy()).to("cuda") for it in inst]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rc = ctx.run_ee_batch(fields, ns, eps, precision=ch.CH_FP32_MIXED, tau0=TAU0, max_steps=steps,
                              m_max=M_MAX, tol=TOL)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    total_steps = sum(x["steps"] for x in st)
    points = sum(n * n for n in ns)
    # one-at-a-time reference on a sample (every 8th instance), scaled to all 64
    idx = list(range(0, len(inst), len(inst) // sequential_sample))
    seq_time, seq_steps = 0.0, 0
    for i in idx:
        y = torch.from_numpy(inst[i].y0.copy()).to("cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s1, _ = ctx.run_ee(ch.Problem(2, ns[i], eps[i], False, ch.CH_FP32_MIXED), y, TAU0, max_steps=steps,
                           m_max=M_MAX, tol=TOL)
        torch.cuda.synchronize()
        seq_time += time.perf_counter() - t1
        seq_steps += s1["steps"]
    seq_rate = seq_steps / seq_time
    # the same batch with its launch shapes tuned together (ch_tune_batch_shapes)
    t_tune = time.perf_counter()
    shapes, best_us, default_us = ctx.tune_batch_shapes(ns, eps, precision=ch.CH_FP32_MIXED, m_max=M_MAX)
    t_tune = time.perf_counter() - t_tune
    fields = [torch.from_numpy(it.y0.copy()).to("cuda") for it in inst]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_t, rc_t = ctx.run_ee_batch(fields, ns, eps, precision=ch.CH_FP32_MIXED, tau0=TAU0, max_steps=steps,
                                  m_max=M_MAX, tol=TOL)
    torch.cuda.synchronize()
    dt_t = time.perf_counter() - t0
    for n in shapes:
        ctx.set_shape(2, n, ch.CH_FP32_MIXED, None)
    return {"workload": "64 ragged 2-D periodic instances, sides {128,192,256,384,512}, eps log-uniform "
                        "[0.01,0.05], 50 adaptive EE2 steps each, FP32-mixed, Krylov dim 30, tol 1e-4",
            "instances": len(inst), "points": points, "instance_steps": total_steps, "seconds": round(dt, 4),
            "instance_steps_per_s": round(total_steps / dt, 1),
            "point_steps_per_s": round(sum(n * n * x["steps"] for n, x in zip(ns, st)) / dt, 1),
            "one_at_a_time_instance_steps_per_s": round(seq_rate, 1),
            "one_at_a_time_sample": f"{len(idx)} of {len(inst)} instances",
            "speedup_vs_one_at_a_time": round(total_steps / dt / seq_rate, 2), "status": rc,
            "tuned": {"instance_steps_per_s": round(sum(x["steps"] for x in st_t) / dt_t, 1),
                      "seconds": round(dt_t, 4), "tuning_seconds": round(t_tune, 3), "status": rc_t,
                      "shapes_by_side": shapes, "batched_iteration_us": round(best_us, 2),
                      "default_batched_iteration_us": round(default_us, 2)}}


def graph_issue(ctx, ch, torch):
    """Adaptive EE2 (FP32-mixed, Krylov dimension 30, tol 1e-4, tau0 1e-5) from
    y0 = 0.1 + U(-0.05, 0.05) at 128^2 (eps 0.02, 300 steps) and 1024^2 (eps
    0.01, 100 steps), with every kernel launched directly and with each Krylov
    cycle's iterations replayed from one captured graph (graph_chunk 31)."""
    from paper_2502_14589_amd.inputs import uniform_field

    out = {}
    for n, eps, steps in ((128, 0.02, 300), (1024, 0.01, 100)):
        prob = ch.Problem(2, n, eps, False, ch.CH_FP32_MIXED)
        y0 = torch.from_numpy(uniform_field(n, 2, 0.1, 0.05, seed=1)).to("cuda")
        res = {}
        for chunk in (0, M_MAX + 1):
            ctx.run_ee(prob, y0.clone(), 1e-5, max_steps=steps, m_max=M_MAX, tol=TOL, graph_chunk=chunk)   # warm
            rates = []
            for _ in range(2):
                y = y0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.run_ee(prob, y, 1e-5, max_steps=steps, m_max=M_MAX, tol=TOL, graph_chunk=chunk)
                torch.cuda.synchronize()
                rates.append(steps / (time.perf_counter() - t0))
            res["graphs" if chunk else "direct"] = round(max(rates), 1)
        res["graph_vs_direct"] = round(res["graphs"] / res["direct"], 3)
        out[f"{n}x{n}"] = res
    out["unit"] = "steps/s (best of two runs)"
    return out


# Constant-step LIM and EE2 runs printed in the paper's Tables 1 (no splitting;
# EE2 with Krylov dimension 100 and the tolerance in the last field) and 2
# (Eyre splitting; EE2(30) with tol 1e-2): tau -> (matvecs, error).
PAPER_TABLE1 = {
    64: {"lim": {1.0: (12960, 9.60e-2), 0.5: (18000, 1.10e-3), 0.25: (27856, 2.52e-3), 0.125: (40000, 8.34e-4),
                 0.0625: (48000, 3.20e-4)},
         "ee": {1.0: (10217, 3.24e-4, 1e-3), 0.5: (24824, 1.55e-4, 1e-5), 0.25: (39138, 3.88e-5, 1e-6),
                0.125: (63039, 9.52e-6, 1e-7)}},
    128: {"lim": {1.0: (50770, 2.90e-2), 0.5: (69908, 1.17e-2), 0.25: (99824, 5.70e-3), 0.125: (136000, 2.14e-3),
                  0.0625: (207350, 1.44e-3)},
          "ee": {1.0: (41266, 1.60e-3, 1e-3), 0.5: (92650, 3.61e-4, 1e-5), 0.25: (141148, 9.08e-5, 1e-6),
                 0.125: (210401, 2.27e-5, 1e-7)}},
}
PAPER_TABLE2 = {
    64: {"lim": {0.5: (21878, 9.93e-1), 0.25: (28000, 6.34e-1), 0.125: (40000, 5.05e-1), 0.0625: (48000, 7.47e-2),
                 0.03125: (96000, 3.85e-2)},
         "ee": {0.5: (13776, 4.84e-1), 0.25: (17391, 5.33e-1), 0.125: (16965, 6.67e-2), 0.0625: (23910, 2.41e-2),
                0.03125: (35818, 1.13e-2)}},
    128: {"lim": {0.5: (70000, 8.02e-1), 0.25: (100000, 5.65e-1), 0.125: (150444, 3.06e-2), 0.0625: (208000, 1.84e-2),
                  0.03125: (288000, 1.03e-2)},
          "ee": {0.5: (54973, 7.98e-1), 0.25: (66443, 4.58e-2), 0.125: (78237, 2.92e-2), 0.0625: (76857, 2.16e-2),
                 0.03125: (110008, 1.15e-2)}},
}
# Adaptive runs printed in Tables 3 (128^2) and 4 (192^2): (method, Krylov
# dimension or None, tol, tau0, matvecs, error); EE2 starts from tau0 = 1.
PAPER_TABLES34 = {
    128: [("lim", None, 1e-2, 1.0, 38940, 2.73e-3), ("lim", None, 1e-3, 0.5, 120476, 3.62e-4),
          ("lim", None, 1e-4, 0.25, 397133, 1.22e-4),
          ("ee", 10, 1e-2, 1.0, 42856, 9.63e-3), ("ee", 10, 1e-3, 1.0, 57100, 3.31e-3),
          ("ee", 10, 1e-4, 1.0, 110088, 7.57e-5),
          ("ee", 30, 1e-2, 1.0, 22800, 4.62e-3), ("ee", 30, 1e-3, 1.0, 44493, 7.03e-4),
          ("ee", 30, 1e-4, 1.0, 73867, 1.28e-4)],
    192: [("lim", None, 1e-2, 1.0, 85843, 1.12e-3), ("lim", None, 1e-3, 0.5, 265411, 1.82e-4),
          ("lim", None, 1e-4, 0.25, 893808, 3.79e-5),
          ("ee", 10, 1e-2, 1.0, 201460, 1.07e-3), ("ee", 10, 1e-3, 1.0, 208018, 1.04e-3),
          ("ee", 10, 1e-4, 1.0, 339418, 4.33e-4), ("ee", 10, 1e-5, 1.0, 546624, 5.35e-6),
          ("ee", 30, 1e-2, 1.0, 75053, 2.99e-3), ("ee", 30, 1e-3, 1.0, 126485, 5.35e-4),
          ("ee", 30, 1e-4, 1.0, 221243, 1.21e-5)],
}


def paper_mode(ctx, ch, torch, grids=(64, 128, 192), ref_tau=1.0 / 64):
    """The constant-step runs of Tables 1 and 2 and the adaptive runs of Tables
    3 and 4 on the paper's problem
    (Section 5.1): homogeneous Neumann conditions on the cell-centred n x n grid
    of (0, 64)^2, eps = eps_4 of the 64^2 grid (eq. eps), y0 ~ U(-0.01, 0.01)
    (seed n), T = 1000, FP64.  Errors as in eq. acc_reached, against an EE2 run
    with tau = ref_tau, Krylov dimension 100 and tol 1e-9 on the same grid
    (the paper's random initial data and reference are not published, so the
    errors compare in magnitude only; the LIM matvec counts do not depend on
    them)."""
    from paper_2502_14589_amd.inputs import paper_field

    eps4 = 4.0 / (2.0 * math.sqrt(2.0) * math.atanh(0.9))
    T = 1000.0
    out = {"workload": "Neumann (0,64)^2, eps_4, y0 ~ U(-0.01,0.01) seed n, T = 1000, FP64; constant tau (Tables 1-2), adaptive tau (Tables 3-4)",
           "reference": f"EE2 tau = {ref_tau:g}, Krylov dimension 100, tol 1e-9", "rows": []}

    def run(kind, n, eyre, tau, tol=0.0, m_max=100, adaptive=False):
        prob = ch.Problem(2, n, eps4, eyre, ch.CH_FP64, ch.CH_BC_NEUMANN, 64.0)
        y = torch.from_numpy(paper_field(n, seed=n)).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "lim":
            st, _ = ctx.run_lim(prob, y, tau, T=T, tol=tol if adaptive else 0.0, raise_on_error=not adaptive)
        else:
            st, _ = ctx.run_ee(prob, y, tau, T=T, m_max=m_max, tol=tol, constant_step=not adaptive,
                               raise_on_error=not adaptive)
        torch.cuda.synchronize()
        return y, st, time.perf_counter() - t0

    for n in grids:
        progress(f"paper mode {n}^2: reference")
        yref, _, tref = run("ee", n, False, ref_tau, tol=1e-9)
        nref = float(torch.linalg.norm(yref))
        for meth, mk, tol, tau0, mv_p, err_p in PAPER_TABLES34.get(n, []):
            y, st, sec = run(meth, n, False, tau0, tol=tol, m_max=mk or 30, adaptive=True)
            err = float(torch.linalg.norm(y - yref)) / nref
            out["rows"].append({
                "grid": n, "table": 3 if n == 128 else 4, "method": "LIM" if meth == "lim" else f"EE2({mk})",
                "adaptive": True, "tau0": tau0, "tol": tol, "status": st.get("rc"), "t_end": st["t"],
                "steps": st["steps"], "restarts": st["restarts"],
                "matvecs": st["matvecs"],
                "matvecs_less_start_vectors": st["matvecs"] - st["steps"] if meth == "ee" else None,
                "paper_matvecs": mv_p, "error": err, "paper_error": err_p, "seconds": round(sec, 3)})
        for table, eyre in ((PAPER_TABLE1, False), (PAPER_TABLE2, True)):
            if n not in table:
                continue
            for kind in ("lim", "ee"):
                for tau, printed in table[n][kind].items():
                    tol = printed[2] if (kind == "ee" and not eyre) else 1e-2
                    m_max = 30 if eyre else 100
                    y, st, sec = run(kind, n, eyre, tau, tol=tol, m_max=m_max)
                    err = float(torch.linalg.norm(y - yref)) / nref
                    out["rows"].append({
                        "grid": n, "table": 2 if eyre else 1, "method": "LIM" if kind == "lim" else f"EE2({m_max})",
                        "tau": tau, "tol": tol if kind == "ee" else None, "status": st["rc"] if "rc" in st else None,
                        "t_end": st["t"], "steps": st["steps"], "matvecs": st["matvecs"],
                        # EE2: the Krylov matvecs without each step's start vector
                        "matvecs_less_start_vectors": st["matvecs"] - st["steps"] if kind == "ee" else None,
                        "paper_matvecs": printed[0], "error": err, "paper_error": printed[1],
                        "seconds": round(sec, 3)})
        out[f"reference_seconds_{n}"] = round(tref, 3)
    return out


def serve_trace(ch, torch, reqs, label):
    """Replay one arrival trace through a server (fields resident on the
    device before it starts); returns latencies and served work."""
    import numpy as np

    count = len(reqs)
    fields = [torch.from_numpy(r.y0.copy()).to("cuda") for r in reqs]
    outs = [torch.empty_like(f) for f in fields]
    torch.cuda.synchronize()
    lat, done, tickets = {}, {}, []
    busy_from = None
    with ch.Server(0, ch.CH_FP32_MIXED, m_max=M_MAX, tol=TOL, hbm_budget=32 << 30, max_slots=128) as srv:
        t0 = time.perf_counter()
        open_ = set()
        while len(done) < count:
            now = time.perf_counter() - t0
            while len(tickets) < count and reqs[len(tickets)].arrival <= now:
                k = len(tickets)
                r = reqs[k]
                tickets.append(srv.submit(fields[k], r.n, r.eps, r.steps, tau0=TAU0))
                open_.add(k)
                if busy_from is None:
                    busy_from = time.perf_counter() - t0
            for k in list(open_):
                state, rc, st, lt = srv.poll(tickets[k], outs[k])
                if state in (ch.CH_REQ_DONE, ch.CH_REQ_FAILED):
                    done[k] = (state, st)
                    lat[k] = lt
                    open_.discard(k)
            if now > 600:
                raise RuntimeError("serving trace did not finish")
            time.sleep(0.0002)
        makespan = time.perf_counter() - t0
    tot = np.array([lat[k][2] for k in range(count)])
    que = np.array([lat[k][0] for k in range(count)])
    steps = sum(done[k][1]["steps"] for k in range(count))
    psteps = sum(done[k][1]["steps"] * reqs[k].n ** 2 for k in range(count))
    rate = count / reqs[-1].arrival
    return {"trace": label, "requests": count, "offered_rate_per_s": round(rate, 2),
            "failed": sum(1 for k in range(count) if done[k][0] != ch.CH_REQ_DONE),
            "makespan_s": round(makespan, 3), "latency_p50_s": round(float(np.percentile(tot, 50)), 4),
            "latency_p99_s": round(float(np.percentile(tot, 99)), 4),
            "queue_p50_s": round(float(np.percentile(que, 50)), 4),
            "queue_p99_s": round(float(np.percentile(que, 99)), 4),
            "request_steps_per_s": round(steps / (makespan - busy_from), 1),
            "point_steps_per_s": round(psteps / (makespan - busy_from), 1),
            "offered_point_steps_per_s": round(rate * float(np.mean([r.n ** 2 * r.steps for r in reqs])), 1)}


def serving(ch, torch, count: int = 2000, rate: float = 200.0, count_sus: int = 1000):
    """Poisson arrivals of 2-D requests: sides 128/256/512/1024 w.p.
    0.4/0.3/0.2/0.1, eps log-uniform [0.005, 0.05], horizons U{10..200}
    adaptive EE2 steps, FP32-mixed, seed 4.  First `count` arrivals at 200/s
    (the configured rate; above capacity, so the server runs saturated and
    its point-step rate is the capacity); then `count_sus` arrivals (seed 5)
    at 80% of the sustainable request rate that capacity implies, where the
    queue stays bounded."""
    import numpy as np

    from paper_2502_14589_amd.inputs import request_trace

    warm = request_trace(8, rate, seed=40)
    serve_trace(ch, torch, warm, "warm-up")
    reqs = request_trace(count, rate)
    hot = serve_trace(ch, torch, reqs, f"{count} arrivals at {rate:g}/s")
    mean_work = float(np.mean([r.n ** 2 * r.steps for r in reqs]))
    del reqs
    sustainable = hot["point_steps_per_s"] / mean_work
    sus = serve_trace(ch, torch, request_trace(count_sus, 0.8 * sustainable, seed=5),
                      f"{count_sus} arrivals at 0.8 x the sustainable rate")
    return {"workload": "Poisson arrivals, sides 128/256/512/1024 (0.4/0.3/0.2/0.1), eps log-uniform "
                        "[0.005,0.05], horizons U{10..200} adaptive EE2 steps, FP32-mixed, Krylov dim 30, tol 1e-4",
            "sustainable_rate_per_s": round(sustainable, 2), "at_200_per_s": hot, "at_0.8_sustainable": sus}


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_14589_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(bytes_per_launch: float):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, if it was taken on the current kernel sources and on the same
    replay (the same algorithmic bytes per launch, to 0.1%); else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            lines = [ln for ln in f if ":" in ln and not ln.startswith(("#", "|", " ", "`"))]
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in (ln.split(":", 1) for ln in lines)}
    if kv.get("source_sha") != kernel_source_sha():
        return None
    try:
        if abs(float(kv["replay_bytes_per_launch"]) - bytes_per_launch) > 1e-3 * bytes_per_launch:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(k, traffic=None):
    achieved = k["achieved_GBps"]
    return {"bound": "hbm", "kernel": DOMINANT, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "bytes_per_launch": round(k["bytes_per_launch"], 1), "avg_launch_us": round(k["avg_launch_us"], 3),
            "launches": k["launches"],
            "note": "back-to-back replay of the timed steps' working launches (same Arnoldi iterations), "
                    "HIP events around the sequence on the launching stream"}


def cpu_baseline(y0, seconds: float):
    """The FP64 oracle on the first adaptive EE2 steps of the workload, one BLAS thread.

    The first step runs at the largest Krylov dimension with the trace (as
    nearly every step of the run to T does); the following ones are the ramp of
    the step size.  Reported: steps/s over the sample, and the seconds of the
    first step alone."""
    from threadpoolctl import threadpool_limits

    from oracle import ch_oracle as O

    prob = O.Problem(2, N_SIDE, EPS)
    js, first = [], None
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        steps = 0
        y, t, tau = y0.copy(), 0.0, TAU0
        while steps < 1 or (time.perf_counter() - t0 < seconds and steps < 50):
            y, rec = O.ee_adaptive(y, prob, tau, T_END - t, TOL, M_MAX, max_steps=1)
            t += rec.t
            tau = O.ee_dt(rec.taus[-1], rec.ests[-1], TOL)
            steps += 1
            js.append(rec.js[-1])
            if first is None:
                first = time.perf_counter() - t0
        dt = time.perf_counter() - t0
    return {"value": round(steps / dt, 5), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "first_step_s_at_m_max": round(first, 3),
            "sample": f"first {steps} adaptive EE2 steps of the 1024^2 workload from y0 (Krylov dimensions "
                      f"{js}; the first traced at 30), FP64 NumPy/SciPy, single thread, {dt:.1f} s on "
                      f"{platform.processor() or platform.machine()}, {os.cpu_count()} host cores present"}


def copy_calibration(torch, mib: int = 256, reps: int = 10):
    """Plain device copies of a known size: the hardware counters' reading for
    them gives the scale of FETCH_SIZE / WRITE_SIZE."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 8, "read_bytes": n * 8, "write_bytes": n * 8, "launches": reps}),
          flush=True)


def progress(msg: str):
    """Progress of the long legs on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed steps of the adaptive LIM window")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--T", type=float, default=T_END, help="horizon of the timed EE2 runs (the workload: 1e-3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and served forms")
    ap.add_argument("--no-extra", action="store_true", help="skip LIM and 3-D")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--counters", action="store_true",
                    help="FP32-mixed run to T, then the replay of its dominant kernel (its own symbol)")
    ap.add_argument("--plan-out", help="--counters: write the replay's Arnoldi iterations to this file")
    ap.add_argument("--plan-in", help="--counters: skip the run to T and replay the iterations of this file "
                                      "(a counter run then sees only one warm step and the replay)")
    ap.add_argument("--only-3d", action="store_true", help="the 256^3 forms alone (profiling runs)")
    ap.add_argument("--only-lim", action="store_true", help="the adaptive LIM form alone (profiling runs)")
    ap.add_argument("--paper", action="store_true",
                    help="the runs of the paper's Tables 1-4 on its Neumann problem (a few minutes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the grid would be split into "
              "slabs with 2-cell halo exchanges and scalar all-reduces per Gram-Schmidt reduction); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch)
        return

    from paper_2502_14589_amd import ch
    from paper_2502_14589_amd.inputs import large_2d_field

    y0 = large_2d_field(SEED, N_SIDE)
    N = N_SIDE * N_SIDE
    T = args.T
    workload = (f"2-D periodic Cahn-Hilliard 1024x1024, eps=0.01, y0=0.1+U(-0.05,0.05) seed 1, adaptive EE2 "
                f"(Fig. 4) tol=1e-4, Krylov dim 30, tau0=1e-3, whole run from y0 to T={T:g}")
    if args.counters:
        # the FP32-mixed run to T; the replay of its dominant kernel runs under
        # a symbol of its own, which a counter run selects by name
        prob = ch.Problem(2, N_SIDE, EPS, False, ch.CH_FP32_MIXED)
        with ch.Context(0) as ctx:
            if args.plan_in:
                with open(args.plan_in) as fh:
                    plan = json.load(fh)
                # one step sets up the workspace the replay runs on
                ctx.run_ee(prob, torch.from_numpy(y0.copy()).to("cuda"), TAU0, T=T, max_steps=1, m_max=M_MAX,
                           tol=TOL)
                rep_mv = replay(ctx, prob, ch.CH_KERNEL_DC_MATVEC, M_MAX, plan["dc_matvec"])
                replayed = plan["replayed"]
            else:
                f, _ = run_ee_form(ctx, ch, torch, prob, y0, TAU0, T, args.warmup, M_MAX, TOL, True, N)
                rep_mv, replayed = f["kernels"]["dc_matvec"], f["replayed_steps"]
                if args.plan_out:
                    with open(args.plan_out, "w") as fh:
                        json.dump({"dc_matvec": f["replay_plan"]["dc_matvec"], "replayed": replayed}, fh)
        print(json.dumps({"mode": "counters", "kernel": DOMINANT, "source_sha": kernel_source_sha(),
                          "workload": workload, "replayed": replayed, "replay": rep_mv}), flush=True)
        return
    if args.only_3d:
        with ch.Context(0) as ctx:
            print(json.dumps({"mode": "only-3d", "c3_3d": c3_form(ctx, ch, torch)}), flush=True)
        return
    if args.paper:
        with ch.Context(0) as ctx:
            print(json.dumps({"mode": "paper", "paper": paper_mode(ctx, ch, torch)}), flush=True)
        return
    if args.only_lim:
        with ch.Context(0) as ctx:
            print(json.dumps({"mode": "only-lim", "lim": lim_form(ctx, ch, torch, y0, args.steps, args.warmup)}),
                  flush=True)
        return
    with ch.Context(0) as ctx:
        progress(f"FP32-mixed EE2 run to T={T:g}")
        f32, y32 = run_ee_form(ctx, ch, torch, ch.Problem(2, N_SIDE, EPS, False, ch.CH_FP32_MIXED), y0, TAU0, T,
                               args.warmup, M_MAX, TOL, True, N)
        progress(f"FP32-mixed: {f32['steps']} steps in {f32['seconds']:.1f} s; FP64 EE2 run to T")
        f64, y64 = run_ee_form(ctx, ch, torch, ch.Problem(2, N_SIDE, EPS, False, ch.CH_FP64), y0, TAU0, T,
                               args.warmup, M_MAX, TOL, False, N)
        progress(f"FP64: {f64['steps']} steps in {f64['seconds']:.1f} s")
        gap = float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64))
        gap_max = float((y32 - y64).abs().max() / y64.abs().max())
        lim = c3 = None
        if not args.no_extra:
            progress("adaptive LIM window")
            lim = lim_form(ctx, ch, torch, y0, args.steps, args.warmup)
            progress("3-D 256^3")
            c3 = c3_form(ctx, ch, torch)
        batch = graphs = None
        if not args.no_batch:
            progress("batched")
            batch = batched(ctx, ch, torch)
            progress("graph-issued Krylov cycles")
            graphs = graph_issue(ctx, ch, torch)
    serve = None
    if not args.no_batch:
        progress("serving")
        serve = serving(ch, torch)

    def kern_summary(f):
        return {k: {"avg_launch_us": round(v["avg_launch_us"], 3), "achieved_GBps": round(v["achieved_GBps"], 1),
                    "launches": v["launches"]} for k, v in f["kernels"].items()}

    def detail(f):
        return {"steps": f["steps"], "seconds": round(f["seconds"], 3), "t_end": f["t_end"],
                "mean_j": round(f["mean_j"], 3), "frac_at_m_max": round(f["frac_at_m_max"], 4),
                "traced_frac": round(f["traced_frac"], 4), "matvecs_per_s": round(f["matvecs_per_s"], 1),
                "sim_time_per_s": f["sim_time_per_s"], "kernels": kern_summary(f),
                "replayed": f["replayed_steps"]}

    mv32 = f32["kernels"]["dc_matvec"]
    out = {
        "metric": METRIC,
        "value": round(f32["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": f32["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload, "grid": [N_SIDE, N_SIDE], "form": "FP32-mixed",
                   "orthogonalisation": "DCGS2", "parallelism": "single GPU",
                   "timed": "the whole run from y0 to T (its step count is set by the controller, not --steps)"},
        "hbm_GBps_effective": round(f32["effective_GBps"], 1),
        "roofline": roofline(mv32, measured_traffic(mv32["bytes_per_launch"])),
        "fp32_detail": detail(f32),
        "fp64_plain": dict(detail(f64), value=round(f64["steps_per_s"], 3), ms_per_step=round(f64["ms_per_step"], 4),
                           hbm_GBps_effective=round(f64["effective_GBps"], 1),
                           roofline=roofline(f64["kernels"]["dc_matvec"])),
        "speedup_fp32_vs_fp64": round(f32["steps_per_s"] / f64["steps_per_s"], 3),
        "time_to_T_speedup_fp32_vs_fp64": round(f64["seconds"] / f32["seconds"], 3),
        "accuracy": {"fp32_vs_fp64_rel_l2_at_T": gap, "fp32_vs_fp64_max_rel_at_T": gap_max,
                     "stated_bound": 1e-5,
                     "compared": "FP32-mixed and FP64 states at the common end time T (both runs clip their last "
                                 "step onto T, Fig. 4)"},
    }
    if lim is not None:
        out["lim"] = lim
        out["c3_3d"] = c3
    if batch is not None:
        out["batched"] = batch
        out["graph_issue"] = graphs
    if serve is not None:
        out["serving"] = serve
    if not args.no_cpu_baseline:
        progress("CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(y0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
