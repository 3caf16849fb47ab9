#!/usr/bin/env python3
"""Throughput of adaptive EE2 steps on one MI355X.

Workload: 2-D periodic Cahn-Hilliard on [0,1]^2, 1024 x 1024 grid (h = 1/1024),
eps = 0.01, y0 = 0.1 + iid U(-0.05, 0.05) (seed 1), adaptive EE2 (Fig. 4) with
tol = 1e-4, Krylov dimension 30, tau0 = T = 1e-3.  A step is one pass of the
whole hot path: Arnoldi with modified Gram-Schmidt driven by the fused Jacobian
stencil matvec, the small-matrix phi with the residual-time trace, the solution
update and the error estimate / step controller (whose stencil also yields the
next start vector).

Forms: FP32-mixed (Krylov basis, matvecs and MGS axpys in FP32; state,
reductions, phi, update and estimate in FP64) and plain FP64.  `value` is the
FP32-mixed steps/s; the FP64 figures and the FP32-vs-FP64 state difference are
reported beside it.  The CPU baseline is the FP64 NumPy/SciPy oracle on the
first steps of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
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
HBM_PEAK_GBPS = 8000.0
METRIC = "CH time steps/s and HBM GB/s at 1024² (EE Krylov), FP32/batched vs FP64 plain"


def ee_step_bytes(j: int, w: int, wy: int, N: int, fp32: bool) -> float:
    """Algorithmic bytes of one EE2 step with Krylov dimension j (each operand vector read/written once).

    Arnoldi iteration k (0-based): matvec reads v_k, y, v_1 and writes w
    (3w + wy); MGS passes 1..k read w, v_{i-1}, v_i and write w (4w each); the
    final pass reads w, v_k and writes w (3w).  Update: reads y and j basis
    columns, writes y^{n+1} (16 + j w).  Estimate: reads y^{n+1}, y^n, f(y^n);
    writes f, v_1 (and the FP32 copy of y) (32 + w (+4)).
    """
    arn = sum((6 + 4 * k) * w + wy for k in range(j))
    return float(N) * (arn + 16 + j * w + 32 + w + (4 if fp32 else 0))


def run_form(ctx, ch, torch, y0, precision: int, steps: int, warmup: int):
    prob = ch.Problem(2, N_SIDE, EPS, False, precision)
    y = torch.from_numpy(y0.copy()).to("cuda")
    st_w, _ = ctx.run_ee(prob, y, TAU0, t0=0.0, T=T_END, max_steps=warmup, m_max=M_MAX, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, recs = ctx.run_ee(prob, y, st_w["tau_next"], t0=st_w["t"], T=T_END, max_steps=steps, m_max=M_MAX,
                          tol=TOL, records=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fp32 = precision == ch.CH_FP32_MIXED
    w, wy = (4, 4) if fp32 else (8, 8)
    N = N_SIDE * N_SIDE
    nbytes = sum(ee_step_bytes(r["j"], w, wy, N, fp32) for r in recs)
    mgs_us, mgs_bytes = ctx.time_kernel(prob, ch.CH_KERNEL_MGS, M_MAX, reps=200)
    mv_us, mv_bytes = ctx.time_kernel(prob, ch.CH_KERNEL_MATVEC, M_MAX, reps=100)
    phi_us, _ = ctx.time_kernel(prob, ch.CH_KERNEL_PHI, M_MAX, reps=20)
    return {
        "steps": st["steps"],
        "seconds": dt,
        "steps_per_s": st["steps"] / dt,
        "ms_per_step": 1000.0 * dt / max(st["steps"], 1),
        "t_end": st["t"],
        "mean_j": sum(r["j"] for r in recs) / max(len(recs), 1),
        "traced_frac": sum(r["traced"] for r in recs) / max(len(recs), 1),
        "matvecs_per_s": st["matvecs"] / dt,
        "sim_time_per_s": (st["t"] - st_w["t"]) / dt,
        "effective_GBps": nbytes / dt / 1e9,
        "mgs_us": mgs_us, "mgs_bytes": mgs_bytes,
        "matvec_us": mv_us, "matvec_bytes": mv_bytes,
        "phi_us": phi_us,
    }


def precision_gap(ctx, ch, torch, y0, steps: int = 10, tau: float = 1e-9):
    """FP32-mixed vs FP64 state after the same constant-step EE2 sequence
    (same tau, Krylov dimension and tol_phi), so only the precision differs."""
    import numpy as np

    out = {}
    for prec in (ch.CH_FP32_MIXED, ch.CH_FP64):
        y = torch.from_numpy(y0.copy()).to("cuda")
        ctx.run_ee(ch.Problem(2, N_SIDE, EPS, False, prec), y, tau, max_steps=steps, m_max=M_MAX,
                   tol_phi_fixed=1e-8, constant_step=True)
        out[prec] = y.cpu().numpy()
    a, b = out[ch.CH_FP32_MIXED], out[ch.CH_FP64]
    return {"fp32_vs_fp64_rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "compared": f"{steps} constant EE2 steps of tau={tau:g} from y0, Krylov dim {M_MAX}, tol_phi 1e-8"}


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
    return {"workload": "64 ragged 2-D periodic instances, sides {128,192,256,384,512}, eps log-uniform "
                        "[0.01,0.05], 50 adaptive EE2 steps each, FP32-mixed, Krylov dim 30, tol 1e-4",
            "instances": len(inst), "points": points, "instance_steps": total_steps, "seconds": round(dt, 4),
            "instance_steps_per_s": round(total_steps / dt, 1),
            "point_steps_per_s": round(sum(n * n * x["steps"] for n, x in zip(ns, st)) / dt, 1),
            "one_at_a_time_instance_steps_per_s": round(seq_rate, 1),
            "one_at_a_time_sample": f"{len(idx)} of {len(inst)} instances",
            "speedup_vs_one_at_a_time": round(total_steps / dt / seq_rate, 2), "status": rc}


def serving(ch, torch, count: int = 60, rate: float = 200.0):
    """Replay `count` Poisson arrivals (rate 200/s) of 2-D requests: sides
    128/256/512/1024 w.p. 0.4/0.3/0.2/0.1, eps log-uniform [0.005, 0.05],
    horizons U{10..200} adaptive EE2 steps, FP32-mixed, seed 4; fields resident
    on the device before the trace starts."""
    from paper_2502_14589_amd.inputs import request_trace

    reqs = request_trace(count, rate)
    fields = [torch.from_numpy(r.y0.copy()).to("cuda") for r in reqs]
    outs = [torch.empty_like(f) for f in fields]
    torch.cuda.synchronize()
    lat, done, tickets = {}, {}, []
    with ch.Server(0, ch.CH_FP32_MIXED, m_max=M_MAX, tol=TOL, hbm_budget=32 << 30, max_slots=128) as srv:
        t0 = time.perf_counter()
        while len(done) < count:
            now = time.perf_counter() - t0
            while len(tickets) < count and reqs[len(tickets)].arrival <= now:
                r = reqs[len(tickets)]
                tickets.append(srv.submit(fields[len(tickets)], r.n, r.eps, r.steps, tau0=TAU0))
            for k, t in enumerate(tickets):
                if k in done:
                    continue
                state, rc, st, lt = srv.poll(t, outs[k])
                if state in (ch.CH_REQ_DONE, ch.CH_REQ_FAILED):
                    done[k] = (state, st)
                    lat[k] = lt
            if now > 300:
                raise RuntimeError("serving trace did not finish")
            time.sleep(0.0005)
        makespan = time.perf_counter() - t0
    import numpy as np

    tot = np.array([lat[k][2] for k in range(count)])
    que = np.array([lat[k][0] for k in range(count)])
    steps = sum(done[k][1]["steps"] for k in range(count))
    psteps = sum(done[k][1]["steps"] * reqs[k].n ** 2 for k in range(count))
    return {"workload": f"{count} Poisson arrivals at {rate:g}/s, sides 128/256/512/1024 (0.4/0.3/0.2/0.1), "
                        "eps log-uniform [0.005,0.05], horizons U{10..200} adaptive EE2 steps, FP32-mixed",
            "requests": count, "failed": sum(1 for k in range(count) if done[k][0] != ch.CH_REQ_DONE),
            "makespan_s": round(makespan, 3), "latency_p50_s": round(float(np.percentile(tot, 50)), 4),
            "latency_p99_s": round(float(np.percentile(tot, 99)), 4),
            "queue_p50_s": round(float(np.percentile(que, 50)), 4),
            "queue_p99_s": round(float(np.percentile(que, 99)), 4),
            "request_steps_per_s": round(steps / makespan, 1), "point_steps_per_s": round(psteps / makespan, 1),
            "offered_point_steps_per_s": round(rate * float(np.mean([r.n ** 2 * r.steps for r in reqs])), 1)}


def roofline(form):
    achieved = form["mgs_bytes"] / (form["mgs_us"] * 1e-6) / 1e9
    return {"bound": "hbm", "kernel": "k_mgs (one modified Gram-Schmidt pass)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
            "bytes_per_launch": form["mgs_bytes"], "avg_launch_us": round(form["mgs_us"], 3)}


def cpu_baseline(y0, seconds: float):
    """The FP64 oracle on the first adaptive EE2 steps of the workload, one BLAS thread."""
    from threadpoolctl import threadpool_limits

    from oracle import ch_oracle as O

    prob = O.Problem(2, N_SIDE, EPS)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        steps = 0
        y, t, tau = y0.copy(), 0.0, TAU0
        while steps < 1 or (time.perf_counter() - t0 < seconds and steps < 50):
            y, rec = O.ee_adaptive(y, prob, tau, T_END - t, TOL, M_MAX, max_steps=1)
            t += rec.t
            tau = rec.taus[-1]
            tau = O.ee_dt(rec.taus[-1], rec.ests[-1], TOL)
            steps += 1
        dt = time.perf_counter() - t0
    return {"value": round(steps / dt, 5), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} adaptive EE2 steps of the 1024^2 workload from y0 (FP64 NumPy/SciPy, "
                      f"single thread), {dt:.1f} s on {platform.processor() or platform.machine()}, "
                      f"{os.cpu_count()} host cores present"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the grid would be split into "
              "slabs with 2-cell halo exchanges and scalar all-reduces per Gram-Schmidt dot); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_14589_amd import ch
    from paper_2502_14589_amd.inputs import large_2d_field

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    y0 = large_2d_field(SEED, N_SIDE)
    with ch.Context(0) as ctx:
        f32 = run_form(ctx, ch, torch, y0, ch.CH_FP32_MIXED, args.steps, args.warmup)
        f64 = run_form(ctx, ch, torch, y0, ch.CH_FP64, args.steps, args.warmup)
        acc = precision_gap(ctx, ch, torch, y0)
        batch = None if args.no_batch else batched(ctx, ch, torch)
    serve = None if args.no_batch else serving(ch, torch)
    t_rel = abs(f32["t_end"] - f64["t_end"]) / f64["t_end"]
    out = {
        "metric": METRIC,
        "value": round(f32["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2-D periodic Cahn-Hilliard 1024x1024, eps=0.01, y0=0.1+U(-0.05,0.05) seed 1, "
                               "adaptive EE2 tol=1e-4, Krylov dim 30, tau0=T=1e-3",
                   "grid": [N_SIDE, N_SIDE], "form": "FP32-mixed", "parallelism": "single GPU"},
        "hbm_GBps_effective": round(f32["effective_GBps"], 1),
        "roofline": roofline(f32),
        "fp64_plain": {"value": round(f64["steps_per_s"], 3), "ms_per_step": round(f64["ms_per_step"], 4),
                       "hbm_GBps_effective": round(f64["effective_GBps"], 1), "roofline": roofline(f64),
                       "mean_j": f64["mean_j"], "traced_frac": f64["traced_frac"],
                       "matvecs_per_s": round(f64["matvecs_per_s"], 1),
                       "sim_time_per_s": f64["sim_time_per_s"], "matvec_us": round(f64["matvec_us"], 3),
                       "phi_us": round(f64["phi_us"], 3)},
        "fp32_detail": {"mean_j": f32["mean_j"], "traced_frac": f32["traced_frac"],
                        "matvecs_per_s": round(f32["matvecs_per_s"], 1), "sim_time_per_s": f32["sim_time_per_s"],
                        "matvec_us": round(f32["matvec_us"], 3), "phi_us": round(f32["phi_us"], 3)},
        "accuracy": dict(acc, adaptive_t_rel_diff=t_rel),
        "speedup_fp32_vs_fp64": round(f32["steps_per_s"] / f64["steps_per_s"], 3),
    }
    if batch is not None:
        out["batched"] = batch
    if serve is not None:
        out["serving"] = serve
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(y0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
