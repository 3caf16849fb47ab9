"""Write tests/golden/c2_prefix50.txt: the oracle's first 50 adaptive EE2 steps
of the 1024^2 workload (Fig. 4; eqs. tol_phi, LIMest, EEdt), reduced to values
a GPU test can compare with its own run: the step sequence (Krylov dimension,
accepted step, estimate, time), the field after step 50 at 4096 seeded sample
points, its norm, its sum and four seeded random projections.

Beside it, the oracle's rounding twin: the same Fig. 4 loop built from the
oracle's functions with the start vector formed as f(y^n) (eq. IVP) instead
of ghat^n - Ahat_n y^n (eq. A_g; the two are equal in exact arithmetic), so
only rounding differs.  Its accepted steps and its distance from the oracle's
field measure how strongly this workload amplifies rounding: a step shortened
by the residual-time trace at the largest Krylov dimension takes the crossing
of a residual built from the last Hessenberg column, and moves by up to ~1e-8
(relative) under a change of rounding alone.  The GPU tests take their
tolerances for those steps from it.

Third, the same workload run to the common end time T_c = t_50 of the first
run (Fig. 4 with T = T_c: the first step is clipped to T_c and the last one
lands on it), reduced the same way (lines "ct ..."): the precision form is
compared with it, at a time both forms reach exactly.

Calls only the oracle (and the seeded input generator).  About eight minutes
of CPU time:

    python tests/golden/make_c2_prefix.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ch_oracle as O  # noqa: E402
from paper_2502_14589_amd.inputs import large_2d_field  # noqa: E402

N_SIDE, EPS, TOL, M_MAX, TAU0, T_END, SEED, STEPS = 1024, 0.01, 1e-4, 30, 1e-3, 1e-3, 1, 50
SAMPLE_SEED, N_SAMPLES, N_PROJ = 1234, 4096, 4
OUT = os.path.join(HERE, "c2_prefix50.txt")


def sample_plan(N: int):
    """Sample indices and projection vectors (uniform in [-1, 1]); the GPU test draws the same."""
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(N, size=N_SAMPLES, replace=False))
    proj = rng.uniform(-1.0, 1.0, size=(N_PROJ, N))
    return idx, proj


def twin_run(y0, prob):
    """The Fig. 4 loop (no final-time clip is reached in 50 steps) with the
    start vector f(y^n); returns the accepted steps and the field."""
    t, tau, y = 0.0, TAU0, y0.copy()
    taus = []
    for _ in range(STEPS):
        assert t + tau <= T_END
        g = O.ghat(y, prob)
        v1 = O.rhs(y, prob)
        beta = float(np.linalg.norm(v1))
        tphi = O.tol_phi_rule(float(np.linalg.norm(g)), beta, TOL)
        y_new, tau_acc, _ = O.krylov_phi_cycle(lambda v: O.ahat_mv(v, y, prob), y, v1, tau, tphi, M_MAX)
        est, _ = O.pc_estimate(y, y_new, tau_acc, prob)
        t += tau_acc
        tau = O.ee_dt(tau_acc, est, TOL)
        y = y_new
        taus.append(tau_acc)
    return taus, y


def main():
    prob = O.Problem(2, N_SIDE, EPS)
    y0 = large_2d_field(SEED, N_SIDE)
    y, rec = O.ee_adaptive(y0, prob, TAU0, T_END, TOL, M_MAX, max_steps=STEPS)
    twin_taus, y_twin = twin_run(y0, prob)
    y_ct, rec_ct = O.ee_adaptive(y0, prob, TAU0, rec.t, TOL, M_MAX)
    assert rec_ct.t == rec.t
    idx, proj = sample_plan(prob.N)
    ts = np.cumsum(rec.taus)
    with open(OUT, "w") as fh:
        fh.write("# Oracle: first 50 adaptive EE2 steps of the 1024^2 workload (Fig. 4), written by\n")
        fh.write("# tests/golden/make_c2_prefix.py.  Workload: periodic [0,1]^2, n = 1024, eps = 0.01,\n")
        fh.write("# y0 = 0.1 + U(-0.05, 0.05) (seed 1), tol 1e-4, Krylov dimension 30, tau0 = T = 1e-3.\n")
        fh.write(f"t_end {rec.t!r}\n")
        fh.write(f"norm {float(np.linalg.norm(y))!r}\n")
        fh.write(f"sum {float(np.sum(y))!r}\n")
        fh.write(f"maxabs {float(np.max(np.abs(y)))!r}\n")
        fh.write(f"twin_rel_l2 {float(np.linalg.norm(y_twin - y) / np.linalg.norm(y))!r}\n")
        fh.write(f"twin_max_rel {float(np.max(np.abs(y_twin - y)) / np.max(np.abs(y)))!r}\n")
        for k in range(N_PROJ):
            fh.write(f"proj {k} {float(proj[k] @ y)!r}\n")
        # step index, Krylov dimension, accepted step, estimate, time, the twin's accepted step
        for s in range(rec.steps):
            fh.write(f"step {s} {rec.js[s]} {rec.taus[s]!r} {rec.ests[s]!r} {float(ts[s])!r} "
                     f"{twin_taus[s]!r}\n")
        for i in idx:
            fh.write(f"y {int(i)} {float(y[i])!r}\n")
        # the run to the common end time T_c = t_end
        fh.write(f"ct steps {rec_ct.steps}\n")
        fh.write(f"ct norm {float(np.linalg.norm(y_ct))!r}\n")
        fh.write(f"ct sum {float(np.sum(y_ct))!r}\n")
        fh.write(f"ct maxabs {float(np.max(np.abs(y_ct)))!r}\n")
        for k in range(N_PROJ):
            fh.write(f"ct proj {k} {float(proj[k] @ y_ct)!r}\n")
        for i in idx:
            fh.write(f"ct y {int(i)} {float(y_ct[i])!r}\n")
    print(f"wrote {OUT}: {rec.steps} steps to t = {rec.t:.6e}")


if __name__ == "__main__":
    main()
