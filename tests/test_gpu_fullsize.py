"""Parity at the full workload sizes, in the configuration bench.py times.

1024^2 (eps = 0.01, y0 = 0.1 + U(-0.05, 0.05)): the first adaptive EE2 steps
from tau0 = T = 1e-3 (the first one runs the residual-time trace from 1e-3
down to ~1e-8), element by element against the oracle; the first 50 steps
against the oracle's stored prefix (step sequence, sampled field, norm, mass,
random projections), in FP64 and, at the prefix's end time, in FP32-mixed.
3-D at the 256^3 workload's parameters (Krylov dimension 40, tol 1e-6) on
64^3, adaptive, element by element.
One LIM step of the same field (p = 33 and 66) and its first 6 adaptive LIM
steps, element by element; LIM steps on 2048^2 and 1999^2, and traced EE2
steps on 1999^2 and 127^3; a traced EE2 step and a batch on 2048^2, whose
waves loop over several strips.
256^3 (eps = 0.02): element-by-element LIM step, the 3-D start-vector stencil
at sampled points, mass conservation of a full EE2 step.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ch_oracle as O
from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import cube_3d_field, large_2d_field, uniform_field


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    c = ch.Context(0)
    yield c
    c.close()


def dev(y):
    import torch

    return torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to("cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """max |a - b| over max |b|: a single wrong halo row cannot hide in a norm."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def large_ref():
    """Oracle: first 3 adaptive EE2 steps of the 1024^2 workload (tol 1e-4, m = 30)."""
    po = O.Problem(2, 1024, 0.01)
    y0 = large_2d_field(1, 1024)
    y3, rec = O.ee_adaptive(y0, po, 1e-3, 1e-3, 1e-4, 30, max_steps=3)
    return y0, y3, rec


def test_large_2d_first_steps_fp64(ctx, large_ref):
    say("1024^2 FP64 first 3 adaptive EE2 steps")
    y0, y_ref, rec_ref = large_ref
    assert rec_ref.js[0] == 30 and rec_ref.taus[0] < 1e-6      # traced from tau0 = 1e-3
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(2, 1024, 0.01), yg, 1e-3, T=1e-3, max_steps=3, m_max=30, tol=1e-4,
                          records=True)
    assert [r["j"] for r in recs] == rec_ref.js
    np.testing.assert_allclose([r["tau"] for r in recs], rec_ref.taus, rtol=1e-10)
    y = yg.cpu().numpy()
    assert rel(y, y_ref) <= 1e-10 and max_rel(y, y_ref) <= 1e-10


def read_prefix():
    """The oracle's first 50 adaptive EE2 steps of the 1024^2 workload
    (tests/golden/make_c2_prefix.py)."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "c2_prefix50.txt")
    g = {"steps": [], "idx": [], "y": [], "proj": []}
    ct = {"idx": [], "y": [], "proj": []}   # the run to the common end time t_50
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if f[0] == "ct":
                if f[1] == "y":
                    ct["idx"].append(int(f[2]))
                    ct["y"].append(float(f[3]))
                elif f[1] == "proj":
                    ct["proj"].append(float(f[3]))
                else:
                    ct[f[1]] = float(f[2])
                continue
            if f[0] == "step":
                g["steps"].append((int(f[2]), float(f[3]), float(f[4]), float(f[5]), float(f[6])))
            elif f[0] == "y":
                g["idx"].append(int(f[1]))
                g["y"].append(float(f[2]))
            elif f[0] == "proj":
                g["proj"].append(float(f[2]))
            else:
                g[f[0]] = float(f[1])
    g["idx"] = np.array(g["idx"])
    g["y"] = np.array(g["y"])
    ct["idx"] = np.array(ct["idx"])
    ct["y"] = np.array(ct["y"])
    g["ct"] = ct
    # Conditioning of the workload, from the oracle's rounding twin: how far a
    # change of rounding alone moves the accepted steps (traced at the largest
    # Krylov dimension) and the field.  FP64 parity is held to 1e-10 or ten
    # times the twin's spread, whichever is larger.
    g["tau_spread"] = max(abs(s[4] - s[1]) / s[1] for s in g["steps"])
    g["state_tol"] = max(1e-10, 10.0 * max(g["twin_rel_l2"], g["twin_max_rel"]))
    return g


def prefix_checks(y, g, N, tol, mass_tol=1e-12):
    """Sampled values, norm, mass and the random projections of y against the
    prefix.  mass_tol: relative to sum |y| (FP64: roundoff; the FP32-mixed form
    keeps its basis orthogonal to the constant vector to FP32 rounding)."""
    import importlib.util
    import os

    spec = importlib.util.spec_from_file_location(
        "make_c2_prefix", os.path.join(os.path.dirname(__file__), "golden", "make_c2_prefix.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    idx, proj = mk.sample_plan(N)
    assert np.array_equal(idx, g["idx"])
    errs = {
        "sampled_max": float(np.max(np.abs(y[idx] - g["y"])) / g["maxabs"]),
        "norm": abs(float(np.linalg.norm(y)) - g["norm"]) / g["norm"],
        "proj": max(abs(float(proj[k] @ y) - g["proj"][k]) / (float(np.linalg.norm(proj[k])) * g["norm"])
                    for k in range(len(g["proj"]))),
    }
    say(f"prefix errors: {errs}")
    assert all(v <= tol for v in errs.values()), errs
    assert abs(float(y.sum()) - g["sum"]) <= mass_tol * float(np.abs(y).sum())
    return errs


def test_large_2d_prefix50_fp64(ctx):
    """The first 50 adaptive EE2 steps of the 1024^2 workload, FP64, against
    the oracle's stored prefix: Krylov dimensions equal; accepted steps, times
    and estimates to 1e-10 (estimates 1e-8) up to the first step the
    residual-time trace shortens, and from there to ten times the spread of the
    oracle's rounding twin (the trace's crossing at the largest Krylov
    dimension moves by up to a few 1e-8 under rounding alone); the field after
    step 50 at 4096 sampled points (max-abs), in norm and in four random
    projections to 1e-10 or ten times the twin's distance."""
    say("1024^2 FP64 first 50 adaptive EE2 steps vs the stored oracle prefix")
    g = read_prefix()
    y0 = large_2d_field(1, 1024)
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(2, 1024, 0.01), yg, 1e-3, T=1e-3, max_steps=50, m_max=30, tol=1e-4,
                          records=True)
    assert st["steps"] == 50 == len(g["steps"])
    assert [r["j"] for r in recs] == [s[0] for s in g["steps"]]
    assert max(r["j"] for r in recs) == 30 and sum(r["traced"] for r in recs) >= 10
    first = next(k for k, r in enumerate(recs) if r["traced"] and k > 0)
    cond = max(1e-10, 10.0 * g["tau_spread"])
    say(f"first traced step {first}; twin spread {g['tau_spread']:.2e}; tolerance past it {cond:.2e}")
    for k, (r, s) in enumerate(zip(recs, g["steps"])):
        tol = 1e-10 if k < first else cond
        assert abs(r["tau"] - s[1]) <= tol * s[1], (k, r["tau"], s[1])
        assert abs(r["t"] - s[3]) <= tol * s[3], (k, r["t"], s[3])
        assert abs(r["est"] - s[2]) <= max(1e-8, 3 * tol) * s[2], (k, r["est"], s[2])
    prefix_checks(yg.cpu().numpy(), g, 1024 * 1024, g["state_tol"])


def test_large_2d_prefix_fp32_mixed_at_common_time(ctx):
    """The precision form against FP64 at a common time: adaptive runs (tol
    1e-4, Krylov dimension 30) from y0 to T_c = t_50 of the prefix (Fig. 4
    with T = T_c: the first step is clipped to T_c, the last lands on it), on
    the GPU in both forms and in the oracle.  FP64 on the GPU matches the
    oracle's run to T_c (to 1e-10 or ten times the rounding twin's distance);
    the FP32-mixed state is within the stated 1e-5 of both."""
    say("1024^2 FP32-mixed vs FP64 at the prefix end time")
    g = read_prefix()
    T = g["t_end"]
    y0 = large_2d_field(1, 1024)
    out = {}
    for prec in (ch.CH_FP64, ch.CH_FP32_MIXED):
        yg = dev(y0)
        st, _ = ctx.run_ee(ch.Problem(2, 1024, 0.01, False, prec), yg, 1e-3, T=T, max_steps=100, m_max=30,
                           tol=1e-4)
        assert st["t"] == T
        out[prec] = (yg.cpu().numpy(), st)
    y64, y32 = out[ch.CH_FP64][0], out[ch.CH_FP32_MIXED][0]
    prefix_checks(y64, g["ct"], 1024 * 1024, g["state_tol"])
    errs = prefix_checks(y32, g["ct"], 1024 * 1024, 1e-5, mass_tol=1e-7)
    gap = rel(y32, y64)
    say(f"FP32-mixed vs FP64 at t = {T:.6e}: rel L2 {gap:.3e}, max {max_rel(y32, y64):.3e}, "
        f"steps {out[ch.CH_FP32_MIXED][1]['steps']} vs {out[ch.CH_FP64][1]['steps']}")
    assert gap <= 1e-5 and max_rel(y32, y64) <= 1e-5


@pytest.mark.parametrize("prec", [ch.CH_FP64, ch.CH_FP32_MIXED])
def test_cube_c3_parameters_adaptive(ctx, prec):
    """The 256^3 workload's parameters (eps 0.02, Krylov dimension 40, tol
    1e-6, tau0 1e-3, y0 = U(-0.05, 0.05) seed 2) on 64^3: five adaptive EE2
    steps.  The first is traced at dimension 40, so the phi tests of
    dimensions 32..39 run on the second stream.  FP64 against the oracle to
    1e-10 (dimensions equal, steps to 1e-10); FP32-mixed to 1e-5."""
    say(f"64^3 adaptive EE2, Krylov dimension 40, tol 1e-6, prec {prec}")
    n = 64
    po = O.Problem(3, n, 0.02)
    y0 = cube_3d_field(2, n)
    y_ref, rec_ref = O.ee_adaptive(y0, po, 1e-3, math.inf, 1e-6, 40, max_steps=5)
    assert rec_ref.js[0] == 40
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(3, n, 0.02, False, prec), yg, 1e-3, max_steps=5, m_max=40, tol=1e-6,
                          records=True)
    assert [r["j"] for r in recs] == rec_ref.js
    y = yg.cpu().numpy()
    if prec == ch.CH_FP64:
        np.testing.assert_allclose([r["tau"] for r in recs], rec_ref.taus, rtol=1e-10)
        assert rel(y, y_ref) <= 1e-10 and max_rel(y, y_ref) <= 1e-10
    else:
        np.testing.assert_allclose([r["tau"] for r in recs], rec_ref.taus, rtol=1e-4)
        say(f"FP32-mixed rel. error vs FP64 oracle: {rel(y, y_ref):.3e}")
        assert rel(y, y_ref) <= 1e-5 and max_rel(y, y_ref) <= 1e-5


def test_large_2d_fp32_mixed_accuracy(ctx):
    """FP32 basis/stencils/axpys with FP64 reductions, phi, update and estimate:
    stated error against the FP64 oracle under the same steps (constant tau,
    so only the precision differs)."""
    say("1024^2 FP32-mixed, 3 constant EE2 steps vs FP64 oracle")
    po = O.Problem(2, 1024, 0.01)
    y0 = large_2d_field(1, 1024)
    y_ref, infos = O.ee_const_run(y0, po, 1e-9, 3, 1e-8, 30)
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(2, 1024, 0.01, False, ch.CH_FP32_MIXED), yg, 1e-9, max_steps=3, m_max=30,
                          tol_phi_fixed=1e-8, constant_step=True, records=True)
    err = rel(yg.cpu().numpy(), y_ref)
    say(f"FP32-mixed rel. error vs FP64 oracle: {err:.3e}")
    assert err <= 1e-6


def test_large_2d_first_steps_fp32_mixed_adaptive(ctx, large_ref):
    """Adaptive FP32-mixed: the residual-time trace reads a small entry of
    tau phi(-tau H) e_1 built from an FP32 basis, so the accepted steps move by
    ~1e-3 relative; the run must stay within 1e-2 in time and conserve mass."""
    say("1024^2 FP32-mixed first 3 adaptive EE2 steps")
    y0, y_ref, rec_ref = large_ref
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(2, 1024, 0.01, False, ch.CH_FP32_MIXED), yg, 1e-3, T=1e-3, max_steps=3,
                          m_max=30, tol=1e-4, records=True)
    t_ref = sum(rec_ref.taus)
    assert [r["j"] for r in recs] == rec_ref.js
    assert abs(st["t"] - t_ref) <= 1e-2 * t_ref
    y = yg.cpu().numpy()
    assert abs(y.sum() - y0.sum()) <= 1e-7 * np.abs(y0).sum()


@pytest.mark.parametrize("tau", [2.5e-7, 1e-6])
def test_large_2d_lim_step_elementwise(ctx, tau):
    """One LIM step of the 1024^2 workload at the adaptive run's first step
    (tau = 2.5e-7: p = 33) and at four times it (p = 66): stage 0 alone, then
    32 or 65 launches of two stages, element by element against the oracle."""
    say(f"1024^2 LIM step tau={tau:g}")
    po, pg = O.Problem(2, 1024, 0.01), ch.Problem(2, 1024, 0.01)
    y0 = large_2d_field(1, 1024)
    y_ref, p = O.lim_step(y0, po, tau)
    assert p == {2.5e-7: 33, 1e-6: 66}[tau]
    yg = dev(y0)
    rec = ctx.step_lim(pg, yg, tau)
    assert rec["j"] == p and rec["matvecs"] == 2 * p - 1
    y = yg.cpu().numpy()
    assert rel(y, y_ref) <= 1e-10
    assert float(np.max(np.abs(y - y_ref))) <= 1e-10 * float(np.max(np.abs(y_ref)))


def test_large_2d_lim_adaptive_first_steps(ctx):
    """The first 6 adaptive LIM steps (Fig. 2) of the 1024^2 workload as the
    benchmark runs them (tol 1e-4, tau0 = 2.5e-7): orders, steps and the
    field against the oracle."""
    say("1024^2 adaptive LIM, 6 steps")
    po, pg = O.Problem(2, 1024, 0.01), ch.Problem(2, 1024, 0.01)
    y0 = large_2d_field(1, 1024)
    y_ref, rec_ref = O.lim_adaptive(y0, po, 2.5e-7, 1e-3, 1e-4, max_steps=6)
    yg = dev(y0)
    st, recs = ctx.run_lim(pg, yg, 2.5e-7, T=1e-3, max_steps=6, tol=1e-4, records=True)
    assert [r["j"] for r in recs] == rec_ref.js
    np.testing.assert_allclose([r["tau"] for r in recs], rec_ref.taus, rtol=1e-10)
    assert rel(yg.cpu().numpy(), y_ref) <= 1e-10


@pytest.mark.parametrize("n", [2048, 1999])
def test_large_2d_lim_step_wide_grids(ctx, n):
    """A LIM step of order 3 (stage 0, then two two-stage launches) on grids
    larger than the workload: 2048^2 (two FP64 values per lane) and the odd
    1999^2 (one value per lane, a ragged last strip in both directions)."""
    say(f"{n}^2 LIM step, p = 3")
    po, pg = O.Problem(2, n, 0.01), ch.Problem(2, n, 0.01)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=700 + n)
    tau = 12.0 / O.lambda_max(y0, po)
    y_ref, p = O.lim_step(y0, po, tau)
    assert p == 3
    yg = dev(y0)
    rec = ctx.step_lim(pg, yg, tau)
    assert rec["j"] == p
    assert rel(yg.cpu().numpy(), y_ref) <= 1e-10


def test_odd_wide_grid_ee_step_traced(ctx):
    """One EE2 step on the odd 1999^2 grid (one value per lane, ragged strips
    in both directions) from tau0 = 1e-8 with Krylov dimension 12: the residual
    test fails at the last dimension and the trace picks the step.  FP64 to
    the parity tolerance, FP32-mixed to 1e-5."""
    n = 1999
    say(f"{n}^2 EE2 step with trace")
    po = O.Problem(2, n, 0.01)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=2700)
    y_ref, tau_ref, info = O.ee_step(y0, po, 1e-8, 1e-8, 12)
    assert not info.converged and info.j == 12
    for prec, tol in ((ch.CH_FP64, 1e-10), (ch.CH_FP32_MIXED, 1e-5)):
        yg = dev(y0)
        rec = ctx.step_ee(ch.Problem(2, n, 0.01, False, prec), yg, 1e-8, m_max=12, tol_phi_fixed=1e-8)
        assert rec["j"] == 12 and rec["traced"] == 1
        assert rec["tau"] == pytest.approx(tau_ref, rel=1e-12 if prec == ch.CH_FP64 else 1e-5)
        y = yg.cpu().numpy()
        assert rel(y, y_ref) <= tol and max_rel(y, y_ref) <= tol


def test_wide_grid_strips_looping_per_wave(ctx):
    """2048^2 needs more than 2048 strip workgroups at one strip per wave, so
    its launches run 512 workgroups whose waves loop over 4 or 5 strips each
    (FP32-mixed, 9216 strips) or 8 or 9 (FP64, 17408 strips).  One traced EE2
    step of Krylov dimension 12 against the oracle (FP64 to the parity
    tolerance, FP32-mixed to 1e-5), and a batch holding the grid and a small
    one equal to their solo runs bit for bit."""
    n = 2048
    say(f"{n}^2 EE2 step, looping strips")
    po = O.Problem(2, n, 0.01)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=2800)
    y_ref, tau_ref, info = O.ee_step(y0, po, 1e-8, 1e-8, 12)
    assert not info.converged and info.j == 12
    for prec, tol in ((ch.CH_FP64, 1e-10), (ch.CH_FP32_MIXED, 1e-5)):
        assert ctx.get_shape(2, n, prec)["wblk"] == 512
        yg = dev(y0)
        rec = ctx.step_ee(ch.Problem(2, n, 0.01, False, prec), yg, 1e-8, m_max=12, tol_phi_fixed=1e-8)
        assert rec["j"] == 12 and rec["traced"] == 1
        assert rec["tau"] == pytest.approx(tau_ref, rel=1e-12 if prec == ch.CH_FP64 else 1e-5)
        y = yg.cpu().numpy()
        assert rel(y, y_ref) <= tol and max_rel(y, y_ref) <= tol
    y1 = uniform_field(128, 2, 0.1, 0.05, seed=2801)
    fields = [dev(y0), dev(y1)]
    st, rc = ctx.run_ee_batch(fields, [n, 128], [0.01, 0.02], precision=ch.CH_FP32_MIXED, tau0=1e-6, max_steps=2,
                              m_max=12, tol=1e-4)
    assert rc == 0 and all(s["steps"] == 2 for s in st)
    for f, y, nn, e in ((fields[0], y0, n, 0.01), (fields[1], y1, 128, 0.02)):
        yg = dev(y)
        ctx.run_ee(ch.Problem(2, nn, e, False, ch.CH_FP32_MIXED), yg, 1e-6, max_steps=2, m_max=12, tol=1e-4)
        assert np.array_equal(yg.cpu().numpy(), f.cpu().numpy()), nn


def test_odd_cube_ee_step_traced(ctx):
    """One EE2 step on the odd 127^3 grid (the marching matvec's 64 x 8 tiles
    and 16-plane runs all ragged) from tau0 = 1e-6 with Krylov dimension 12:
    traced.  FP64 to the parity tolerance, FP32-mixed to 1e-5."""
    n = 127
    say(f"{n}^3 EE2 step with trace")
    po = O.Problem(3, n, 0.02)
    y0 = uniform_field(n, 3, 0.0, 0.05, seed=3127)
    y_ref, tau_ref, info = O.ee_step(y0, po, 1e-6, 1e-8, 12)
    assert not info.converged and info.j == 12
    for prec, tol in ((ch.CH_FP64, 1e-10), (ch.CH_FP32_MIXED, 1e-5)):
        yg = dev(y0)
        rec = ctx.step_ee(ch.Problem(3, n, 0.02, False, prec), yg, 1e-6, m_max=12, tol_phi_fixed=1e-8)
        assert rec["j"] == 12 and rec["traced"] == 1
        assert rec["tau"] == pytest.approx(tau_ref, rel=1e-12 if prec == ch.CH_FP64 else 1e-5)
        y = yg.cpu().numpy()
        assert rel(y, y_ref) <= tol and max_rel(y, y_ref) <= tol


def test_cube_3d_lim_step_elementwise(ctx):
    say("256^3 LIM step")
    po, pg = O.Problem(3, 256, 0.02), ch.Problem(3, 256, 0.02)
    y0 = cube_3d_field(2, 256)
    lam = O.lambda_max(y0, po)
    tau = 3.0 / lam                      # p = 2: three stages
    y_ref, p = O.lim_step(y0, po, tau)
    assert p == 2
    yg = dev(y0)
    rec = ctx.step_lim(pg, yg, tau)
    assert rec["j"] == p
    assert rec["lambda_max"] == pytest.approx(lam, rel=1e-13)
    assert rel(yg.cpu().numpy(), y_ref) <= 1e-10


def test_cube_3d_start_vector_sampled(ctx):
    """With m_max = 1 the phi action is y + u f(y) for a scalar u: check f(y) of
    the 25-point stencil at 4096 sampled points (oracle computes them one by one)."""
    say("256^3 start vector at sampled points")
    import torch

    n, eps = 256, 0.02
    pg = ch.Problem(3, n, eps)
    y0 = cube_3d_field(2, n)
    yg = dev(y0)
    out = torch.empty_like(yg)
    ctx.phiv(pg, yg, out, 1e-9, mode=ch.CH_PHI_SHRINK, tol_phi=1.0, m_max=1)
    dy = (out - yg).cpu().numpy()
    Y = y0.reshape(n, n, n)
    h2 = 1.0 / n ** 2
    rng = np.random.default_rng(7)
    idx = rng.integers(0, n, size=(4096, 3))

    def lap_at(F, z, y, x):
        return (6 * F(z, y, x) - F(z - 1, y, x) - F(z + 1, y, x) - F(z, y - 1, x) - F(z, y + 1, x)
                - F(z, y, x - 1) - F(z, y, x + 1)) / h2

    def yv(z, y, x):
        return Y[z % n, y % n, x % n]

    def inner(z, y, x):   # F'(y) + eps^2 A y at one point (eq. IVP)
        v = yv(z, y, x)
        return v * (v * v - 1) + eps ** 2 * lap_at(yv, z, y, x)

    f = np.array([-lap_at(inner, z, y, x) for z, y, x in idx])
    g = dy.reshape(n, n, n)[idx[:, 0], idx[:, 1], idx[:, 2]]
    u = float(g @ f / (f @ f))
    assert u > 0
    assert np.max(np.abs(g - u * f)) <= 1e-9 * np.max(np.abs(u * f))


def test_cube_3d_ee_step_mass_and_determinism(ctx):
    say("256^3 EE2 step (m = 40, tol 1e-6)")
    pg = ch.Problem(3, 256, 0.02)
    y0 = cube_3d_field(2, 256)
    a, b = dev(y0), dev(y0)
    st, recs = ctx.run_ee(pg, a, 1e-3, T=math.inf, max_steps=1, m_max=40, tol=1e-6, records=True)
    ctx.run_ee(pg, b, 1e-3, T=math.inf, max_steps=1, m_max=40, tol=1e-6)
    assert st["steps"] == 1 and recs[0]["j"] == 40 and recs[0]["traced"] == 1
    ya = a.cpu().numpy()
    assert np.array_equal(ya, b.cpu().numpy())
    assert abs(ya.sum() - y0.sum()) <= 1e-12 * np.abs(y0).sum()
    assert not np.array_equal(ya, y0)


def test_largest_krylov_dimension(ctx):
    say("m_max = CH_MMAX")
    po, pg = O.Problem(2, 48, 0.05), ch.Problem(2, 48, 0.05)
    y0 = uniform_field(48, 2, 0.1, 0.05, seed=21)
    y_ref, tau_ref, info = O.ee_step(y0, po, 1e-2, 1e-9, ch.CH_MMAX)
    yg = dev(y0)
    rec = ctx.step_ee(pg, yg, 1e-2, m_max=ch.CH_MMAX, tol_phi_fixed=1e-9)
    assert rec["j"] == info.j
    assert rec["tau"] == pytest.approx(tau_ref, rel=1e-12)
    y = yg.cpu().numpy()
    assert rel(y, y_ref) <= 1e-10 and max_rel(y, y_ref) <= 1e-10


def test_cube_512_beyond_32_bit_offsets():
    """512^3 (134M points; a 41-column FP64 basis of 44 GB, element offsets
    past 2^32): two adaptive EE2 steps at Krylov dimension 40, tol 1e-6, in
    both forms on the same field.  Mass is conserved, the Krylov dimensions
    agree, and the FP32-mixed state matches the FP64 one to 1e-5."""
    import torch

    n = 512
    say("512^3 adaptive EE2, FP64 and FP32-mixed")
    g = torch.Generator(device="cuda").manual_seed(5)
    y0 = (torch.rand(n ** 3, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 0.1
    m0 = float(y0.sum())
    out = {}
    with ch.Context(0) as c:
        for prec in (ch.CH_FP64, ch.CH_FP32_MIXED):
            y = y0.clone()
            st, recs = c.run_ee(ch.Problem(3, n, 0.01, precision=prec), y, 1e-4, max_steps=2, m_max=40, tol=1e-6,
                                records=True)
            assert st["steps"] == 2 and bool(torch.isfinite(y).all())
            out[prec] = (y, [r["j"] for r in recs])
    y64, j64 = out[ch.CH_FP64]
    y32, j32 = out[ch.CH_FP32_MIXED]
    assert j64 == j32 and j64[0] == 40
    scale = float(y64.abs().sum())
    assert abs(float(y64.sum()) - m0) <= 1e-12 * scale
    assert float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64)) <= 1e-5
