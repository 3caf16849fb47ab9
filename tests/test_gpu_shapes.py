"""Launch shapes per grid (ch_set_shape / ch_get_shape) and the shape tuners
(ch_tune_shape for one grid, ch_tune_batch_shapes for a batch's grids together).

A shape only changes how the work of a launch is split over workgroups (and so
the order in which partial dot products are added): runs under unusual shapes
(a few workgroups looping over many strips, tiles or chunks; one column per
lane) must match the FP64 oracle to the usual 1e-10, batches must still equal
their members' solo runs bit for bit, and the tuner must keep the fastest
shape it timed.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ch_oracle as O
from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import uniform_field

TOL_FP64 = 1e-10


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture()
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


def test_shape_round_trip_and_limits(ctx):
    d = ctx.get_shape(2, 96, ch.CH_FP32_MIXED)
    assert d["vx"] in (1, 2, 4) and 96 % d["vx"] == 0 and d["wblk"] >= 1 and d["cblk"] >= 1
    ctx.set_shape(2, 96, ch.CH_FP32_MIXED, {"vx": 1, "wblk": 5, "cblk": 3})
    assert ctx.get_shape(2, 96, ch.CH_FP32_MIXED) == {"vx": 1, "wblk": 5, "cblk": 3}
    assert ctx.get_shape(2, 96, ch.CH_FP64) != {"vx": 1, "wblk": 5, "cblk": 3}   # per precision
    ctx.set_shape(2, 96, ch.CH_FP32_MIXED, None)
    assert ctx.get_shape(2, 96, ch.CH_FP32_MIXED) == d
    bad = [(2, 96, ch.CH_FP64, {"vx": 4, "wblk": 1, "cblk": 1}),    # FP64 strips take 1 or 2 columns
           (2, 98, ch.CH_FP32_MIXED, {"vx": 4, "wblk": 1, "cblk": 1}),   # 4 does not divide 98
           (2, 96, ch.CH_FP64, {"vx": 3, "wblk": 1, "cblk": 1}),
           (2, 96, ch.CH_FP64, {"vx": 2, "wblk": 0, "cblk": 1}),
           (2, 96, ch.CH_FP64, {"vx": 2, "wblk": 2049, "cblk": 1}),
           (3, 32, ch.CH_FP64, {"vx": 1, "wblk": 4, "cblk": 513}),
           (2, 4, ch.CH_FP64, {"vx": 1, "wblk": 1, "cblk": 1})]
    for dim, n, prec, s in bad:
        with pytest.raises(ch.ChError):
            ctx.set_shape(dim, n, prec, s)


def test_built_in_workgroup_counts(ctx):
    """The built-in counts: 2-D one workgroup per four strips (1024^2: 2560
    strips in FP32, 4608 in FP64), 512 once that exceeds 2048 (2048^2); 3-D
    one per work item, with FP32 runs sized to fill whole rounds of 768
    co-resident workgroups while the items at 16-plane runs fit 2048 (256^3:
    runs of 22, 768 items; 210^3: runs of 17, 728 items), else 16-plane runs
    capped at 2048 (384^3); FP64 16-plane runs (256^3: 2048 items)."""
    F32, F64 = ch.CH_FP32_MIXED, ch.CH_FP64
    for dim, n, prec, w in ((2, 1024, F32, 640), (2, 1024, F64, 1152), (2, 2048, F32, 512), (2, 2048, F64, 512),
                            (3, 256, F32, 768), (3, 210, F32, 728), (3, 384, F32, 2048), (3, 256, F64, 2048),
                            (3, 24, F32, 4)):
        assert ctx.get_shape(dim, n, prec)["wblk"] == w, (dim, n, prec)


@pytest.mark.parametrize("prec,shape", [(ch.CH_FP64, {"vx": 1, "wblk": 3, "cblk": 1}),
                                        (ch.CH_FP64, {"vx": 2, "wblk": 1, "cblk": 2}),
                                        (ch.CH_FP32_MIXED, {"vx": 1, "wblk": 2, "cblk": 1}),
                                        (ch.CH_FP32_MIXED, {"vx": 2, "wblk": 7, "cblk": 4})])
def test_ee_and_lim_under_unusual_2d_shapes(ctx, prec, shape):
    say(f"2-D shape {shape} prec={prec}")
    n = 96
    po = O.Problem(2, n, 0.03)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=7300)
    ctx.set_shape(2, n, prec, shape)
    y_ref, rec = O.ee_adaptive(y0, po, 1e-5, np.inf, 1e-4, 30, max_steps=6)
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(2, n, 0.03, precision=prec), yg, 1e-5, max_steps=6, m_max=30, records=True)
    tol = TOL_FP64 if prec == ch.CH_FP64 else 1e-5
    assert rel(yg.cpu().numpy(), y_ref) <= tol
    if prec == ch.CH_FP64:
        assert [r["j"] for r in recs] == rec.js
        # LIM takes the FP64 shape of the grid: strips, two-stage launches, estimate
        y_lim, rl = O.lim_adaptive(y0, po, 1e-6, np.inf, 1e-4, max_steps=5)
        yg = dev(y0)
        st, recs = ctx.run_lim(ch.Problem(2, n, 0.03), yg, 1e-6, max_steps=5, tol=1e-4, records=True)
        assert [r["j"] for r in recs] == rl.js
        assert rel(yg.cpu().numpy(), y_lim) <= TOL_FP64


def test_ee_under_a_3d_shape(ctx):
    n = 24
    po = O.Problem(3, n, 0.05)
    y0 = uniform_field(n, 3, 0.0, 0.05, seed=7400)
    ctx.set_shape(3, n, ch.CH_FP64, {"vx": 1, "wblk": 2, "cblk": 1})
    y_ref, rec = O.ee_adaptive(y0, po, 1e-4, np.inf, 1e-4, 30, max_steps=4)
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(3, n, 0.05), yg, 1e-4, max_steps=4, m_max=30, records=True)
    assert [r["j"] for r in recs] == rec.js
    assert rel(yg.cpu().numpy(), y_ref) <= TOL_FP64


def test_batch_equals_solo_runs_under_set_shapes(ctx):
    """Each member's shape follows from its own grid, so a batch still equals
    its members run one at a time, bit for bit."""
    ns = [64, 96, 64, 130]
    eps = [0.03, 0.02, 0.04, 0.02]
    ctx.set_shape(2, 96, ch.CH_FP64, {"vx": 1, "wblk": 4, "cblk": 2})
    ctx.set_shape(2, 130, ch.CH_FP64, {"vx": 2, "wblk": 9, "cblk": 3})
    y0s = [uniform_field(n, 2, 0.1, 0.05, seed=7500 + i) for i, n in enumerate(ns)]
    fields = [dev(y) for y in y0s]
    st, rc = ctx.run_ee_batch(fields, ns, eps, max_steps=10, tau0=1e-5)
    assert rc == 0
    for i, n in enumerate(ns):
        yg = dev(y0s[i])
        ctx.run_ee(ch.Problem(2, n, eps[i]), yg, 1e-5, max_steps=10, m_max=30)
        assert np.array_equal(yg.cpu().numpy(), fields[i].cpu().numpy()), n


@pytest.mark.parametrize("dim,n,prec", [(2, 256, ch.CH_FP32_MIXED), (2, 128, ch.CH_FP64), (3, 48, ch.CH_FP64)])
def test_tuner_keeps_the_fastest_shape(ctx, dim, n, prec):
    say(f"tune dim={dim} n={n} prec={prec}")
    prob = ch.Problem(dim, n, 0.02, precision=prec)
    shape, best_us, default_us = ctx.tune_shape(prob, m_max=30)
    assert 0.0 < best_us <= default_us
    assert ctx.get_shape(dim, n, prec) == shape
    # a run after tuning uses the tuned shape and still matches the oracle
    po = O.Problem(dim, n, 0.02)
    y0 = uniform_field(n, dim, 0.1, 0.05, seed=7600 + n)
    y_ref, rec = O.ee_adaptive(y0, po, 1e-5, np.inf, 1e-4, 30, max_steps=2)
    yg = dev(y0)
    st, recs = ctx.run_ee(prob, yg, 1e-5, max_steps=2, m_max=30, records=True)
    tol = TOL_FP64 if prec == ch.CH_FP64 else 1e-5
    assert rel(yg.cpu().numpy(), y_ref) <= tol


def test_batch_tuner_keeps_shapes_that_speed_up_the_batch(ctx):
    """The batch tuner starts from the built-in shapes and keeps only changes
    that make the batched iteration faster; the batch then still equals its
    members' solo runs bit for bit and matches the oracle."""
    ns = [64, 96, 128, 96, 64, 128]
    eps = [0.03, 0.02, 0.02, 0.04, 0.05, 0.03]
    shapes, best_us, default_us = ctx.tune_batch_shapes(ns, eps, precision=ch.CH_FP64, m_max=20)
    assert 0.0 < best_us <= default_us
    assert set(shapes) == {64, 96, 128}
    y0s = [uniform_field(n, 2, 0.1, 0.05, seed=7700 + i) for i, n in enumerate(ns)]
    fields = [dev(y) for y in y0s]
    st, rc = ctx.run_ee_batch(fields, ns, eps, max_steps=6, tau0=1e-5, m_max=20)
    assert rc == 0
    for i in (0, 2):
        yg = dev(y0s[i])
        ctx.run_ee(ch.Problem(2, ns[i], eps[i]), yg, 1e-5, max_steps=6, m_max=20)
        assert np.array_equal(yg.cpu().numpy(), fields[i].cpu().numpy())
        y_ref, _ = O.ee_adaptive(y0s[i], O.Problem(2, ns[i], eps[i]), 1e-5, np.inf, 1e-4, 20, max_steps=6)
        assert rel(fields[i].cpu().numpy(), y_ref) <= TOL_FP64
