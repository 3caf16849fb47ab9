"""DCGS2 Arnoldi iterations replayed from captured HIP graphs (ch_ee_opts.graph_chunk).

The graphs hold the same launches as direct issue, so every run must equal its
directly issued twin bit for bit: whole adaptive runs (each step replays the
cached graphs, with the step's other launches and the host's lookahead waits
between replays), FP64 and FP32-mixed, chunk sizes from one iteration to a
whole cycle, Krylov dimensions whose tests would use the second stream, the
batched driver, and direct and graph runs interleaved on one context (the
device's count of update launches must stay in step with the host's).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ch_oracle as O
from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import batch_instances, uniform_field


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


def run(ctx, prob, y0, chunk, **kw):
    yg = dev(y0)
    st, recs = ctx.run_ee(prob, yg, kw.pop("tau0", 1e-5), graph_chunk=chunk, records=True, **kw)
    return yg.cpu().numpy(), st, recs


@pytest.mark.parametrize("prec", [ch.CH_FP64, ch.CH_FP32_MIXED])
@pytest.mark.parametrize("n,m_max", [(128, 30), (200, 12)])
def test_graph_runs_equal_direct_runs(ctx, prec, n, m_max):
    say(f"graphs n={n} m_max={m_max} prec={prec}")
    prob = ch.Problem(2, n, 0.02, precision=prec)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=7000 + n)
    ref, st_ref, rec_ref = run(ctx, prob, y0, 0, max_steps=40, m_max=m_max)
    assert st_ref["steps"] == 40
    for chunk in (1, 4, m_max + 1):
        for _ in range(2):   # the second run replays graphs captured by the first
            y, st, recs = run(ctx, prob, y0, chunk, max_steps=40, m_max=m_max)
            assert np.array_equal(y, ref), chunk
            assert st["matvecs"] == st_ref["matvecs"] and st["t"] == st_ref["t"]
            assert [r["j"] for r in recs] == [r["j"] for r in rec_ref]
        # a direct run after graph runs still matches (launch counts in step)
        y, st, _ = run(ctx, prob, y0, 0, max_steps=40, m_max=m_max)
        assert np.array_equal(y, ref)


def test_graph_run_with_tests_beyond_the_update_launch(ctx):
    """m_max = 40, constant steps with linear residual-time restarts (every cycle
    reaches dimension 33 or more): the tests of dimensions 32..39 go to the
    second stream when issued directly and stay on the main stream inside the
    graphs."""
    n = 96
    prob = ch.Problem(2, n, 0.01)
    y0 = uniform_field(n, 2, 0.0, 0.05, seed=7100)
    kw = dict(max_steps=4, m_max=40, tau0=1e-3, constant_step=True, tol_phi_fixed=1e-8)
    ref, st_ref, _ = run(ctx, prob, y0, 0, **kw)
    assert st_ref["restarts"] >= 8
    for chunk in (3, 41):
        y, st, _ = run(ctx, prob, y0, chunk, **kw)
        assert np.array_equal(y, ref)
        assert st["matvecs"] == st_ref["matvecs"] and st["restarts"] == st_ref["restarts"]


def test_graph_run_matches_the_oracle(ctx):
    """A graph run against the FP64 oracle directly (5 adaptive steps)."""
    n = 64
    po = O.Problem(2, n, 0.03)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=7200)
    y_ref, rec = O.ee_adaptive(y0, po, 1e-5, np.inf, 1e-4, 30, max_steps=5)
    y, st, recs = run(ctx, ch.Problem(2, n, 0.03), y0, 5, max_steps=5, m_max=30)
    assert [r["j"] for r in recs] == rec.js
    assert np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref) <= 1e-10


def test_graph_batch_equals_direct_batch(ctx):
    """The batched driver with graphs: every instance bit-identical to direct issue."""
    insts = batch_instances(count=12, seed=3, sides=(128, 192, 256))
    outs = []
    for chunk in (0, 4, 0, 31):
        fields = [dev(it.y0) for it in insts]
        st, rc = ctx.run_ee_batch(fields, [it.n for it in insts], [it.eps for it in insts], max_steps=25,
                                  tau0=1e-5, graph_chunk=chunk)
        assert rc == 0 and all(s["steps"] == 25 for s in st)
        outs.append([f.cpu().numpy() for f in fields])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_graph_chunk_out_of_range_is_rejected(ctx):
    prob = ch.Problem(2, 64, 0.03)
    yg = dev(np.zeros(64 * 64))
    for bad in (-1, ch.CH_MMAX + 2):
        with pytest.raises(ch.ChError):
            ctx.run_ee(prob, yg, 1e-5, max_steps=1, graph_chunk=bad)


@pytest.mark.parametrize("kind", ["neumann", "mobility"])
def test_graph_runs_with_boundary_and_mobility_variants(ctx, kind):
    """The Neumann and variable-mobility kernels replayed from graphs equal
    their direct issue bit for bit (the graph key holds the instance record)."""
    n = 96
    if kind == "neumann":
        prob = ch.Problem(2, n, 0.05, bc=ch.CH_BC_NEUMANN, length=2.0)
    else:
        prob = ch.Problem(2, n, 0.02, mobility=(0.2, 1.0))
    y0 = uniform_field(n, 2, 0.1, 0.3, seed=7800)
    ref, st_ref, rec_ref = run(ctx, prob, y0, 0, max_steps=15, m_max=30)
    for chunk in (4, 31):
        y, st, recs = run(ctx, prob, y0, chunk, max_steps=15, m_max=30)
        assert np.array_equal(y, ref)
        assert [r["j"] for r in recs] == [r["j"] for r in rec_ref]


@pytest.mark.parametrize("prec", [ch.CH_FP64, ch.CH_FP32_MIXED])
@pytest.mark.parametrize("n", [24, 65])
def test_graph_runs_equal_direct_runs_3d(ctx, n, prec):
    """The 3-D marching kernels replayed from graphs (chunks of 4 iterations and
    a whole cycle) equal their direct issue bit for bit, and the run matches
    the FP64 oracle."""
    say(f"3-D graphs n={n} prec={prec}")
    prob = ch.Problem(3, n, 0.05, precision=prec)
    y0 = uniform_field(n, 3, 0.1, 0.05, seed=7900 + n)
    ref, st_ref, rec_ref = run(ctx, prob, y0, 0, max_steps=8, m_max=30, tau0=1e-4)
    for chunk in (4, 31):
        y, st, recs = run(ctx, prob, y0, chunk, max_steps=8, m_max=30, tau0=1e-4)
        assert np.array_equal(y, ref), chunk
        assert [r["j"] for r in recs] == [r["j"] for r in rec_ref]
    if prec == ch.CH_FP64:
        y_or, rec = O.ee_adaptive(y0, O.Problem(3, n, 0.05), 1e-4, np.inf, 1e-4, 30, max_steps=8)
        assert [r["j"] for r in rec_ref] == rec.js
        assert np.linalg.norm(ref - y_or) / np.linalg.norm(y_or) <= 1e-10
