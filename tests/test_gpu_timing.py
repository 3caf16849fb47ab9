"""The kernel-timing entry point (ch_time_kernel): argument checks, the
algorithmic byte count it reports, and that a later run is unaffected by the
values it leaves in the workspace."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import uniform_field


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


def run_steps(ctx, pg, y0, m):
    y = dev(y0)
    st, recs = ctx.run_ee(pg, y, 1e-3, T=1e-3, max_steps=2, m_max=m, tol=1e-4, records=True)
    return y.cpu().numpy(), recs


@pytest.mark.parametrize("prec", [ch.CH_FP64, ch.CH_FP32_MIXED])
def test_time_kernel_bytes_and_workspace(ctx, prec):
    n, m = 96, 12
    say(f"ch_time_kernel 96^2 prec={prec}")
    pg = ch.Problem(2, n, 0.05, False, prec)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=611)
    ya, recs = run_steps(ctx, pg, y0, m)
    last_j = recs[-1]["j"]
    assert last_j >= 2
    w, N = (8 if prec == ch.CH_FP64 else 4), n * n
    mv = list(range(m + 1)) + [0, m]
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_DC_MATVEC, m, mv)
    assert us > 0 and nb == sum((k + 2 + (1 if k < m else 0)) * w * N for k in mv)
    up = list(range(m))
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_DC_UPDATE, m, up)
    assert us > 0 and nb == sum((k + 4) * w * N for k in up)
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_DC_ITER, m, up)
    assert us > 0 and nb == sum((2 * k + 7) * w * N for k in up)
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_PHI, m, list(range(1, min(last_j, m - 1) + 1)))
    assert us > 0 and nb == 0
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_MATVEC, m, [0, 1, m - 1])
    assert nb == 3 * 4 * w * N
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_MGS, m, [1, m - 1])
    assert nb == 2 * 4 * w * N
    # out-of-range iterations are refused before anything is launched
    for kernel, k in ((ch.CH_KERNEL_DC_MATVEC, m + 1), (ch.CH_KERNEL_DC_UPDATE, m), (ch.CH_KERNEL_MGS, 0),
                      (ch.CH_KERNEL_PHI, last_j + 1 if last_j + 1 < m else m), (ch.CH_KERNEL_DC_MATVEC, -1)):
        with pytest.raises(ch.ChError):
            ctx.time_kernel(pg, kernel, m, [k])
    with pytest.raises(ch.ChError):
        ctx.time_kernel(pg, ch.CH_KERNEL_DC_MATVEC, ch.CH_MMAX + 1, [0])
    # a run after the timing launches starts from a fresh workspace state
    yb, recs_b = run_steps(ctx, pg, y0, m)
    assert [r["j"] for r in recs_b] == [r["j"] for r in recs]
    assert np.array_equal(ya, yb)


def test_time_kernel_lim_stage(ctx):
    n = 96
    say("ch_time_kernel LIM stage 96^2")
    pg = ch.Problem(2, n, 0.05)
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=612)
    y = dev(y0)
    ctx.run_lim(pg, y, 1e-7, T=1e-6, max_steps=2, tol=1e-4)
    us, nb = ctx.time_kernel(pg, ch.CH_KERNEL_LIM_STAGE, 1, count=7)
    assert us > 0 and nb == 7 * 24 * n * n
    with pytest.raises(ch.ChError):
        ctx.time_kernel(pg, ch.CH_KERNEL_LIM_STAGE, 1, count=0)
    us2, nb2 = ctx.time_kernel(pg, ch.CH_KERNEL_LIM_STAGE2, 1, count=5)
    assert us2 > 0 and nb2 == 5 * 24 * n * n


def test_time_kernel_lim_stage_pair_is_2d_only(ctx):
    n = 12
    say("ch_time_kernel LIM stage pair on 12^3: rejected")
    pg = ch.Problem(3, n, 0.05)
    y = dev(uniform_field(n, 3, 0.1, 0.05, seed=613))
    ctx.run_lim(pg, y, 1e-7, T=1e-6, max_steps=1, tol=1e-4)
    ctx.time_kernel(pg, ch.CH_KERNEL_LIM_STAGE, 1, count=2)
    with pytest.raises(ch.ChError):
        ctx.time_kernel(pg, ch.CH_KERNEL_LIM_STAGE2, 1, count=2)


def test_time_kernel_needs_workspace():
    """A fresh context has no workspace to time on."""
    c = ch.Context(0)
    try:
        with pytest.raises(ch.ChError):
            c.time_kernel(ch.Problem(2, 64, 0.05), ch.CH_KERNEL_DC_MATVEC, 4, [0])
    finally:
        c.close()
