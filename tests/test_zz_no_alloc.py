"""The entry point that allocates nothing (ch_step_lim_noalloc) against the
one it is a variant of (ch_step_lim): same kernels, same inputs, so the same
bits.  Two calls in a row on one context, the second on a smaller grid (the
shared scratch keeps the first call's contents), and a grid above the
scratch's limit, which must be refused with an error."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import uniform_field


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(y):
    import torch

    return torch.from_numpy(np.ascontiguousarray(y, dtype=np.float64)).to("cuda")


CASES = [
    # (dim, n, eps, mean, tau, tol): adaptive 2-D at 1024^2 (the limit), then a smaller 2-D
    # constant step, then 3-D
    (2, 1024, 0.01, 0.1, 2.5e-7, 1e-4),
    (2, 96, 0.03, 0.2, 4e-6, 0.0),
    (3, 40, 0.05, 0.0, 2e-6, 1e-4),
]


def test_noalloc_lim_step_equals_lim_step():
    import torch

    with ch.Context(0) as ctx:
        for k, (dim, n, eps, mean, tau, tol) in enumerate(CASES):
            say(f"no-alloc LIM step: dim {dim}, n {n}, tol {tol}")
            y0 = uniform_field(n, dim, mean, 0.05, seed=800 + k)
            pg = ch.Problem(dim, n, eps)
            a, b = dev(y0), dev(y0)
            rec_a = ctx.step_lim(pg, a, tau, T=1.0, tol=tol)
            rec_b, rc = ctx.step_lim_noalloc(pg, b, tau, T=1.0, tol=tol)
            torch.cuda.synchronize()
            assert rc == ch.CH_OK
            assert rec_b == rec_a
            assert rec_b["j"] >= 2 and rec_b["matvecs"] == 2 * rec_b["j"] - 1
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
            assert not np.array_equal(b.cpu().numpy(), y0)


def test_noalloc_lim_step_refuses_grids_above_the_limit():
    say("no-alloc LIM step above the limit")
    n = 1025
    assert n * n > ch.CH_NOALLOC_MAX_POINTS
    y0 = uniform_field(n, 2, 0.1, 0.05, seed=899)
    with ch.Context(0) as ctx:
        y = dev(y0)
        with pytest.raises(ch.ChError) as e:
            ctx.step_lim_noalloc(ch.Problem(2, n, 0.01), y, 2.5e-7, T=1.0, tol=1e-4)
        assert e.value.status == ch.CH_EINVAL and "CH_NOALLOC_MAX_POINTS" in str(e.value)
        assert np.array_equal(y.cpu().numpy(), y0)
