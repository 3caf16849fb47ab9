"""3-D grids of every awkward size for the z-marching kernels (the DCGS2
matvec with its dot phase and the EE2 estimate pass).

In FP64 a workgroup owns a 64 x 8 block of (x, y) columns and a run of 16
planes, and each thread a pair of consecutive x; in FP32 a 64 x 16 block and
four consecutive x, with runs whose length is chosen per grid so that the work
items fill whole rounds of workgroups (16 on small grids, 17 at 210^3, 22 at
256^3).  The sizes here cover:
- grids narrower than the block in x and y, whose halos wrap several times (n = 5, 6, 7);
- odd n (the pair as two scalar points) and even n (one vector);
- a single block (16) and runs whose last one has 1 plane (33, 65);
- two blocks in x with a ragged second one (65, 66).

- FP32 grids whose runs are not 16 planes (210, 256).

Adaptive EE2 (Fig. 4) against the FP64 oracle: equal Krylov dimensions, the
field to 1e-10 (relative L2 and max-abs).  FP32-mixed: one step to 1e-5.  A
batch mixing odd and even sizes (the per-instance pair form): every member
bit-equal to its solo run.  The FP32 grids with longer runs: a batch (run
length found per instance on the device) bit-equal to the solo runs (length
from the host), and within 1e-5 of the FP64 run with the same Krylov
dimensions.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ch_oracle as O
from paper_2502_14589_amd import ch
from paper_2502_14589_amd.inputs import uniform_field

SIZES = [5, 6, 7, 9, 16, 33, 65, 66]


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
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n", SIZES)
def test_march_sizes_adaptive_fp64(ctx, n):
    say(f"3-D adaptive EE2 n={n}")
    eps = 0.3 if n < 10 else 0.05
    po = O.Problem(3, n, eps)
    y0 = uniform_field(n, 3, 0.1, 0.05, seed=8100 + n)
    y_ref, rec = O.ee_adaptive(y0, po, 1e-4, np.inf, 1e-4, 30, max_steps=3)
    yg = dev(y0)
    st, recs = ctx.run_ee(ch.Problem(3, n, eps), yg, 1e-4, max_steps=3, m_max=30, tol=1e-4, records=True)
    assert [r["j"] for r in recs] == rec.js
    y = yg.cpu().numpy()
    assert rel(y, y_ref) <= 1e-10 and max_rel(y, y_ref) <= 1e-10


@pytest.mark.parametrize("n", SIZES)
def test_march_sizes_fp32_mixed_step(ctx, n):
    eps = 0.3 if n < 10 else 0.05
    po = O.Problem(3, n, eps)
    y0 = uniform_field(n, 3, 0.1, 0.05, seed=8200 + n)
    y_ref, tau_ref, info = O.ee_step(y0, po, 1e-4, 1e-8, 20)
    yg = dev(y0)
    ctx.step_ee(ch.Problem(3, n, eps, precision=ch.CH_FP32_MIXED), yg, 1e-4, m_max=20, tol_phi_fixed=1e-8)
    assert rel(yg.cpu().numpy(), y_ref) <= 1e-5


def test_march_batch_of_odd_and_even_sizes(ctx):
    ns = [5, 6, 9, 16, 33, 6]
    eps = [0.3, 0.3, 0.3, 0.05, 0.05, 0.2]
    y0s = [uniform_field(n, 3, 0.1, 0.05, seed=8300 + i) for i, n in enumerate(ns)]
    fields = [dev(y) for y in y0s]
    st, rc = ctx.run_ee_batch(fields, ns, eps, dim=3, tau0=1e-4, max_steps=4, m_max=20, tol=1e-4)
    assert rc == 0
    for i, n in enumerate(ns):
        yg = dev(y0s[i])
        ctx.run_ee(ch.Problem(3, n, eps[i]), yg, 1e-4, max_steps=4, m_max=20, tol=1e-4)
        assert np.array_equal(yg.cpu().numpy(), fields[i].cpu().numpy()), n
    y_ref, _ = O.ee_adaptive(y0s[4], O.Problem(3, 33, 0.05), 1e-4, np.inf, 1e-4, 20, max_steps=4)
    assert rel(fields[4].cpu().numpy(), y_ref) <= 1e-10


def test_fp32_longer_runs_batch_equals_solo_and_fp64(ctx):
    ns = [210, 24, 256]
    eps = [0.02, 0.05, 0.02]
    kw = dict(tau0=1e-4, max_steps=3, m_max=20, tol=1e-4)
    y0s = [uniform_field(n, 3, 0.1, 0.05, seed=8400 + i) for i, n in enumerate(ns)]
    say("3-D FP32 batch with runs of 17, 16 and 22 planes")
    fields = [dev(y) for y in y0s]
    st, rc = ctx.run_ee_batch(fields, ns, eps, dim=3, precision=ch.CH_FP32_MIXED, **kw)
    assert rc == 0 and all(s["steps"] == 3 for s in st)
    for i, n in enumerate(ns):
        yg = dev(y0s[i])
        ctx.run_ee(ch.Problem(3, n, eps[i], precision=ch.CH_FP32_MIXED), yg, kw["tau0"], max_steps=3, m_max=20,
                   tol=1e-4)
        assert np.array_equal(yg.cpu().numpy(), fields[i].cpu().numpy()), n
    y64 = dev(y0s[0])
    _, r64 = ctx.run_ee(ch.Problem(3, 210, 0.02), y64, kw["tau0"], max_steps=3, m_max=20, tol=1e-4, records=True)
    y32 = dev(y0s[0])
    _, r32 = ctx.run_ee(ch.Problem(3, 210, 0.02, precision=ch.CH_FP32_MIXED), y32, kw["tau0"], max_steps=3,
                        m_max=20, tol=1e-4, records=True)
    assert [r["j"] for r in r32] == [r["j"] for r in r64]
    assert rel(y32.cpu().numpy(), y64.cpu().numpy()) <= 1e-5
