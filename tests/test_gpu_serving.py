"""Serving (continuous batching): each result equals the same request run
alone, whatever else shares the GPU; admission waits for slots and memory."""
import sys
import time

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


REQS = [(40, 0.05, 6), (64, 0.03, 11), (33, 0.06, 3), (96, 0.02, 8), (70, 0.04, 14), (50, 0.05, 1), (80, 0.03, 5)]


def wait_all(srv, tickets, outs, timeout=60.0):
    results = {}
    t_end = time.time() + timeout
    while len(results) < len(tickets) and time.time() < t_end:
        for k, t in enumerate(tickets):
            if k in results:
                continue
            state, rc, st, lat = srv.poll(t, outs[k])
            if state in (ch.CH_REQ_DONE, ch.CH_REQ_FAILED):
                results[k] = (state, rc, st, lat)
        time.sleep(0.002)
    return results


@pytest.mark.parametrize("prec,slots,budget", [(ch.CH_FP64, 64, 1 << 30), (ch.CH_FP64, 2, 1 << 30),
                                               (ch.CH_FP32_MIXED, 3, 3 << 20)])
def test_served_results_equal_solo_runs(prec, slots, budget):
    say(f"serving prec={prec} slots={slots} budget={budget}")
    import torch

    ys = [uniform_field(n, 2, 0.05 * (k % 3), 0.05, seed=1000 + k) for k, (n, e, s) in enumerate(REQS)]
    with ch.Server(0, prec, m_max=12, tol=1e-4, hbm_budget=budget, max_slots=slots) as srv:
        tickets = [srv.submit(dev(y), n, e, s, tau0=1e-3) for y, (n, e, s) in zip(ys, REQS)]
        outs = [torch.empty(n * n, dtype=torch.float64, device="cuda") for n, _, _ in REQS]
        res = wait_all(srv, tickets, outs)
    assert len(res) == len(REQS)
    with ch.Context(0) as ctx:
        for k, ((n, e, s), y) in enumerate(zip(REQS, ys)):
            state, rc, st, lat = res[k]
            assert state == ch.CH_REQ_DONE and rc == ch.CH_OK and st["steps"] == s
            assert lat[0] >= 0 and lat[1] > 0 and lat[2] >= lat[1]
            solo = dev(y)
            ctx.run_ee(ch.Problem(2, n, e, False, prec), solo, 1e-3, max_steps=s, m_max=12, tol=1e-4)
            assert np.array_equal(solo.cpu().numpy(), outs[k].cpu().numpy()), k


def test_serving_rejects_what_can_never_fit_and_unknown_tickets():
    say("serving errors")
    with ch.Server(0, ch.CH_FP64, m_max=12, tol=1e-4, hbm_budget=1 << 20, max_slots=2) as srv:
        with pytest.raises(ch.ChError) as e:
            srv.submit(dev(np.zeros(128 * 128)), 128, 0.05, 3)
        assert e.value.status == ch.CH_ENOMEM
        state, rc, _, _ = srv.poll(12345)
        assert rc == ch.CH_ENOENT
        t = srv.submit(dev(uniform_field(32, 2, 0.0, 0.05, seed=5)), 32, 0.05, 2)
        import torch
        out = torch.empty(32 * 32, dtype=torch.float64, device="cuda")
        res = wait_all(srv, [t], [out])
        assert res[0][0] == ch.CH_REQ_DONE
        assert srv.poll(t)[1] == ch.CH_ENOENT      # released after the result was taken


def test_served_lim_and_ee_mix_with_host_fields_final_times_and_tolerances():
    """Requests of both methods in one server: LIM (Fig. 2) and EE2 (Fig. 4)
    members advance in the same batch steps; fields given in host memory;
    per-request tolerances and final times (the last step clipped onto T).
    Each result equals the same request run alone, bit for bit."""
    say("serving: LIM and EE2 mix, host fields, final times, tolerances")
    import torch

    reqs = [  # (n, eps, method, steps, T, tau0, tol, on_host)
        (40, 0.05, ch.CH_METHOD_LIM, 5, float("inf"), 2e-7, 1e-4, False),
        (64, 0.03, ch.CH_METHOD_EE, 0, 3e-6, 1e-3, 1e-3, True),
        (33, 0.06, ch.CH_METHOD_LIM, 0, 2e-6, 3e-7, 0.0, True),
        (96, 0.02, ch.CH_METHOD_EE, 7, float("inf"), 1e-3, 0.0, False),
        (50, 0.04, ch.CH_METHOD_LIM, 3, float("inf"), 1e-7, 1e-5, False),
    ]
    ys = [uniform_field(n, 2, 0.05 * k, 0.05, seed=1300 + k) for k, (n, *_rest) in enumerate(reqs)]
    with ch.Server(0, ch.CH_FP64, m_max=12, tol=1e-4, hbm_budget=1 << 30, max_slots=8) as srv:
        tickets = []
        for y, (n, e, meth, steps, T, tau0, tol, host_y) in zip(ys, reqs):
            y0 = y.copy() if host_y else dev(y)
            tickets.append(srv.submit(y0, n, e, steps, tau0=tau0, method=meth, T=T, tol=tol))
        outs = [torch.empty(n * n, dtype=torch.float64, device="cuda") for n, *_ in reqs]
        res = wait_all(srv, tickets, outs)
    assert len(res) == len(reqs)
    with ch.Context(0) as ctx:
        for k, ((n, e, meth, steps, T, tau0, tol, _), y) in enumerate(zip(reqs, ys)):
            state, rc, st, lat = res[k]
            assert state == ch.CH_REQ_DONE and rc == ch.CH_OK, (k, state, rc)
            solo = dev(y)
            if meth == ch.CH_METHOD_LIM:
                tl = tol if tol > 0 else 1e-4          # the server's tolerance
                s1, _ = ctx.run_lim(ch.Problem(2, n, e), solo, tau0, T=T, max_steps=steps, tol=tl)
            else:
                tl = tol if tol > 0 else 1e-4
                s1, _ = ctx.run_ee(ch.Problem(2, n, e), solo, tau0, T=T, max_steps=steps, m_max=12, tol=tl)
            assert st["steps"] == s1["steps"] and st["t"] == s1["t"], k
            if T < float("inf"):
                assert st["t"] == T
            assert np.array_equal(solo.cpu().numpy(), outs[k].cpu().numpy()), k
