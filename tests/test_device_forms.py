"""Reformulations the device kernels rely on, checked on the CPU against the
oracle (no GPU; the kernels themselves are covered by the GPU parity tests)."""
import math

import numpy as np
import pytest

from oracle import ch_oracle as O


def leja_order_from_log_sine_table(p: int) -> list:
    """The LIM node order as the plan kernel forms it: with
    theta_i = pi (2i + 1) / (2p), cos a - cos b = -2 sin((a + b)/2) sin((a - b)/2)
    gives log|beta_i - beta_r| = log 2 + L[i + r + 1] + L[|i - r|] with
    L[k] = log sin(pi k / (2p)); the sums are accumulated in that form, and the
    pick rule (largest sum; within 1e-9 relative of it, the smallest index) is
    the one of Fig. 1's node ordering (reading R6)."""
    k = np.arange(2 * p, dtype=float)
    with np.errstate(divide="ignore"):
        L = np.log(np.sin(math.pi * k / (2.0 * p)))
    L[0] = 0.0
    idx = np.arange(p)
    score = np.zeros(p)
    taken = np.zeros(p, dtype=bool)
    order, r = [], 0
    for s in range(p):
        order.append(r)
        taken[r] = True
        score += math.log(2.0) + (L[idx + r + 1] + L[np.abs(idx - r)])
        if s == p - 1:
            break
        cand = np.where(taken, -np.inf, score)
        best = cand.max()
        r = int(np.flatnonzero(cand >= best - 1e-9 * max(1.0, abs(best)))[0])
    return order


@pytest.mark.parametrize("p", list(range(1, 65)) + [97, 128, 209, 300, 513, 1000])
def test_leja_order_log_sine_table_matches_oracle(p):
    assert leja_order_from_log_sine_table(p) == O.lim_node_order(p)
