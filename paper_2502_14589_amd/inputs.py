"""Seeded synthetic inputs for the Cahn-Hilliard workloads.

Random draws only: this module holds none of the method's arithmetic.  Both the
HIP path (through the binding) and the CPU oracle are fed from it, so a test
compares the two on identical arrays.  Every generator uses
numpy.random.default_rng(seed) (PCG64) and draws in the order documented per
function.  Fields are FP64, flat, row-major with x fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def uniform_field(n: int, dim: int, mean: float, amp: float, seed: int) -> np.ndarray:
    """mean + iid U(-amp, amp) on an n^dim grid (one draw of n^dim values)."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=n ** dim)


# The five workloads: sizes, parameters and seeds.
def small_2d_field(seed: int = 0) -> np.ndarray:
    """64^2, zero mean, U(-0.05, 0.05) noise (constant-step EE2/LIM workload)."""
    return uniform_field(64, 2, 0.0, 0.05, seed)


def large_2d_field(seed: int = 1, n: int = 1024) -> np.ndarray:
    """1024^2, mean 0.1, U(-0.05, 0.05) noise (adaptive EE2/LIM workload)."""
    return uniform_field(n, 2, 0.1, 0.05, seed)


def cube_3d_field(seed: int = 2, n: int = 256) -> np.ndarray:
    """256^3, zero mean, U(-0.05, 0.05) noise (3-D adaptive EE2 workload)."""
    return uniform_field(n, 3, 0.0, 0.05, seed)


def paper_field(n: int, seed: int) -> np.ndarray:
    """The paper's initial data (Section 5.1): iid U(-0.01, 0.01) on an n^2 grid."""
    return uniform_field(n, 2, 0.0, 0.01, seed)


@dataclass
class Instance:
    n: int
    eps: float
    mean: float
    y0: np.ndarray


BATCH_SIDES = (128, 192, 256, 384, 512)


def batch_instances(count: int = 64, seed: int = 3, sides=BATCH_SIDES,
                    eps_range=(0.01, 0.05)) -> list[Instance]:
    """Ragged batch of 2-D instances.

    Draw order: sides (uniform over `sides`), eps (log-uniform), means
    (U(-0.3, 0.3)), then the noise of each field in instance order
    (U(-0.05, 0.05)).
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sides), size=count)
    lo, hi = np.log(eps_range[0]), np.log(eps_range[1])
    eps = np.exp(rng.uniform(lo, hi, size=count))
    means = rng.uniform(-0.3, 0.3, size=count)
    out = []
    for k in range(count):
        n = int(ns[k])
        y0 = means[k] + rng.uniform(-0.05, 0.05, size=n * n)
        out.append(Instance(n, float(eps[k]), float(means[k]), y0))
    return out


@dataclass
class Request:
    arrival: float      # seconds after the start of the trace
    n: int
    eps: float
    steps: int          # horizon in accepted adaptive EE2 steps
    y0: np.ndarray


def request_trace(count: int, rate: float = 200.0, seed: int = 4,
                  sides=(128, 256, 512, 1024), probs=(0.4, 0.3, 0.2, 0.1),
                  eps_range=(0.005, 0.05), horizon=(10, 200)) -> list[Request]:
    """Poisson arrivals of 2-D solve requests.

    Draw order: exponential inter-arrival gaps (mean 1/rate), sides (by
    probs), eps (log-uniform), horizons (uniform integers, inclusive), means
    (U(-0.3, 0.3)), then each field's noise (U(-0.05, 0.05)) in request order.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps)
    ns = rng.choice(np.asarray(sides), size=count, p=np.asarray(probs))
    eps = np.exp(rng.uniform(np.log(eps_range[0]), np.log(eps_range[1]), size=count))
    hz = rng.integers(horizon[0], horizon[1] + 1, size=count)
    means = rng.uniform(-0.3, 0.3, size=count)
    out = []
    for k in range(count):
        n = int(ns[k])
        y0 = means[k] + rng.uniform(-0.05, 0.05, size=n * n)
        out.append(Request(float(arrivals[k]), n, float(eps[k]), int(hz[k]), y0))
    return out


def fourier_mode(n: int, dim: int, k: tuple, amp: float, mean: float = 0.0) -> np.ndarray:
    """mean + amp cos(2 pi k.x) at the nodes x_i = i h (deterministic test field)."""
    axes = np.meshgrid(*([np.arange(n) / n] * dim), indexing="ij")
    # axes[0] is the slowest index; reverse so k[0] multiplies x (fastest)
    phase = sum(kk * ax for kk, ax in zip(k, reversed(axes)))
    return (mean + amp * np.cos(2 * np.pi * phase)).ravel()
