"""Oracle: plain, slow, FP64 CPU implementation of the explicit Cahn-Hilliard
time integrators of Botchev, "Explicit adaptive time stepping for the
Cahn-Hilliard equation by exponential Krylov subspace and Chebyshev polynomial
methods" (arXiv 2502.14589).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this module.  The product path (the HIP
library and its Python binding) never imports, calls or links it, and this
module imports nothing from the product package.

Conventions (the paper's notation):
  * ``y`` is the grid vector (length N = n**dim), row-major with x fastest,
    on the periodic cube [0,L)^dim with h = L/n (L = 1 by default), or, with
    bc = "neumann", on the cell-centred grid x_i = (i + 1/2) h of (0,L)^dim
    with the homogeneous Neumann conditions of the paper's problem (Section 2,
    eq. CH; Section 5.1): the mirror ghost cell y_{-1} = y_0, y_n = y_{n-1}.
  * ``A`` is the symmetric positive semidefinite matrix whose negative is the
    standard second-order Laplacian (Section 2, eq. IVP).
  * F'(y) = y(y^2 - 1) (eq. F); J_n = 3 diag(y^2) - I (eq. J).
  * Ahat_n = A (J_n + eps^2 A) and ghat^n = A (J_n y^n - F'(y^n)) (eq. A_g), or
    with the Eyre splitting Ahat_n = A (J_n + eps^2 A + I),
    ghat^n = A (J_n y^n + y^n - F'(y^n)) (eq. A_g_cs).
  * Norms are Euclidean (Section 1, last paragraph).
  * Variable mobility (Section 2, Remark 1; reading R12): with
    mobility = (m0, m1) the equation is c_t = div(M(c) grad mu),
    M(c) = max(m0 + m1 (1 - c^2), 0), discretised as
    y' = -A_M(y) (F'(y) + eps^2 A y) with the flux-form matrix
    (A_M(y) v)_i = h^-2 sum over the neighbours k of (M_i + M_k)/2 (v_i - v_k).
    A step freezes A_M at y^n: Ahat_n = A_M(y^n) (J_n + eps^2 A [+ I]),
    ghat^n = A_M(y^n) (J_n y^n [+ y^n] - F'(y^n)).  Periodic grids only.

Every function follows the definition or the algorithm box it cites, step by
step, with library primitives (``numpy`` array arithmetic, ``scipy.linalg.expm``)
as the only helpers.  Where the paper is silent the reading taken is stated in
the docstring (these readings are listed in the design notes as well):

  R1  the "trace resnorm for s in [0, tau0]" of the Krylov algorithm (Fig. 3)
      is a dyadic search for the largest bracket [tau0 2^-k, tau0 2^(1-k)]
      whose left end satisfies the residual test, then bisection of that
      bracket to a relative width of 2^-50; the left end is returned.
  R2  the constant-step EE2 with linear residual-time restarting (Section 4.1,
      last paragraph) keeps Ahat_n and ghat^n frozen at y^n and repeats the
      Fig. 3 cycle from the current sub-step state with start vector
      ghat^n - Ahat_n z and initial step tau - (time already covered).
  R3  beta = 0 (y^n is a steady state of the linearised problem): the step is
      y^{n+1} = y^n with tau = tau0.  A lucky breakdown (h_{j+1,j} = 0) is a
      converged step (its residual is zero).
  R4  est = 0: EE2 takes tau_new = 5/4 tau (the limit of eq. EEdt); LIM keeps
      tau (eq. LIMdt would divide by zero).
  R5  the final-time clip sets t = T exactly when the clipped step was taken
      in full.
  R6  the Chebyshev nodes of the LIM step (Fig. 1 fixes only beta_1 =
      cos(pi/2p) as the first of its "ordered set") are taken in Leja order:
      beta_1, then each time the node that maximises the product of distances
      to the nodes already taken (lim_node_order).  Any order gives the same
      step in exact arithmetic (the stage factors commute); in floating point
      the order decides how far intermediate stages grow.  Taking i = 1..p
      instead lets a stage amplify rounding by 10^16 at p = 33 and by 10^105
      at p = 209 (max over the spectrum of the partial product times the
      remaining one), which destroys the adaptive 1024^2 run; Leja order keeps
      it below 10^7.2 up to p = 4096.  Both sweeps (m = 1..p, then 2..p) follow
      the same order.
  R12 variable mobility (Remark 1 gives only the structure A_M(y)): M(c) =
      max(m0 + m1 (1 - c^2), 0), faces take the arithmetic mean of the two
      cell mobilities, the step freezes A_M at y^n, the LIM bound is the
      1-norm of the assembled Ahat_n, and the estimate of eq. LIMest is the
      trapezoidal rule y_PC = y^n + tau/2 (f(y^n) + f(y^{n+1})) (with M = 1
      it is eq. LIMest exactly).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import expm


class TauUnderflow(RuntimeError):
    """The residual-time trace could not find an admissible step >= tau_min."""


@dataclass(frozen=True)
class Problem:
    """Space discretisation of the Cahn-Hilliard problem (eq. IVP).

    dim: 2 or 3; n: grid points per direction (periodic, h = 1/n);
    eps: interface parameter epsilon; eyre: use the Eyre splitting (eq. A_g_cs).
    """

    dim: int
    n: int
    eps: float
    eyre: bool = False
    bc: str = "periodic"       # or "neumann"
    length: float = 1.0        # side L of the domain
    mobility: tuple | None = None   # (m0, m1): M(c) = max(m0 + m1 (1 - c^2), 0); None: M = 1

    @property
    def h(self) -> float:
        return self.length / self.n

    @property
    def N(self) -> int:
        return self.n ** self.dim

    @property
    def shape(self):
        return (self.n,) * self.dim


# ---------------------------------------------------------------------------
# Space discretisation (Section 2, eqs. F, IVP; Section 3.1, eqs. J, A_g;
# Section 3.3, eq. A_g_cs)
# ---------------------------------------------------------------------------

def lap(y: np.ndarray, prob: Problem) -> np.ndarray:
    """A y, where -A is the standard (2*dim+1)-point Laplacian (eq. IVP): periodic,
    or with homogeneous Neumann conditions on the cell-centred grid, whose ghost
    values mirror the boundary cells (np.pad in "edge" mode)."""
    Y = np.asarray(y, dtype=np.float64).reshape(prob.shape)
    out = (2.0 * prob.dim) * Y
    if prob.bc == "neumann":
        P = np.pad(Y, 1, mode="edge")
        inner = tuple(slice(1, -1) for _ in range(prob.dim))
        for ax in range(prob.dim):
            lo = list(inner)
            hi = list(inner)
            lo[ax] = slice(0, -2)
            hi[ax] = slice(2, None)
            out = out - P[tuple(lo)] - P[tuple(hi)]
        return (out / prob.h ** 2).ravel()
    for ax in range(prob.dim):
        out = out - np.roll(Y, 1, axis=ax) - np.roll(Y, -1, axis=ax)
    return (out / prob.h ** 2).ravel()


def mobility_of(y: np.ndarray, prob: Problem) -> np.ndarray:
    """M(c) = max(m0 + m1 (1 - c^2), 0) (reading R12 of Section 2, Remark 1)."""
    m0, m1 = prob.mobility
    return np.maximum(m0 + m1 * (1.0 - y * y), 0.0)


def lap_M(v: np.ndarray, y: np.ndarray, prob: Problem) -> np.ndarray:
    """A_M(y) v = h^-2 sum over the neighbours k of (M_i + M_k)/2 (v_i - v_k): the
    flux form of -div(M grad) on the periodic grid (Section 2, Remark 1)."""
    if prob.bc != "periodic":
        raise ValueError("variable mobility is defined on periodic grids")
    V = np.asarray(v, dtype=np.float64).reshape(prob.shape)
    M = mobility_of(np.asarray(y, dtype=np.float64), prob).reshape(prob.shape)
    out = np.zeros_like(V)
    for ax in range(prob.dim):
        for shift in (1, -1):
            Mk = np.roll(M, shift, axis=ax)
            Vk = np.roll(V, shift, axis=ax)
            out = out + 0.5 * (M + Mk) * (V - Vk)
    return (out / prob.h ** 2).ravel()


def outer(v: np.ndarray, y: np.ndarray, prob: Problem) -> np.ndarray:
    """The outer operator of the splitting: A v, or A_M(y) v with variable mobility."""
    return lap(v, prob) if prob.mobility is None else lap_M(v, y, prob)


def Fprime(y: np.ndarray) -> np.ndarray:
    """F'(c) = c (c^2 - 1), the derivative of F(c) = (1 - c^2)^2 / 4 (eq. F)."""
    return y * (y * y - 1.0)


def Fenergy(y: np.ndarray) -> np.ndarray:
    """F(c) = (1 - c^2)^2 / 4 (eq. F)."""
    return 0.25 * (1.0 - y * y) ** 2


def rhs(y: np.ndarray, prob: Problem) -> np.ndarray:
    """f(y) = -A (F'(y) + eps^2 A y), the semi-discrete right-hand side (eq. IVP);
    -A_M(y) (F'(y) + eps^2 A y) with variable mobility."""
    return -outer(Fprime(y) + prob.eps ** 2 * lap(y, prob), y, prob)


def jac_diag(y: np.ndarray, prob: Problem) -> np.ndarray:
    """Diagonal of J_n = 3 diag(y^2) - I (eq. J); plus I with the Eyre splitting."""
    d = 3.0 * y * y - 1.0
    if prob.eyre:
        d = d + 1.0
    return d


def ahat_mv(v: np.ndarray, y: np.ndarray, prob: Problem) -> np.ndarray:
    """Ahat_n v = A ((J_n + eps^2 A [+ I]) v) (eq. A_g / A_g_cs), frozen at y^n = y
    (A_M(y^n) in place of the outer A with variable mobility)."""
    return outer(jac_diag(y, prob) * v + prob.eps ** 2 * lap(v, prob), y, prob)


def ghat(y: np.ndarray, prob: Problem) -> np.ndarray:
    """ghat^n = A (J_n y^n - F'(y^n)) (eq. A_g), or A (J_n y^n + y^n - F'(y^n)) (eq. A_g_cs)."""
    Jy = (3.0 * y * y - 1.0) * y
    inner = Jy - Fprime(y)
    if prob.eyre:
        inner = inner + y
    return outer(inner, y, prob)


def assemble_A(prob: Problem):
    """A as a scipy.sparse matrix (Kronecker sum of 1-D second differences: periodic,
    or Neumann on the cell-centred grid, whose end rows read (y_0 - y_1) / h^2)."""
    import scipy.sparse as sp

    n, h = prob.n, prob.h
    e = np.ones(n)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="lil")
    if prob.bc == "neumann":
        T[0, 0] = 1.0
        T[n - 1, n - 1] = 1.0
    else:
        T[0, n - 1] = -1.0
        T[n - 1, 0] = -1.0
    T = sp.csr_matrix(T) / h ** 2
    I = sp.identity(n, format="csr")
    if prob.dim == 2:
        # y is stored with x fastest: index = iy*n + ix
        return (sp.kron(I, T) + sp.kron(T, I)).tocsr()
    return (sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I))).tocsr()


def assemble_AM(y: np.ndarray, prob: Problem):
    """A_M(y) as a scipy.sparse matrix: D^T W D with D the (edge x point)
    incidence matrix of the periodic grid (one row per edge i -> i + e_ax,
    entries +1 at i and -1 at its neighbour) and W = diag((M_i + M_k)/2) / h^2."""
    import scipy.sparse as sp

    N = prob.N
    idx = np.arange(N).reshape(prob.shape)
    M = mobility_of(np.asarray(y, dtype=np.float64), prob).reshape(prob.shape)
    rows, cols, vals, w = [], [], [], []
    e = 0
    for ax in range(prob.dim):
        nb = np.roll(idx, -1, axis=ax).ravel()
        Mk = np.roll(M, -1, axis=ax).ravel()
        m = idx.size
        rows += [np.arange(e, e + m)] * 2
        cols += [idx.ravel(), nb]
        vals += [np.ones(m), -np.ones(m)]
        w.append(0.5 * (M.ravel() + Mk))
        e += m
    D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(e, N))
    W = sp.diags(np.concatenate(w) / prob.h ** 2)
    return (D.T @ W @ D).tocsr()


def assemble_ahat(y: np.ndarray, prob: Problem):
    """Ahat_n = A (J_n + eps^2 A [+ I]) assembled as a sparse matrix (eq. A_g / A_g_cs);
    A_M(y^n) (J_n + eps^2 A [+ I]) with variable mobility."""
    import scipy.sparse as sp

    A = assemble_A(prob)
    Aout = A if prob.mobility is None else assemble_AM(y, prob)
    return (Aout @ (sp.diags(jac_diag(y, prob)) + prob.eps ** 2 * A)).tocsr()


# ---------------------------------------------------------------------------
# Small dense phi evaluation (Section 4.1, eqs. phi, yt_m, rm)
# ---------------------------------------------------------------------------

def phiv_small(Hj: np.ndarray, s: float) -> np.ndarray:
    """u = s phi(-s H_{j,j}) e_1 for the small Hessenberg matrix (Fig. 3, "u := s phi(-sH)e1").

    phi(z) = (e^z - 1)/z (eq. phi).  Computed as the last column (top j entries)
    of exp([[-s H, s e_1], [0, 0]]), the block-triangular identity
    exp([[X, b], [0, 0]]) = [[e^X, phi(X) b], [0, 1]], with scipy's expm.
    """
    j = Hj.shape[0]
    M = np.zeros((j + 1, j + 1))
    M[:j, :j] = -s * Hj
    M[0, j] = s
    return expm(M)[:j, j]


def resnorm_at(Hj: np.ndarray, h_next: float, s: float) -> float:
    """||r(t_n + s)|| / beta = h_{j+1,j} |e_j^T s phi(-s H) e_1| (eq. rm, phi_stop)."""
    return h_next * abs(phiv_small(Hj, s)[-1])


def rt_trace(Hj: np.ndarray, h_next: float, tau0: float, tol_phi: float,
             tau_min: float = 0.0, rel_width: float = 2.0 ** -50) -> float:
    """tau := max{s in [0, tau0] : resnorm(s) <= tol_phi} (Fig. 3, trace branch).

    Reading R1: the largest dyadic step tau0 2^-k (k >= 1) that passes the
    residual test is located first; its bracket [tau0 2^-k, tau0 2^(1-k)] is then
    bisected until its relative width is <= rel_width, keeping
    resnorm(lo) <= tol_phi < resnorm(hi).  Returns lo.  For a monotone residual
    (Section 4.1) this is the maximum the box asks for.
    """
    k = 1
    while True:
        s = tau0 * 2.0 ** (-k)
        if s < tau_min or s == 0.0:
            raise TauUnderflow(f"trace found no step >= tau_min={tau_min}")
        if resnorm_at(Hj, h_next, s) <= tol_phi:
            break
        k += 1
    lo, hi = s, 2.0 * s
    while hi - lo > rel_width * lo:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if resnorm_at(Hj, h_next, mid) <= tol_phi:
            lo = mid
        else:
            hi = mid
    return lo


@dataclass
class KrylovInfo:
    """Outcome of one Fig. 3 cycle."""

    j: int                 # Krylov dimension used (number of matvecs with Ahat inside the cycle)
    tau: float             # accepted step
    converged: bool        # residual test passed at tau0 (no trace)
    resnorm: float         # ||r(tau)|| / beta at the returned tau
    beta: float
    H: np.ndarray = field(repr=False, default=None)   # H_{j+1,j}
    V: np.ndarray = field(repr=False, default=None)   # V_{j+1}
    u: np.ndarray = field(repr=False, default=None)   # tau phi(-tau H_jj) e_1


def krylov_phi_cycle(matvec, y: np.ndarray, v1: np.ndarray, tau0: float, tol_phi: float,
                     m_max: int, tau_min: float = 0.0, keep_basis: bool = False):
    """One run of the Krylov algorithm of Fig. 3 on y' = -Ahat y + ghat, y(0) = y.

    matvec(v) returns Ahat v; v1 = ghat - Ahat y is the start vector.
    Arnoldi with modified Gram-Schmidt (eq. Arn), the residual test
    of eq. phi_stop at s = tau0 and, at j = m_max, the trace of
    the residual over s (reading R1).  Returns y + V_j (beta u)
    (the solution update), the accepted tau and a KrylovInfo.
    """
    N = y.size
    beta = float(np.linalg.norm(v1))
    if beta == 0.0:                                          # reading R3
        return y.copy(), tau0, KrylovInfo(0, tau0, True, 0.0, 0.0)
    # basis vector i is the row V[i] (contiguous), H is (m_max + 1) x m_max
    V = np.zeros((m_max + 1, N))
    H = np.zeros((m_max + 1, m_max))
    V[0] = v1 / beta
    tau = tau0
    converged = False
    for j in range(1, m_max + 1):
        w = matvec(V[j - 1])
        for i in range(1, j + 1):
            H[i - 1, j - 1] = w @ V[i - 1]
            w = w - H[i - 1, j - 1] * V[i - 1]
        H[j, j - 1] = np.linalg.norm(w)
        Hj = H[:j, :j]
        u = phiv_small(Hj, tau0)
        resnorm = H[j, j - 1] * abs(u[-1])
        if resnorm <= tol_phi:
            tau = tau0
            converged = True
            break
        if j == m_max:
            tau = rt_trace(Hj, H[j, j - 1], tau0, tol_phi, tau_min)
            u = phiv_small(Hj, tau)
            resnorm = H[j, j - 1] * abs(u[-1])
            break
        V[j] = w / H[j, j - 1]
    y_new = y + (beta * u) @ V[:j]
    info = KrylovInfo(j, tau, converged, float(resnorm), beta)
    if keep_basis:
        info.H = H[: j + 1, :j].copy()
        info.V = V[: j + 1].T.copy()                         # columns v_1 .. v_{j+1}
        info.V[:, j] = w / H[j, j - 1] if H[j, j - 1] != 0 else 0.0
        info.u = u.copy()
    return y_new, tau, info


# ---------------------------------------------------------------------------
# EE2 step (Section 4, eqs. IVPlin, EE2, yt; Fig. 3)
# ---------------------------------------------------------------------------

def ee_step(y: np.ndarray, prob: Problem, tau0: float, tol_phi: float, m_max: int,
            tau_min: float = 0.0, keep_basis: bool = False):
    """One EE2 step with the nonlinear residual-time restart (Fig. 3).

    The linear IVP y' = -Ahat_n y + ghat^n is frozen at y^n (eq. IVPlin); its
    exact solution is y^n + t phi(-t Ahat_n)(ghat^n - Ahat_n y^n) (eq. yt).  The
    returned tau may be smaller than tau0 (it is the accepted step).
    """
    g = ghat(y, prob)
    v1 = g - ahat_mv(y, y, prob)
    return krylov_phi_cycle(lambda v: ahat_mv(v, y, prob), y, v1, tau0, tol_phi, m_max,
                            tau_min, keep_basis)


@dataclass
class ConstStepInfo:
    restarts: int       # Krylov cycles beyond the first
    matvecs: int        # matvecs with Ahat_n, counting each start vector as one
    js: list


def ee_step_const(y: np.ndarray, prob: Problem, tau: float, tol_phi: float, m_max: int,
                  tau_min: float = 0.0):
    """One constant-step EE2 step with linear residual-time restarting (Section 4.1; reading R2).

    Ahat_n and ghat^n stay frozen at y^n; each cycle of Fig. 3 advances the
    linear IVP (eq. IVPlin) by the step its residual allows, until the whole
    tau is covered.
    """
    g = ghat(y, prob)
    mv = lambda v: ahat_mv(v, y, prob)
    z = y.copy()
    covered = 0.0
    js, matvecs, cycles = [], 0, 0
    while True:
        v1 = g - mv(z)
        remaining = tau - covered
        z, s, info = krylov_phi_cycle(mv, z, v1, remaining, tol_phi, m_max, tau_min)
        cycles += 1
        matvecs += 1 + info.j
        js.append(info.j)
        if info.converged:
            break
        covered += s
    return z, ConstStepInfo(cycles - 1, matvecs, js)


def tol_phi_rule(gnorm: float, beta: float, tol: float) -> float:
    """tol_phi = max{min{||ghat||/(10 beta), 1/10, 10 tol}, 1e-7} (eq. tol_phi)."""
    first = gnorm / (10.0 * beta) if beta > 0 else math.inf
    return max(min(first, 0.1, 10.0 * tol), 1e-7)


def pc_estimate(y_n: np.ndarray, y_np1: np.ndarray, tau: float, prob: Problem):
    """Predictor-corrector estimate (eq. LIMest).

    y_PC = y^n - tau/2 A (F'(y^n) + F'(y^{n+1}) + eps^2 A (y^n + y^{n+1}));
    est = ||y^{n+1} - y_PC|| / ||y_PC||.  Returns (est, y_PC).  With variable
    mobility the outer operators of the two states differ: y_PC = y^n +
    tau/2 (f(y^n) + f(y^{n+1})) (reading R12).
    """
    if prob.mobility is not None:
        y_pc = y_n + 0.5 * tau * (rhs(y_n, prob) + rhs(y_np1, prob))
        return float(np.linalg.norm(y_np1 - y_pc) / np.linalg.norm(y_pc)), y_pc
    inner = Fprime(y_n) + Fprime(y_np1) + prob.eps ** 2 * lap(y_n + y_np1, prob)
    y_pc = y_n - 0.5 * tau * lap(inner, prob)
    return float(np.linalg.norm(y_np1 - y_pc) / np.linalg.norm(y_pc)), y_pc


def ee_dt(tau: float, est: float, tol: float) -> float:
    """tau_new = min{5/4 tau, sqrt(tol/est) tau} (eq. EEdt); est = 0 -> 5/4 tau (reading R4)."""
    if est == 0.0:
        return 1.25 * tau
    return min(1.25 * tau, math.sqrt(tol / est) * tau)


def lim_dt(tau: float, est: float, tol: float) -> float:
    """tau_new = tol/est tau (eq. LIMdt); est = 0 keeps tau (reading R4)."""
    if est == 0.0:
        return tau
    return tol / est * tau


@dataclass
class RunRecord:
    t: float
    steps: int
    matvecs: int
    taus: list
    js: list
    ests: list


def ee_adaptive(y0: np.ndarray, prob: Problem, tau0: float, T: float, tol: float, m_max: int,
                max_steps: int | None = None, tol_phi_fixed: float | None = None,
                tau_min: float = 0.0):
    """Adaptive EE2 time stepping (Fig. 4; eqs. tol_phi, LIMest, EEdt).

    Runs until t >= T or max_steps accepted steps (T = inf with max_steps gives
    a fixed number of steps).  Steps are never rejected.  tol_phi_fixed, when
    given, replaces eq. tol_phi.  Returns (y, RunRecord).
    """
    t, tau, y = 0.0, tau0, np.array(y0, dtype=np.float64, copy=True)
    rec = RunRecord(0.0, 0, 0, [], [], [])
    while t < T and (max_steps is None or rec.steps < max_steps):
        clipped = False
        if t + tau > T:
            tau = T - t
            clipped = True
        g = ghat(y, prob)
        v1 = g - ahat_mv(y, y, prob)
        beta = float(np.linalg.norm(v1))
        tphi = tol_phi_fixed if tol_phi_fixed is not None else tol_phi_rule(float(np.linalg.norm(g)), beta, tol)
        y_new, tau_acc, info = krylov_phi_cycle(lambda v: ahat_mv(v, y, prob), y, v1, tau, tphi,
                                                m_max, tau_min)
        est, _ = pc_estimate(y, y_new, tau_acc, prob)
        t = T if (clipped and info.converged) else t + tau_acc          # reading R5
        tau = ee_dt(tau_acc, est, tol)
        y = y_new
        rec.steps += 1
        rec.matvecs += 1 + info.j
        rec.taus.append(tau_acc)
        rec.js.append(info.j)
        rec.ests.append(est)
    rec.t = t
    return y, rec


def ee_const_run(y0: np.ndarray, prob: Problem, tau: float, n_steps: int, tol_phi: float,
                 m_max: int):
    """n_steps constant-step EE2 steps (linear RT restarting, reading R2)."""
    y = np.array(y0, dtype=np.float64, copy=True)
    infos = []
    for _ in range(n_steps):
        y, info = ee_step_const(y, prob, tau, tol_phi, m_max)
        infos.append(info)
    return y, infos


# ---------------------------------------------------------------------------
# LIM step (Section 3.1, eq. p; Fig. 1) and its adaptive driver (Fig. 2)
# ---------------------------------------------------------------------------

def _stencil_columns(prob: Problem):
    """Columns of A and A^2 through the origin, as {offset: coefficient} maps.

    Obtained by applying lap() to a unit impulse (so they are A e_0 and A A e_0
    literally); requires n >= 5 so that no two offsets alias on the torus.
    """
    small = Problem(prob.dim, 9, prob.eps, prob.eyre)
    e0 = np.zeros(small.N)
    centre = tuple([4] * prob.dim)
    e0[np.ravel_multi_index(centre, small.shape)] = 1.0
    a_col = lap(e0, small).reshape(small.shape) * (small.h ** 2) / (prob.h ** 2)
    b_col = lap(lap(e0, small), small).reshape(small.shape) * (small.h ** 4) / (prob.h ** 4)
    offs = {}
    for idx in np.argwhere((a_col != 0) | (b_col != 0)):
        off = tuple(int(i) - 4 for i in idx)
        offs[off] = (float(a_col[tuple(idx)]), float(b_col[tuple(idx)]))
    return offs


def lambda_max(y: np.ndarray, prob: Problem) -> float:
    """lambda_max := ||Ahat_n||_1 = max_j sum_i |ahat_ij| (the spectral bound of Fig. 1).

    Column j of Ahat_n = A diag(d) + eps^2 A^2 is d_j A e_j + eps^2 A^2 e_j, so
    its absolute sum is a sum over the stencil offsets of
    |d_j a_off + eps^2 b_off|.  With Neumann boundaries the columns near the
    boundary differ, and with variable mobility every column differs; there the
    1-norm is taken from the assembled sparse matrix.
    """
    if prob.bc == "neumann" or prob.mobility is not None:
        M = abs(assemble_ahat(y, prob))
        return float(np.asarray(M.sum(axis=0)).max())
    if prob.n < 5:
        raise ValueError("n >= 5 required (stencil offsets alias on smaller tori)")
    d = jac_diag(y, prob)
    colsum = np.zeros_like(d)
    for a, b in _stencil_columns(prob).values():
        colsum += np.abs(d * a + prob.eps ** 2 * b)
    return float(colsum.max())


def lim_order(tau: float, lam: float) -> int:
    """p = ceil((pi/4) / (pi/2 - arctan sqrt(tau lambda_max))) (eq. p)."""
    return int(math.ceil((math.pi / 4.0) / (math.pi / 2.0 - math.atan(math.sqrt(tau * lam)))))


def lim_coefficients(p: int, lam: float):
    """Chebyshev nodes beta_i = cos(pi (2i - 1) / (2p)) and a_i = lambda_max
    (z_1 - beta_i) / (1 + z_1), z_1 = beta_1, indexed by i = 1..p (Fig. 1)."""
    betas = [math.cos(math.pi * (2 * i - 1) / (2 * p)) for i in range(1, p + 1)]
    z1 = betas[0]
    a = [lam / (1.0 + z1) * (z1 - b) for b in betas]
    return betas, a


LEJA_TIE = 1e-9


def lim_node_order(p: int) -> list:
    """Order in which a LIM step takes the nodes (reading R6): 0-based indices
    into lim_coefficients, beta_1 first, then the Leja rule -- the node with
    the largest sum of log-distances to the nodes taken so far; among nodes
    within LEJA_TIE (relative) of the largest sum, the smallest index."""
    betas, _ = lim_coefficients(p, 1.0)
    b = np.array(betas)
    taken = np.zeros(p, dtype=bool)
    score = np.zeros(p)
    order = []
    r = 0
    for _ in range(p):
        order.append(r)
        taken[r] = True
        with np.errstate(divide="ignore"):
            score += np.log(np.abs(b - b[r]))
        if len(order) == p:
            break
        cand = np.where(taken, -np.inf, score)
        best = cand.max()
        r = int(np.flatnonzero(cand >= best - LEJA_TIE * max(1.0, abs(best)))[0])
    return order


def lim_iterate(matvec, g: np.ndarray, y: np.ndarray, tau: float, lam: float):
    """The Chebyshev iteration of Fig. 1 for y' = -Ahat y + g, y(0) = y, given lambda_max.

    Stages: the nodes in lim_node_order (first sweep), then the same order
    without beta_1 (second sweep).  Returns (y^{n+1}, p); 2p - 1 matvecs are made.
    """
    p = lim_order(tau, lam)
    _, a = lim_coefficients(p, lam)
    order = lim_node_order(p)
    yprev = y
    for i in order + order[1:]:
        am = a[i]
        yprev = (y + tau * am * yprev + tau * (g - matvec(yprev))) / (1.0 + tau * am)
    return yprev, p


def lim_step(y: np.ndarray, prob: Problem, tau: float):
    """One LIM step (Fig. 1) with Ahat_n, ghat^n from eq. A_g (or A_g_cs). Returns (y_new, p)."""
    lam = lambda_max(y, prob)
    return lim_iterate(lambda v: ahat_mv(v, y, prob), ghat(y, prob), y, tau, lam)


def lim_adaptive(y0: np.ndarray, prob: Problem, tau0: float, T: float, tol: float,
                 max_steps: int | None = None):
    """Adaptive LIM time stepping (Fig. 2; eqs. LIMest, LIMdt)."""
    t, tau, y = 0.0, tau0, np.array(y0, dtype=np.float64, copy=True)
    rec = RunRecord(0.0, 0, 0, [], [], [])
    while t < T and (max_steps is None or rec.steps < max_steps):
        clipped = False
        if t + tau > T:
            tau = T - t
            clipped = True
        y_new, p = lim_step(y, prob, tau)
        est, _ = pc_estimate(y, y_new, tau, prob)
        t = T if clipped else t + tau                                   # reading R5
        tau_used = tau
        tau = lim_dt(tau, est, tol)
        y = y_new
        rec.steps += 1
        rec.matvecs += 2 * p - 1
        rec.taus.append(tau_used)
        rec.js.append(p)
        rec.ests.append(est)
    rec.t = t
    return y, rec


def lim_const_run(y0: np.ndarray, prob: Problem, tau: float, n_steps: int):
    y = np.array(y0, dtype=np.float64, copy=True)
    ps = []
    for _ in range(n_steps):
        y, p = lim_step(y, prob, tau)
        ps.append(p)
    return y, ps


# ---------------------------------------------------------------------------
# Diagnostics (Section 5: eqs. acc_reached, Ediscr; mass)
# ---------------------------------------------------------------------------

def energy(y: np.ndarray, prob: Problem) -> float:
    """Discrete Ginzburg-Landau energy (eq. Ediscr): periodic with wrap-around, or
    on the Neumann grid, where the differences to the mirror ghost cells vanish.

    E_h = h^d sum F(y) + eps^2/2 h^(d-2) sum over grid edges of (difference)^2.
    """
    Y = y.reshape(prob.shape)
    h, d = prob.h, prob.dim
    if prob.bc == "neumann":
        grad2 = sum(np.sum(np.diff(Y, axis=ax) ** 2) for ax in range(d))
    else:
        grad2 = sum(np.sum((np.roll(Y, -1, axis=ax) - Y) ** 2) for ax in range(d))
    return float(h ** d * np.sum(Fenergy(Y)) + 0.5 * prob.eps ** 2 * h ** (d - 2) * grad2)


def mass(y: np.ndarray) -> float:
    """m = sum_j y_j (Section 5, mass deviation figures)."""
    return float(np.sum(y))


def rel_error(y: np.ndarray, y_ref: np.ndarray) -> float:
    """||y - y_ref|| / ||y_ref|| (eq. acc_reached)."""
    return float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))
