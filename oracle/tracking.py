"""Real-time tracking of the reduced-space optimum: FP64 CPU oracle.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this module; the library never
does, and this module shares no code with it.

What is computed (Sec. 6.3, eq. (nonlinearoptreduced_time) and eq.
(qp_rto)): at time t, with loads w_t = (P^d_t, Q^d_t) and control p_t,

* Step 1: the power flow g(x, p_t; w_t) = 0 by Newton (started from the
  previous state), the reduced gradient g_t = grad_p F(p_t; w_t) and the
  reduced Hessian H_t (Algorithm 2 on the columns of the identity);
* Step 2: H_t d_t = -g_t by a dense Cholesky factorisation, and
  p_{t+1} = p_t + d_t.

Readings where the paper is silent:

* the update is projected on caller-given bounds lo <= p <= hi and on
  per-step ramp limits |p_{t+1} - p_t| <= r (each optional).  The tracked
  problem is an OPF whose controls carry bounds, and set-points of a
  real-time controller move at limited rates, while the step of eq.
  (qp_rto) has neither; with free voltage set-points the cost keeps falling
  as voltages rise (losses shrink), and plain steps leave the region where
  the power flow is solvable.
* the factorisation reads only the lower triangle of H_t (the computed H_t
  is symmetric only up to rounding).
* H_t is not positive definite everywhere on the synthetic grids (its
  smallest eigenvalue falls with the loading), where eq. (qp_rto) has no
  Cholesky factor and -H_t^{-1} g_t need not descend.  The step then
  factorises H_t + tau I with the smallest tau of a doubling sequence that
  succeeds (Cholesky with an added multiple of the identity, Nocedal and
  Wright, Algorithm 3.3); tau = 0, the paper's step, whenever H_t is
  positive definite.

A library triangular solve (scipy) serves as the substitution step.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .powerflow import Oracle, Solved


def cholesky(A):
    """A = L L^T with L lower triangular, column by column from the lower
    triangle of A (the strict upper triangle is never read).  Returns
    (L, j): j = -1 on success, else the first column whose pivot
    A_jj - sum_k L_jk^2 is not positive (L is then complete up to j - 1)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    for j in range(n):
        s = A[j, j] - L[j, :j] @ L[j, :j]
        if not s > 0.0:
            return L, j
        L[j, j] = np.sqrt(s)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, -1


def solve_spd(A, B, shift=0.0):
    """X with (A + shift I) X = B by cholesky() and the two triangular
    substitutions; raises np.linalg.LinAlgError at a non-positive pivot."""
    A = np.asarray(A, dtype=np.float64)
    As = A + shift * np.eye(A.shape[0]) if shift else A
    L, j = cholesky(As)
    if j >= 0:
        raise np.linalg.LinAlgError(f"leading minor {j + 1} is not positive definite")
    Y = sla.solve_triangular(L, B, lower=True)
    return sla.solve_triangular(L.T, Y, lower=False)


def shifted_cholesky(A, shift=0.0, beta_rel=1e-3, max_tries=64):
    """Cholesky with an added multiple of the identity (Nocedal and Wright,
    Numerical Optimization, Algorithm 3.3): tau_0 = shift if every diagonal
    entry of A + shift I is positive, else -min_i a_ii + beta; on a failed
    factorisation of A + tau I, tau <- max(2 tau, beta), with
    beta = beta_rel * max_i |a_ii|.  Returns (L, tau, tries)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    dg = np.diag(A)
    beta = beta_rel * (float(np.max(np.abs(dg))) if n else 0.0)
    if beta == 0.0:
        beta = beta_rel
    tau = float(shift) if n == 0 or float(np.min(dg)) + shift > 0.0 else float(-np.min(dg) + beta)
    for tries in range(1, max_tries + 1):
        L, j = cholesky(A + tau * np.eye(n) if tau else A)
        if j < 0:
            return L, tau, tries
        tau = max(2.0 * tau, beta)
    raise np.linalg.LinAlgError("no shift made the matrix positive definite")


def newton_direction(H, g, shift=0.0):
    """d with (H + tau I) d = -g, tau from shifted_cholesky (tau = 0 when H
    is positive definite and shift = 0: the step of eq. (qp_rto)).  Returns
    (d, tau, tries)."""
    L, tau, tries = shifted_cholesky(H, shift=shift)
    y = sla.solve_triangular(L, -np.asarray(g, dtype=np.float64), lower=True)
    return sla.solve_triangular(L.T, y, lower=False), tau, tries


def step(grid, p, x0=None, shift=0.0, tol=1e-13):
    """One tracking update at control p on `grid` (whose loads are w_t):
    returns (solved operating point, g_t, H_t, d_t, tau)."""
    s = Solved(Oracle(grid), p=p, tol=tol, x0=x0)
    H = s.reduced_hessian()
    d, tau, _ = newton_direction(H, s.grad, shift=shift)
    return s, s.grad.copy(), H, d, tau


def project(p, d, lo=None, hi=None, ramp=None):
    """p + d clipped to lo <= . <= hi and |. - p| <= ramp (any may be None)."""
    q = p + d
    if ramp is not None:
        q = np.minimum(np.maximum(q, p - ramp), p + ramp)
    if lo is not None:
        q = np.maximum(q, lo)
    if hi is not None:
        q = np.minimum(q, hi)
    return q


def trajectory(grid, Pd_seq, Qd_seq, p0=None, lo=None, hi=None, ramp=None, shift=0.0):
    """T tracking updates over the load sequence (T rows of P^d and Q^d).
    Returns per step the control p_t, the objective F(p_t; w_t), |g_t|_inf,
    d_t and the shift tau."""
    g = grid.copy()
    p = Oracle(grid).p0() if p0 is None else np.array(p0, dtype=np.float64)
    x = None
    out = []
    for Pd, Qd in zip(Pd_seq, Qd_seq):
        g.Pd = np.asarray(Pd, dtype=np.float64).copy()
        g.Qd = np.asarray(Qd, dtype=np.float64).copy()
        s, gr, _, d, tau = step(g, p, x0=x, shift=shift)
        out.append({"p": p.copy(), "F": s.F, "grad_inf": float(np.max(np.abs(gr))), "d": d, "tau": tau})
        x = s.x
        p = project(p, d, lo, hi, ramp)
    return out
