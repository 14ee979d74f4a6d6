"""Pins of the tracking oracle (Sec. 6.3, eq. (qp_rto)) against facts that do
not come from its own formulas: a library Cholesky, eigenvalues, Newton's
quadratic convergence on F, and finite differences of F."""
import numpy as np
import pytest

import gridgen
from oracle import powerflow as pf
from oracle import tracking


def _spd(n, seed, lo=1.0, hi=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * rng.uniform(lo, hi, n)) @ Q.T


@pytest.mark.parametrize("n", [1, 7, 40])
def test_cholesky_matches_library_and_reads_only_the_lower_triangle(n):
    A = _spd(n, seed=n)
    L, j = tracking.cholesky(A)
    assert j == -1
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=0, atol=1e-13 * np.abs(A).max())
    assert np.all(np.triu(L, 1) == 0.0)
    B = A.copy()
    B[np.triu_indices(n, 1)] = np.nan  # the strict upper triangle is never read
    L2, j2 = tracking.cholesky(B)
    assert j2 == -1 and np.array_equal(L2, L)


def test_cholesky_reports_the_first_failing_column():
    # leading minors 0 .. 11 positive definite; the pivot of column 12 is -1
    A = _spd(20, seed=3)
    L0 = np.linalg.cholesky(A)
    A[12, 12] -= L0[12, 12] ** 2 + 1.0
    _, j = tracking.cholesky(A)
    ev = [np.linalg.eigvalsh(A[:m, :m]).min() for m in range(1, 21)]
    first_bad = next(m for m in range(20) if ev[m] <= 0.0)
    assert j == first_bad == 12


def test_solve_spd_matches_library_solve():
    A = _spd(30, seed=5)
    B = np.random.default_rng(6).standard_normal((30, 3))
    X = tracking.solve_spd(A, B)
    np.testing.assert_allclose(X, np.linalg.solve(A, B), rtol=1e-12, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        tracking.solve_spd(-A, B)


def test_shift_is_zero_on_spd_and_the_first_sufficient_doubling_otherwise():
    A = _spd(25, seed=7)
    _, tau, tries = tracking.shifted_cholesky(A)
    assert tau == 0.0 and tries == 1
    # indefinite: eigenvalues in [-3, 5]
    rng = np.random.default_rng(8)
    Q, _ = np.linalg.qr(rng.standard_normal((25, 25)))
    lam = np.linspace(-3.0, 5.0, 25)
    M = (Q * lam) @ Q.T
    L, tau, tries = tracking.shifted_cholesky(M)
    assert tries > 1
    # the factor is that of M + tau I, which is positive definite ...
    np.testing.assert_allclose(L @ L.T, M + tau * np.eye(25), atol=1e-12)
    assert lam.min() + tau > 0.0
    # ... and the previous shift of the sequence was not enough (either
    # tau = 2 tau_prev, or tau_prev was the first shift -min diag + beta)
    beta = 1e-3 * np.abs(np.diag(M)).max()
    tau0 = -np.diag(M).min() + beta
    prev = tau / 2.0 if tau > tau0 * 1.5 else None
    if prev is not None:
        assert lam.min() + prev <= 0.0


def test_fixed_loads_make_tracking_newton_on_F_with_quadratic_convergence():
    """With the loads held, p <- p + d is Newton's method on F (H the exact
    Hessian, g the exact gradient): ||g|| must fall quadratically.  A wrong
    term anywhere in H (or a sign in g) turns this into linear convergence or
    divergence."""
    grid = gridgen.config_grid("c0", 0)
    p = pf.Oracle(grid).p0()
    x = None
    norms = []
    for _ in range(12):
        s, g, H, d, tau = tracking.step(grid, p, x0=x)
        norms.append(float(np.abs(g).max()))
        assert tau == 0.0  # H positive definite along this path
        x, p = s.x, p + d
        if norms[-1] < 1e-12:
            break
    assert norms[-1] < 1e-11
    quad = [(a, b) for a, b in zip(norms, norms[1:]) if 1e-7 < a < 1e-2]
    assert len(quad) >= 2
    for a, b in quad:
        assert b <= 50.0 * a * a, (a, b)


def test_step_is_a_descent_direction_with_the_directional_derivative_of_F():
    """Central differences of F(p) = f(x(p), p) along d (each point solved by
    Newton) give g^T d, which is negative for d = -H^{-1} g with H positive
    definite."""
    grid = gridgen.config_grid("c0", 0)
    orc = pf.Oracle(grid)
    s, g, H, d, tau = tracking.step(grid, orc.p0())
    assert tau == 0.0
    u = d / np.abs(d).max()
    h = 1e-5
    Fp = pf.solve(grid, p=s.p + h * u).F
    Fm = pf.solve(grid, p=s.p - h * u).F
    fd = (Fp - Fm) / (2 * h)
    assert abs(fd - g @ u) <= 1e-6 * max(1.0, abs(g @ u))
    assert g @ d < 0.0


def test_projection_keeps_bounds_and_ramps():
    rng = np.random.default_rng(9)
    p = rng.uniform(-1, 1, 50)
    d = rng.uniform(-2, 2, 50)
    lo, hi = np.full(50, -0.8), np.full(50, 0.9)
    ramp = rng.uniform(0.0, 0.3, 50)
    q = tracking.project(p, d, lo, hi, ramp)
    assert np.all(q >= lo) and np.all(q <= hi)
    inside = (p >= lo) & (p <= hi)
    assert np.all(np.abs(q - p)[inside] <= ramp[inside] + 1e-15)
    free = (np.abs(d) <= ramp) & (p + d >= lo) & (p + d <= hi)
    np.testing.assert_array_equal(q[free], (p + d)[free])


def test_load_trajectory_recipe():
    grid = gridgen.config_grid("c1", 0)
    Pd, Qd = gridgen.load_trajectory(grid, steps=60, amp=0.03, noise=0.005, seed=2)
    assert Pd.shape == Qd.shape == (60, grid.n_bus)
    s = Pd / np.where(grid.Pd == 0, 1.0, grid.Pd)[None, :]
    loaded = grid.Pd != 0
    assert np.all(np.abs(s[:, loaded] - 1.0) < 2 * 0.03 + 6 * 0.005)
    assert np.all(np.abs(s[0, loaded] - 1.0) < 6 * 0.005)  # starts at the base loads
    np.testing.assert_allclose(Pd[:, loaded] / grid.Pd[loaded], Qd[:, loaded] / grid.Qd[loaded])
