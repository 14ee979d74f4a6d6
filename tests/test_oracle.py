"""Pins of the FP64 oracle against mathematics the paper fixes (CPU only).

Each test checks the oracle against something other than itself: closed
forms, a direct-direct Hessian from autograd tensors, finite differences, the
Taylor remainder, symmetry, an exactly known special case, the paper's
Table 1 bookkeeping, and the quadratic rate of Newton's method.
"""
from pathlib import Path

import mpmath as mp
import numpy as np
import pytest

import gridgen
from oracle.powerflow import Oracle, Solved, solve
from tests.brute_force import Brute

GOLDEN = Path(__file__).resolve().parent / "golden"


def _relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- T10 (Table 1)
def test_table1_bookkeeping():
    """n_x = n_v - 1 + n_pq and n_p = 2 n_gen - 1 must partition the buses.

    For every case of Table 1, n_pq = n_x - n_v + 1 and n_gen = (n_p + 1)/2
    must be whole and add up to n_v (reading of the parameter vector as
    [Pg_pv; v_ref; v_pv]).
    """
    rows = [ln.split() for ln in (GOLDEN / "table1_dims.txt").read_text().splitlines()
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 6
    for name, nv, ne, nx, npar in rows:
        nv, nx, npar = int(nv), int(nx), int(npar)
        n_pq = nx - nv + 1
        assert (npar + 1) % 2 == 0, name
        n_gen = (npar + 1) // 2
        assert n_pq > 0 and n_pq + n_gen == nv, name


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_dims_of_synthetic_grids(name):
    g = gridgen.config_grid(name, 0)
    o = Oracle(g)
    assert o.n_x == g.n_bus - 1 + g.n_pq
    assert o.n_p == 2 * g.n_gen - 1
    assert o.n_x == g.n_x and o.n_p == g.n_p


# ---------------------------------------------------------- T1: 2-bus closed form
R, X, P, Q, V1, C2, C1 = 0.02, 0.1, 1.2, 0.4, 1.03, 1.5, 3.0


def _two_bus_closed(v1):
    """Reference bus at v1, PQ bus with load P + jQ over z = R + jX, no charging.

    v2^2 = u solves u^2 - a u + |z|^2 |S|^2 = 0, a = v1^2 - 2 (R P + X Q)
    (high-voltage root); the slack supplies P plus the loss R |S|^2 / u.
    """
    a = v1 ** 2 - 2 * (R * P + X * Q)
    z2s2 = (R * R + X * X) * (P * P + Q * Q)
    u = (a + mp.sqrt(a * a - 4 * z2s2)) / 2
    Pg = P + R * (P * P + Q * Q) / u
    F = C2 * Pg ** 2 + C1 * Pg
    # angle of V2: v1 v2 e^{-j theta2} = u + z conj(S)
    th2 = -mp.arg(mp.mpc(u + R * P + X * Q, X * P - R * Q))
    return F, mp.sqrt(u), th2


def test_two_bus_pq_closed_form():
    mp.mp.dps = 40
    g = gridgen.two_bus(R, X, P, Q, V1, C2, C1)
    s = solve(g)
    F, v2, th2 = _two_bus_closed(mp.mpf(V1))
    dF = mp.diff(lambda t: _two_bus_closed(t)[0], mp.mpf(V1), 1)
    d2F = mp.diff(lambda t: _two_bus_closed(t)[0], mp.mpf(V1), 2)
    assert s.o.n_x == 2 and s.o.n_p == 1
    assert abs(s.x[0] - float(th2)) < 1e-13
    assert abs(s.x[1] - float(v2)) < 1e-13
    assert abs(s.F - float(F)) < 1e-12 * abs(float(F))
    assert abs(s.grad[0] - float(dF)) < 1e-11 * abs(float(dF))
    H = s.reduced_hessian()
    assert abs(H[0, 0] - float(d2F)) < 1e-10 * abs(float(d2F))


def test_two_bus_pv_closed_form():
    """Reference bus + PV bus: theta_2 from the PV bus's active balance in closed form.

    With y = g + j b = 1/(r + jx): P_2 = g v2^2 - v1 v2 (g cos t + b sin t), so
    g cos t + b sin t = k, t = phi - arccos(k / rho) (the small-angle root),
    phi = atan2(b, g), rho = |y|.  The slack supplies
    P_1 = g v1^2 - v1 v2 (g cos t - b sin t).
    """
    mp.mp.dps = 40
    r, x, Pd2, Qd2 = 0.03, 0.12, 0.5, 0.2
    c2a, c1a, c2b, c1b = 1.2, 2.5, 0.8, 3.5
    p0 = (mp.mpf("1.1"), mp.mpf("1.02"), mp.mpf("1.04"))  # Pg2, v1, v2
    y = 1 / mp.mpc(r, x)
    gg, bb = y.real, y.imag

    def F(Pg2, v1, v2):
        k = (gg * v2 ** 2 - (Pg2 - Pd2)) / (v1 * v2)
        rho = mp.sqrt(gg * gg + bb * bb)
        phi = mp.atan2(bb, gg)
        cands = [phi - mp.acos(k / rho), phi + mp.acos(k / rho)]
        t = min(cands, key=lambda c: abs(c))
        P1 = gg * v1 ** 2 - v1 * v2 * (gg * mp.cos(t) - bb * mp.sin(t))
        return c2a * P1 ** 2 + c1a * P1 + c2b * Pg2 ** 2 + c1b * Pg2

    g = gridgen.two_bus(r, x, Pd2, Qd2, float(p0[1]), c2a, c1a, pv=True, Pg2=float(p0[0]),
                        v2=float(p0[2]), c2b=c2b, c1b=c1b)
    s = solve(g)
    assert s.o.n_x == 1 and s.o.n_p == 3
    Hc = np.zeros((3, 3))
    gc = np.zeros(3)
    for i in range(3):
        o = [0, 0, 0]
        o[i] = 1
        gc[i] = float(mp.diff(F, p0, tuple(o)))
        for j in range(3):
            o2 = [0, 0, 0]
            o2[i] += 1
            o2[j] += 1
            Hc[i, j] = float(mp.diff(F, p0, tuple(o2)))
    assert abs(s.F - float(F(*p0))) < 1e-12 * abs(float(F(*p0)))
    assert _relerr(s.grad, gc) < 1e-11
    assert _relerr(s.reduced_hessian(), Hc) < 1e-10


# ------------------------------------------------- T4: direct-direct brute force
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_direct_direct(seed):
    g = gridgen.ring9(seed)
    s = solve(g)
    b = Brute(g)
    Hb, gb, res = b.hessian(s.x, s.p)
    assert np.max(np.abs(res)) < 1e-12  # oracle state solves the independent g
    assert _relerr(s.grad, gb) < 1e-12
    H = s.reduced_hessian()
    assert _relerr(H, Hb) < 1e-11


def test_brute_force_14_bus():
    """A second topology: a 14-bus planar grid from the geometric generator."""
    g = gridgen.geometric(14, 20, 4, seed=5, alpha=0.3)
    s = solve(g)
    Hb, gb, _ = Brute(g).hessian(s.x, s.p)
    assert _relerr(s.grad, gb) < 1e-12
    assert _relerr(s.reduced_hessian(), Hb) < 1e-11


# ----------------------------------------- planted mistakes must fail the pins
@pytest.mark.parametrize("mutation", ["drop_slack_rank1", "flip_psi", "flip_hxp_sign",
                                      "drop_pg_diag"])
def test_planted_mistakes_are_caught(mutation, monkeypatch):
    g = gridgen.ring9(0)
    ref = Brute(g)
    orig_lh = Oracle.lagrangian_hessian

    def mutated_lh(self, x, p, lam):
        H = orig_lh(self, x, p, lam).toarray()
        nx = self.n_x
        if mutation == "drop_slack_rank1":
            th, v, _ = self.unpack(x, p)
            a = self._slack_row(th, v)
            r = self.gen_of_bus[self.ref]
            H -= 2.0 * self.grid.c2[r] * np.outer(a, a)
        elif mutation == "flip_hxp_sign":
            H[:nx, nx:] *= -1.0
        elif mutation == "drop_pg_diag":
            d = np.arange(nx, nx + self.npv)
            H[d, d] = 0.0
        import scipy.sparse as sp
        return sp.csr_matrix(H)

    monkeypatch.setattr(Oracle, "lagrangian_hessian", mutated_lh)
    s = solve(g)
    if mutation == "flip_psi":
        orig_hvp = Solved.hvp

        def bad_hvp(self, W):
            W2 = np.asarray(W, dtype=np.float64)
            B = self.Gp @ W2
            Z = -self.lu.solve(B)
            Y = self.Hl @ np.vstack([Z, W2])
            Psi = -self.lu.solve(Y[:self.o.n_x], trans="T")
            return Y[self.o.n_x:] - self.Gp.T @ Psi

        monkeypatch.setattr(Solved, "hvp", bad_hvp)
        assert orig_hvp is not None
    Hb, _, _ = ref.hessian(s.x, s.p)
    assert _relerr(s.reduced_hessian(), Hb) > 1e-6


# --------------------------------------------------- T5: finite differences
def _F_at(g, p, x0):
    o = Oracle(g)
    x, _, ok = o.newton(p, tol=1e-14, x0=x0)
    assert ok
    return o.objective(x, p), x


def test_gradient_and_hessian_against_central_differences():
    g = gridgen.ring9(1)
    s = solve(g)
    n_p = s.o.n_p
    h = 1e-5
    H = s.reduced_hessian()
    fd_grad = np.zeros(n_p)
    fd_H = np.zeros((n_p, n_p))
    for j in range(n_p):
        e = np.zeros(n_p)
        e[j] = h
        Fp, xp = _F_at(g, s.p + e, s.x)
        Fm, xm = _F_at(g, s.p - e, s.x)
        fd_grad[j] = (Fp - Fm) / (2 * h)
        gp = Solved(Oracle(g), p=s.p + e).grad
        gm = Solved(Oracle(g), p=s.p - e).grad
        fd_H[:, j] = (gp - gm) / (2 * h)
    assert _relerr(s.grad, fd_grad) < 1e-7
    assert _relerr(H, fd_H) < 1e-6


# ------------------------------------------------------- T6: Taylor remainder
def test_taylor_remainder_is_third_order():
    g = gridgen.ring9(2)
    s = solve(g)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(s.o.n_p)
    w /= np.linalg.norm(w)
    Hw = s.hvp(w)
    eps = np.array([4e-3, 2e-3, 1e-3, 5e-4])
    rem = []
    for e in eps:
        Fe, _ = _F_at(g, s.p + e * w, s.x)
        rem.append(abs(Fe - s.F - e * s.grad @ w - 0.5 * e * e * w @ Hw))
    slope = np.polyfit(np.log(eps), np.log(rem), 1)[0]
    assert 2.8 < slope < 3.3, (slope, rem)


# --------------------------------------------------------------- T7: symmetry
def test_hessian_symmetry_1k():
    s = solve(gridgen.config_grid("c1", 0))
    H = s.reduced_hessian(64)
    assert np.max(np.abs(H - H.T)) / np.max(np.abs(H)) < 1e-12


# ---------------------------------------- T3: lossless special case (any size)
@pytest.mark.parametrize("name", ["c0", "c1"])
def test_lossless_case_has_known_hessian(name):
    """With r = 0 the injections sum to zero, so Pg_ref = sum Pd - sum Pg_pv.

    F then depends on p only through the PV outputs:
    H = [diag(2 c2_pv) + 2 c2_ref 1 1^T, 0; 0, 0] although lambda != 0.
    """
    g = gridgen.lossless(gridgen.config_grid(name, 0))
    s = solve(g)
    o = s.o
    assert np.max(np.abs(s.lam)) > 1e-3
    npv = o.npv
    gi = o.gen_of_bus
    Hx = np.zeros((o.n_p, o.n_p))
    Hx[:npv, :npv] = np.diag(2 * g.c2[gi[o.pv]]) + 2 * g.c2[gi[o.ref]]
    H = s.reduced_hessian(64)
    assert np.max(np.abs(H - Hx)) / np.max(np.abs(Hx)) < 1e-10


# ------------------------------------------------ T8: Algorithm 1 == Algorithm 2
def test_sequential_equals_batched():
    s = solve(gridgen.config_grid("c1", 1))
    W = gridgen.directions(s.o.n_p, 16, 11)
    HW = s.hvp(W)
    for j in (0, 7, 15):
        assert _relerr(s.hvp(W[:, j]), HW[:, j]) < 1e-13


# ------------------------------------------------- T9: relabelling invariance
def test_relabelling_permutes_hessian():
    g = gridgen.ring9(0)
    perm = np.random.default_rng(4).permutation(g.n_bus)
    g2 = gridgen.relabel(g, perm)
    s1, s2 = solve(g), solve(g2)

    def keys(o):
        npv = o.npv
        k = [("Pg", int(b)) for b in o.pv] + [("v", o.ref)] + [("v", int(b)) for b in o.pv]
        return k, npv

    k1, _ = keys(s1.o)
    k2, _ = keys(s2.o)
    k1 = [(t, int(perm[b])) for t, b in k1]
    idx = [k2.index(k) for k in k1]
    H1 = s1.reduced_hessian()
    H2 = s2.reduced_hessian()
    assert _relerr(H2[np.ix_(idx, idx)], H1) < 1e-12


# ------------------------------------------------------------- T11: Newton rate
def test_newton_converges_quadratically():
    s = solve(gridgen.config_grid("c1", 0))
    h = s.hist
    seen = 0
    for a, b in zip(h[:-1], h[1:]):
        if 1e-10 < a < 1e-2:
            assert b <= 50.0 * a * a, h
            seen += 1
    assert seen >= 1, h


# ---------------------------------------------------------- T12: Jacobians by FD
def test_jacobians_against_central_differences():
    g = gridgen.ring9(0)
    o = Oracle(g)
    s = solve(g)
    Gx, Gp = o.jacobians(s.x, s.p)
    h = 1e-6
    fdx = np.zeros((o.n_x, o.n_x))
    for j in range(o.n_x):
        e = np.zeros(o.n_x)
        e[j] = h
        fdx[:, j] = (o.residual(s.x + e, s.p) - o.residual(s.x - e, s.p)) / (2 * h)
    fdp = np.zeros((o.n_x, o.n_p))
    for j in range(o.n_p):
        e = np.zeros(o.n_p)
        e[j] = h
        fdp[:, j] = (o.residual(s.x, s.p + e) - o.residual(s.x, s.p - e)) / (2 * h)
    assert np.max(np.abs(Gx.toarray() - fdx)) < 1e-7
    assert np.max(np.abs(Gp.toarray() - fdp)) < 1e-7


def test_grids_converge_for_the_workloads():
    """Every instance used by tests and benchmarks solves from its initial guess."""
    for name, insts in (("c0", [0, 1, 2]), ("c1", [0, 1, 2, 3]), ("c2", [0])):
        for i in insts:
            s = solve(gridgen.config_grid(name, i))
            assert s.hist[-1] <= 1e-13 or s.ok
