"""FP64 CPU oracle for the batched adjoint-adjoint reduced Hessian.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this module; the library never
does, and this module shares no code with it.

What is computed (paper: "Batched Second-Order Adjoint Sensitivity for
Reduced Space Methods"):

* power injections in the *bus form* of eq. (powerflow), with the sum taken
  over the adjacent buses and the bus itself, (g_ij + j b_ij) being the
  bus-admittance entries (Sec. 3.1);
* the balance equations g(x, p) of eq. (powerflowvec) with
  x = [theta_pv; theta_pq; v_pq] and p = [Pg_pv; v_ref; v_pv]
  (parameter count 2 n_gen - 1 as in Table 1);
* Newton-Raphson on g(., p) = 0 (Sec. 3.2);
* the first-order adjoint and reduced gradient, eq. (lagrangian) and
  eq. (reduced_gradient) (Sec. 3.3);
* the explicit sparse Lagrangian Hessian  d2 l = d2 f + sum_k lambda_k d2 g_k,
  assembled from second derivatives of each injection term (Sec. 4.1-4.2);
* the batched reduction of Algorithm 2 (Sec. 4.3): B = G_p W,
  Z = -G_x^{-1} B, [Y_x; Y_p] = d2 l [Z; W], Psi = -G_x^{-T} Y_x,
  H W = Y_p + G_p^T Psi.

Readings where the paper is silent or misprinted: the cost is quadratic over
all generators with the reference generator's output taken from its own bus
balance, P^g_ref = P^inj_ref + P^d_ref; the first adjoint system is read as
G_x z = -G_p w and the Hessian-vector product as d2_pp l w + d2_px l z +
G_p^T psi (dimensionally consistent forms of eq. (socadjoint) and
eq. (hessvecprod), matching Algorithms 1 and 2).

A library sparse LU (scipy's SuperLU) serves as the linear-solve step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PQ, PV, REF = 1, 2, 3


class Oracle:
    """Plain FP64 reference for one network."""

    def __init__(self, grid):
        self.grid = grid
        n = grid.n_bus
        self.n = n
        t = np.asarray(grid.bus_type)
        refs = np.flatnonzero(t == REF)
        if refs.size != 1:
            raise ValueError("exactly one reference bus is required")
        self.ref = int(refs[0])
        self.pv = np.flatnonzero(t == PV)
        self.pq = np.flatnonzero(t == PQ)
        npv, npq = self.pv.size, self.pq.size
        self.npv, self.npq = npv, npq
        self.n_x = npv + 2 * npq
        self.n_p = 2 * npv + 1
        gen_of_bus = np.full(n, -1)
        gen_of_bus[grid.gen_bus] = np.arange(grid.n_gen)
        self.gen_of_bus = gen_of_bus
        if np.any(gen_of_bus[self.pv] < 0) or gen_of_bus[self.ref] < 0:
            raise ValueError("every PV bus and the reference bus need a generator")

        # bus-space coordinates: theta_b -> b, v_b -> n + b; rows P_b -> b, Q_b -> n + b
        self.x_cols = np.concatenate([self.pv, self.pq, n + self.pq])
        self.g_rows = np.concatenate([self.pv, self.pq, n + self.pq])
        self.p_vcols = np.concatenate([[n + self.ref], n + self.pv])

        # bus admittance matrix (reading: series y = 1/(r + jx), half the
        # charging at each end, off-diagonals minus the series admittance)
        f = np.asarray(grid.br_from, dtype=np.int64)
        tt = np.asarray(grid.br_to, dtype=np.int64)
        ys = 1.0 / (np.asarray(grid.br_r) + 1j * np.asarray(grid.br_x))
        ysh = 0.5j * np.asarray(grid.br_b)
        rows = np.concatenate([f, tt, f, tt])
        cols = np.concatenate([f, tt, tt, f])
        vals = np.concatenate([ys + ysh, ys + ysh, -ys, -ys])
        Y = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
        Y.sum_duplicates()
        Yc = Y.tocoo()
        self.Yi = Yc.row.astype(np.int64)
        self.Yj = Yc.col.astype(np.int64)
        self.Gij = Yc.data.real.copy()
        self.Bij = Yc.data.imag.copy()

        # the coordinate selection E : (x, p) -> bus space (theta, v)
        nxp = self.n_x + self.n_p
        sel_rows = np.concatenate([self.x_cols, self.p_vcols])
        sel_cols = np.concatenate([np.arange(self.n_x), self.n_x + npv + np.arange(npv + 1)])
        self.E = sp.csr_matrix((np.ones(sel_rows.size), (sel_rows, sel_cols)), shape=(2 * n, nxp))

    # ------------------------------------------------------------------ state
    def p0(self) -> np.ndarray:
        g = self.grid
        gi = self.gen_of_bus
        return np.concatenate([g.Pg[gi[self.pv]], [g.Vg[gi[self.ref]]], g.Vg[gi[self.pv]]])

    def flat_start(self) -> np.ndarray:
        """Angles 0; PQ magnitudes from the grid's guess ``v0`` if it has one, else 1."""
        v0 = getattr(self.grid, "v0", None)
        vpq = np.ones(self.npq) if v0 is None else np.asarray(v0, dtype=np.float64)[self.pq]
        return np.concatenate([np.zeros(self.npv + self.npq), vpq])

    def unpack(self, x, p):
        n, npv, npq = self.n, self.npv, self.npq
        theta = np.zeros(n)
        v = np.zeros(n)
        theta[self.pv] = x[:npv]
        theta[self.pq] = x[npv:npv + npq]
        v[self.pq] = x[npv + npq:]
        v[self.ref] = p[npv]
        v[self.pv] = p[npv + 1:]
        return theta, v, p[:npv]

    # ------------------------------------------------------ eq. (powerflow)
    def injections(self, theta, v):
        """P_i, Q_i summed over the bus-admittance row of i (bus itself included)."""
        i, j = self.Yi, self.Yj
        a = theta[i] - theta[j]
        vv = v[i] * v[j]
        P = np.bincount(i, weights=vv * (self.Gij * np.cos(a) + self.Bij * np.sin(a)), minlength=self.n)
        Q = np.bincount(i, weights=vv * (self.Gij * np.sin(a) - self.Bij * np.cos(a)), minlength=self.n)
        return P, Q

    # ---------------------------------------------------- eq. (powerflowvec)
    def residual(self, x, p):
        theta, v, Pg = self.unpack(x, p)
        P, Q = self.injections(theta, v)
        g = self.grid
        return np.concatenate([
            P[self.pv] - Pg + g.Pd[self.pv],
            P[self.pq] + g.Pd[self.pq],
            Q[self.pq] + g.Qd[self.pq],
        ])

    def _term_parts(self, theta, v):
        """Per admittance entry: v_i, v_j and h, dh/da for the P and Q terms.

        Each term has the form v_i v_j h(theta_i - theta_j) with
        h_P = G cos a + B sin a and h_Q = G sin a - B cos a.
        """
        i, j = self.Yi, self.Yj
        a = theta[i] - theta[j]
        c, s = np.cos(a), np.sin(a)
        G, B = self.Gij, self.Bij
        return v[i], v[j], G * c + B * s, -G * s + B * c, G * s - B * c, G * c + B * s

    def jac_bus(self, theta, v):
        """d(P, Q)/d(theta, v) as a (2n x 2n) sparse matrix.

        For a term v_i v_j h(theta_i - theta_j): d/dtheta_i = v_i v_j h',
        d/dtheta_j = -v_i v_j h', d/dv_i = v_j h, d/dv_j = v_i h.  Scatter-adding
        all slots also covers the bus's own term (i = j).
        """
        n = self.n
        i, j = self.Yi, self.Yj
        vi, vj, hP, hPp, hQ, hQp = self._term_parts(theta, v)
        rows, cols, vals = [], [], []
        for roff, h, hp in ((0, hP, hPp), (n, hQ, hQp)):
            r = roff + i
            rows += [r, r, r, r]
            cols += [i, j, n + i, n + j]
            vals += [vi * vj * hp, -vi * vj * hp, vj * h, vi * h]
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(2 * n, 2 * n)).tocsr()

    def jacobians(self, x, p):
        """G_x = d g / d x  and  G_p = d g / d p."""
        theta, v, _ = self.unpack(x, p)
        J = self.jac_bus(theta, v)
        Jr = J[self.g_rows]
        Gx = Jr[:, self.x_cols].tocsc()
        Gpg = sp.coo_matrix((-np.ones(self.npv), (np.arange(self.npv), np.arange(self.npv))),
                            shape=(self.n_x, self.npv))
        Gp = sp.hstack([Gpg, Jr[:, self.p_vcols]]).tocsr()
        return Gx, Gp

    # ------------------------------------------------------------ objective
    def slack_power(self, x, p):
        theta, v, _ = self.unpack(x, p)
        P, _ = self.injections(theta, v)
        return P[self.ref] + self.grid.Pd[self.ref]

    def objective(self, x, p):
        """f = sum over PV of c2 Pg^2 + c1 Pg + c0, plus the same for the slack."""
        g = self.grid
        gi = self.gen_of_bus
        Pg = p[:self.npv]
        c2, c1, c0 = g.c2[gi[self.pv]], g.c1[gi[self.pv]], g.c0[gi[self.pv]]
        r = gi[self.ref]
        Pr = self.slack_power(x, p)
        return float(np.sum(c2 * Pg ** 2 + c1 * Pg + c0) + g.c2[r] * Pr ** 2 + g.c1[r] * Pr + g.c0[r])

    def _slack_row(self, theta, v):
        """Gradient of P^inj_ref in (x, p) coordinates (zero on the Pg block)."""
        J = self.jac_bus(theta, v)
        row = np.asarray(J[self.ref].todense()).ravel()
        return np.concatenate([row[self.x_cols], np.zeros(self.npv), row[self.p_vcols]])

    def grad_f(self, x, p):
        g = self.grid
        gi = self.gen_of_bus
        theta, v, Pg = self.unpack(x, p)
        r = gi[self.ref]
        Pr = self.slack_power(x, p)
        d = self._slack_row(theta, v) * (2.0 * g.c2[r] * Pr + g.c1[r])
        d[self.n_x:self.n_x + self.npv] += 2.0 * g.c2[gi[self.pv]] * Pg + g.c1[gi[self.pv]]
        return d[:self.n_x], d[self.n_x:]

    # --------------------------------------------------------------- Newton
    def newton(self, p, tol=1e-13, max_iter=30, x0=None):
        """x_{k+1} = x_k - G_x^{-1} g(x_k, p); returns (x, residual history, converged)."""
        x = self.flat_start() if x0 is None else np.array(x0, dtype=np.float64)
        hist = []
        for _ in range(max_iter + 1):
            gv = self.residual(x, p)
            r = float(np.max(np.abs(gv))) if gv.size else 0.0
            hist.append(r)
            if not np.isfinite(r):
                return x, hist, False
            if r <= tol:
                return x, hist, True
            if len(hist) > 3 and r >= 0.5 * hist[-2] and r < 1e-11:
                return x, hist, True  # stagnated at rounding level
            Gx, _ = self.jacobians(x, p)
            x = x - spla.splu(Gx).solve(gv)
        return x, hist, False

    # ------------------------------------------------ first-order adjoint
    def adjoint(self, x, p, lu=None):
        """lambda = -G_x^{-T} (grad_x f)^T."""
        Gx, _ = self.jacobians(x, p)
        lu = lu or spla.splu(Gx)
        fx, _ = self.grad_f(x, p)
        return -lu.solve(fx, trans="T")

    def reduced_gradient(self, x, p, lam=None):
        """grad F = grad_p f + G_p^T lambda."""
        _, Gp = self.jacobians(x, p)
        lam = self.adjoint(x, p) if lam is None else lam
        _, fp = self.grad_f(x, p)
        return fp + Gp.T @ lam

    # --------------------------------------------- second-order information
    def _bus_hessian(self, theta, v, wP, wQ):
        """Hessian in (theta, v) of sum_b wP_b P_b + wQ_b Q_b, as a sparse matrix.

        For one term v_i v_j h(a), a = theta_i - theta_j, in the slots
        (theta_i, theta_j, v_i, v_j):
            theta_i theta_i: -v_i v_j h   theta_i theta_j: +v_i v_j h   theta_j theta_j: -v_i v_j h
            theta_i v_i:  v_j h'          theta_i v_j:  v_i h'
            theta_j v_i: -v_j h'          theta_j v_j: -v_i h'
            v_i v_j: h                    v_i v_i = v_j v_j = 0
        (using h'' = -h).
        """
        n = self.n
        i, j = self.Yi, self.Yj
        vi, vj, hP, hPp, hQ, hQp = self._term_parts(theta, v)
        h = wP[i] * hP + wQ[i] * hQ
        hp = wP[i] * hPp + wQ[i] * hQp
        ti, tj, ui, uj = i, j, n + i, n + j
        ent = [
            (ti, ti, -vi * vj * h), (ti, tj, vi * vj * h), (tj, ti, vi * vj * h), (tj, tj, -vi * vj * h),
            (ti, ui, vj * hp), (ui, ti, vj * hp), (ti, uj, vi * hp), (uj, ti, vi * hp),
            (tj, ui, -vj * hp), (ui, tj, -vj * hp), (tj, uj, -vi * hp), (uj, tj, -vi * hp),
            (ui, uj, h), (uj, ui, h),
        ]
        rows = np.concatenate([e[0] for e in ent])
        cols = np.concatenate([e[1] for e in ent])
        vals = np.concatenate([e[2] for e in ent])
        return sp.coo_matrix((vals, (rows, cols)), shape=(2 * n, 2 * n)).tocsr()

    def lagrangian_hessian(self, x, p, lam):
        """d2 l = d2 f + sum_k lambda_k d2 g_k over the (x, p) coordinates."""
        g = self.grid
        gi = self.gen_of_bus
        n, npv, npq = self.n, self.npv, self.npq
        theta, v, _ = self.unpack(x, p)
        r = gi[self.ref]
        Pr = self.slack_power(x, p)
        # multipliers of the injections: lambda on the balance rows, and the
        # slack cost's first derivative on P_ref (from d2 f)
        wP = np.zeros(n)
        wQ = np.zeros(n)
        wP[self.pv] = lam[:npv]
        wP[self.pq] = lam[npv:npv + npq]
        wQ[self.pq] = lam[npv + npq:]
        wP[self.ref] += 2.0 * g.c2[r] * Pr + g.c1[r]
        Hb = self._bus_hessian(theta, v, wP, wQ)
        H = (self.E.T @ Hb @ self.E).tocsr()
        a = self._slack_row(theta, v)
        nz = np.flatnonzero(a)
        # d2 f also holds 2 c2_ref (grad P_ref)(grad P_ref)^T and 2 c2 on each Pg
        Hs = sp.coo_matrix((2.0 * g.c2[r] * np.outer(a[nz], a[nz]).ravel(),
                            (np.repeat(nz, nz.size), np.tile(nz, nz.size))), shape=H.shape)
        d = np.zeros(self.n_x + self.n_p)
        d[self.n_x:self.n_x + npv] = 2.0 * g.c2[gi[self.pv]]
        return (H + Hs + sp.diags(d)).tocsr()


class Solved:
    """An operating point: Newton solution, factorised G_x, lambda, d2 l."""

    def __init__(self, orc: Oracle, p=None, tol=1e-13, max_iter=30, x0=None):
        self.o = orc
        self.p = orc.p0() if p is None else np.asarray(p, dtype=np.float64)
        self.x, self.hist, self.ok = orc.newton(self.p, tol=tol, max_iter=max_iter, x0=x0)
        if not self.ok:
            raise RuntimeError(f"Newton did not converge: {self.hist}")
        self.Gx, self.Gp = orc.jacobians(self.x, self.p)
        self.lu = spla.splu(self.Gx)
        fx, self.fp = orc.grad_f(self.x, self.p)
        self.lam = -self.lu.solve(fx, trans="T")
        self.grad = self.fp + self.Gp.T @ self.lam
        self.F = orc.objective(self.x, self.p)
        self.Hl = orc.lagrangian_hessian(self.x, self.p, self.lam)

    def hvp(self, W):
        """Algorithm 2 on a block W (n_p x k): returns H W."""
        W = np.asarray(W, dtype=np.float64)
        one = W.ndim == 1
        W2 = W[:, None] if one else W
        n_x = self.o.n_x
        B = self.Gp @ W2  # SpMul
        Z = -self.lu.solve(B)  # BatchSparseSolve
        Y = self.Hl @ np.vstack([Z, W2])  # BatchTensorProjection
        Yx, Yp = Y[:n_x], Y[n_x:]
        Psi = -self.lu.solve(Yx, trans="T")  # BatchSparseSolve (transposed)
        HW = Yp + self.Gp.T @ Psi  # SpMulAdd
        return HW[:, 0] if one else HW

    def reduced_hessian(self, k=None):
        """Full H by blocks of k columns of the identity, ceil(n_p / k) blocks."""
        n_p = self.o.n_p
        k = n_p if k is None else int(k)
        H = np.empty((n_p, n_p))
        for s in range(0, n_p, k):
            e = min(n_p, s + k)
            W = np.zeros((n_p, e - s))
            W[np.arange(s, e), np.arange(e - s)] = 1.0
            H[:, s:e] = self.hvp(W)
        return H


def solve(grid, p=None, tol=1e-13, max_iter=30) -> Solved:
    return Solved(Oracle(grid), p=p, tol=tol, max_iter=max_iter)
