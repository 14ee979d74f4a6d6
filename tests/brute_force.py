"""Direct-direct reduced Hessian from explicit derivative tensors (test helper).

Independent of the oracle: it writes the balance equations from the complex
power S = V * conj(Y V) (dense bus admittance matrix) in PyTorch and lets
autograd form grad g, the third-order tensors d2_xx g, d2_xp g, d2_pp g and
d2 f.  With S = -G_x^{-1} G_p (dense) the reduced Hessian is
    H = d2_pp l + S^T d2_xp l + d2_px l S + S^T d2_xx l S,
l = f + lambda^T g, lambda = -G_x^{-T} grad_x f  (the direct-direct scheme the
paper names among the Hessian reduction schemes, Sec. 4.1; the tensors are
the ones of Sec. 1).  For tiny networks only.
"""
import numpy as np
import torch

PQ, PV, REF = 1, 2, 3


class Brute:
    def __init__(self, grid):
        n = grid.n_bus
        t = np.asarray(grid.bus_type)
        self.n = n
        self.ref = int(np.flatnonzero(t == REF)[0])
        self.pv = np.flatnonzero(t == PV)
        self.pq = np.flatnonzero(t == PQ)
        self.npv, self.npq = self.pv.size, self.pq.size
        self.n_x = self.npv + 2 * self.npq
        self.n_p = 2 * self.npv + 1
        Y = np.zeros((n, n), dtype=np.complex128)
        for f, tt, r, x, b in zip(grid.br_from, grid.br_to, grid.br_r, grid.br_x, grid.br_b):
            y = 1.0 / complex(r, x)
            Y[f, f] += y + 0.5j * b
            Y[tt, tt] += y + 0.5j * b
            Y[f, tt] -= y
            Y[tt, f] -= y
        self.Y = torch.tensor(Y)
        gi = np.full(n, -1)
        gi[grid.gen_bus] = np.arange(grid.n_gen)
        self.gi = gi
        self.grid = grid
        self.Pd = torch.tensor(grid.Pd)
        self.Qd = torch.tensor(grid.Qd)

    def bus_vectors(self, z):
        nx, npv, npq = self.n_x, self.npv, self.npq
        x, p = z[:nx], z[nx:]
        theta = torch.zeros(self.n, dtype=torch.float64)
        v = torch.zeros(self.n, dtype=torch.float64)
        theta = theta.index_put((torch.tensor(self.pv),), x[:npv])
        theta = theta.index_put((torch.tensor(self.pq),), x[npv:npv + npq])
        v = v.index_put((torch.tensor(self.pq),), x[npv + npq:])
        v = v.index_put((torch.tensor([self.ref]),), p[npv:npv + 1])
        v = v.index_put((torch.tensor(self.pv),), p[npv + 1:])
        return theta, v, p[:npv]

    def power(self, z):
        theta, v, Pg = self.bus_vectors(z)
        V = v * torch.exp(1j * theta)
        S = V * torch.conj(self.Y @ V)
        return S.real, S.imag, Pg

    def g(self, z):
        P, Q, Pg = self.power(z)
        pv, pq = torch.tensor(self.pv), torch.tensor(self.pq)
        return torch.cat([P[pv] - Pg + self.Pd[pv], P[pq] + self.Pd[pq], Q[pq] + self.Qd[pq]])

    def f(self, z):
        P, _, Pg = self.power(z)
        g = self.grid
        gpv = self.gi[self.pv]
        c2 = torch.tensor(g.c2[gpv])
        c1 = torch.tensor(g.c1[gpv])
        c0 = torch.tensor(g.c0[gpv])
        r = self.gi[self.ref]
        Pr = P[self.ref] + self.Pd[self.ref]
        return (c2 * Pg ** 2 + c1 * Pg + c0).sum() + g.c2[r] * Pr ** 2 + g.c1[r] * Pr + g.c0[r]

    def hessian(self, x, p):
        z = torch.tensor(np.concatenate([x, p]))
        nx = self.n_x
        J = torch.autograd.functional.jacobian(self.g, z)
        Hg = torch.autograd.functional.jacobian(
            lambda zz: torch.autograd.functional.jacobian(self.g, zz, create_graph=True), z)
        gf = torch.autograd.functional.jacobian(self.f, z)
        Hf = torch.autograd.functional.hessian(self.f, z)
        Gx, Gp = J[:, :nx], J[:, nx:]
        lam = -torch.linalg.solve(Gx.T, gf[:nx])
        Hl = Hf + torch.einsum("k,kij->ij", lam, Hg)
        S = -torch.linalg.solve(Gx, Gp)
        Hxx, Hxp = Hl[:nx, :nx], Hl[:nx, nx:]
        Hpx, Hpp = Hl[nx:, :nx], Hl[nx:, nx:]
        H = Hpp + S.T @ Hxp + Hpx @ S + S.T @ Hxx @ S
        grad = gf[nx:] + Gp.T @ lam
        return H.numpy(), grad.numpy(), self.g(z).numpy()
