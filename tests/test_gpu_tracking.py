"""Real-time tracking on the device (Sec. 6.3, eq. (qp_rto)) against the
oracle: the dense Cholesky solve, the reduced gradient, one tracking update
and a short trajectory.  FP64 throughout; tolerances are far inside the
1e-9 relative bound of the FP64 mode."""
import numpy as np
import pytest
import scipy.linalg as sla

import gridgen
from oracle import powerflow as pf
from oracle import tracking

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_00241_amd import rh  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = rh.Context(0)
    yield c
    c.close()


def _spd(n, seed, lo=1.0, hi=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * rng.uniform(lo, hi, n)) @ Q.T


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("n,nrhs,pad", [(1, 1, 0), (5, 2, 0), (31, 1, 3), (32, 1, 0), (33, 3, 0),
                                        (64, 1, 0), (65, 2, 5), (100, 1, 0), (257, 3, 0),
                                        (700, 2, 7), (2085, 1, 0)])
def test_cholesky_solve_matches_oracle(ctx, n, nrhs, pad):
    print(f"cholesky n={n} nrhs={nrhs} lda={n + pad}", flush=True)
    M = _spd(n, seed=n)
    Ac = M.copy()
    Ac[np.triu_indices(n, 1)] = 7.0  # the strict upper triangle is neither read nor written
    lda = n + pad
    big = np.full((n, lda), -3.0)  # row j = column j of the matrix, padded to lda
    big[:, :n] = Ac.T
    A_t = _dev(big)
    B = np.random.default_rng(n + 1).standard_normal((n, nrhs))
    B_t = _dev(B.T)
    assert ctx.cholesky_solve_device(A_t[:, :n], B_t) == -1
    L_or, j = tracking.cholesky(Ac)
    assert j == -1
    X_or = sla.solve_triangular(L_or.T, sla.solve_triangular(L_or, B, lower=True), lower=False)
    out = A_t.cpu().numpy()
    L_dev = out[:, :n].T
    assert np.all(out[:, n:] == -3.0)
    assert np.all(L_dev[np.triu_indices(n, 1)] == 7.0)
    err_L = np.abs(np.tril(L_dev) - L_or).max() / np.abs(L_or).max()
    X_dev = B_t.cpu().numpy().T
    err_X = np.abs(X_dev - X_or).max() / np.abs(X_or).max()
    print(f"  max rel err L {err_L:.2e} X {err_X:.2e}", flush=True)
    assert err_L <= 1e-12 and err_X <= 1e-11


@pytest.mark.parametrize("n,e", [(70, -1000), (97, 900)])
def test_cholesky_solve_extreme_scales(ctx, n, e):
    """A = 2^e M: with e = -1000 every pivot is far below 2^-900, where the
    pivot is scaled by a power of two before the reciprocal square root;
    with e = 900 every pivot is far above 1.  L scales by 2^(e/2) and X not
    at all (B is scaled by 2^e too), so the scaled call must agree with the
    unscaled one as closely as with the oracle."""
    print(f"cholesky extreme scale n={n} 2^{e}", flush=True)
    M = _spd(n, seed=7 * n)
    B0 = np.random.default_rng(n).standard_normal((n, 1))
    s = 2.0 ** e
    A_t, B_t = _dev((s * M).T), _dev((s * B0).T)
    assert ctx.cholesky_solve_device(A_t, B_t) == -1
    U_t, C_t = _dev(M.T), _dev(B0.T)
    assert ctx.cholesky_solve_device(U_t, C_t) == -1
    L_or, j = tracking.cholesky(s * M)
    assert j == -1
    X_or = sla.solve_triangular(L_or.T, sla.solve_triangular(L_or, s * B0, lower=True), lower=False)
    L_dev = np.tril(A_t.cpu().numpy().T)
    L_ref = np.tril(U_t.cpu().numpy().T) * 2.0 ** (e // 2)
    X_dev, X_ref = B_t.cpu().numpy().T, C_t.cpu().numpy().T
    assert np.all(np.isfinite(L_dev)) and np.all(np.isfinite(X_dev))
    err_L = np.abs(L_dev - L_or).max() / np.abs(L_or).max()
    err_X = np.abs(X_dev - X_or).max() / np.abs(X_or).max()
    d_L = np.abs(L_dev - L_ref).max() / np.abs(L_ref).max()
    d_X = np.abs(X_dev - X_ref).max() / np.abs(X_ref).max()
    print(f"  vs oracle L {err_L:.2e} X {err_X:.2e}; vs unscaled L {d_L:.2e} X {d_X:.2e}", flush=True)
    assert err_L <= 1e-12 and err_X <= 1e-11
    assert d_L <= 1e-14 and d_X <= 1e-13


@pytest.mark.parametrize("n,bad", [(40, 12), (300, 201), (97, 96)])
def test_cholesky_reports_the_oracle_failing_column(ctx, n, bad):
    print(f"cholesky failure n={n} col={bad}", flush=True)
    A = _spd(n, seed=3 * n)
    L0 = np.linalg.cholesky(A)
    A[bad, bad] -= L0[bad, bad] ** 2 + 1.0
    _, j = tracking.cholesky(A)
    assert j == bad
    A_t, B_t = _dev(A.T), _dev(np.ones((1, n)))
    with pytest.raises(rh.RhError) as ei:
        ctx.cholesky_solve_device(A_t, B_t)
    assert ei.value.status == rh.RH_ESINGULAR and ei.value.failed_col == bad


def _bounds(orc, p0):
    """Box and ramp limits in the parameter order [Pg at PV; v_ref; v at PV]."""
    npv = orc.npv
    lo = np.concatenate([np.zeros(npv), np.full(npv + 1, 0.94)])
    hi = np.concatenate([2.0 * np.maximum(p0[:npv], 0.1), np.full(npv + 1, 1.06)])
    ramp = np.concatenate([np.full(npv, 0.01), np.full(npv + 1, 0.002)])
    return lo, hi, ramp


@pytest.mark.parametrize("name,scale", [("c1", 1.0), ("c1", 0.96), ("c2", 1.0)])
def test_tracking_step_matches_oracle(ctx, name, scale):
    print(f"tracking step {name} load scale {scale}", flush=True)
    g = gridgen.config_grid(name, 0)
    g.Pd = g.Pd * scale
    g.Qd = g.Qd * scale
    orc = pf.Oracle(g)
    p0 = orc.p0()
    lo, hi, ramp = _bounds(orc, p0)
    net = rh.Network(ctx, g)
    net.solve_device()
    n_p = net.n_p
    gd = torch.empty(n_p, dtype=torch.float64, device="cuda")
    net.reduced_gradient_device(gd)
    d = torch.empty(n_p, dtype=torch.float64, device="cuda")
    info = net.tracking_step_device(lo=lo, hi=hi, ramp=ramp, d=d)
    s, gr, H, d_or, tau_or = tracking.step(g, p0)
    err_g = np.abs(gd.cpu().numpy() - gr).max() / np.abs(gr).max()
    d_dev = d.cpu().numpy()
    err_d = np.abs(d_dev - d_or).max() / np.abs(d_or).max()
    print(f"  tau dev {info['tau']:.6e} oracle {tau_or:.6e} tries {info['tries']}; rel err g {err_g:.2e} "
          f"d {err_d:.2e}; ms grad {info['ms_gradient']:.3f} hess {info['ms_hessian']:.3f} "
          f"solve {info['ms_solve']:.3f}", flush=True)
    assert err_g <= 1e-11
    assert abs(info["tau"] - tau_or) <= 1e-12 * max(1.0, tau_or)
    if scale < 1.0:
        assert tau_or > 0.0  # H is indefinite at this light loading
    assert err_d <= 1e-10
    assert abs(info["grad_inf"] - np.abs(gr).max()) <= 1e-11 * np.abs(gr).max()
    p1 = net.get_parameters()
    np.testing.assert_allclose(p1, tracking.project(p0, d_or, lo, hi, ramp), rtol=0, atol=1e-10)


def test_tracking_trajectory_matches_oracle(ctx):
    g = gridgen.config_grid("c1", 0)
    orc = pf.Oracle(g)
    p0 = orc.p0()
    lo, hi, ramp = _bounds(orc, p0)
    T = 6
    Pd, Qd = gridgen.load_trajectory(g, steps=60, seed=5)
    ref = tracking.trajectory(g, Pd[:T], Qd[:T], p0=np.clip(p0, lo, hi), lo=lo, hi=hi, ramp=ramp)
    net = rh.Network(ctx, g)
    net.set_parameters(np.clip(p0, lo, hi))
    for t in range(T):
        print(f"trajectory step {t}", flush=True)
        net.set_loads(Pd[t], Qd[t])
        net.solve_device()
        np.testing.assert_allclose(net.get_parameters(), ref[t]["p"], rtol=0, atol=1e-9)
        assert abs(net.objective() - ref[t]["F"]) <= 1e-10 * abs(ref[t]["F"])
        info = net.tracking_step_device(lo=lo, hi=hi, ramp=ramp)
        assert abs(info["tau"] - ref[t]["tau"]) <= 1e-10 * max(1.0, ref[t]["tau"])
