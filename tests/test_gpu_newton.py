"""Device-resident Newton with the LU refactorisation on the GPU (needs an
MI355X).

rh_solve_powerflow_device runs every Newton step on the device (mismatch,
G_x on its fixed pattern, P G_x P^T = L U with static pivots, the two solves)
and reads back only max |g| per step.  The state and the factors it ends with
must match the host solve of the same operating point, and the state the
oracle's, to 1e-12; products after it match the oracle.
"""
import time

import numpy as np
import pytest

import gridgen
from oracle import solve

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def rhmod():
    import torch

    from paper_2201_00241_amd import rh

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rh.load()
    return rh


@pytest.fixture(scope="module")
def ctx(rhmod):
    c = rhmod.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# The refactorisation treats the last min(128, n_x) rows as one dense block:
# c0 (n_x = 14) and geo60 (113) are one dense block, geo75 (142) has a
# sparse part of 14 rows, geo150 (284) and the 1k and 10k grids larger ones.
# The solves keep the vector in LDS up to n_x = 19,968: geo11k (20,899) takes
# the global-memory path.
GRIDS = {
    "c2": lambda: gridgen.config_grid("c2", 0),
    "c1": lambda: gridgen.config_grid("c1", 0),
    "c0": lambda: gridgen.config_grid("c0", 0),
    "geo60": lambda: gridgen.geometric(60, 81, 6, seed=560, alpha=0.3, kappa=0.0255),
    "geo75": lambda: gridgen.geometric(75, 101, 7, seed=575, alpha=0.3, kappa=0.0255),
    "geo150": lambda: gridgen.geometric(150, 202, 15, seed=650, alpha=0.3, kappa=0.0255),
    "geo11k": lambda: gridgen.geometric(11000, 14850, 1100, seed=611, alpha=0.22, kappa=0.0187),
}


@pytest.mark.parametrize("name,seed", [("c2", 81), ("c1", 82), ("c0", 0), ("geo60", 83), ("geo75", 84),
                                       ("geo150", 85), ("geo11k", 86)])
def test_device_newton_matches_host_and_oracle(ctx, rhmod, name, seed):
    base = GRIDS[name]()
    g = gridgen.perturb_loads(base, seed=seed) if name != "c0" else base
    dev = rhmod.Network(ctx, g)
    host = rhmod.Network(ctx, g)
    t0 = time.perf_counter()
    it_d, r_d = dev.solve_device(1e-13, 30)
    t_dev = time.perf_counter() - t0
    t0 = time.perf_counter()
    it_h, r_h = host.solve(1e-13, 30)
    t_host = time.perf_counter() - t0
    _say(f"{name}: device Newton {it_d} steps ({t_dev * 1e3:.1f} ms), host {it_h} steps ({t_host * 1e3:.1f} ms), "
         f"residuals {r_d:.1e} {r_h:.1e}")
    assert r_d <= 1e-13 and it_d == it_h
    xd, xh = dev.state(), host.state()
    s = solve(g)
    assert _rel(xd, xh) <= 1e-12
    assert _rel(xd, s.x) <= 1e-12
    Ld, Ud = dev.factors()
    Lh, Uh = host.factors()
    assert _rel(Ld, Lh) <= 1e-12 and _rel(Ud, Uh) <= 1e-12
    _say(f"  state vs host {_rel(xd, xh):.1e}, L {_rel(Ld, Lh):.1e}, U {_rel(Ud, Uh):.1e}")
    # the product path set up from the device solve
    W = gridgen.directions(dev.n_p, min(16, dev.n_p), 90 + seed)
    ref = s.hvp(W)
    assert _rel(dev.hvp(W), ref) <= 1e-9
    assert abs(dev.objective() - s.F) <= 1e-12 * abs(s.F)
    dev.close()
    host.close()


def test_device_newton_reports_failures(ctx, rhmod):
    g = gridgen.config_grid("c1", 0)
    net = rhmod.Network(ctx, g)
    with pytest.raises(rhmod.RhError) as ei:
        net.solve_device(1e-13, 1)  # one step cannot reach the tolerance
    assert ei.value.status == rhmod.RH_ENOCONV
    W = gridgen.directions(net.n_p, 2, 3)
    with pytest.raises(rhmod.RhError) as ei:
        net.hvp(W)  # no accepted state
    assert ei.value.status == rhmod.RH_ESTATE
    net.solve_device()
    assert np.all(np.isfinite(net.hvp(W)))
    net.close()


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_device_newton_singular_and_non_finite_starts(ctx, rhmod, name):
    """A zero start makes G_x singular (every flow and partial vanishes at
    the PQ buses): the device refactorisation must say so, as the host
    factorisation does (c0 is all one dense block, c1 mostly sparse rows);
    a start of 1e200 overflows the flows: a non-finite residual."""
    g = GRIDS[name]()
    net = rhmod.Network(ctx, g)
    for x0, status in ((np.zeros(net.n_x), rhmod.RH_ESINGULAR), (np.full(net.n_x, 1e200), rhmod.RH_ENOCONV)):
        net.set_initial_state(x0)
        with pytest.raises(rhmod.RhError) as ei:
            net.solve_device(1e-13, 30)
        assert ei.value.status == status, str(ei.value)
        _say(f"{name}: {ei.value}")
    # a flat start then solves, and matches the host
    net.set_initial_state(None)
    host = rhmod.Network(ctx, g)
    net.solve_device(1e-13, 30)
    host.solve(1e-13, 30)
    assert _rel(net.state(), host.state()) <= 1e-12
    net.close()
    host.close()


def test_distinct_networks_on_two_threads(ctx, rhmod):
    """Two networks solved on the device and projected on two host threads at
    once (the upload's host arrays come from a shared pool; distinct handles
    may be used from different threads): every state and product equals the
    same work done one network after the other, bit for bit."""
    import threading

    grids = [gridgen.perturb_loads(GRIDS["c1"](), seed=91), gridgen.perturb_loads(GRIDS["geo150"](), seed=92)]
    Ws = [None, None]

    def work(net, i, out):
        for step in range(3):  # three operating points: loads scaled by 1, 1.01, 1.02
            Pd, Qd = grids[i].Pd * (1 + 0.01 * step), grids[i].Qd * (1 + 0.01 * step)
            net.set_loads(Pd, Qd)
            net.solve_device(1e-13, 30)
            out.append((net.state(), net.hvp(Ws[i])))

    serial = [[], []]
    for i in range(2):
        net = rhmod.Network(ctx, grids[i])
        Ws[i] = gridgen.directions(net.n_p, min(8, net.n_p), 95 + i)
        work(net, i, serial[i])
        net.close()
    nets = [rhmod.Network(ctx, g) for g in grids]
    par = [[], []]
    errs = []

    def run(i):
        try:
            work(nets[i], i, par[i])
        except Exception as e:  # reported below, in the main thread
            errs.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in th) and not errs, errs
    for i in range(2):
        for (xs, hs), (xp, hp) in zip(serial[i], par[i]):
            assert np.array_equal(xs, xp) and np.array_equal(hs, hp)
        assert len(par[i]) == 3
    _say("two threads: states and products equal to the serial runs")
    for n in nets:
        n.close()


def test_device_newton_70k_matches_host(ctx, rhmod):
    """The 70,000-bus grid (n_x = 134,999: the solves' vector in global
    memory, LU rows of up to 732 positions in the refactorisation's LDS
    buffers): state and factors of the device solve against the host's."""
    g = gridgen.perturb_loads(gridgen.config_grid("c3", 0), seed=87)
    dev = rhmod.Network(ctx, g)
    host = rhmod.Network(ctx, g)
    t0 = time.perf_counter()
    it_d, r_d = dev.solve_device(1e-12, 30)
    t_dev = time.perf_counter() - t0
    it_h, r_h = host.solve(1e-12, 30)
    _say(f"c3: device Newton {it_d} steps ({t_dev * 1e3:.0f} ms), host {it_h} steps, residuals {r_d:.1e} {r_h:.1e}")
    assert r_d <= 1e-12 and it_d == it_h
    assert _rel(dev.state(), host.state()) <= 1e-12
    Ld, Ud = dev.factors()
    Lh, Uh = host.factors()
    assert _rel(Ld, Lh) <= 1e-12 and _rel(Ud, Uh) <= 1e-12
    _say(f"  state vs host {_rel(dev.state(), host.state()):.1e}, L {_rel(Ld, Lh):.1e}, U {_rel(Ud, Uh):.1e}")
    dev.close()
    host.close()
