"""Parity of the launch configurations beyond the headline one (needs an MI355X).

Every kernel instantiation that a workload can reach is compared with the
FP64 oracle on the same seeded inputs: the 70k-bus grid of the batched
workload (vectors in global memory, one and four directions per workgroup,
FP64 and refined FP32), the refined mode with two and four directions per
workgroup in LDS and in global memory, a loading close to the grid's limit,
the per-column refinement figures of the ABI, and the server with 10k- and
70k-bus networks in the mix.
"""
import numpy as np
import pytest

import gridgen
from oracle import solve

pytestmark = pytest.mark.gpu

TOL64 = 1e-9   # FP64 mode: max |H - H*| / max |H*|
TOL32 = 1e-8   # refined mode: the same per column


def _say(msg):
    print(msg, flush=True)


def _percol(a, b):
    return np.max(np.abs(a - b), axis=0) / np.max(np.abs(b), axis=0)


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


@pytest.fixture(scope="module")
def c3_pair(ctx, rhmod):
    """Two load-perturbed operating points of the 70k-bus grid, 16 Gaussian
    directions each, with the oracle's products."""
    base = gridgen.config_grid("c3", 0)
    out = []
    for i in range(2):
        g = gridgen.perturb_loads(base, seed=5000 + i)
        net = rhmod.Network(ctx, g)
        net.solve()
        W = gridgen.directions(net.n_p, 16, 7000 + i)
        out.append((net, W, solve(g).hvp(W)))
    return out


@pytest.mark.parametrize("dirs", ["auto", "4"])
@pytest.mark.parametrize("prec", ["fp64", "refined"])
def test_70k_two_operating_points_in_one_launch(ctx, rhmod, c3_pair, monkeypatch, prec, dirs):
    import torch

    if dirs != "auto":
        monkeypatch.setenv("RH_DIRS_PER_GROUP", dirs)
    p = rhmod.RH_FP64 if prec == "fp64" else rhmod.RH_FP32_REFINED
    nets = [c[0] for c in c3_pair]
    Ws = [torch.from_numpy(np.ascontiguousarray(c[1].T)).cuda() for c in c3_pair]
    HWs = [torch.zeros_like(W) for W in Ws]
    _say(f"70k: 2 operating points x 16 directions, one launch, {prec}, dirs/group {dirs}")
    ctx.hvp_batch_device(nets, Ws, HWs, stream=torch.cuda.current_stream().cuda_stream, prec=p)
    torch.cuda.synchronize()
    rep = ctx.report()
    assert rep["last_launches"] == 1
    if dirs != "auto":
        assert rep["dirs_per_group"] == int(dirs)
    for (net, W, ref), HW in zip(c3_pair, HWs):
        e = _percol(HW.cpu().numpy().T, ref)
        _say(f"  per-column error max {e.max():.2e} median {np.median(e):.2e}")
        if prec == "fp64":
            assert np.max(np.abs(HW.cpu().numpy().T - ref)) / np.max(np.abs(ref)) <= TOL64
        else:
            assert e.max() <= TOL32


@pytest.fixture(scope="module")
def c1(ctx, rhmod):
    g = gridgen.config_grid("c1", 0)
    net = rhmod.Network(ctx, g)
    net.solve()
    return g, net, solve(g)


def test_refined_every_grouping_and_vector_placement_1k(c1, rhmod, monkeypatch):
    """Refined mode with 1, 2 and 4 directions per workgroup, the FP32
    correction in LDS and in global memory: bitwise the same results (each
    direction's arithmetic and stopping decision are its own), each column
    within 1e-8 of the oracle."""
    g, net, s = c1
    W = gridgen.directions(net.n_p, 48, 44)
    ref = s.hvp(W)
    base = None
    for lds in ("lds", "global"):
        if lds == "global":
            monkeypatch.setenv("RH_NO_LDS", "1")
        for c in ("1", "2", "4"):
            monkeypatch.setenv("RH_DIRS_PER_GROUP", c)
            HW = net.hvp(W, prec=rhmod.RH_FP32_REFINED)
            assert net.report()["dirs_per_group"] == int(c)
            e = _percol(HW, ref)
            _say(f"refined 1k, {c} dirs/group, {lds}: per-column error max {e.max():.2e}")
            assert e.max() <= TOL32
            if base is None:
                base = HW
            else:
                np.testing.assert_array_equal(HW, base)


def test_refinement_report_tracks_the_oracle_error(c1, ctx, rhmod):
    """Per-column figures through the ABI: with the tolerance at 0 every
    column takes exactly the requested corrections; the backward errors and
    the error against the oracle shrink together as corrections are added,
    and the error stays within the bound the backward error and the
    condition of G_x give."""
    g, net, s = c1
    W = gridgen.directions(net.n_p, 32, 45)
    ref = s.hvp(W)
    cond = np.linalg.cond(s.Gx.toarray())
    errs, berrs = [], []
    ctx.set_refinement_tol(0.0)
    try:
        for steps in (0, 1, 2):
            ctx.set_refinement(steps)
            HW = net.hvp(W, prec=rhmod.RH_FP32_REFINED)
            rep = net.refinement_report(32)
            assert np.all(rep["steps_z"] == steps) and np.all(rep["steps_psi"] == steps)
            e = _percol(HW, ref)
            b = np.maximum(rep["berr_z"], rep["berr_psi"])
            _say(f"refined 1k, {steps} corrections: error max {e.max():.2e}, backward error max {b.max():.2e}")
            errs.append(e.max())
            berrs.append(b.max())
            assert e.max() <= 1e3 * cond * b.max() + 1e-13
    finally:
        ctx.set_refinement(4)
        ctx.set_refinement_tol(1e-13)
    assert errs[0] > errs[1] > errs[2] or errs[2] <= 1e-12
    assert berrs[0] > berrs[1] > berrs[2] or berrs[2] <= 1e-15
    with pytest.raises(rhmod.RhError):
        net.refinement_report(33)  # more columns than the last call had


def test_refined_near_the_loading_limit_1k(ctx, rhmod):
    """The 1k grid loaded to about 97 % of its loading limit (Newton fails
    beyond a loading factor of about 0.61 for this instance), where G_x is
    worse conditioned: FP64 within 1e-9, refined within 1e-8 per column."""
    c = gridgen.CONFIGS["c1"]
    alpha = 0.59
    g = gridgen.geometric(c["n_bus"], c["n_branch"], c["n_gen"], 1000, alpha,
                          kappa=c["kappa"] * alpha / c["alpha"], name="c1-i0-heavy")
    net = rhmod.Network(ctx, g)
    net.solve()
    s = solve(g)
    W = gridgen.directions(net.n_p, 32, 46)
    ref = s.hvp(W)
    H64 = net.hvp(W)
    assert np.max(np.abs(H64 - ref)) / np.max(np.abs(ref)) <= TOL64
    e = _percol(net.hvp(W, prec=rhmod.RH_FP32_REFINED), ref)
    _say(f"refined 1k at loading {alpha}: per-column error max {e.max():.2e}")
    assert e.max() <= TOL32


def test_served_mix_with_10k_and_70k_networks_equals_solo(ctx, rhmod, c1):
    """Continuous batching over 1k, 10k and 70k networks (FP64 and refined
    requests, a full 10k Hessian among them): every result is bitwise its solo
    result, and the 10k full Hessian matches the oracle."""
    import torch

    from paper_2201_00241_amd.serving import Request, Server

    g1, net1, s1 = c1
    g2 = gridgen.perturb_loads(gridgen.config_grid("c2", 0), seed=9001)
    net2 = rhmod.Network(ctx, g2)
    net2.solve()
    g3 = gridgen.perturb_loads(gridgen.config_grid("c3", 0), seed=9002)
    net3 = rhmod.Network(ctx, g3)
    net3.solve()
    nets = {"c1": net1, "c2": net2, "c3": net3}
    plan = [("c2", 0, 0), ("c3", 16, 0), ("c1", 1, 1), ("c2", 16, 1), ("c3", 128, 0),
            ("c1", 16, 0), ("c2", 1, 0), ("c3", 1, 1), ("c1", 128, 0), ("c2", 128, 1)]
    rng = np.random.default_rng(5)
    reqs = []
    for i, (key, k, refined) in enumerate(plan):
        W = None if k == 0 else gridgen.directions(nets[key].n_p, k, 200 + i)
        reqs.append(Request(rid=i, key=key, k=k, W=W, arrival=float(i * rng.exponential(1e-3)),
                            prec=rhmod.RH_FP32_REFINED if refined else rhmod.RH_FP64))
    _say("serving: 10 requests over 1k/10k/70k networks, FP64 and refined")
    srv = Server(ctx, nets, max_inflight=3, dirs_per_launch=1024, block=256)
    done = srv.run(reqs)
    assert len(done) == len(reqs) and all(r.error is None for r in done)
    stream = torch.cuda.current_stream().cuda_stream
    for r in done:
        net = nets[r.key]
        if r.k:
            W = torch.from_numpy(np.ascontiguousarray(r.W.T)).cuda()
            solo = torch.zeros_like(W)
            net.hvp_device(W, solo, stream=stream, prec=r.prec)
        else:
            solo = torch.zeros((net.n_p, net.n_p), dtype=torch.float64, device="cuda")
            net.reduced_hessian_device(solo, k_block=256, stream=stream, prec=r.prec)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(r.result, solo.cpu().numpy().T)
    full = [r for r in done if r.key == "c2" and r.k == 0][0]
    Ho = solve(g2).reduced_hessian(256)
    assert np.max(np.abs(full.result - Ho)) / np.max(np.abs(Ho)) <= TOL64


def test_server_evicts_a_failing_request_and_serves_the_rest(ctx, rhmod, c1):
    """A request on a network whose operating point was invalidated (loads
    changed, no new solve) makes its batched launch fail: the server retries
    each request of that launch alone, evicts the failing one with its error,
    and every other request completes with its solo result.  A request with
    non-finite directions is rejected at arrival."""
    import torch

    from paper_2201_00241_amd.serving import Request, Server

    g1, net1, s1 = c1
    gb = gridgen.perturb_loads(g1, seed=31)
    bad = rhmod.Network(ctx, gb)
    bad.solve()
    nets = {"good": net1, "bad": bad}
    reqs = [Request(rid=i, key="good", k=16, W=gridgen.directions(net1.n_p, 16, 400 + i)) for i in range(4)]
    reqs.append(Request(rid=4, key="bad", k=16, W=gridgen.directions(bad.n_p, 16, 404)))
    nanW = gridgen.directions(net1.n_p, 4, 405)
    nanW[3, 2] = np.nan
    reqs.append(Request(rid=5, key="good", k=4, W=nanW))
    srv = Server(ctx, nets, max_inflight=1, dirs_per_launch=4096, block=256)
    bad.set_loads(gb.Pd * 1.01, gb.Qd * 1.01)  # invalidates the solution: products now fail
    _say("serving: one request on an invalidated network, one with NaN directions")
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    by = {r.rid: r for r in done}
    assert by[4].error is not None and by[4].retried
    assert by[5].error is not None and by[5].launches == 0
    stream = torch.cuda.current_stream().cuda_stream
    for i in range(4):
        r = by[i]
        assert r.error is None and r.retried
        W = torch.from_numpy(np.ascontiguousarray(r.W.T)).cuda()
        solo = torch.zeros_like(W)
        net1.hvp_device(W, solo, stream=stream)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(r.result, solo.cpu().numpy().T)
    assert srv._mem_used == 0
