"""Batched launches recorded as a HIP graph and replayed (needs an MI355X).

rh_batch_create records the one batched launch of rh_hvp_batch_device (Sec.
4.3: direction blocks are independent across instances) once; every replay
must give bitwise the products of the eager batched call on the same inputs,
with the inputs changed between replays and unrelated eager work and
synchronisations in between, in FP64 and in the refined mode.  A network
re-solved after the recording makes the replay refuse.
"""
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


@pytest.fixture(scope="module")
def nets(ctx, rhmod):
    """Two load-perturbed operating points of the 1k grid and a 9-bus grid."""
    base = gridgen.config_grid("c1", 0)
    grids = [gridgen.perturb_loads(base, seed=61), gridgen.perturb_loads(base, seed=62),
             gridgen.config_grid("c0", 1)]
    out = []
    for g in grids:
        n = rhmod.Network(ctx, g)
        n.solve()
        out.append((g, n))
    return out


@pytest.mark.parametrize("prec_name", ["fp64", "refined"])
def test_graph_replays_equal_the_eager_batched_launch(ctx, rhmod, nets, prec_name):
    import torch

    prec = rhmod.RH_FP64 if prec_name == "fp64" else rhmod.RH_FP32_REFINED
    ks = [40, 24, 5]
    Ws = [torch.zeros((k, n.n_p), dtype=torch.float64, device="cuda") for (g, n), k in zip(nets, ks)]
    HWs = [torch.full_like(W, float("nan")) for W in Ws]
    batch = ctx.batch([n for _, n in nets], Ws, HWs, prec=prec)
    info = batch.info()
    assert info["directions"] == sum(ks) and info["workgroups"] >= 1 and info["dirs_per_group"] in (1, 2, 4)
    stream = torch.cuda.current_stream().cuda_stream
    other = torch.from_numpy(np.ascontiguousarray(gridgen.directions(nets[0][1].n_p, 8, 99).T)).cuda()
    other_out = torch.zeros_like(other)
    for rep in range(3):
        for i, (W, (g, n)) in enumerate(zip(Ws, nets)):
            W.copy_(torch.from_numpy(np.ascontiguousarray(gridgen.directions(n.n_p, W.shape[0], 700 + 10 * rep + i).T)))
        _say(f"graph replay {rep}, {prec_name}")
        batch.launch(stream)
        torch.cuda.synchronize()
        got = [h.clone() for h in HWs]
        # eager work between replays, then the eager batched call for reference
        nets[1][1].hvp_device(other, other_out, stream=stream, prec=prec)
        torch.cuda.synchronize()
        ref = [torch.full_like(W, float("nan")) for W in Ws]
        ctx.hvp_batch_device([n for _, n in nets], Ws, ref, stream=stream, prec=prec)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)
    # the products themselves against the oracle (last replay)
    tol = 1e-9 if prec_name == "fp64" else 1e-8
    for (g, n), W, H in zip(nets, Ws, got):
        ref = solve(g).hvp(W.cpu().numpy().T)
        e = np.max(np.abs(H.cpu().numpy().T - ref), axis=0) / np.max(np.abs(ref), axis=0)
        assert e.max() <= tol
    batch.close()


def test_graph_refuses_after_a_network_moves(ctx, rhmod, nets):
    import torch

    g, n = nets[0]
    W = torch.from_numpy(np.ascontiguousarray(gridgen.directions(n.n_p, 4, 5).T)).cuda()
    HW = torch.zeros_like(W)
    batch = ctx.batch([n], [W], [HW])
    batch.launch()
    torch.cuda.synchronize()
    n.set_loads(g.Pd * 1.001, g.Qd * 1.001)
    n.solve()
    with pytest.raises(rhmod.RhError) as ei:
        batch.launch()
    assert ei.value.status == rhmod.RH_ESTATE
    batch.close()
    n.set_loads(g.Pd, g.Qd)
    n.solve()
