"""The allocation-free product entry point (needs an MI355X).

rh_hvp_device_noalloc takes its launch scratch from the library's fixed
device array instead of allocating.  Three calls in a row, each on a smaller
input than the one before (a 70k-bus network whose full launch scratch does
not fit the array, so fewer workgroups take several direction chunks each;
then the 10k and 1k networks), in FP64 and in the refined mode: every product
is bitwise the product of rh_hvp_device on the same inputs, and the 10k and
1k products are within the FP64 tolerance of the oracle.
"""
import numpy as np
import pytest

import gridgen
from oracle import solve

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-8


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
def nets(rhmod):
    ctx = rhmod.Context(0)
    out = {}
    for name in ("c3", "c2", "c1"):
        g = gridgen.config_grid(name, 0)
        net = rhmod.Network(ctx, g)
        net.solve()
        out[name] = (g, net)
    yield out
    for g, net in out.values():
        net.close()
    ctx.close()


@pytest.mark.parametrize("prec_name", ["fp64", "refined"])
def test_noalloc_equals_the_allocating_entry_point(rhmod, nets, prec_name):
    import torch

    prec = rhmod.RH_FP64 if prec_name == "fp64" else rhmod.RH_FP32_REFINED
    stream = torch.cuda.current_stream().cuda_stream
    # largest input first: at 70k buses and 64 directions one workgroup's
    # scratch (vector and Y_x in global memory) is 2.2 MB, so the 128 MiB array
    # holds fewer workgroups than the launch has direction chunks
    for name, k, seed in (("c3", 64, 81), ("c2", 256, 82), ("c1", 16, 83)):
        g, net = nets[name]
        W = gridgen.directions(net.n_p, k, seed)
        dW = torch.from_numpy(np.ascontiguousarray(W.T)).cuda()
        ref = torch.full_like(dW, float("nan"))
        out = torch.full_like(dW, float("nan"))
        _say(f"noalloc: {name} ({net.n_x} states), k={k}, {prec_name}")
        net.hvp_device(dW, ref, stream=stream, prec=prec)
        net.hvp_device_noalloc(dW, out, stream=stream, prec=prec)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
        if name != "c3":
            HW = solve(g).hvp(W)
            e = np.max(np.abs(a.T - HW), axis=0) / np.max(np.abs(HW), axis=0)
            _say(f"  per-column error vs oracle: max {e.max():.2e}")
            assert e.max() <= (TOL64 if prec_name == "fp64" else TOL32)


def test_noalloc_rejects_bad_arguments(rhmod, nets):
    import torch

    g, net = nets["c1"]
    W = torch.zeros((4, net.n_p), dtype=torch.float64, device="cuda")
    HW = torch.zeros_like(W)
    with pytest.raises(rhmod.RhError) as ei:
        rhmod.rh_hvp_device_noalloc(net.h, 4, W.data_ptr(), net.n_p - 1, HW.data_ptr(), net.n_p)
    assert ei.value.status == rhmod.RH_EINVAL
    with pytest.raises(rhmod.RhError) as ei:
        rhmod.rh_hvp_device_noalloc(net.h, 4, W.data_ptr(), net.n_p, HW.data_ptr(), net.n_p, prec=7)
    assert ei.value.status == rhmod.RH_EINVAL
    # zero directions: nothing to do
    rhmod.rh_hvp_device_noalloc(net.h, 0, W.data_ptr(), net.n_p, HW.data_ptr(), net.n_p)
