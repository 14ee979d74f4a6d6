"""The launch-shape tuner (needs an MI355X).

rh_autotune times the candidate launch shapes (full-Hessian launch size,
directions per workgroup, sweep-schedule parameters) and applies the
fastest; a shape measured for one operating point of a grid is read back
from the cache file for another operating point of the same grid.  Products
with the tuned shapes match the oracle.
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


def _valid(t, n_p):
    return (t["k"] in (128, 256, 512, 1024, n_p) and t["dirs_per_group"] in (1, 2, 4)
            and t["block_rows"] in (16, 32, 64) and t["wave_steps"] in (0, 1) and t["ms_per_hessian"] > 0)


def test_autotune_measures_caches_and_applies(ctx, rhmod, tmp_path, monkeypatch):
    cache = tmp_path / "tiles.txt"
    monkeypatch.setenv("RH_TUNE_CACHE", str(cache))
    g = gridgen.config_grid("c1", 0)
    net = rhmod.Network(ctx, g)
    net.solve()
    _say("tune: 1k grid, FP64, empty cache")
    t = net.autotune()
    _say(f"  chosen {t}")
    assert t["source"] == 1 and _valid(t, net.n_p)
    assert net.report()["tile"][0] == t
    H = net.reduced_hessian(k_block=0)
    assert net.report()["last_k"] == t["k"]
    Ho = solve(g).reduced_hessian()
    assert np.max(np.abs(H - Ho)) / np.max(np.abs(Ho)) <= 1e-9
    # another operating point of the same grid: the shape comes from the cache
    g2 = gridgen.perturb_loads(g, seed=71)
    net2 = rhmod.Network(ctx, g2)
    net2.solve()
    t2 = net2.autotune()
    assert t2["source"] == 2
    assert {k: t2[k] for k in ("k", "dirs_per_group", "block_rows", "wave_steps")} == \
        {k: t[k] for k in ("k", "dirs_per_group", "block_rows", "wave_steps")}
    W = gridgen.directions(net2.n_p, 24, 72)
    ref = solve(g2).hvp(W)
    assert np.max(np.abs(net2.hvp(W) - ref)) / np.max(np.abs(ref)) <= 1e-9
    # measuring again on request
    t3 = net2.autotune(flags=rhmod.RH_TUNE_MEASURE)
    assert t3["source"] == 1 and _valid(t3, net2.n_p)
    # the refined mode has a shape of its own
    tr = net.autotune(prec=rhmod.RH_FP32_REFINED)
    _say(f"  refined {tr}")
    assert _valid(tr, net.n_p)
    e = np.max(np.abs(net.hvp(W, prec=rhmod.RH_FP32_REFINED) - solve(g).hvp(W)), axis=0)
    assert np.all(e / np.max(np.abs(solve(g).hvp(W)), axis=0) <= 1e-8)
    lines = cache.read_text().splitlines()
    assert len(lines) >= 3 and all(ln.startswith("v1 ") for ln in lines)
    # no cache at all
    t4 = net2.autotune(flags=rhmod.RH_TUNE_NO_CACHE | rhmod.RH_TUNE_MEASURE)
    assert t4["source"] == 1 and len(cache.read_text().splitlines()) == len(lines)
    net.close()
    net2.close()
