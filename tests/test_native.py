"""CPU checks of the library's host planner through a small native driver.

The driver (tests/native/check_planner.cpp) links the planner sources with
g++ and checks the fixed-pattern LU against dense elimination and the device
sweep schedules (levels + dense-inverse blocks) against plain sweeps, by
emulating on the host exactly what the kernel does per step.
"""
import subprocess
from pathlib import Path

import numpy as np
import pytest

import gridgen

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2201_00241_amd" / "csrc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = tmp_path_factory.mktemp("native") / "check_planner"
    subprocess.run(["g++", "-O2", "-std=c++17", str(ROOT / "tests/native/check_planner.cpp"),
                    str(CSRC / "network.cpp"), str(CSRC / "sparse_lu.cpp"), "-o", str(out)],
                   check=True)
    return out


def _dump(g, path):
    with open(path, "wb") as f:
        np.array([g.n_bus, g.n_branch, g.n_gen], np.int32).tofile(f)
        for a in (g.br_from, g.br_to):
            np.asarray(a, np.int32).tofile(f)
        for a in (g.br_r, g.br_x, g.br_b):
            np.asarray(a, np.float64).tofile(f)
        np.asarray(g.bus_type, np.int32).tofile(f)
        for a in (g.Pd, g.Qd):
            np.asarray(a, np.float64).tofile(f)
        np.asarray(g.gen_bus, np.int32).tofile(f)
        for a in (g.Pg, g.Vg, g.c2, g.c1, g.c0):
            np.asarray(a, np.float64).tofile(f)
        if g.v0 is not None:
            np.asarray(g.v0, np.float64).tofile(f)


GRIDS = {
    "c0": lambda: gridgen.config_grid("c0", 0),
    "geo60": lambda: gridgen.geometric(60, 81, 6, seed=560, alpha=0.3, kappa=0.0255),
    "geo75": lambda: gridgen.geometric(75, 101, 7, seed=575, alpha=0.3, kappa=0.0255),
    "geo120": lambda: gridgen.geometric(120, 162, 12, seed=77, alpha=0.3, kappa=0.0255),
    "c1": lambda: gridgen.config_grid("c1", 0),
    "c2": lambda: gridgen.config_grid("c2", 0),
}


@pytest.mark.parametrize("name", list(GRIDS))
def test_planner_lu_and_sweep_schedules(driver, tmp_path, name):
    g = GRIDS[name]()
    f = tmp_path / "grid.bin"
    _dump(g, f)
    res = subprocess.run([str(driver), str(f)], capture_output=True, text=True, check=True)
    errs = {}
    for ln in res.stdout.splitlines():
        parts = ln.split()
        if parts and parts[0] == "max_err":
            errs[parts[1]] = float(parts[2])
    assert "order_violations 0" in res.stdout, res.stdout
    assert "refactor_level_violations 0" in res.stdout, res.stdout
    assert "max_err device_refactor" in res.stdout, res.stdout
    assert "max_err device_solve" in res.stdout, res.stdout
    assert "order_violations_composed" not in res.stdout
    assert "record_mismatch" not in res.stdout, res.stdout
    assert "pack_reuse_mismatch" not in res.stdout, res.stdout
    assert "sweeps_reuse_mismatch" not in res.stdout, res.stdout
    assert any(k.startswith("sweep_") for k in errs), res.stdout
    if g.n_x <= 400:
        assert "lu_solve" in errs and "lu_solve_t" in errs
    for k, v in errs.items():
        assert v < 1e-12, (k, v, res.stdout)


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    """The same driver and planner sources built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only; any report aborts the run)."""
    out = tmp_path_factory.mktemp("native_san") / "check_planner_san"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    str(ROOT / "tests/native/check_planner.cpp"), str(CSRC / "network.cpp"),
                    str(CSRC / "sparse_lu.cpp"), "-o", str(out)], check=True)
    return out


@pytest.mark.parametrize("name", ["c0", "geo60", "geo75", "geo120", "c1"])
def test_planner_under_sanitizers(sanitized_driver, tmp_path, name):
    """Network set-up, Newton, the LU, the four sweep schedules with their
    packing and records, and the device refactorisation's maps, with every
    memory access and integer operation checked."""
    f = tmp_path / "grid.bin"
    _dump(GRIDS[name](), f)
    res = subprocess.run([str(sanitized_driver), str(f)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    assert "order_violations 0" in res.stdout and "refactor_level_violations 0" in res.stdout, res.stdout
