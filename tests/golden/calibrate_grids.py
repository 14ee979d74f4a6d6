"""Calibrate the loading factor and loss factor of the synthetic workloads.

Run by hand (``python tests/golden/calibrate_grids.py c2 0 1 2``); it calls
only the generator and the oracle; Newton starts from the generator's voltage
guess ``v0`` (angles 0).  For each instance it

1. solves the power flow at a light loading ``alpha0`` and reads off the
   fraction of the total load that the slack bus supplies (the losses),
2. sets the loss factor ``kappa`` to that fraction scaled linearly in the
   loading factor (losses grow with the square of the load),
3. bisects the largest loading factor for which Newton converges, to 0.01.

The values chosen in ``gridgen.CONFIGS`` keep every listed instance at or
below 0.8 of its limit; ``tests/test_oracle.py::test_grids_converge_for_the_workloads``
checks convergence there.
"""
import json
import sys
from pathlib import Path

sys.path.insert(0, str(Path(__file__).resolve().parents[2]))

import numpy as np  # noqa: E402

import gridgen  # noqa: E402
from oracle.powerflow import Oracle  # noqa: E402


def _grid(name, inst, alpha, kappa):
    c = gridgen.CONFIGS[name]
    return gridgen.geometric(c["n_bus"], c["n_branch"], c["n_gen"],
                             1000 * gridgen.CONFIG_INDEX[name] + inst, alpha, kappa=kappa)


def converges(name, inst, alpha, kappa):
    g = _grid(name, inst, alpha, kappa)
    o = Oracle(g)
    _, _, ok = o.newton(o.p0(), max_iter=25)
    return ok


def loss_fraction(name, inst, alpha0):
    g = _grid(name, inst, alpha0, 0.0)
    o = Oracle(g)
    x, _, ok = o.newton(o.p0(), max_iter=25)
    if not ok:
        raise RuntimeError("light-load solve failed")
    # the slack covers losses plus its own cell's load
    own = g.Pd.sum() - g.Pg[1:].sum()
    return (o.slack_power(x, o.p0()) - own) / g.Pd.sum()


def main(name, insts, alpha0=0.05):
    alpha0 = 0.02 if name == "c3" else alpha0
    out = {}
    for inst in insts:
        lf = loss_fraction(name, inst, alpha0)
        kap = lambda a: lf * a / alpha0  # noqa: E731
        lo, hi = 0.0, 1.0
        while hi - lo > 0.01:
            mid = 0.5 * (lo + hi)
            if converges(name, inst, mid, kap(mid)):
                lo = mid
            else:
                hi = mid
        out[inst] = {"loss_fraction_at_alpha0": lf, "alpha_max": lo,
                     "kappa_per_alpha": lf / alpha0}
        print(name, inst, out[inst], flush=True)
    return out


if __name__ == "__main__":
    name = sys.argv[1]
    insts = [int(v) for v in sys.argv[2:]] or [0]
    print(json.dumps(main(name, insts), indent=1))
