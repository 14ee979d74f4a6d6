"""Benchmark: reduced-Hessian HVPs per second on the 10k-bus synthetic grid.

One step = the full dense reduced Hessian (n_p = 2,799 directions) computed
through the C ABI in k = 256 direction blocks, one kernel launch per block,
with every input already resident on the GPU.  The timed region brackets
exactly `--steps` steps with device synchronisations.  Prints one JSON line.

Roofline: the block kernel is the only kernel of a step.  Its algorithmic HBM
bytes per launch are (10 n_x + 5 n_p) * 8 per direction (every intermediate
written and read once, W read twice, H written) plus the factor entries of
the four triangular sweeps (12 bytes each), the per-incidence coefficients and
G_p; achieved GB/s = those bytes / the average launch duration from HIP events
recorded on the launch stream.  Peak: 8 TB/s (MI355X HBM3E).

The CPU baseline runs the FP64 oracle (single-threaded SuperLU solves and
sparse products) on the same grid for a bounded sample of identity blocks.
"""
import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0


def algorithmic_bytes_per_launch(rep, g, k):
    n_x, n_p = rep["n_x"], rep["n_p"]
    per_dir = (10 * n_x + 5 * n_p) * 8
    factors = 2 * (rep["nnz_l"] + rep["nnz_u"]) * 12  # L, U, U^T, L^T sweeps
    tape = 2 * g.n_branch * (5 * 8 + 4) + g.n_bus * 8 * 3
    gp = 2 * (n_x + 2 * g.n_branch * 2) * 12
    return per_dir * k + factors + tape + gp


def cpu_baseline(g, k, budget_s=12.0):
    """Oracle on blocks of k identity columns until the time budget is spent."""
    from oracle import solve

    t0 = time.perf_counter()
    s = solve(g)
    setup = time.perf_counter() - t0
    n_p = s.o.n_p
    done = 0
    t1 = time.perf_counter()
    while done < n_p and time.perf_counter() - t1 < budget_s:
        kb = min(k, n_p - done)
        W = np.zeros((n_p, kb))
        W[np.arange(done, done + kb), np.arange(kb)] = 1.0
        s.hvp(W)
        done += kb
    el = time.perf_counter() - t1
    return {
        "value": done / el, "unit": "HVP/s", "cores": 1, "kind": "oracle",
        "sample": f"{done} of {n_p} identity directions in k={k} blocks ({el:.1f} s); "
                  f"Newton+LU+lambda set-up {setup:.1f} s not included",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(direction blocks would shard across GPUs, see DESIGN.md)"}))
        sys.exit(2)

    import torch

    import gridgen
    from paper_2201_00241_amd import rh

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    g = gridgen.config_grid(args.config, 0)
    ctx = rh.Context(0)
    net = rh.Network(ctx, g)
    t0 = time.perf_counter()
    net.solve(1e-13, 30)
    setup_s = time.perf_counter() - t0
    n_p = net.n_p
    k = min(args.k, n_p)
    H = torch.empty((n_p, n_p), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    for _ in range(args.warmup):
        net.reduced_hessian_device(H, k_block=k, stream=sptr)
    torch.cuda.synchronize()

    ctx.set_timing(True)
    net.report()  # open a fresh timing window
    step_ms = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        net.reduced_hessian_device(H, k_block=k, stream=sptr)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    trep = net.report()  # launch durations of the timed region
    ctx.set_timing(False)
    for i in range(args.steps):
        step_ms.append(ev[i].elapsed_time(ev[i + 1]))
    total_ms = ev[0].elapsed_time(ev[-1])
    ms_per_step = total_ms / args.steps
    value = n_p * args.steps / (total_ms / 1e3)

    # one more step with in-kernel phase stamps (outside the timed region)
    ctx.set_timing(2)
    net.reduced_hessian_device(H, k_block=k, stream=sptr)
    torch.cuda.synchronize()
    prep = net.report()
    ctx.set_timing(0)

    rep = trep
    launches = trep["last_launches"]
    avg_launch_ms = trep["last_kernel_ms"] / launches
    bytes_launch = algorithmic_bytes_per_launch(rep, g, k)
    achieved = bytes_launch / (avg_launch_ms / 1e3) / 1e9
    out = {
        "metric": "reduced-Hessian HVPs/sec at 10k buses (k=256) vs plain; p50/p99 latency",
        "value": value,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"full reduced Hessian of a {g.n_bus}-bus synthetic grid "
                        f"({g.n_branch} branches, {g.n_gen} generators) in k={k} blocks",
            "n_x": rep["n_x"], "n_p": n_p, "k": k,
            "launches_per_step": launches // args.steps,
            "dirs_per_group": rep["dirs_per_group"],
            "levels_l": rep["levels_l"], "levels_u": rep["levels_u"],
            "nnz_l": rep["nnz_l"], "nnz_u": rep["nnz_u"],
            "steps_l": rep["steps_l"], "steps_u": rep["steps_u"],
        },
        "phase_us": dict(zip(["spmul", "L", "U", "projection", "Ut", "Lt", "spmuladd"],
                             [round(v, 2) for v in prep["phase_us"]])),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99)),
                       "what": "one full reduced Hessian"},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": None,
            "kernel": "block_kernel", "avg_launch_ms": avg_launch_ms,
            "algorithmic_bytes_per_launch": bytes_launch,
        },
        "setup_s": setup_s,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
