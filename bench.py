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
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = ROOT / "profiles" / "block_kernel_10k_hbm_traffic.txt"


def sources_digest():
    """SHA-256 over the library sources (kernels, planner, ABI), in name order."""
    h = hashlib.sha256()
    for f in sorted((ROOT / "paper_2201_00241_amd" / "csrc").iterdir()):
        if f.suffix in (".hip", ".cpp", ".h"):
            h.update(f.name.encode())
            h.update(f.read_bytes())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the block kernel from the committed counter
    summary, or None if the kernel sources changed since it was measured."""
    if not TRAFFIC_FILE.exists():
        return None
    kv = {}
    for line in TRAFFIC_FILE.read_text().splitlines():
        if ":" in line and not line.startswith(("#", " ", "|")):
            key, val = line.split(":", 1)
            kv[key.strip()] = val.strip()
    if kv.get("sources_sha256") != sources_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    ap.add_argument("--workload", default="hessian",
                    choices=["hessian", "batch", "serving"],
                    help="hessian: full reduced Hessian (the headline metric); batch: many "
                         "operating points of one grid in one launch; serving: Poisson "
                         "request mix through the continuous-batching server")
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes, 10 times "
                         "(reference for scaling HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(direction blocks are independent and would shard across "
                                   "GPUs by block, which is not implemented)"}))
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                          "launches": 10}), flush=True)
        return

    import gridgen
    from paper_2201_00241_amd import rh

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)
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

    # the refined FP32 mode on the same workload ("vs plain"), after the timed region
    H64 = H.clone()
    for _ in range(args.warmup):
        net.reduced_hessian_device(H, k_block=k, stream=sptr, prec=rh.RH_FP32_REFINED)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    for _ in range(args.steps):
        net.reduced_hessian_device(H, k_block=k, stream=sptr, prec=rh.RH_FP32_REFINED)
    r1.record(stream)
    torch.cuda.synchronize()
    refined_ms = r0.elapsed_time(r1) / args.steps
    refined_dev = float((H - H64).abs().max() / H64.abs().max())
    H.copy_(H64)

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
    traffic = measured_traffic()
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
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "kernel": "block_kernel", "avg_launch_ms": avg_launch_ms,
            "algorithmic_bytes_per_launch": bytes_launch,
        },
        "refined_fp32": {"value": n_p / (refined_ms / 1e3), "unit": "HVP/s", "ms_per_step": refined_ms,
                         "max_rel_dev_from_fp64": refined_dev,
                         "what": "same workload, FP32 sweeps with two FP64 refinement steps"},
        "setup_s": setup_s,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, k)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Operating points of one grid (loads perturbed by up to 10 %), each with
    128 Gaussian directions, in one launch per step."""
    import torch

    import gridgen
    from paper_2201_00241_amd import rh

    base = gridgen.config_grid(args.config if args.config != "c2" else "c3", 0)
    ctx = rh.Context(0)
    nets, t0 = [], time.perf_counter()
    for i in range(args.instances):
        g = gridgen.perturb_loads(base, seed=5000 + i)
        n = rh.Network(ctx, g)
        n.solve(1e-13, 30)
        nets.append(n)
    setup_s = time.perf_counter() - t0
    k = 128
    Ws = [torch.from_numpy(np.ascontiguousarray(gridgen.directions(n.n_p, k, 7000 + i).T)).cuda()
          for i, n in enumerate(nets)]
    HWs = [torch.empty_like(W) for W in Ws]
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.hvp_batch_device(nets, Ws, HWs, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    ctx.set_timing(1)
    ctx.report()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        ctx.hvp_batch_device(nets, Ws, HWs, stream=stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    rep = ctx.report()
    ctx.set_timing(0)
    ms = e0.elapsed_time(e1) / args.steps
    n_x, n_p = nets[0].n_x, nets[0].n_p
    # the same batch with FP32 sweeps and FP64 refinement, after the timed
    # region: its rate and its largest deviation from the FP64 results
    HW64 = [h.clone() for h in HWs]
    ctx.hvp_batch_device(nets, Ws, HWs, stream=stream.cuda_stream, prec=rh.RH_FP32_REFINED)
    torch.cuda.synchronize()
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record(stream)
    for _ in range(args.steps):
        ctx.hvp_batch_device(nets, Ws, HWs, stream=stream.cuda_stream, prec=rh.RH_FP32_REFINED)
    r1.record(stream)
    torch.cuda.synchronize()
    refined_ms = r0.elapsed_time(r1) / args.steps
    refined_dev = max(float((h - g).abs().max() / g.abs().max()) for h, g in zip(HWs, HW64))
    print(json.dumps({
        "metric": "batched instances: HVPs/sec", "value": len(nets) * k / (ms / 1e3),
        "unit": "HVP/s", "ms_per_step": ms, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(nets)} operating points of a {base.n_bus}-bus grid "
                               f"x {k} Gaussian directions, one launch",
                   "n_x": n_x, "n_p": n_p, "launches_per_step": rep["last_launches"] // args.steps,
                   "dirs_per_group": rep["dirs_per_group"]},
        "avg_launch_ms": rep["last_kernel_ms"] / max(1, rep["last_launches"]),
        "refined_fp32": {"value": len(nets) * k / (refined_ms / 1e3), "unit": "HVP/s",
                         "ms_per_step": refined_ms, "max_rel_dev_from_fp64": refined_dev,
                         "what": "same batch, FP32 sweeps with two FP64 refinement steps"},
        "setup_s": setup_s}), flush=True)


def bench_serving(args):
    """Poisson arrivals over resident 1k, 10k and 70k networks (4 operating
    points each), requests for 1, 16 or 128 directions or the full Hessian."""
    import gridgen
    from paper_2201_00241_amd import rh
    from paper_2201_00241_amd.serving import Request, Server, latency_summary

    ctx = rh.Context(0)
    nets = {}
    for name in ("c1", "c2", "c3"):
        base = gridgen.config_grid(name, 0)
        for i in range(4):
            n = rh.Network(ctx, gridgen.perturb_loads(base, seed=9000 + i))
            n.solve(1e-13, 30)
            nets[f"{name}/{i}"] = n
    keys = sorted(nets)
    rng = np.random.default_rng(11)

    def make(n_req, rate):
        t, reqs = 0.0, []
        for i in range(n_req):
            key = keys[rng.integers(len(keys))]
            k = int(rng.choice([1, 16, 128, 0], p=[0.3, 0.3, 0.3, 0.1]))
            if k == 0 and key.startswith("c3"):
                k = 128  # a full 70k-bus Hessian would dominate the mix
            W = None if k == 0 else rng.standard_normal((nets[key].n_p, k))
            if rate:
                t += rng.exponential(1.0 / rate)
            reqs.append(Request(rid=i, key=key, k=k, W=W, arrival=t))
        return reqs

    srv = Server(ctx, nets, max_inflight=3, dirs_per_launch=4096, block=256)
    srv.run(make(20, 0))  # warm-up
    t0 = time.perf_counter()
    closed = srv.run(make(120, 0))
    peak = len(closed) / (time.perf_counter() - t0)
    reqs = make(200, 0.8 * peak)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    hvps = sum((r.k if r.k else nets[r.key].n_p) for r in done)
    print(json.dumps({
        "metric": "served reduced-Hessian requests: p50/p99 latency", "unit": "ms",
        "latency": latency_summary(done), "requests_per_s": len(done) / wall,
        "hvp_per_s": hvps / wall, "peak_requests_per_s": peak, "arrival_rate": 0.8 * peak,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Poisson mix over 1k/10k/70k-bus grids, 4 operating points "
                               "each; k in {1,16,128} or the full Hessian (1k, 10k)"}}),
          flush=True)


if __name__ == "__main__":
    main()
