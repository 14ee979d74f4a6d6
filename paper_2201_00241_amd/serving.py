"""Continuous-batching server for reduced-Hessian requests on one GPU.

Requests ask for k Hessian-vector products of one resident network (a grid
at an operating point whose LU factors, adjoint and branch coefficients stay
on the device) or for its full reduced Hessian, in FP64 or in the refined
FP32 mode.  The server splits every request into work items of at most
`block` directions (a full Hessian becomes identity blocks, Sec. 5.3) and
keeps up to `max_inflight` batched launches in flight, each on its own
stream.  Whenever a launch completes, the items that arrived meanwhile are
admitted into the next launch, as far as the direction budget per launch and
the device-memory budget allow; a request's blocks may be spread over several
launches.  A launch carries one precision.  Every direction's arithmetic is
independent of the launch it lands in, so a result is bitwise the same alone
and in the mix.

Admission counts device memory: the resident bytes of every network (held
for the server's lifetime) are taken off the budget at start; a request then
needs its W and H W buffers plus the launch scratch of its directions.

Failures: a request whose directions are not finite is rejected at arrival.
If a batched launch fails, each request in it is retried alone; a request that
fails alone is evicted (its buffers released, `error` set) and the others
continue.

All computation runs in librh (rh_hvp_batch_device); this module only
schedules, moves buffers and measures latency.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import rh


@dataclass
class Request:
    rid: int
    key: str                      # resident network
    k: int                        # directions; 0 = the full reduced Hessian
    W: np.ndarray | None = None   # host directions (n_p x k), None for a full Hessian
    arrival: float = 0.0          # scheduled arrival, seconds from the start
    prec: int = rh.RH_FP64
    # filled by the server
    result: np.ndarray | None = None
    error: str | None = None
    t_first_launch: float = -1.0
    t_done: float = -1.0
    launches: int = 0
    retried: bool = False
    _dW: object = None
    _dHW: object = None
    _blocks_left: int = 0
    _bytes: int = 0

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class _Item:
    req: Request
    j0: int
    kb: int


@dataclass
class _Launch:
    stream: object
    event: object
    items: list = field(default_factory=list)


class Server:
    def __init__(self, ctx: rh.Context, networks: dict, max_inflight: int = 3,
                 dirs_per_launch: int = 4096, block: int = 256,
                 mem_budget_bytes: int = 64 << 30, keep_results: bool = True):
        import torch

        self.torch = torch
        self.ctx = ctx
        self.nets = networks
        self.max_inflight = max_inflight
        self.dirs_per_launch = dirs_per_launch
        self.block = block
        self.keep_results = keep_results
        self.streams = [torch.cuda.Stream() for _ in range(max_inflight)]
        self.resident = {key: n.device_bytes()[0] for key, n in networks.items()}
        self.mem_budget = mem_budget_bytes
        self.budget_left = mem_budget_bytes - sum(self.resident.values())
        if self.budget_left <= 0:
            raise ValueError("resident networks exceed the device-memory budget")

    def footprint_bytes(self, req: Request) -> int:
        """Device bytes a request holds while admitted: W and H W, and the launch
        scratch of as many of its directions as one launch may run."""
        net = self.nets[req.key]
        kk = req.k if req.k else net.n_p
        _, per_dir = net.device_bytes(req.prec)
        bufs = (2 * req.k if req.k else net.n_p) * net.n_p * 8
        return bufs + min(kk, self.dirs_per_launch) * per_dir

    # ---- request life cycle -------------------------------------------------
    def _admit(self, req: Request) -> bool:
        """Allocate the request's device buffers if the memory budget allows."""
        torch = self.torch
        net = self.nets[req.key]
        nbytes = self.footprint_bytes(req)
        if self._mem_used + nbytes > self.budget_left:
            return False
        kk = req.k if req.k else net.n_p
        if req.k:
            req._dW = torch.from_numpy(np.ascontiguousarray(np.asarray(req.W).T)).cuda().contiguous()
        req._dHW = torch.empty((kk, net.n_p), dtype=torch.float64, device="cuda")
        req._bytes = nbytes
        self._mem_used += nbytes
        req._blocks_left = (kk + self.block - 1) // self.block
        for j0 in range(0, kk, self.block):
            self._items.append(_Item(req, j0, min(self.block, kk - j0)))
        return True

    def _release(self, req: Request):
        req._dW = req._dHW = None
        self._mem_used -= req._bytes
        req._bytes = 0

    def _enqueue(self, stream, items, prec):
        torch = self.torch
        nets, ks, dWs, ldws, dHWs, ldhws, idf = [], [], [], [], [], [], []
        for it in items:
            r = it.req
            net = self.nets[r.key]
            nets.append(net.h)
            ks.append(it.kb)
            # both buffers are contiguous (rows, n_p): leading dimension n_p
            if r.k:
                dWs.append(r._dW[it.j0].data_ptr())
                idf.append(-1)
            else:
                dWs.append(0)
                idf.append(it.j0)
            ldws.append(net.n_p)
            dHWs.append(r._dHW[it.j0].data_ptr())
            ldhws.append(net.n_p)
        stream.wait_stream(torch.cuda.current_stream())  # uploads of admitted W blocks
        with torch.cuda.stream(stream):
            rh.rh_hvp_batch_device(self.ctx.h, nets, ks, dWs, ldws, dHWs, ldhws,
                                   identity_from=idf, prec=prec, stream=stream.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return ev

    def _launch(self, stream, items, now, done):
        prec = items[0].req.prec
        for it in items:
            if it.req.t_first_launch < 0:
                it.req.t_first_launch = now
            it.req.launches += 1
        try:
            return _Launch(stream, self._enqueue(stream, items, prec), items)
        except rh.RhError:
            pass
        # the batched launch failed: retry each request alone; a request that
        # fails alone is evicted
        ok = []
        by_req = {}
        for it in items:
            by_req.setdefault(it.req.rid, []).append(it)
        for its in by_req.values():
            r = its[0].req
            r.retried = True
            try:
                self._enqueue(stream, its, prec)
                ok.extend(its)
            except rh.RhError as e:
                r.error = str(e)
                r.t_done = time.perf_counter() - self._t0
                self._items = deque(x for x in self._items if x.req is not r)
                self._release(r)
                done.append(r)
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return _Launch(stream, ev, ok)

    def _finish(self, launch: _Launch, now: float, done: list):
        for it in launch.items:
            r = it.req
            if r.error is not None:  # evicted after this launch was enqueued
                continue
            r._blocks_left -= 1
            if r._blocks_left == 0:
                r.t_done = now
                if self.keep_results:
                    r.result = r._dHW.cpu().numpy().T
                self._release(r)
                done.append(r)

    # ---- event loop ---------------------------------------------------------
    def run(self, requests: list, poll_s: float = 5e-5) -> list:
        """Serve `requests` (arrival times relative to now); returns them completed."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()     # arrived, not yet admitted
        self._items: deque = deque()  # admitted blocks not yet launched
        self._mem_used = 0
        inflight: list = []
        done: list = []
        free_streams = list(self.streams)
        self._t0 = t0 = time.perf_counter()
        while pending or waiting or self._items or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                if r.k and not np.all(np.isfinite(r.W)):
                    r.error = "directions are not finite"
                elif self.footprint_bytes(r) > self.budget_left:
                    r.error = "request exceeds the device-memory budget"
                if r.error is not None:
                    r.t_done = now
                    done.append(r)
                    continue
                waiting.append(r)
            for L in list(inflight):
                if L.event.query():
                    inflight.remove(L)
                    free_streams.append(L.stream)
                    self._finish(L, time.perf_counter() - t0, done)
            while waiting and self._admit(waiting[0]):
                waiting.popleft()
            if self._items and free_streams:
                # the next launch: blocks of the head item's precision, in order
                prec = self._items[0].req.prec
                batch, dirs, rest = [], 0, deque()
                while self._items:
                    it = self._items.popleft()
                    if it.req.prec == prec and dirs + it.kb <= self.dirs_per_launch:
                        batch.append(it)
                        dirs += it.kb
                    elif it.req.prec == prec and not batch:
                        batch.append(it)  # one block larger than the budget: alone
                        dirs += it.kb
                    else:
                        rest.append(it)
                self._items = rest
                L = self._launch(free_streams.pop(0), batch, now, done)
                inflight.append(L)
                continue
            if not inflight and not self._items and not waiting and pending:
                time.sleep(max(0.0, min(pending[0].arrival - now, 1e-3)))
            else:
                time.sleep(poll_s)
        self.torch.cuda.synchronize()
        return done


def latency_summary(reqs: list) -> dict:
    lat = np.array([r.latency for r in reqs if r.error is None]) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "n": int(lat.size)}
