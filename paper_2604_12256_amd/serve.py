"""Continuous-batching request loop for circuit simulation on one GPU.

Requests (circuits of 10..30 qubits) arrive over time.  The server

* admits a request as soon as its device memory fits in the HBM budget and
  a slot is free, in arrival order.  The memory of a request is its state
  vector (2^n x 16 B for complex128, 8 B for complex64) plus the buffers its
  context holds (booster sub-states, operator tables, stage programs,
  descriptors): a reserve at admission, replaced by the context's own count
  once the circuit is planned.  A request that does not fit yet waits at the
  head of the queue; a later request may pass it if it fits.  Passing counts
  as a bypass only when the later request takes what the head waits for (a
  stream, or memory the head needs); after `max_bypass` bypasses such
  requests wait behind the head (no starvation), while requests that take
  nothing the head needs (small circuits while the head waits for a stream)
  are still admitted;
* runs every admitted large circuit on a stream of its own (plan on the
  host, then the optimised plan on the device), overlapping on the GPU;
* collects admitted small and mid-size circuits (up to BATCH_MAX qubits)
  and runs all pending ones together whenever the batch stream is idle:
  states that fit one workgroup's LDS in one launch, the others with their
  full-state stages launched together (one launch per stage step);
* detects completion by polling stream events, records latency =
  completion - arrival, and releases the memory, which admits more requests.

`serve_sequential_plain` is the baseline: one request at a time in arrival
order on the gate-by-gate path.

The scheduler talks to a backend (`GpuBackend` here, a fake one in the CPU
tests), so its admission / batching / accounting logic is testable without a
device.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import workloads as W

AMP_BYTES = {"c128": 16, "c64": 8}
SMALL_MAX = {"c128": 13, "c64": 14}   # whole state in one workgroup's LDS
BATCH_MAX = {"c128": 18, "c64": 19}   # run in the batch rather than on a stream of their own


@dataclass
class Result:
    rid: int
    n: int
    dtype: str
    gates: int
    arrival: float
    start: float = 0.0
    done: float = 0.0
    mode: str = ""          # "batch" | "stream" | "plain"

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def state_bytes(n: int, dtype: str) -> int:
    return AMP_BYTES[dtype] << n


def is_small(n: int, dtype: str) -> bool:
    return n <= SMALL_MAX[dtype]


def is_batched(n: int, dtype: str) -> bool:
    return n <= BATCH_MAX[dtype]


def reserve_bytes(n: int, dtype: str) -> int:
    """Device memory reserved for a request at admission: its state and an
    allowance for its context's own buffers (tables, programs, sub-states),
    which the context's own count replaces once the circuit is planned."""
    extra = (1 << 20) if is_small(n, dtype) else (64 << 20)
    return state_bytes(n, dtype) + extra


# ------------------------------------------------------------------ backends
class GpuBackend:
    """Runs requests through the HIP library (one Simulator per request)."""

    def __init__(self, opt: int, n_streams: int = 4, keep_states: bool = False) -> None:
        import torch
        from . import qsim
        self.torch, self.qsim = torch, qsim
        self.opt = opt
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.batch_stream = torch.cuda.Stream()
        self.keep_states = keep_states
        self.kept: Dict[int, np.ndarray] = {}
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait(self, dt: float) -> None:
        time.sleep(dt)

    def budget_bytes(self) -> int:
        free, _total = self.torch.cuda.mem_get_info()
        return int(min(288e9, free)) - (2 << 30)

    def prepare(self, req: W.Request, stream_idx: Optional[int]) -> object:
        stream = self.streams[stream_idx] if stream_idx is not None else self.batch_stream
        sim = self.qsim.Simulator(req.n, dtype=req.dtype, opt=self.opt, stream=stream)
        sim.load(req.circuit())
        return sim

    def start_stream(self, sim, stream_idx: int):
        stream = self.streams[stream_idx]
        sim.run_async()
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def start_batch(self, sims: Sequence) -> object:
        for dtype in ("c128", "c64"):   # one launch per dtype, both on the batch stream
            group = [s for s in sims if s.dtype == dtype]
            if group:
                self.qsim.run_batch(group, stream=self.batch_stream)
        ev = self.torch.cuda.Event()
        ev.record(self.batch_stream)
        return ev

    def done(self, token) -> bool:
        return token.query()

    def held_bytes(self, sim) -> int:
        """Device bytes the request's context holds beside its state."""
        return sim.device_bytes()

    def release(self, rid: int, sim) -> None:
        if self.keep_states:
            self.kept[rid] = sim.amplitudes()
        sim.close()
        del sim

    def run_plain(self, req: W.Request) -> None:
        sim = self.qsim.Simulator(req.n, dtype=req.dtype, opt=0)
        sim.load(req.circuit())
        sim.run()
        if self.keep_states:
            self.kept[req.rid] = sim.amplitudes()
        sim.close()


# ------------------------------------------------------------------ scheduler
@dataclass
class _Slot:
    req: W.Request
    handle: object
    token: object = None
    stream_idx: Optional[int] = None
    nbytes: int = 0                    # device memory it holds (state + context buffers)


def held_bytes(backend, handle) -> int:
    f = getattr(backend, "held_bytes", None)
    return int(f(handle)) if f else 0


def serve(requests: Sequence[W.Request], backend, max_streams: int = 4, max_bypass: int = 8,
          poll_s: float = 2e-4, progress=None) -> List[Result]:
    """Runs the request stream through the continuous-batching server.
    `progress(n_done, n_total)` is called after each completion, if given."""
    pending = sorted(requests, key=lambda r: r.arrival_s)
    results: Dict[int, Result] = {r.rid: Result(r.rid, r.n, r.dtype, 0, r.arrival_s) for r in pending}
    queue: List[W.Request] = []
    used = 0
    free_streams = list(range(max_streams))
    running: List[_Slot] = []          # large circuits on their own streams
    small_ready: List[_Slot] = []      # admitted batched circuits waiting for the batch
    batch: Optional[List[_Slot]] = None
    batch_token = None
    bypassed = 0
    nxt = 0
    n_done = 0
    budget = backend.budget_bytes()
    while n_done < len(pending):
        now = backend.now()
        while nxt < len(pending) and pending[nxt].arrival_s <= now:
            queue.append(pending[nxt])
            nxt += 1
        progressed = False
        # admission in arrival order, by device memory
        i = 0
        head_mem = head_stream = False   # what a blocked head request waits for
        while i < len(queue):
            req = queue[i]
            small = is_batched(req.n, req.dtype)   # runs in the batch: takes no stream
            need = reserve_bytes(req.n, req.dtype)
            mem_ok = used + need <= budget
            stream_ok = small or bool(free_streams)
            if i == 0 and not (mem_ok and stream_ok):
                head_mem, head_stream = not mem_ok, not stream_ok
                i += 1
                continue
            if not (mem_ok and stream_ok):
                i += 1
                continue
            if i > 0:
                # passing the blocked head: a bypass if it takes what the head waits for
                head = queue[0]
                takes = (head_stream and not small) or head_mem or \
                    used + need + reserve_bytes(head.n, head.dtype) > budget
                if takes:
                    if bypassed >= max_bypass:
                        i += 1         # hold the line for the head request
                        continue
                    bypassed += 1
            else:
                bypassed = 0
            queue.pop(i)
            used += need
            res = results[req.rid]
            res.gates = W.layered_gate_count(req.n, req.layers)
            if small:
                slot = _Slot(req, backend.prepare(req, None))
                small_ready.append(slot)
            else:
                si = free_streams.pop(0)
                slot = _Slot(req, backend.prepare(req, si), stream_idx=si)
            # the context's own count replaces the admission reserve
            slot.nbytes = state_bytes(req.n, req.dtype) + held_bytes(backend, slot.handle)
            used += slot.nbytes - need
            if not small:
                res.start = backend.now()
                slot.token = backend.start_stream(slot.handle, slot.stream_idx)
                res.mode = "stream"
                running.append(slot)
            progressed = True
        # one batched run of every admitted batched circuit when idle
        if batch is None and small_ready:
            batch, small_ready = small_ready, []
            t = backend.now()
            for s in batch:
                results[s.req.rid].start = t
                results[s.req.rid].mode = "batch"
            batch_token = backend.start_batch([s.handle for s in batch])
            progressed = True
        # completions
        for slot in list(running):
            if backend.done(slot.token):
                t = backend.now()
                results[slot.req.rid].done = t
                backend.release(slot.req.rid, slot.handle)
                used -= slot.nbytes
                free_streams.append(slot.stream_idx)
                running.remove(slot)
                n_done += 1
                progressed = True
                if progress:
                    progress(n_done, len(pending))
        if batch is not None and backend.done(batch_token):
            t = backend.now()
            for s in batch:
                results[s.req.rid].done = t
                backend.release(s.req.rid, s.handle)
                used -= s.nbytes
                n_done += 1
                if progress:
                    progress(n_done, len(pending))
            batch, batch_token = None, None
            progressed = True
        if not progressed:
            backend.wait(poll_s)
    return [results[r.rid] for r in pending]


def serve_sequential_plain(requests: Sequence[W.Request], backend, progress=None) -> List[Result]:
    """Baseline: FIFO, one request at a time, gate-by-gate path."""
    out = []
    for req in sorted(requests, key=lambda r: r.arrival_s):
        now = backend.now()
        if now < req.arrival_s:
            backend.wait(req.arrival_s - now)
        res = Result(req.rid, req.n, req.dtype, W.layered_gate_count(req.n, req.layers), req.arrival_s)
        res.start = backend.now()
        backend.run_plain(req)
        res.done = backend.now()
        res.mode = "plain"
        out.append(res)
        if progress:
            progress(len(out), len(requests))
    return out


def summarize(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    t_first = min(r.arrival for r in results)
    t_last = max(r.done for r in results)
    gates = sum(r.gates for r in results)
    amp_updates = sum(r.gates * float(2 ** r.n) for r in results)
    span = t_last - t_first
    return {"requests": len(results), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "makespan_s": span, "gate_apps_per_s": gates / span, "amp_updates_per_s": amp_updates / span,
            "batched": sum(1 for r in results if r.mode == "batch")}


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=0.8, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--n-min", type=int, default=10)
    ap.add_argument("--n-max", type=int, default=30)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--skip-plain", action="store_true")
    args = ap.parse_args(argv)
    from . import qsim

    def progress(tag):
        def f(done, total):
            if done % 20 == 0 or done == total:
                print(f"[serve] {tag}: {done}/{total} done", file=sys.stderr, flush=True)
        return f
    reqs = W.serving_stream(args.requests, args.rate, args.seed, args.n_min, args.n_max)
    out = {"config": vars(args)}
    be = GpuBackend(qsim.OPT_ALL, n_streams=args.streams)
    out["served"] = summarize(serve(reqs, be, max_streams=args.streams, progress=progress("served")))
    print(json.dumps({"served": out["served"]}), flush=True)
    if not args.skip_plain:
        bp = GpuBackend(0)
        out["sequential_plain"] = summarize(serve_sequential_plain(reqs, bp, progress=progress("plain")))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
