"""Scheduler of the serving loop on the CPU with a fake executor: admission by
memory, batching of small circuits, overlap, latency accounting and the
sequential baseline.  Service times are a model (bytes of all passes at a
fixed rate), time is virtual."""
import numpy as np
import pytest

from paper_2604_12256_amd import serve as S
from paper_2604_12256_amd import workloads as W


class FakeBackend:
    def __init__(self, budget, bw=5e12, overlap=True):
        self.t = 0.0
        self.budget = budget
        self.bw = bw
        self.overlap = overlap
        self.busy_until = 0.0
        self.in_use = 0
        self.peak = 0
        self.batches = []
        self.events = []

    def now(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 1e-4)

    def budget_bytes(self):
        return self.budget

    def service(self, req, plain=False):
        passes = W.layered_gate_count(req.n, req.layers) if plain else max(3, req.layers // 2)
        return 1e-5 + passes * 2 * S.state_bytes(req.n, req.dtype) / self.bw

    def prepare(self, req, stream_idx):
        self.in_use += S.state_bytes(req.n, req.dtype)
        self.peak = max(self.peak, self.in_use)
        assert self.in_use <= self.budget
        return req

    def start_stream(self, req, stream_idx):
        start = self.t if self.overlap else max(self.t, self.busy_until)
        self.busy_until = start + self.service(req)
        self.events.append(("stream", req.rid, start))
        return self.busy_until

    def start_batch(self, reqs):
        self.batches.append([r.rid for r in reqs])
        return self.t + max(self.service(r) for r in reqs)

    def done(self, token):
        return self.t >= token

    def release(self, rid, req):
        self.in_use -= S.state_bytes(req.n, req.dtype)

    def run_plain(self, req):
        self.t += self.service(req, plain=True)


def stream(n_req=60, rate=5.0, seed=1, n_min=10, n_max=24):
    return W.serving_stream(n_req, rate, seed, n_min, n_max)


def test_every_request_completes_once_and_latency_positive():
    reqs = stream()
    be = FakeBackend(budget=1 << 34)
    res = S.serve(reqs, be)
    assert sorted(r.rid for r in res) == sorted(r.rid for r in reqs)
    assert all(r.done >= r.start >= r.arrival for r in res)
    assert be.in_use == 0


def test_small_circuits_are_batched():
    reqs = stream(n_req=80, rate=20000.0, n_min=10, n_max=14)
    be = FakeBackend(budget=1 << 34)
    res = S.serve(reqs, be)
    small = [r for r in res if r.n <= S.BATCH_MAX[r.dtype]]
    assert small and all(r.mode == "batch" for r in small)
    assert max(len(b) for b in be.batches) > 1          # several circuits in one launch
    assert sum(len(b) for b in be.batches) == len(small)


def test_mid_size_circuits_join_the_batch_large_ones_take_streams():
    reqs = [W.Request(0, 0.0, 16, 10, "c128", 1), W.Request(1, 0.0, 18, 10, "c128", 2),
            W.Request(2, 0.0, 19, 10, "c64", 3), W.Request(3, 0.0, 19, 10, "c128", 4),
            W.Request(4, 0.0, 20, 10, "c64", 5)]
    be = FakeBackend(budget=1 << 34)
    res = {r.rid: r for r in S.serve(reqs, be)}
    assert [res[i].mode for i in range(5)] == ["batch", "batch", "batch", "stream", "stream"]


def test_admission_respects_memory_budget():
    reqs = stream(n_req=40, rate=100.0, n_min=20, n_max=26)
    budget = 3 * S.state_bytes(26, "c128")
    be = FakeBackend(budget=budget)
    S.serve(reqs, be)
    assert be.peak <= budget


def test_oversized_head_request_does_not_starve():
    """A request that cannot fit yet lets at most max_bypass later ones pass."""
    big = W.Request(0, 0.0, 27, 10, "c128", 1)
    smalls = [W.Request(i, 0.001 * i, 22, 10, "c128", 10 + i) for i in range(1, 30)]
    budget = S.state_bytes(27, "c128") + S.state_bytes(22, "c128")
    be = FakeBackend(budget=budget)
    res = {r.rid: r for r in S.serve([big] + smalls, be, max_bypass=3)}
    later = sorted(r.start for r in res.values() if r.rid != 0)
    assert res[0].start <= later[4]


def test_small_requests_pass_a_head_waiting_for_a_stream():
    """A large head request that waits only for a stream does not hold back
    small circuits behind it (they take no stream and little memory), and
    they are not counted as bypasses of the head."""
    big = [W.Request(0, 0.0, 28, 60, "c128", 1), W.Request(1, 0.001, 28, 60, "c128", 2)]
    small = [W.Request(2, 0.020, 10, 10, "c128", 3), W.Request(3, 0.030, 10, 10, "c64", 4)]
    be = FakeBackend(budget=1 << 36)
    res = {r.rid: r for r in S.serve(big + small, be, max_streams=1, max_bypass=0)}
    assert be.service(big[0]) > 0.04            # the second large request waits for the stream
    assert res[1].start >= res[0].done - 1e-9
    for rid in (2, 3):
        assert res[rid].start - res[rid].arrival < 1e-3, (rid, res[rid].start, res[rid].arrival)
        assert res[rid].mode == "batch"


def test_bypass_count_limits_competing_requests_only():
    """With max_bypass = 1, one large request may take a stream past a head
    that waits for memory; the next large one waits behind the head."""
    head = W.Request(0, 0.001, 27, 10, "c128", 1)
    first = W.Request(9, 0.0, 26, 60, "c128", 9)       # holds memory while the head arrives
    later = [W.Request(i, 0.002 + 0.0001 * i, 20, 10, "c128", 10 + i) for i in range(1, 4)]
    budget = S.reserve_bytes(27, "c128") + S.reserve_bytes(20, "c128") + S.reserve_bytes(26, "c128") // 2
    be = FakeBackend(budget=budget)
    res = {r.rid: r for r in S.serve([first, head] + later, be, max_bypass=1)}
    passed = [rid for rid in (1, 2, 3) if res[rid].start < res[0].start]
    assert len(passed) == 1, (passed, {k: (v.start, v.done) for k, v in res.items()})


def test_admission_counts_context_buffers():
    """A context that holds buffers beside its state is charged for them."""
    class Held(FakeBackend):
        def held_bytes(self, req):
            return 1 << 30
    reqs = [W.Request(i, 0.0, 26, 10, "c128", i) for i in range(4)]
    budget = 2 * S.state_bytes(26, "c128") + (1 << 30)   # two reserves fit, not two contexts
    be = Held(budget=budget)
    res = S.serve(reqs, be)
    starts = sorted(r.start for r in res)
    # the second request cannot be admitted beside the first: 2 states + 2 GiB of buffers exceed the budget
    assert starts[1] > starts[0]


def test_served_beats_sequential_plain_on_fake_costs():
    reqs = stream(n_req=60, rate=2.0, n_min=12, n_max=24)
    served = S.summarize(S.serve(reqs, FakeBackend(budget=1 << 36)))
    plain = S.summarize(S.serve_sequential_plain(reqs, FakeBackend(budget=1 << 36)))
    assert served["p99_latency_s"] < plain["p99_latency_s"]
    assert served["gate_apps_per_s"] > plain["gate_apps_per_s"]


def test_summary_fields():
    res = [S.Result(0, 10, "c128", 100, 0.0, 0.1, 1.0), S.Result(1, 12, "c64", 200, 0.5, 0.6, 2.0)]
    s = S.summarize(res)
    assert s["requests"] == 2
    assert s["p50_latency_s"] == pytest.approx(np.percentile([1.0, 1.5], 50))
    assert s["gate_apps_per_s"] == pytest.approx(300 / 2.0)
