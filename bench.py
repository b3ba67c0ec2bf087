#!/usr/bin/env python3
"""Benchmark of the full-state simulation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = plan the circuit on the host (booster, diagonal detector, stages,
fusion) and execute it on the GPU from |0...0> to the final state, for the
30-qubit random layered circuit (40 layers, 2,680 gates, complex128).  The
state (16 GiB) stays resident in HBM.  Prints one JSON line:

* value: input gates applied per second over the timed steps (gate-apps/s);
* roofline: the dominant kernel's achieved rate against the MI355X peak that
  bounds it, from HIP events around its launches inside the timed steps;
* cpu_baseline: the CPU oracle (one gate per full pass, complex128) timed on a
  bounded prefix of the same circuit at the same size on the host cores;
* precision: complex64 (and the forced 5-qubit fused-GEMM form on FP32 MFMA)
  against the complex128 GPU path at 28 and 32 qubits, time and infidelity;
* serving: a shortened Poisson request stream through the continuous-batching
  server and through sequential plain solves, p50/p99 latency and gate-apps/s;
* offload: the same 30-qubit circuit with its state in host memory and two
  4 GiB device windows, gate-apps/s and host-link GB/s.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_workload(name, dtype, opt, steps, warmup, profile=True):
    import torch
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import workloads as W
    n, gates = W.config_circuit(name)
    n_gates = len(gates)
    gates = qsim.Circuit(gates)  # marshalled once; every step still validates and plans it
    sim = qsim.Simulator(n, dtype=dtype, opt=opt)
    sim.set_profiling(profile)
    for i in range(warmup):
        sim.load(gates)
        sim.run()
        log(f"[bench] {name} warmup {i + 1}/{warmup}: {sim.stats()['run_ms']:.1f} ms")
    per_kind = {}
    plan_ms = run_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        sim.load(gates)
        sim.run()
        st = sim.stats()
        plan_ms += st["plan_ms"]
        run_ms += st["run_ms"]
        if profile:
            for t in sim.op_timings():
                if t["buffer"] != 0:
                    continue
                d = per_kind.setdefault(t["kind"], {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
                d["ms"] += t["ms"]
                d["launches"] += 1
                d["flops"] += t["flops"]
                d["bytes"] += t["bytes"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    norm = sim.norm()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"n": n, "gates": n_gates, "wall_s": t1 - t0, "plan_ms": plan_ms / steps, "run_ms": run_ms / steps,
            "per_kind": per_kind, "stats": st, "norm": norm}


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch of the kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a copy kernel of known size),
    only while the kernel source is the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{dtype}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2604_12256_amd", "csrc", "kernel_stage.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("source_sha256"):
            return None
    return round(rec["traffic_bytes_per_launch"])


def roofline(per_kind, dtype, steps, workload=None):
    kind = max(per_kind, key=lambda k: per_kind[k]["ms"])
    d = per_kind[kind]
    avg_s = d["ms"] / d["launches"] / 1e3
    flops = d["flops"] / d["launches"]
    byts = d["bytes"] / d["launches"]
    peak_fl = FP64_PEAK_TFLOPS if dtype == "c128" else FP32_PEAK_TFLOPS
    intensity = flops / byts if byts else float("inf")
    ridge = peak_fl * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity > ridge:
        ach = flops / avg_s / 1e12
        r = {"bound": "alu", "achieved": round(ach, 3), "peak": peak_fl, "unit": "TFLOP/s",
             "frac": round(ach / peak_fl, 4)}
    else:
        ach = byts / avg_s / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
    r.update({"kernel": {"STAGE": "k_stage", "DENSE": "k_dense", "DIAG": "k_diag", "KRON": "k_kron",
                         "INIT": "k_init"}.get(kind, kind),
              "avg_launch_ms": round(avg_s * 1e3, 4), "launches_per_step": d["launches"] // steps,
              "flops_per_launch": flops, "bytes_per_launch": byts,
              "hbm_GBps_of_kernel": round(byts / avg_s / 1e9, 1),
              "traffic": measured_traffic("k_stage", workload, dtype) if kind == "STAGE" and workload else None})
    return r


def copy_reference(gib=16, reps=3):
    """Achievable HBM bandwidth: the library's plain copy kernel (K11) on
    `gib` GiB, read + write bytes / time."""
    import torch
    from paper_2604_12256_amd import qsim
    a = torch.zeros(gib << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        qsim.device_copy(b, a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * a.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return round(best, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, n_prefix=100, n_one_thread=4):
    """The oracle (plain one-gate-per-pass complex128 simulator, OpenMP over
    the host cores) on a bounded prefix of the same circuit at full size.
    Only the gate loop is timed: the |0...0> state is allocated and set
    before the clock starts.  A second figure runs the next few gates on one
    thread."""
    import numpy as np
    from oracle import oracle
    from paper_2604_12256_amd import workloads as W
    oracle.build(force=False)
    n, gates = W.config_circuit(name)
    state = np.zeros(1 << n, dtype=np.complex128)
    state[0] = 1.0
    sample = gates[:n_prefix]
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.apply_inplace(n, sample, state)
    dt = time.perf_counter() - t0
    one = gates[n_prefix:n_prefix + n_one_thread]
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.apply_inplace(n, one, state)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    del state
    return {"value": round(len(sample) / dt, 4), "unit": "gate-apps/s", "cores": threads, "kind": "oracle",
            "sample": f"gates 1..{len(sample)} of {name} ({n} qubits, full 2^{n} complex128 state, one pass per "
                      f"gate), gate loop only ({dt:.1f} s); |0...0> set up outside the timed region",
            "cpu": cpu_model(),
            "one_thread": {"value": round(len(one) / dt1, 4), "unit": "gate-apps/s", "cores": 1,
                           "sample": f"gates {n_prefix + 1}..{n_prefix + len(one)} of {name}, one thread "
                                     f"({dt1:.1f} s)"}}


def precision_leg():
    """The precision form: complex64 storage (FP32 arithmetic; 5-qubit fused
    gates as batched 32x32 complex GEMMs on FP32 MFMA in the forced-fusion
    form) against the complex128 GPU path, on the 28- and 32-qubit layered
    circuits.  Infidelity 1 - |<a|b>|^2 / (<a|a><b|b>) in FP64 on the device;
    times are validate + plan + run (second of two runs)."""
    import torch
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import workloads as W

    def timed(sim, circ):
        sim.load(circ)
        sim.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.load(circ)
        sim.run()
        return (time.perf_counter() - t0) * 1e3

    rows = []
    for name in ("layered28", "layered32"):
        n, gates = W.config_circuit(name)
        circ = qsim.Circuit(gates)
        log(f"[bench] precision {name}")
        ref = qsim.Simulator(n, dtype="c128", opt=qsim.OPT_ALL)
        t_ref = timed(ref, circ)
        row = {"workload": f"{name}: {n}-qubit random layered circuit, {len(gates)} gates",
               "c128_all_passes_ms": round(t_ref, 2)}
        for key, kw in (("c64_all_passes", dict(opt=qsim.OPT_ALL)),
                        ("c64_fused_k5_fp32_mfma", dict(opt=qsim.OPT_FUSE, force_fuse_k=5))):
            low = qsim.Simulator(n, dtype="c64", **kw)
            t = timed(low, circ)
            ip = ref.inner(low)
            inf = 1.0 - abs(ip) ** 2 / (ref.norm() * low.norm())
            row[key] = {"ms": round(t, 2), "infidelity": float(f"{inf:.3e}"),
                        "full_passes": low.stats()["full_passes"]}
            low.close()
            del low
            torch.cuda.empty_cache()
        if name == "layered28":
            plain = qsim.Simulator(n, dtype="c128", opt=0, state=ref.state)
            plain.load(circ)
            t0 = time.perf_counter()
            plain.run()
            row["c128_plain_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
            plain.close()
        ref.close()
        del ref
        torch.cuda.empty_cache()
        rows.append(row)
    return rows


def offload_leg(window=28):
    """Host-memory offload on the 30-qubit layered circuit: the 16 GiB
    complex128 state in pinned host memory, two device windows of 2^window
    amplitudes; one warm-up run, then one timed run (plan + run)."""
    import torch
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import workloads as W
    n, gates = W.config_circuit("layered30")
    circ = qsim.Circuit(gates)
    log(f"[bench] offload layered30, windows of 2^{window}")
    sim = qsim.Simulator(n, dtype="c128", opt=qsim.OPT_ALL, offload_window=window)
    sim.load(circ)
    sim.run()
    log("[bench] offload warm-up done")
    t0 = time.perf_counter()
    sim.load(circ)
    sim.run()
    dt = time.perf_counter() - t0
    st = sim.stats()
    norm = sim.norm()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"workload": f"layered30 complex128 (16 GiB state in pinned host memory), two device windows of "
                        f"2^{window} amplitudes ({2 * 16 * 2 ** window / 2 ** 30:.0f} GiB of device memory)",
            "gate_apps_per_s": round(len(gates) / dt, 1), "ms_per_step": round(dt * 1e3, 1),
            "run_ms": round(st["run_ms"], 1), "offload_passes": st["offload_passes"],
            "device_passes": st["full_passes"],
            "host_link_GBps": round(st["pcie_bytes"] / (st["run_ms"] / 1e3) / 1e9, 1),
            "norm_error": abs(norm - 1.0)}


def serving_leg(n_requests=40, rate=0.8, seed=5):
    """A shortened serving stream: Poisson arrivals of random layered
    circuits (10..30 qubits, 10..60 layers, half complex128 and half
    complex64), through the continuous-batching server and through
    sequential plain (gate-by-gate, one request at a time) on the same GPU."""
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import serve as S
    from paper_2604_12256_amd import workloads as W
    reqs = W.serving_stream(n_requests, rate, seed, 10, 30)

    def progress(tag):
        def f(done, total):
            log(f"[bench] serving {tag}: {done}/{total}")
        return f
    served = S.summarize(S.serve(reqs, S.GpuBackend(qsim.OPT_ALL, n_streams=4), max_streams=4,
                                 progress=progress("served")))
    plain = S.summarize(S.serve_sequential_plain(reqs, S.GpuBackend(0), progress=progress("plain")))
    keep = ("p50_latency_s", "p99_latency_s", "mean_latency_s", "makespan_s", "gate_apps_per_s", "batched")
    return {"stream": f"{n_requests} requests, Poisson rate {rate}/s, seed {seed}, 10..30 qubits, 10..60 layers, "
                      f"half complex128",
            "served": {k: round(served[k], 4) if isinstance(served[k], float) else served[k] for k in keep},
            "sequential_plain": {k: round(plain[k], 4) if isinstance(plain[k], float) else plain[k] for k in keep},
            "mid_size_batch": mid_size_batch()}


def mid_size_batch(count=48, n=16, layers=20, seed=60):
    """Device time of `count` planned 16-qubit layered circuits (complex128):
    one after the other on one stream (sim_run_async each) against one
    staged batch (sim_run_batch: their full-state stages in shared launches).
    Plans are built before the clock starts; best of three."""
    import torch
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import workloads as W
    stream = torch.cuda.Stream()
    sims = []
    for i in range(count):
        sim = qsim.Simulator(n, opt=qsim.OPT_ALL, stream=stream)
        sim.load(W.layered(n, layers, seed + i))
        sims.append(sim)

    def timed(fn):
        best = 1e9
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            stream.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    def solo():
        for sim in sims:
            sim.run_async()

    solo_ms = timed(solo)
    batch_ms = timed(lambda: qsim.run_batch(sims, stream=stream))
    stages = sims[0].stats()["n_stages"]
    for sim in sims:
        sim.close()
    gates = count * W.layered_gate_count(n, layers)
    return {"circuits": count, "qubits": n, "layers": layers, "dtype": "c128", "stages_each": stages,
            "one_by_one_ms": round(solo_ms, 3), "staged_batch_ms": round(batch_ms, 3),
            "one_by_one_gate_apps_per_s": round(gates / solo_ms * 1e3, 1),
            "staged_batch_gate_apps_per_s": round(gates / batch_ms * 1e3, 1)}


def kernel_table(n=30):
    """Per-kernel device time and HBM rate at `n` qubits (both dtypes), each
    kernel driven through the C ABI: full-pass dense gates on the VALU
    (k = 1..3) and on MFMA (k = 4, 5), full-pass diagonals, the tensor
    product of the merge booster, |0...0>, the output reductions (marginal,
    inner product, amplitude gather), measurement (sampling, Z strings,
    collapse) and the batched small-state kernel.
    Rates are algorithmic bytes (one read and one write of the state for a
    pass) over the measured time."""
    import numpy as np
    import torch
    from paper_2604_12256_amd import qsim
    from paper_2604_12256_amd import workloads as W
    from paper_2604_12256_amd.workloads import Gate
    rng = np.random.default_rng(11)
    rows = []

    def events(fn, reps=3):
        best = 1e9
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    for dtype in ("c128", "c64"):
        b = 16 if dtype == "c128" else 8
        state_bytes = b << n
        a = torch.empty((2 if dtype == "c128" else 1) << n, dtype=torch.float64, device="cuda")
        other = torch.empty_like(a)

        def op_ms(gates, opt, kind):
            sim = qsim.Simulator(n, dtype=dtype, opt=opt, state=a)
            sim.set_profiling(True)
            sim.load(gates)
            best = 1e9
            for _ in range(3):
                sim.run()
                best = min(best, sum(t["ms"] for t in sim.op_timings() if t["kind"] == kind and t["buffer"] == 0))
            sim.close()
            return best

        def add(kernel, what, ms, nbytes):
            rows.append({"dtype": dtype, "kernel": kernel, "op": what, "ms": round(ms, 3),
                         "GBps": round(nbytes / ms / 1e6, 1), "hbm_frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 3)})
            log(f"[kernels] {dtype} {kernel} {what}: {ms:.3f} ms")

        add("k_init", "|0...0>", op_ms([], 0, "INIT"), state_bytes)
        for k in (1, 2, 3):
            g = [Gate("U", tuple(range(7, 7 + k)), data=W.haar_unitary(rng, 1 << k))]
            kern = "k_dense_mfma" if (k == 3 and dtype == "c64") else "k_dense"   # FP32 MFMA from k = 3
            add(kern, f"dense k={k} (qubits 7..)", op_ms(g, 0, "DENSE"), 2 * state_bytes)
        for k in (4, 5):
            g = [Gate("U", tuple(range(7, 7 + k)), data=W.haar_unitary(rng, 1 << k))]
            add("k_dense_mfma", f"dense k={k} (qubits 7..)", op_ms(g, 0, "DENSE"), 2 * state_bytes)
        for k in (1, 6):
            g = [Gate("DIAG", tuple(range(20, 20 + k)), data=np.exp(1j * rng.uniform(0, 6.3, 1 << k)))]
            add("k_diag", f"diagonal k={k} (qubits 20..)", op_ms(g, 0, "DIAG"), 2 * state_bytes)
        add("k_kron", "tensor product of two 15-qubit sub-states",
            op_ms(W.product_circuit(n, 2, 5), qsim.OPT_BOOST | qsim.OPT_STAGES, "KRON"), state_bytes)
        sim = qsim.Simulator(n, dtype=dtype, opt=0, state=a)
        sim.load([Gate("H", (q,)) for q in range(3)])
        sim.run()
        add("k_marg_partial_lanes", "marginal over qubits 0..9",
            events(lambda: sim.probabilities(list(range(10)))), state_bytes)
        add("k_marg_partial", "marginal over qubits 20..29",
            events(lambda: sim.probabilities(list(range(20, 30)))), state_bytes)
        sim2 = qsim.Simulator(n, dtype=dtype, opt=0, state=other)
        sim2.load([Gate("H", (q,)) for q in range(2)])
        sim2.run()
        add("k_inner_*", "inner product of two states", events(lambda: sim.inner(sim2)), 2 * state_bytes)
        idx = np.sort(rng.choice(1 << n, 1 << 20, replace=False)).astype(np.uint64)
        add("k_gather", "2^20 sampled amplitudes incl. host index upload and copy-out",
            events(lambda: sim.amplitudes(idx)), (1 << 20) * b)
        sim2.close()
        # measurement on the uniform state (every block of the sampler is hit)
        sim.load([Gate("H", (q,)) for q in range(n)])
        sim.run()
        u = rng.random(100000)
        add("k_marg + k_sample", "10^5 shots, uniform state, incl. host sort and copies",
            events(lambda: sim.sample(u)), 2 * state_bytes)
        masks = [int(x) for x in rng.integers(0, 1 << n, 16)]
        add("k_expect_z_*", "16 Z strings, one pass", events(lambda: sim.expect_z(masks)), state_bytes)
        add("k_marg + k_collapse", "measure one qubit (marginal, then collapse in place)",
            events(lambda: sim.measure(5, 0.3), reps=1), 3 * state_bytes)
        sim.close()
        del a, other
        torch.cuda.empty_cache()
        # batched small circuits: 128 circuits of 12 qubits, 20 layers each
        sims = []
        for i in range(128):
            s_ = qsim.Simulator(12, dtype=dtype, opt=qsim.OPT_ALL)
            s_.load(W.layered(12, 20, seed=100 + i))
            sims.append(s_)
        ms = events(lambda: qsim.run_batch(sims))
        rows.append({"dtype": dtype, "kernel": "k_small_ptrs", "op": "128 circuits x 12 qubits x 540 gates, one launch",
                     "ms": round(ms, 3), "gate_apps_per_s": round(128 * 540 / (ms / 1e3), 1)})
        log(f"[kernels] {dtype} k_small_ptrs: {ms:.3f} ms")
        for s_ in sims:
            s_.close()
    return rows


# The benchmark circuits of Sec. 5 on one GPU, with the paper's own figure
# for the same circuit family and size (NVIDIA H100, complex128) as context.
PAPER_BENCHMARKS = (
    ("qaoa30", "30-qubit 5-level fully-connected QAOA (H, then per level RZZ on all 435 pairs and RX on "
               "every qubit), 2355 gates",
     {"paper_s": 0.99, "paper": "Table 3, all optimisations, one H100"}),
    ("qaoa31", "31-qubit 5-level fully-connected QAOA (RZZ on all 465 pairs and RX on every qubit per level), "
               "2511 gates",
     {"paper_ms_per_gate": 2.35, "paper": "Table 2, QAOA with the booster, one H100, per gate"}),
    ("qft31", "31-qubit QFT of a seeded basis state (X prep, H + 465 controlled phases, 15 closing SWAPs)",
     {"paper_ms_per_gate": 1.26, "paper": "Table 2, QFT with the booster, one H100, per gate"}),
    ("rzz30", "30-qubit H layer + RZZ on all 435 pairs (gate-level benchmark)",
     {"paper_s": 0.02, "paper": "Table 1, all optimisations, 64 H100s (context only)"}),
    ("rzz33", "33-qubit H layer + RZZ on all 528 pairs, a 128 GiB state",
     {"paper_s": 0.04, "paper": "Table 1, all optimisations, 64 H100s (context only)"}),
    ("rzz34", "34-qubit H layer + RZZ on all 561 pairs, a 256 GiB state",
     {"paper_s": 0.07, "paper": "Table 1, all optimisations, 64 H100s (context only)"}),
)


def describe(name, r, dtype):
    passes = ("|0...0> init, all optimiser passes (booster, diagonal detector, cache-blocked stages, fusion, "
              "qubit relabelling)")
    if name.startswith("layered"):
        return (f"{name}: {r['n']}-qubit random layered circuit (Haar U(2) on every qubit, CZ on floor(n/4) random "
                f"disjoint pairs, RZ on every qubit), {r['gates']} gates, {dtype}, {passes}")
    for key, what, _ in PAPER_BENCHMARKS:
        if key == name:
            return f"{name}: {what}, {dtype}, {passes}"
    return f"{name}: {r['n']} qubits, {r['gates']} gates, {dtype}, {passes}"


def paper_benchmarks(steps=3, warmup=1):
    from paper_2604_12256_amd import qsim
    rows = []
    import torch
    for name, what, ref in PAPER_BENCHMARKS:
        n = int(name[-2:])
        free, _ = torch.cuda.mem_get_info()
        if free < (16 << n) + (4 << 30):
            log(f"[bench] {name}: skipped, {free / 2**30:.0f} GiB free")
            continue
        log(f"[bench] {name}")
        try:
            d = run_workload(name, "c128", qsim.OPT_ALL, steps, warmup, profile=False)
        except (torch.cuda.OutOfMemoryError, qsim.QsimError) as e:  # a state that does not fit this device
            log(f"[bench] {name}: skipped ({type(e).__name__}: {str(e)[:120]})")
            torch.cuda.empty_cache()
            continue
        ms = d["wall_s"] / steps * 1e3
        hb = d["stats"]["algorithmic_bytes"] / (d["run_ms"] / 1e3) / 1e9
        row = {"workload": f"{name}: {what}, complex128, all passes", "ms_per_step": round(ms, 3),
               "gate_apps_per_s": round(d["gates"] / (ms / 1e3), 1), "ms_per_gate": round(ms / d["gates"], 5),
               "plan_ms": round(d["plan_ms"], 3), "run_ms": round(d["run_ms"], 3),
               "full_passes": d["stats"]["full_passes"], "hbm_GBps": round(hb, 1),
               "norm_error": abs(d["norm"] - 1.0)}
        row.update(ref)
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered30")
    ap.add_argument("--dtype", default="c128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-prefix", type=int, default=100)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-offload", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--kernels", action="store_true",
                    help="print a per-kernel time / HBM-rate table at 30 qubits instead of the benchmark line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this simulator runs on one GPU only (the state vector is not sharded across "
              "GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    from paper_2604_12256_amd import qsim
    if args.kernels:
        print(json.dumps({"kernels": kernel_table()}), flush=True)
        return
    log(f"[bench] workload {args.workload} {args.dtype} steps={args.steps} warmup={args.warmup}")
    r = run_workload(args.workload, args.dtype, qsim.OPT_ALL, args.steps, args.warmup)
    ms_per_step = r["wall_s"] / args.steps * 1e3
    value = r["gates"] / (ms_per_step / 1e3)
    st = r["stats"]
    hbm = st["algorithmic_bytes"] / (r["run_ms"] / 1e3) / 1e9
    out = {
        "metric": "gate-apps/s + HBM GB/s (% peak) at 30q; served p50/p99 latency vs plain",
        "value": round(value, 2),
        "unit": "gate-apps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": describe(args.workload, r, args.dtype),
                   "qubits": r["n"], "gates": r["gates"], "state_GiB": (16 if args.dtype == 'c128' else 8) *
                   2 ** r["n"] / 2 ** 30},
        "plan_ms": round(r["plan_ms"], 3),
        "run_ms": round(r["run_ms"], 3),
        "hbm_GBps": round(hbm, 1),
        "hbm_frac": round(hbm / HBM_PEAK_GBS, 4),
        "full_passes": st["full_passes"],
        "stages": st["n_stages"],
        "plan_flops": st["flops"],
        "norm_error": abs(r["norm"] - 1.0),
        "roofline": roofline(r["per_kind"], args.dtype, args.steps, args.workload),
        "per_kind_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in r["per_kind"].items()},
    }
    out["hbm_copy_GBps"] = copy_reference()
    if not args.no_secondary:
        d = run_workload("diag30", "c128", qsim.OPT_ALL, 3, 1)
        ms = d["wall_s"] / 3 * 1e3
        dh = d["stats"]["algorithmic_bytes"] / (d["run_ms"] / 1e3) / 1e9
        out["secondary"] = {"workload": "diag30: 30-qubit diagonal-heavy circuit, 200 gates (160 diagonal), "
                                        "complex128, all passes",
                            "gate_apps_per_s": round(d["gates"] / (ms / 1e3), 2), "ms_per_step": round(ms, 3),
                            "hbm_GBps": round(dh, 1), "hbm_frac": round(dh / HBM_PEAK_GBS, 4),
                            "full_passes": d["stats"]["full_passes"],
                            "roofline": roofline(d["per_kind"], "c128", 3, "diag30")}
        out["paper_benchmarks"] = paper_benchmarks()
    if not args.no_precision:
        out["precision"] = precision_leg()
    if not args.no_serving:
        out["serving"] = serving_leg()
    if not args.no_offload:
        out["offload"] = offload_leg()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_prefix)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
