#!/usr/bin/env python3
"""Benchmark of the single-graph blocked Floyd–Warshall solve on one MI355X.

Workload: one directed graph, n = 32768 (a 4 GiB int32 matrix), edge
probability 0.1, integer weights b + pi(i) - pi(j) with b uniform in
[1, 1000] and pi(v) = floor(100 v / (n-1)) (negative weights only on i<j
edges, no negative cycles), distances only.  A step is one complete solve
(every round, all three phases, the wrap-up pass) preceded by a
device-to-device restore of the input from a pristine copy; inputs are
resident in HBM before the timed region starts.

Metric: min-plus GOPS = 2 n^3 / t (one add and one min per (i, j, k)).
One JSON line is printed (see the fields below); ``--gpus`` above 1 is
refused: the benchmark measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published float32 vector peak: 157.3 TFLOP/s = 256 CUs x 2.4 GHz x
# 256 flops per CU-cycle (an FMA counts 2 flops).  A min-plus relaxation
# (one add, one min) counts 2 ops the same way, so 157.3 T ops/s is the
# published ALU peak this path is reported against.  The instruction-set
# ceiling of the actual float32 min-plus step (2 v_add_f32 + 1 v_min3_f32 per
# two relaxations; no fused add-min exists) is measured on the device by the
# library's steady-state VALU probes and reported beside it.
PEAK_F32_VECTOR = 157.3e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, budget_s: float, c1_W=None, batch=None):
    """The oracle on the host, built here with gcc -O3 -march=native (OpenMP
    over rows): (a) the headline input, first K iterations of k over the full
    matrix (a bounded sample of the same solve), K grown until the budget is
    spent, with all host threads and with one, reported as 2 n^2 K / t;
    (b) the n=1024 workload solved whole, one thread and all threads;
    (c) every graph of the 4096-graph batch, one graph per thread."""
    import tempfile

    import numpy as np

    import oracle  # test infrastructure: only this leg of the benchmark uses it

    tmp = tempfile.mkdtemp(prefix="apsp_oracle_")
    orc = oracle.Oracle(oracle.load(oracle.build_native(tmp)))
    n = W.shape[0]
    threads = oracle.default_threads()

    def sample(nthreads, budget):
        D = W.copy()
        k = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget and k < n:
            orc.fw_steps(D, k, k + 1, threads=nthreads)
            k += 1
        t = time.perf_counter() - t0
        return k, t

    k_all, t_all = sample(threads, budget_s)
    k_one, t_one = sample(1, budget_s / 3.0)
    out = {
        "value": round(2.0 * n * n * k_all / t_all / 1e9, 3),
        "unit": "GOPS",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {k_all} of {n} k-iterations of the oracle's plain triple loop on the same "
                  f"n={n} int32 input ({t_all:.1f} s, {threads} threads)",
        "build": "gcc -O3 -march=native -fopenmp (the oracle source, built on this host)",
        "cpu_model": cpu_model(),
        "nproc": os.cpu_count(),
        "affinity_cpus": len(os.sched_getaffinity(0)),
        "one_thread": {"value": round(2.0 * n * n * k_one / t_one / 1e9, 3), "unit": "GOPS",
                       "sample": f"first {k_one} k-iterations ({t_one:.1f} s)"},
    }
    if c1_W is not None:
        m = c1_W.shape[0]
        res = {}
        for label, nt in (("one_thread", 1), ("all_threads", threads)):
            t0 = time.perf_counter()
            orc.fw(c1_W, threads=nt)
            t = time.perf_counter() - t0
            res[label] = {"ms": round(t * 1e3, 2), "gops": round(2.0 * m ** 3 / t / 1e9, 2)}
        out["c1_n1024_full"] = res
    if batch is not None:
        graphs = [batch.graph(b) for b in range(len(batch.ns))]
        ops = float((2.0 * batch.ns.astype(np.float64) ** 3).sum())
        t0 = time.perf_counter()
        orc.fw_many(graphs, workers=threads)
        t = time.perf_counter() - t0
        out["batched_4096_graphs"] = {"s": round(t, 2), "solves_per_s": round(len(graphs) / t, 1),
                                      "gops": round(ops / t / 1e9, 2), "threads": threads,
                                      "mode": "one graph per thread"}
    return out


def sweep_leg(sizes, modes):
    """The paper's size sweep (Section "Experimental Design": powers of two
    from 4096 to 65536) on one GPU: float32 with the path matrix (the paper's
    own configuration) and int32 distances.  Weights are integers 1..1000,
    edge probability 0.3, synthetic.  One warm-up solve, then timed solves
    (HIP events on the current stream)."""
    import torch

    import paper_1811_01201_amd as apsp
    import synth

    rows = []
    for n in sizes:
        for mode in modes:
            log(f"[sweep] n={n} {mode}: generating")
            if mode == "f32pred":
                W = synth.single_f32int(n, p=0.3, seed=synth.BASE_SEED + 10)
            else:
                W = synth.single_int32(n, p=0.3, seed=synth.BASE_SEED + 10)
            pristine = torch.from_numpy(W).cuda()
            del W
            work = torch.empty_like(pristine)
            pred = torch.empty(pristine.shape, dtype=torch.int32, device="cuda") if mode == "f32pred" else None
            used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            reps = 1 if n >= 32768 else 3
            times = []
            for r in range(reps + 1):
                work.copy_(pristine)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                apsp.solve(work, pred, arith_used=used)
                e1.record()
                torch.cuda.synchronize()
                log(f"[sweep] n={n} {mode}: solve {r} {e0.elapsed_time(e1):.1f} ms")
                if r > 0:
                    times.append(e0.elapsed_time(e1))
            t = min(times)
            rows.append({"n": n, "mode": mode, "ms": round(t, 3), "gops": round(2.0 * n ** 3 / (t / 1e3) / 1e9, 1),
                         "arithmetic": (("float32 distances + key product (exact)" if int(used.item()) == 1
                                         else "fp64 keys") if mode == "f32pred" else
                                        "float32 (exact)" if int(used.item()) == 1 else "int32")})
            del pristine, work, pred
            torch.cuda.empty_cache()
    return rows


def batched_leg(replays: int, graph_replays: bool = True):
    """4096 graphs (n uniform in [16, 512], p uniform in [0.05, 0.9], int32
    weights 1..1000) in the plan's fused launches per replay, against the same graphs
    solved one apsp_solve launch sequence per graph on one stream."""
    import numpy as np
    import torch

    import paper_1811_01201_amd as apsp
    import synth

    bt = synth.batch()
    pristine = torch.from_numpy(bt.pack_int32()).cuda()
    d = torch.empty_like(pristine)
    plan = apsp.BatchPlan(bt.ns, bt.offsets, "int32")
    ops = float((2.0 * bt.ns.astype(np.float64) ** 3).sum())
    status = torch.full((len(bt.ns),), -1, dtype=torch.int32, device="cuda")
    times = []
    for r in range(replays + 1):
        d.copy_(pristine)
        status.fill_(-1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.execute(d, status=status)
        e1.record()
        torch.cuda.synchronize()
        if not bool((status == apsp.SUCCESS).all()):
            raise RuntimeError("a batched solve reported a non-success status")
        if r > 0:
            times.append(e0.elapsed_time(e1))
    med = float(np.median(times))
    # the same launches captured once into a hipGraph and replayed
    gtimes = []
    if graph_replays:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.execute(d)
    for r in range(replays + 1 if graph_replays else 0):
        d.copy_(pristine)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            gtimes.append(e0.elapsed_time(e1))
    if graph_replays:
        del graph
    views = [d[int(o):int(o) + int(n) * int(n)].view(int(n), int(n)) for n, o in zip(bt.ns, bt.offsets)]
    d.copy_(pristine)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for v in views:
        apsp.solve(v)
    e1.record()
    torch.cuda.synchronize()
    loop_ms = e0.elapsed_time(e1)
    plan.destroy()
    return {
        "workload": "4096 graphs, n uniform int [16,512], edge prob uniform [0.05,0.9], int32 w in [1,1000], "
                    "packed ragged, fused launches (int32-arithmetic graphs, then float32-arithmetic graphs)",
        "solves_per_s": round(4096 / (med / 1e3), 1),
        "batch_ms_median": round(med, 3),
        "batch_ms_p99": round(float(np.percentile(times, 99)), 3),
        "replays": replays,
        "gops": round(ops / (med / 1e3) / 1e9, 1),
        "hipgraph_replay": {"batch_ms_median": round(float(np.median(gtimes)), 3),
                            "batch_ms_p99": round(float(np.percentile(gtimes, 99)), 3)} if gtimes else None,
        "one_graph_per_launch": {"solves_per_s": round(4096 / (loop_ms / 1e3), 1), "batch_ms": round(loop_ms, 3)},
        "speedup_vs_one_graph_per_launch": round(loop_ms / med, 2),
    }


def serving_leg(count: int, rate_fractions=(0.25, 0.5, 0.75, 0.9, 1.1), per_rate_s: float = 6.0):
    """Poisson request streams (n log-uniform in [32, 8192], int32 / float32
    integer weights 1..1000 half each, p=0.2, predecessors for 30%) through
    the continuous-batching server and a FIFO one-request-at-a-time server:
    both saturated (all requests submitted at once), then both at the same
    offered rates, fractions of the continuous-batching saturated rate
    (about per_rate_s seconds of requests each)."""
    import threading

    import torch

    import paper_1811_01201_amd as apsp
    import synth

    nmax = 8192
    base = {"int32": torch.from_numpy(synth.single_int32(nmax, 0.2, seed=synth.BASE_SEED + 4)).pin_memory(),
            "float32": torch.from_numpy(synth.single_f32int(nmax, 0.2, seed=synth.BASE_SEED + 4)).pin_memory()}

    def run(rate, n_req, fifo=False, slice_rounds=0):
        reqs = synth.requests(n_req, rate if rate else 1e9)
        kw = dict(max_inflight=1, batch_max_n=-1) if fifo else dict(max_inflight=64, n_streams=8,
                                                                      slice_rounds=slice_rounds)
        sv = apsp.Server(**kw)
        tickets = []
        done = threading.Event()
        errors = []

        def drain():
            i = 0
            while True:
                while i >= len(tickets):
                    if done.is_set():
                        return
                    time.sleep(0.0002)
                st = sv.wait(tickets[i])
                if st != apsp.SUCCESS:
                    errors.append(st)
                sv.release(tickets[i])
                i += 1

        th = threading.Thread(target=drain)
        th.start()
        t0 = time.perf_counter()
        for r in reqs:
            if rate:
                now = time.perf_counter() - t0
                if r.arrival_s > now:
                    time.sleep(r.arrival_s - now)
            # a request's graph is the leading n x n block of a pinned base matrix
            # (a principal submatrix of a p=0.2 random graph is one too)
            tickets.append(sv.submit(base[r.dtype], n=r.n, want_pred=r.want_pred, borrow=True))
        done.set()
        th.join()
        s = sv.stats()
        sv.destroy()
        if errors:
            raise RuntimeError(f"serving requests failed: {errors[:5]}")
        out = {"offered_rate": round(rate, 1) if rate else "saturated", "requests": n_req,
               "solves_per_s": round(s["solves_per_s"], 1), "p50_ms": round(s["p50_latency_ms"], 3),
               "p99_ms": round(s["p99_latency_ms"], 3)}
        if not fifo:  # coalesced (n <= 512) and large requests separately
            out.update({"small_p50_ms": round(s["p50_small_ms"], 3), "small_p99_ms": round(s["p99_small_ms"], 3),
                        "large_p50_ms": round(s["p50_large_ms"], 3), "large_p99_ms": round(s["p99_large_ms"], 3)})
        if slice_rounds:
            out["slice_rounds"] = slice_rounds
        return out

    sat = run(None, count)
    fifo_sat = run(None, count, fifo=True)
    out = {"workload": "Poisson stream, n=round(exp U[ln32,ln8192]), int32/float32 integer weights "
                       "[1,1000] half each, p=0.2, predecessors for 30%",
           "continuous_batching": [sat], "fifo_one_at_a_time": [fifo_sat],
           "saturated_speedup_vs_fifo": round(sat["solves_per_s"] / fifo_sat["solves_per_s"], 3)}
    # the same Poisson streams (rates relative to the continuous-batching
    # server's saturated rate) through both servers
    for f in rate_fractions:
        rate = f * sat["solves_per_s"]
        m = max(200, min(count, int(rate * per_rate_s)))
        log(f"[bench] serving at {f:.2f}x saturation ({rate:.0f}/s, {m} requests)")
        cb = run(rate, m)
        cb["load"] = f
        ff = run(rate, m, fifo=True)
        ff["load"] = f
        out["continuous_batching"].append(cb)
        out["fifo_one_at_a_time"].append(ff)
    # round-level preemption: large solves issued 4 rounds at a time
    out["continuous_batching_sliced"] = [run(0.9 * sat["solves_per_s"], count, slice_rounds=4)]
    return out


def paper_config_leg(steps: int):
    """The paper's own configuration: float32 weights (integers 1..1000,
    p=0.3) with the path matrix, n=8192; one warm-up and `steps` timed solves
    (HIP events, input restored by a device copy each step).  Reports the
    route that held and the predecessor key product's rate from the
    library's per-launch events."""
    import torch

    import paper_1811_01201_amd as apsp
    import synth

    n = 8192
    W = synth.single_f32int(n, p=0.3, seed=synth.BASE_SEED + 1)
    pristine = torch.from_numpy(W).cuda()
    del W
    work = torch.empty_like(pristine)
    pred = torch.empty(pristine.shape, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")

    def step():
        work.copy_(pristine)
        apsp.solve(work, pred, arith_used=used)

    step()
    torch.cuda.synchronize()
    apsp.profile_begin()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    prof = apsp.profile_end()
    t = e0.elapsed_time(e1) / 1e3 / steps
    pp = prof["pred_product"]
    out = {"workload": "single graph n=8192, float32 integer weights [1,1000], p=0.3, distances + predecessors",
           "ms_per_solve": round(t * 1e3, 3), "gops": round(2.0 * n ** 3 / t / 1e9, 1),
           "route": ("float32 distances + predecessor key product (exact)" if int(used.item()) == 1
                     else "fp64-key recurrence")}
    if pp["launches"]:
        ms = pp["total_ms"] / pp["launches"]
        rate = 2.0 * pp["updates"] / pp["launches"] / (ms / 1e3) / 1e12
        out["key_product"] = {"avg_launch_ms": round(ms, 4), "achieved": round(rate, 2), "unit": "Tops/s",
                              "frac": round(rate * 1e12 / PEAK_F32_VECTOR, 4)}
    del work, pristine, pred
    torch.cuda.empty_cache()
    return out


def device_state():
    """Clock, temperature and power right after the timed region (through
    torch's SMI bindings; None where unavailable)."""
    import torch
    out = {"name": torch.cuda.get_device_name(0)}
    for key, fn in (("clock_mhz", "clock_rate"), ("temperature_c", "temperature"), ("power_w", "power_draw")):
        try:
            out[key] = getattr(torch.cuda, fn)(0)  # ROCm builds read these through amd-smi (W, MHz, C)
        except Exception:
            out[key] = None
    return out


def isa_ceiling():
    """Steady-state VALU rates of the float32 min-plus step and of its two
    instructions alone (library probes), and the ceilings they give in
    metric ops per second (2 per relaxation)."""
    import paper_1811_01201_amd as apsp
    rates = {k: apsp.probe_valu(k)["lane_instr_per_s"] for k in ("mix_f32", "add_f32", "min3_f32")}
    # two relaxations per lane take 3 instructions of the mix, or, issued one
    # after another, 2 adds at the add rate and 1 three-input minimum at its rate
    mix = rates["mix_f32"] * 2.0 / 3.0 * 2.0
    serial = 2.0 * 2.0 / (2.0 / rates["add_f32"] + 1.0 / rates["min3_f32"])
    return {"value": round(mix / 1e12, 3), "unit": "Tops/s",
            "derivation": "measured rate of the float32 min-plus step (2 v_add_f32 + 1 v_min3_f32 per two "
                          "relaxations, every CU busy, steady state) x 2/3 relaxations per instruction x 2 ops",
            "from_single_instruction_rates": round(serial / 1e12, 3),
            "lane_instr_per_s": {k: round(v / 1e12, 3) for k, v in rates.items()},
            "lane_instr_unit": "1e12 lane-instructions/s"}, mix


def single_leg(args, n):
    """Timed single-graph solves; returns (host weights, JSON fields)."""
    import torch

    import paper_1811_01201_amd as apsp
    from paper_1811_01201_amd import profiling
    import synth

    log(f"[bench] generating n={n} potential-weight graph")
    W = synth.potential_int32(n, p=0.1, seed=synth.BASE_SEED + 2)
    pristine = torch.from_numpy(W).cuda()
    work = torch.empty_like(pristine)
    torch.cuda.synchronize()

    arith_used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    status = torch.full((max(args.steps, args.warmup, 1),), -1, dtype=torch.int32, device="cuda")

    def step(i):
        work.copy_(pristine)
        apsp.solve(work, block_size=args.block_size, arith=args.arith, arith_used=arith_used,
                   status=status[i:i + 1])

    for i in range(args.warmup):
        log(f"[bench] warmup {i + 1}/{args.warmup}")
        step(i)
    torch.cuda.synchronize()
    status.fill_(-1)

    apsp.profile_begin()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        step(i)
        log(f"[bench] step {i + 1}/{args.steps} enqueued")
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = apsp.profile_end()
    dev_state = device_state()
    st = status[:args.steps].cpu().tolist()
    if any(x != apsp.SUCCESS for x in st):
        raise RuntimeError(f"timed solves reported status {st}: the line is not a valid measurement")
    t = e0.elapsed_time(e1) / 1e3
    ms_per_step = t / args.steps * 1e3
    gops = 2.0 * n ** 3 * args.steps / t / 1e9

    # dominant kernel: the remaining-block products (kRest launches under the
    # two-stream schedule, plus the last round's full launch); rate = summed
    # algorithmic ops / summed launch durations = per-launch ops / average duration
    p3 = prof["phase3"]
    per_launch_ops = 2.0 * p3["updates"] / max(1, p3["launches"])
    avg_ms = p3["total_ms"] / max(1, p3["launches"])
    achieved = per_launch_ops / (avg_ms / 1e3) / 1e12
    ceiling, ceiling_ops = isa_ceiling()
    if achieved * 1e12 <= ceiling_ops:
        ceiling["frac"] = round(achieved * 1e12 / ceiling_ops, 4)
    else:
        ceiling["note"] = "the kernel ran faster than the probe's mix: no fraction is reported"
    roofline = {
        "bound": "alu",
        "kernel": "phase3_kernel kRest (remaining-block min-plus products, 128x128 tiles, one launch per round "
                  "beside the next round's closure and panels)",
        "achieved": round(achieved, 3),
        "peak": round(PEAK_F32_VECTOR / 1e12, 1),
        "unit": "TFLOP/s-equivalent: 2 ops per (i,j,k) relaxation (one add, one min), as an FMA counts 2 flops",
        "frac": round(achieved * 1e12 / PEAK_F32_VECTOR, 4),
        "peak_basis": "MI355X published float32 vector peak, 256 CUs x 2.4 GHz x 256 flops per CU-cycle",
        "isa_ceiling": ceiling,
        "avg_launch_ms": round(avg_ms, 4),
        "launches": p3["launches"],
        "traffic": None,
    }
    # under the two-stream schedule the phases overlap: each figure is the
    # summed span between the events around its launches (waiting for free
    # compute units included), not its own work
    phases = {k: {"launches": v["launches"], "event_span_ms_per_step": round(v["total_ms"] / args.steps, 3)}
              for k, v in prof.items() if v["launches"]}
    phases["note"] = ("event spans of launches on two streams that overlap; phase 1 and 2 spans include "
                      "waiting behind the other stream's remaining-block products")

    # algorithmic HBM bytes of one launch: its C elements read and written
    # once (8 bytes), plus the panel rows and columns they need, once
    # (the library's automatic block size for distance solves)
    bs = args.block_size or (64 if n <= 5888 else 128 if n < 7168 else 256)
    m = n - 2 * bs
    c_elems = p3["updates"] / max(1, p3["launches"]) / bs
    algo = int(c_elems * 8 + (c_elems / m + m) * bs * 4)
    roofline["algorithmic_bytes_per_launch"] = algo
    traffic = None
    tr = profiling.read_traffic_file(os.path.join(ROOT, "profiles", f"phase3_int32_n{n}_traffic.txt"))
    if tr and tr.get("source_sha256") == profiling.kernel_source_hash() and not args.block_size:
        traffic = int(float(tr["traffic_bytes_per_launch"]))
        roofline["traffic_kernel"] = tr.get("kernel")
        roofline["traffic_vs_algorithmic"] = round(traffic / algo, 3)
    roofline["traffic"] = traffic
    roofline["arithmetic"] = ("float32 on integer values: exact, every operand below 2^23 checked on the device"
                              if int(arith_used.item()) == 1 else "int32")
    del work, pristine
    torch.cuda.empty_cache()
    return W, {"value": round(gops, 2), "ms_per_step": round(ms_per_step, 3), "wall_s": round(wall, 3),
               "dtype": "f32" if int(arith_used.item()) == 1 else "int32", "step_status": "all success",
               "roofline": roofline, "phases": phases, "device": dev_state}


def c1_leg(reps: int):
    """The small single-graph workload: n=1024, p=0.5, int32 weights
    1..1000, distances only; `reps` solves timed one by one (HIP events,
    input restored by a device copy outside the events), median and p99,
    eager and replayed from a captured hipGraph."""
    import numpy as np
    import torch

    import paper_1811_01201_amd as apsp
    import synth

    n = 1024
    W = synth.single_int32(n, p=0.5, seed=synth.BASE_SEED + 0)
    pristine = torch.from_numpy(W).cuda()
    work = torch.empty_like(pristine)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    out = {"workload": "single directed graph n=1024, edge prob 0.5, int32 weights [1,1000], distances only"}
    with torch.cuda.stream(stream):
        for label, kw in (("eager", {}), ("hipgraph_replay", {"use_graph": True})):
            times = []
            for r in range(reps + 2):
                work.copy_(pristine)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                apsp.solve(work, status=st, **kw)
                e1.record(stream)
                stream.synchronize()
                if int(st.item()) != apsp.SUCCESS:
                    raise RuntimeError(f"n=1024 solve reported status {int(st.item())}")
                if r >= 2:
                    times.append(e0.elapsed_time(e1))
            med = float(np.median(times))
            out[label] = {"ms_median": round(med, 4), "ms_p99": round(float(np.percentile(times, 99)), 4),
                          "gops": round(2.0 * n ** 3 / (med / 1e3) / 1e9, 1), "solves": reps}
    del work, pristine
    torch.cuda.empty_cache()
    return out, W


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768, help="override the graph size (quick runs)")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--arith", type=int, default=0, help="0 automatic, 1 int32, 2 float32 (exact, checked)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-single", action="store_true", help="batched/serving legs only")
    ap.add_argument("--sweep", default="",
                    help="only the paper's size sweep, e.g. 4096,8192,16384,32768,65536 (one JSON line)")
    ap.add_argument("--sweep-modes", default="f32pred,int32",
                    help="sweep runs: f32pred (float32 + predecessors), int32 (distances)")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-paper-config", action="store_true",
                    help="skip the n=8192 float32 + predecessors leg")
    ap.add_argument("--skip-serving", action="store_true")
    ap.add_argument("--batched-replays", type=int, default=10)
    ap.add_argument("--no-batched-graph", action="store_true",
                    help="skip the hipGraph replays of the batched plan (counter collection runs)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rate-seconds", type=float, default=6.0,
                    help="seconds of Poisson arrivals per offered rate")
    ap.add_argument("--skip-c1", action="store_true", help="skip the n=1024 leg")
    ap.add_argument("--c1-reps", type=int, default=20)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU: there is no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_01201_amd as apsp

    if args.sweep:
        torch.cuda.set_device(0)
        apsp.lib()
        modes = [m for m in args.sweep_modes.split(",") if m]
        if not modes or any(m not in ("f32pred", "int32") for m in modes):
            ap.error("--sweep-modes takes f32pred and/or int32")
        rows = sweep_leg([int(x) for x in args.sweep.split(",")], modes)
        print(json.dumps({"sweep": rows, "data": "synthetic", "n_gpus": 1}), flush=True)
        return

    n = args.n
    torch.cuda.set_device(0)
    apsp.lib()  # fails loudly without the HIP library
    out = {
        "metric": "min-plus GOPS (2n^3/t) vs VALU peak at n=32768; batched solves/s + p99 latency",
        "value": None, "unit": "GOPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {
            "workload": f"single directed graph n={n}, edge prob 0.1, int32 weights b+pi(i)-pi(j) "
                        f"(b uniform [1,1000], pi(v)=floor(100v/(n-1))), distances only",
            "n": n, "block_size": args.block_size or "auto", "parallelism": "single GPU"},
    }
    W = None
    if not args.skip_single:
        W, single = single_leg(args, n)
        out.update(single)
    c1 = None
    c1_W = None
    if not args.skip_c1:
        log("[bench] n=1024 leg")
        c1, c1_W = c1_leg(args.c1_reps)
    paper = None
    if not args.skip_single and not args.skip_paper_config:
        log("[bench] paper configuration leg (n=8192, float32 + predecessors)")
        paper = paper_config_leg(args.steps)
    batched = None
    if not args.skip_batched:
        log("[bench] batched leg")
        batched = batched_leg(args.batched_replays, not args.no_batched_graph)
    serving = None
    if not args.skip_serving:
        log("[bench] serving leg")
        serving = serving_leg(args.serving_requests, per_rate_s=args.serving_rate_seconds)

    cpu = None
    if not args.no_cpu_baseline and W is not None:
        log(f"[bench] cpu baseline ({args.cpu_seconds:.0f} s budget)")
        import synth
        cpu = cpu_baseline(W, args.cpu_seconds, c1_W=c1_W, batch=None if args.skip_batched else synth.batch())

    out["cpu_baseline"] = cpu
    out["c1_n1024"] = c1
    out["paper_config"] = paper
    out["batched"] = batched
    out["serving"] = serving
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
