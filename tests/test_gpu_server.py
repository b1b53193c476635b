"""GPU tests of the serving runtime: every result in a mixed, overlapping
request stream equals the same request solved alone (bit for bit) and the
oracle; admission by device-memory budget, queue limits, cancellation and
error propagation; concurrent requests that take the dataflow kernels (the
single launch for small graphs solved in place, the phase-1 closure of
large ones) on several streams at once."""
import threading
import time

import numpy as np
import pytest

import synth
from gpu_util import describe, gpu_solve

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _mix(count, seed, n_hi=1500):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        n = int(round(np.exp(rng.uniform(np.log(8), np.log(n_hi)))))
        dtype = "int32" if rng.random() < 0.5 else "float32"
        pred = bool(rng.random() < 0.3)
        if dtype == "int32":
            W = synth.int32_rows(n, 0.2, 1, 1000, seed, g=r)
        else:
            W = synth.single_f32int(n, 0.2, seed=seed, g=r)
        reqs.append((W, pred))
    return reqs


def test_mix_equals_alone_and_oracle(orc):
    import paper_1811_01201_amd as apsp
    describe("server mix == alone")
    reqs = _mix(40, seed=3)
    with apsp.Server(n_streams=3) as sv:
        tickets = [sv.submit(W, want_pred=p) for W, p in reqs]
        for t, (W, p) in zip(tickets, reqs):
            assert sv.wait(t) == apsp.SUCCESS
            D, P = sv.result(t)
            Da, Pa, st = gpu_solve(W, pred=p)
            assert st == 0
            assert np.array_equal(D, Da)
            if p:
                assert np.array_equal(P, Pa)
            D0, P0, _ = orc.fw(W, pred=p)
            assert np.array_equal(D, D0.astype(D.dtype))
            if p:
                assert np.array_equal(P, P0)
            assert sv.release(t) == apsp.SUCCESS
        s = sv.stats()
        assert s["completed"] == len(reqs) and s["failed"] == 0 and s["inflight"] == 0
        assert s["p99_latency_ms"] >= s["p50_latency_ms"] > 0


def test_alone_vs_in_mix_bitwise():
    """The same request submitted to an idle server and inside a busy mixed
    stream gives identical bits."""
    import paper_1811_01201_amd as apsp
    describe("server alone vs mix")
    probe = [(synth.single_f32int(700, 0.2, seed=77), True), (synth.single_int32(40, 0.2, seed=78), True),
             (synth.single_int32(2000, 0.2, seed=79), False)]
    alone = []
    with apsp.Server() as sv:
        for W, p in probe:
            t = sv.submit(W, want_pred=p)
            assert sv.wait(t) == apsp.SUCCESS
            alone.append(sv.result(t))
            sv.release(t)
    mix = _mix(30, seed=5)
    with apsp.Server() as sv:
        ts = [sv.submit(W, want_pred=p) for W, p in mix[:15]]
        tp = [sv.submit(W, want_pred=p) for W, p in probe]
        ts += [sv.submit(W, want_pred=p) for W, p in mix[15:]]
        for t, (D0, P0) in zip(tp, alone):
            assert sv.wait(t) == apsp.SUCCESS
            D, P = sv.result(t)
            assert np.array_equal(D, D0)
            assert (P is None and P0 is None) or np.array_equal(P, P0)
        for t in ts + tp:
            assert sv.wait(t) == apsp.SUCCESS
            sv.release(t)


def test_budget_admission_and_release():
    """With a budget that holds only one large request at a time, requests
    wait for releases; results are still correct."""
    import paper_1811_01201_amd as apsp
    describe("server budget admission")
    n = 1536  # a multiple of the block size: solved in place, no work memory
    per = n * n * 4 + 4096
    graphs = [synth.single_int32(n, 0.2, seed=200 + i) for i in range(4)]
    with apsp.Server(hbm_budget_bytes=int(1.5 * per), batch_max_n=-1) as sv:
        ts = [sv.submit(W) for W in graphs]
        assert sv.wait(ts[0]) == apsp.SUCCESS
        time.sleep(0.05)
        assert sv.poll(ts[1]) == apsp.NOT_READY  # blocked by the budget
        assert sv.stats()["queued"] >= 2
        for t, W in zip(ts, graphs):
            assert sv.wait(t, timeout_us=20_000_000) == apsp.SUCCESS
            D, _ = sv.result(t)
            Da, _, _ = gpu_solve(W)
            assert np.array_equal(D, Da)
            sv.release(t)
        too_big = np.zeros((2000, 2000), dtype=np.int32)
        assert sv.submit(too_big, check=False) == apsp.OUT_OF_MEMORY


def test_errors_queue_full_cancel_and_negative_cycle():
    import paper_1811_01201_amd as apsp
    describe("server errors")
    W = synth.single_int32(120, 0.1, seed=4)
    W[3, 9], W[9, 3] = 2, -7
    with apsp.Server() as sv:
        t = sv.submit(W)
        assert sv.wait(t) == apsp.NEGATIVE_CYCLE
        assert sv.poll(t) == apsp.NEGATIVE_CYCLE
        assert sv.release(t) == apsp.SUCCESS
        assert sv.poll(t) == apsp.UNKNOWN_TICKET
        assert sv.wait(12345) == apsp.UNKNOWN_TICKET
    # a full queue: one slot, one long request in flight
    big = synth.single_int32(4096, 0.2, seed=5)
    small = synth.single_int32(50, 0.2, seed=6)
    sv = apsp.Server(max_inflight=1, max_queue=2, batch_max_n=-1)
    t0 = sv.submit(big)
    t1 = sv.submit(small)
    t2 = sv.submit(small)
    st = sv.submit(small, check=False)
    assert st == apsp.QUEUE_FULL
    # destroy while t1/t2 wait for the slot held by t0 (never released)
    results = {}

    def waiter(t):
        results[t] = sv.wait(t)

    th = [threading.Thread(target=waiter, args=(t,)) for t in (t1, t2)]
    for x in th:
        x.start()
    assert sv.wait(t0) == apsp.SUCCESS
    time.sleep(0.05)
    sv.destroy()
    for x in th:
        x.join(timeout=30)
    assert results == {t1: apsp.CANCELLED, t2: apsp.CANCELLED}


def test_borrowed_strided_submission():
    import torch

    import paper_1811_01201_amd as apsp
    describe("server borrowed strided")
    base = torch.from_numpy(synth.single_int32(900, 0.2, seed=8)).pin_memory()
    with apsp.Server() as sv:
        ts = [(n, sv.submit(base, n=n, borrow=True)) for n in (900, 700, 333, 40)]
        for n, t in ts:
            assert sv.wait(t) == apsp.SUCCESS
            D, _ = sv.result(t)
            Da, _, _ = gpu_solve(np.ascontiguousarray(base.numpy()[:n, :n]))
            assert np.array_equal(D, Da)
            sv.release(t)


def test_large_int32_request_float32_arithmetic(orc):
    """An int32 request above n = 4096 runs in float32 arithmetic inside the
    server (work memory from the server's budget): equal to the solo solve
    and to the row oracle."""
    import paper_1811_01201_amd as apsp
    describe("server large int32 request")
    n = 5000
    W = synth.potential_int32(n, p=0.05, seed=61)
    with apsp.Server() as sv:
        t = sv.submit(W)
        assert sv.wait(t, timeout_us=60_000_000) == apsp.SUCCESS
        D, _ = sv.result(t)
        sv.release(t)
    Da, _, st = gpu_solve(W)
    assert st == 0 and np.array_equal(D, Da)
    for src in (0, n - 1):
        dr, _, s = orc.row(W, src)
        assert s == 0 and np.array_equal(D[src], dr)


@pytest.mark.parametrize("slice_rounds", [1, 4])
def test_sliced_large_requests_equal_alone(orc, slice_rounds):
    """Round-level preemption: large requests issued slice_rounds rounds at a
    time, interleaved with small batched requests and each other, give the
    bits of the same request solved alone; per-class latencies are reported."""
    import paper_1811_01201_amd as apsp
    describe(f"server sliced rounds={slice_rounds}")
    reqs = _mix(24, seed=11, n_hi=3000)
    reqs += [(synth.single_f32int(4500, 0.2, seed=12), True), (synth.potential_int32(5000, p=0.1, seed=13), False)]
    with apsp.Server(n_streams=2, slice_rounds=slice_rounds) as sv:
        tickets = [sv.submit(W, want_pred=p) for W, p in reqs]
        for t, (W, p) in zip(tickets, reqs):
            assert sv.wait(t) == apsp.SUCCESS
            D, P = sv.result(t)
            Da, Pa, st = gpu_solve(W, pred=p)
            assert st == 0 and np.array_equal(D, Da)
            if p:
                assert np.array_equal(P, Pa)
            if W.shape[0] <= 300:
                D0, _, _ = orc.fw(W)
                assert np.array_equal(D, D0.astype(D.dtype))
            assert sv.release(t) == apsp.SUCCESS
        s = sv.stats()
        assert s["completed"] == len(reqs) and s["failed"] == 0
        assert s["p99_large_ms"] >= s["p50_large_ms"] > 0
        assert s["p99_small_ms"] >= s["p50_small_ms"] > 0


def test_sliced_negative_cycle_reported():
    import paper_1811_01201_amd as apsp
    describe("server sliced negative cycle")
    W = synth.single_int32(900, p=0.05, seed=21)
    W[10, 150], W[150, 10] = 5, -9
    with apsp.Server(slice_rounds=2, batch_max_n=-1) as sv:
        t = sv.submit(W)
        assert sv.wait(t) == apsp.NEGATIVE_CYCLE
        sv.release(t)


def test_concurrent_dataflow_requests(orc):
    """Requests that run the task-graph kernels concurrently on several
    streams: in-place int32 graphs of n = 64 k (the single launch) and
    n ~ 6000 (256-wide blocks, the phase-1 closure), interleaved with small
    batched ones.  Every workgroup of those launches only waits for work
    that running workgroups hold, so each completes beside the others; the
    small and single-launch results equal the oracle, the large ones its
    rows (16 sampled rows each)."""
    import paper_1811_01201_amd as apsp
    describe("server: concurrent single-launch and closure requests")
    rng = np.random.default_rng(41)
    reqs = []
    for k, n in enumerate([640, 5960, 1024, 128, 6100, 768, 1984, 5900, 256, 1024, 64, 1536]):
        reqs.append(synth.single_int32(n, p=0.2, seed=900 + k))
    small = [synth.single_int32(int(rng.integers(16, 200)), p=0.3, seed=950 + k) for k in range(24)]
    with apsp.Server(n_streams=6, max_inflight=32) as sv:
        order = []
        for k, W in enumerate(reqs):
            order.append((sv.submit(W), W))
            order.append((sv.submit(small[2 * k]), small[2 * k]))
            order.append((sv.submit(small[2 * k + 1]), small[2 * k + 1]))
        for t, W in order:
            assert sv.wait(t) == apsp.SUCCESS, W.shape
            D, _ = sv.result(t)
            n = W.shape[0]
            if n <= 2048:
                D0, _, st0 = orc.fw(W)
                assert st0 == 0
                assert np.array_equal(D, D0), n
            else:
                srcs = [int(x) for x in rng.choice(n, 16, replace=False)]
                for src, (dr, _, s0) in zip(srcs, orc.rows(W, srcs)):
                    assert s0 == 0
                    assert np.array_equal(D[src], dr), (n, src)
            assert sv.release(t) == apsp.SUCCESS
        s = sv.stats()
        assert s["failed"] == 0
