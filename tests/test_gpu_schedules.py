"""The production schedule against the full oracle at sizes the oracle solves
whole.

The automatic configuration uses the two-stream split (phase 3 of round r
as the next round's panels plus the rest, the rest on a second stream beside
phases 1-2 of round r+1) only from a padded order of 4096 (3072 for the
fp64-key recurrence), and phase 1 as the dataflow closure of the diagonal
block (4-byte distances in 128- and 256-wide blocks) with one launch of the
remaining phase-3 tiles per round.  The options schedule=2 and phase1=2/3
force the split and either closure at any size, so the exact
launch sequence the headline runs is compared here element by element with
the oracle, for every arithmetic (int32, float32 watched with its int32
redo, float32 weights, the float32 predecessor route and the fp64-key
recurrence), distances and canonical predecessors, on 3 to 8 rounds.  The
library's per-launch profile confirms that the split and the blocked
closure really ran (Section "Data Locality": phase 1, then phases 2 and 3,
per round; the split only reorders independent tiles)."""
import numpy as np
import pytest

import oracle
import pins
import synth
from gpu_util import describe, first_mismatch, oracle_expect

pytestmark = pytest.mark.gpu
INF32 = synth.INF32

_EXPECT = {}


def _graph(kind, n):
    seed = 4242 + n
    if kind == "int":
        return synth.single_int32(n, p=0.3, seed=seed)
    if kind == "pot":
        return synth.potential_int32(n, p=0.1, seed=seed)
    if kind == "f32":
        return synth.single_f32int(n, p=0.3, seed=seed)
    if kind == "sparse":
        return synth.single_int32(n, p=2.0 / n, seed=seed)
    raise ValueError(kind)


def _expect(orc, kind, n):
    """Oracle distances and predecessors of one graph, computed once."""
    key = (kind, n)
    if key not in _EXPECT:
        W = _graph(kind, n)
        D0, P0, st0 = oracle_expect(orc, W, True)
        assert st0 == oracle.OK
        _EXPECT[key] = (W, D0, P0)
    return _EXPECT[key]


def _solve_profiled(W, pred, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    apsp.profile_begin()
    apsp.solve(d, p, status=st, arith_used=used, **kw)
    torch.cuda.synchronize()
    prof = apsp.profile_end()
    return (d.cpu().numpy(), p.cpu().numpy() if pred else None, int(st.item()), int(used.item()), prof)


SIZES = [768, 1000, 1280, 2048]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind,arith", [("int", 1), ("int", 2), ("pot", 1), ("pot", 2), ("f32", 0)])
def test_split_and_blocked_phase1_distances(orc, n, kind, arith):
    """256-wide blocks, the blocked diagonal closure and one kRest launch per
    round on the second stream, as at n = 32768."""
    describe(f"schedule forced: distances n={n} {kind} arith={arith} bs=256 split+blocked")
    W, D0, _ = _expect(orc, kind, n)
    D, _, st, used, prof = _solve_profiled(W, False, block_size=256, schedule=2, phase1=2, arith=arith)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    R = (n + 255) // 256
    assert prof["phase3_cross"]["launches"] == R - 1, prof["phase3_cross"]
    assert prof["phase1_blocked"]["launches"] == R, prof["phase1_blocked"]
    # one kRest launch per round but the last, plus the last round's whole phase 3
    assert prof["phase3"]["launches"] == R, prof["phase3"]
    if kind != "f32":
        assert used == (1 if arith == 2 else 0)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["int", "pot", "f32"])
def test_split_and_blocked_phase1_float32_predecessor_route(orc, n, kind):
    """Predecessors by the float32 route with its distance rounds in the
    production schedule (256-wide blocks, split, blocked closure), then the
    key product."""
    describe(f"schedule forced: float32 predecessor route n={n} {kind}")
    W, D0, P0 = _expect(orc, kind, n)
    D, P, st, used, prof = _solve_profiled(W, True, block_size=256, schedule=2, phase1=2, arith=2)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    R = (n + 255) // 256
    assert prof["phase1_blocked"]["launches"] == R
    assert prof["phase3_cross"]["launches"] == R - 1
    assert used == 1


def test_split_float32_predecessor_route_falls_back(orc):
    """Negative weights together with keys D 2^S + v at or above 2^24 rule the
    key product out: the fp64-key recurrence (128-wide blocks, rounds in
    order) runs after a split float32 distance pass, exactly."""
    describe("schedule forced: float32 predecessor route, fallback to the recurrence")
    n = 1000
    rng = np.random.default_rng(5)
    B = pins.random_graph(rng, n, 0.01, 3000, 8000)
    pot = (np.arange(n, dtype=np.int64) * 10000) // (n - 1)
    W = np.where(B != INF32, B + pot[:, None] - pot[None, :], INF32)
    np.fill_diagonal(W, 0)
    W = W.astype(np.int32)
    assert (W < 0).any()
    D0, P0, st0 = orc.fw(W, pred=True)
    assert st0 == oracle.OK and (D0[D0 != INF32] >= 2 ** 14).any()
    D, P, st, used, prof = _solve_profiled(W, True, block_size=256, schedule=2, phase1=2, arith=2)
    assert st == 0 and used == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    assert prof["phase3_cross"]["launches"] == (n + 255) // 256 - 1


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["int", "pot", "f32"])
def test_split_fp64_key_recurrence(orc, n, kind):
    """The exact fp64-key recurrence for predecessors on two streams
    (128-wide blocks, the two-launch kRest)."""
    describe(f"schedule forced: fp64-key recurrence n={n} {kind}")
    W, D0, P0 = _expect(orc, kind, n)
    D, P, st, used, prof = _solve_profiled(W, True, block_size=128, schedule=2, arith=1)
    assert st == 0 and used == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    R = (n + 127) // 128
    assert prof["phase3_cross"]["launches"] == R - 1
    assert prof["phase1_blocked"]["launches"] == 0


@pytest.mark.parametrize("n,bs,tt", [(1000, 64, 4), (1280, 64, 8), (2048, 128, 8), (1000, 256, 8)])
@pytest.mark.parametrize("kind", ["int", "f32", "sparse"])
def test_split_two_launch_rest(orc, n, bs, tt, kind):
    """The split with the stepwise diagonal kernel and kRest in two launches
    per round (the schedule wherever phase 1 is the stepwise kernel: the
    fp64-key recurrence, 64-wide blocks, or phase1=1)."""
    describe(f"schedule forced: split two-launch rest n={n} bs={bs} tt={tt} {kind}")
    W, D0, _ = _expect(orc, kind, n)
    kw = dict(block_size=bs, thread_tile=tt, schedule=2, phase1=1)
    if kind != "f32":
        kw["arith"] = 2
    D, _, st, _, prof = _solve_profiled(W, False, **kw)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    R = (n + bs - 1) // bs
    assert prof["phase3_cross"]["launches"] == R - 1
    assert prof["phase1_blocked"]["launches"] == 0
    assert prof["phase3"]["launches"] == 2 * (R - 1) + 1


@pytest.mark.parametrize("case", ["chain", "long_paths"])
def test_split_float32_pass_redone_in_int32(orc, case):
    """Operands reaching 2^23 in the split float32 pass make the device redo
    the solve in int32 (rounds in order, blocked closure): still exact.  A
    chain of near-bound weights certainly passes 2^23; random long paths may
    or may not."""
    describe(f"schedule forced: float32 watch fallback {case}")
    n = 900
    rng = np.random.default_rng(11)
    bound = (2 ** 28 - 1) // (n - 1)
    if case == "chain":
        W = pins.random_graph(rng, n, 0.002, bound // 2, bound)
        for i in range(n - 1):
            W[i, i + 1] = bound - (i % 7)
    else:
        W = pins.random_graph(rng, n, 0.05, max(1, bound // 2), bound)
    D0, _, st0 = orc.fw(W)
    assert st0 == oracle.OK
    D, _, st, used, prof = _solve_profiled(W, False, block_size=256, schedule=2, phase1=2, arith=2)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    if case == "chain":
        assert used == 0
    assert prof["phase3_cross"]["launches"] == (n + 255) // 256 - 1


def test_split_negative_cycle_reported():
    describe("schedule forced: negative cycle")
    n = 800
    W = synth.single_int32(n, p=0.05, seed=12)
    W[10, 600], W[600, 10] = 5, -9
    for arith in (1, 2):
        _, _, st, _, _ = _solve_profiled(W, False, block_size=256, schedule=2, phase1=2, arith=arith)
        assert st == 3, arith


# ------------------------------------------------------------------------
# Phase 1 as the dataflow closure (phase1=3): the diagonal block solved by
# the blocked schedule over 32-wide sub-blocks in one launch, on the exact
# routes (int32 arithmetic; float32 arithmetic watched for exactness).


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bs", [128, 256])
@pytest.mark.parametrize("kind,arith", [("int", 1), ("int", 2), ("pot", 1), ("pot", 2), ("sparse", 2)])
def test_dataflow_closure_distances(orc, n, bs, kind, arith):
    describe(f"phase-1 closure: distances n={n} bs={bs} {kind} arith={arith}")
    W, D0, _ = _expect(orc, kind, n)
    R = (n + bs - 1) // bs
    for schedule in (1, 2):
        D, _, st, used, prof = _solve_profiled(W, False, block_size=bs, schedule=schedule, phase1=3, arith=arith)
        assert st == 0
        assert first_mismatch(D, D0) is None, (schedule, first_mismatch(D, D0))
        assert prof["phase1_flow"]["launches"] == R, prof["phase1_flow"]
        assert prof["phase1"]["launches"] == R
        assert used == (1 if arith == 2 else 0)


@pytest.mark.parametrize("n", [1000, 2048])
@pytest.mark.parametrize("kind", ["int", "pot", "f32"])
def test_dataflow_closure_float32_predecessor_route(orc, n, kind):
    """The float32 route's distance rounds (watched float32) with the closure
    and the two-stream split, then the key product."""
    describe(f"phase-1 closure: float32 predecessor route n={n} {kind}")
    W, D0, P0 = _expect(orc, kind, n)
    D, P, st, used, prof = _solve_profiled(W, True, block_size=256, schedule=2, phase1=3, arith=2)
    assert st == 0 and used == 1
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    assert prof["phase1_flow"]["launches"] == (n + 255) // 256


def test_dataflow_closure_watch_fallback_and_cycles(orc):
    """Operands reaching 2^23 inside the closure raise the watch, and the
    int32 redo (closure too) is exact; negative cycles are reported."""
    describe("phase-1 closure: watch fallback, negative cycle")
    n = 900
    rng = np.random.default_rng(11)
    bound = (2 ** 28 - 1) // (n - 1)
    W = pins.random_graph(rng, n, 0.002, bound // 2, bound)
    for i in range(n - 1):
        W[i, i + 1] = bound - (i % 7)
    D0, _, st0 = orc.fw(W)
    assert st0 == oracle.OK
    D, _, st, used, prof = _solve_profiled(W, False, block_size=256, schedule=1, phase1=3, arith=2)
    assert st == 0 and used == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert prof["phase1_flow"]["launches"] >= (n + 255) // 256
    Wc = synth.single_int32(800, p=0.05, seed=12)
    Wc[10, 600], Wc[600, 10] = 5, -9
    for arith in (1, 2):
        _, _, st, _, _ = _solve_profiled(Wc, False, block_size=256, phase1=3, arith=arith)
        assert st == 3, arith


def test_dataflow_closure_real_float32_every_path_agrees(orc):
    """Real-valued float32 weights: the closure rounds otherwise than the
    stepwise kernel (within float32 rounding of the oracle), and every way of
    issuing the solve -- direct, a hipGraph replay, a stepper in slices, the
    no-allocation entry point -- makes the same choice, bit for bit."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("phase-1 closure: real float32, every path")
    n = 700
    W = synth.single_f32real(n, p=0.05, lo=0.5, hi=100.0, seed=23)
    D, _, st, _, prof = _solve_profiled(W, False, block_size=256)
    assert st == 0
    assert prof["phase1_flow"]["launches"] == (n + 255) // 256
    D0, _, _ = orc.fw(W)
    fin = np.isfinite(D0)
    assert np.array_equal(np.isfinite(D), fin)
    rel = np.abs(D[fin].astype(np.float64) - D0[fin]) / np.maximum(1.0, np.abs(D0[fin]))
    assert rel.max() <= 1e-6, rel.max()
    s = torch.cuda.Stream()
    w = torch.from_numpy(W).cuda()
    # hipGraph (captured, then replayed)
    d = torch.empty_like(w)
    for _ in range(2):
        d.copy_(w)
        torch.cuda.synchronize()
        apsp.solve(d, stream=s, use_graph=True, block_size=256)
        s.synchronize()
        assert np.array_equal(d.cpu().numpy().view(np.uint32), D.view(np.uint32))
    # stepper, two rounds per slice
    st_ = apsp.Stepper(n, "float32", block_size=256)
    d = w.clone()
    torch.cuda.synchronize()
    st_.begin(d, stream=s)
    while not st_.step(2):
        pass
    s.synchronize()
    st_.destroy()
    assert np.array_equal(d.cpu().numpy().view(np.uint32), D.view(np.uint32))
    # no allocation
    d = w.clone()
    torch.cuda.synchronize()
    apsp.solve_noalloc(d, stream=s, block_size=256)
    s.synchronize()
    assert np.array_equal(d.cpu().numpy().view(np.uint32), D.view(np.uint32))


def test_dataflow_closure_in_a_graph_replayed(orc):
    """The closure recorded into a hipGraph (its scratch made beforehand),
    replayed several times with eager work in between: every replay exact."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("phase-1 closure: hipGraph replays")
    n = 2100
    W = _graph("int", n)
    D0, _, _ = oracle_expect(orc, W)
    s = torch.cuda.Stream()
    for rep in range(3):
        d = torch.from_numpy(W).cuda()
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        apsp.solve(d, status=st, stream=s, use_graph=True, block_size=256, phase1=3, arith=2)
        s.synchronize()
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert first_mismatch(d.cpu().numpy(), D0) is None, rep
