"""The single-launch schedule (all rounds of the blocked algorithm in one
ordinary launch of the task-graph kernel) against the full oracle.

Section "Data Locality" orders each round as the diagonal block, then its
block row and column, then the remaining blocks; the single launch numbers
those tasks so that every task's operands come from smaller numbers, lets
workgroups claim numbers from a counter and wait on per-block round
counters instead of launch boundaries, and closes the next round's diagonal
block as soon as its own phase-3 product is done.  Every size here runs
with schedule=3 (forced) and is compared element by element with the
oracle; the library's profile confirms that exactly one launch did the
rounds.  Sizes span one round (n <= 64), ragged last blocks and padded
orders up to 3000 (int32 in 32 x 32 blocks up to a padded order of 768,
else 64 x 64).
Real-valued float32 weights are compared
with the multi-launch schedule bit for bit (the same products over the same
operands) and with the oracle within float32 rounding."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import describe, first_mismatch, oracle_expect

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _graph(kind, n):
    seed = 9100 + n
    if kind == "int":
        return synth.single_int32(n, p=0.3, seed=seed)
    if kind == "pot":
        return synth.potential_int32(n, p=0.1, seed=seed)
    if kind == "f32":
        return synth.single_f32int(n, p=0.3, seed=seed)
    if kind == "sparse":
        return synth.single_int32(n, p=2.0 / max(n, 2), seed=seed)
    raise ValueError(kind)


def _run(W, profile=True, stream=None, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    if profile:
        apsp.profile_begin()
    apsp.solve(d, status=st, stream=stream, **kw)
    torch.cuda.synchronize()
    prof = apsp.profile_end() if profile else None
    return d.cpu().numpy(), int(st.item()), prof


def _assert_one_launch(prof):
    assert prof["single_launch"]["launches"] == 1, prof["single_launch"]
    for k in ("phase1", "phase2", "phase3", "phase3_cross"):
        assert prof[k]["launches"] == 0, (k, prof[k])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130, 300, 777, 1000, 1024, 1025, 1280, 1536, 2048, 2100, 2500,
                               3000])
@pytest.mark.parametrize("kind", ["int", "pot", "f32", "sparse"])
def test_single_launch_matches_oracle(orc, n, kind):
    describe(f"single launch: n={n} {kind}")
    W = _graph(kind, n)
    D0, _, st0 = oracle_expect(orc, W)
    assert st0 == oracle.OK
    D, st, prof = _run(W, schedule=3)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    _assert_one_launch(prof)


@pytest.mark.parametrize("n", [200, 1000, 2048])
def test_single_launch_real_weights_bitwise(orc, n):
    """Real-valued float32 weights: the single launch equals the rounds in
    order bit for bit, and the oracle within float32 rounding."""
    describe(f"single launch: real float32 weights n={n}")
    W = synth.single_f32real(n, p=0.05, lo=0.5, hi=100.0, seed=17 + n)
    D1, st1, prof = _run(W, schedule=3)
    _assert_one_launch(prof)
    D2, st2, _ = _run(W, profile=False, schedule=1)
    assert st1 == 0 and st2 == 0
    assert np.array_equal(D1.view(np.uint32), D2.view(np.uint32))
    D0, _, _ = orc.fw(W)
    fin = np.isfinite(D0)
    assert np.array_equal(np.isfinite(D1), fin)
    rel = np.abs(D1[fin].astype(np.float64) - D0[fin]) / np.maximum(1.0, np.abs(D0[fin]))
    assert rel.max() <= 1e-6, rel.max()


def test_single_launch_is_automatic_for_small_graphs(orc):
    """Default options: the single launch up to a padded order of 4096 (int32
    at 4096 itself too, ahead of the float32 route), the per-phase launches
    beyond it."""
    for n, single in ((1024, True), (2048, True), (2049, True), (4096, True), (4100, False)):
        describe(f"single launch: automatic choice n={n}")
        W = _graph("int", n)
        D, st, prof = _run(W)
        assert st == 0
        if n < 4096:  # (the per-phase launches have parity tests of their own)
            D0, _, _ = oracle_expect(orc, W)
            assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
        elif single:  # the per-phase rounds in float32 arithmetic, element by element
            D1, st1, _ = _run(W, profile=False, schedule=1)
            assert st1 == 0
            assert first_mismatch(D, D1) is None, first_mismatch(D, D1)
            for src in (0, n // 2 + 1, n - 1):
                dr, _, s_ = orc.row(W, src)
                assert s_ == 0 and np.array_equal(D[src], dr.astype(D.dtype)), src
        if single:
            _assert_one_launch(prof)
        else:
            assert prof["single_launch"]["launches"] == 0
            assert prof["phase1"]["launches"] > 0


def test_single_launch_back_to_back_and_on_a_stream(orc):
    """Consecutive solves of different sizes on one stream reuse one set of
    task words (cleared before each launch): every result stays exact."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("single launch: back to back on a side stream")
    s = torch.cuda.Stream()
    cases = [(_graph("int", n), n) for n in (520, 1100, 130, 520)]
    outs = []
    with torch.cuda.stream(s):
        for W, _ in cases:
            d = torch.from_numpy(W).cuda()
            st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            apsp.solve(d, status=st, schedule=3, stream=s)
            outs.append((d, st))
    s.synchronize()
    for (W, n), (d, st) in zip(cases, outs):
        D0, _, _ = oracle_expect(orc, W)
        assert int(st.item()) == 0
        assert first_mismatch(d.cpu().numpy(), D0) is None, n


def test_single_launch_negative_cycle_and_validation():
    import torch

    import paper_1811_01201_amd as apsp
    describe("single launch: negative cycle, invalid weights")
    n = 700
    W = synth.single_int32(n, p=0.05, seed=12)
    W[10, 600], W[600, 10] = 5, -9
    _, st, prof = _run(W, schedule=3)
    assert st == apsp.NEGATIVE_CYCLE
    _assert_one_launch(prof)
    Wf = synth.single_f32int(n, p=0.05, seed=13)
    Wf[3, 400], Wf[400, 3] = 2.0, -7.0
    _, st, _ = _run(Wf, schedule=3)
    assert st == apsp.NEGATIVE_CYCLE
    # a nonzero diagonal fails validation: the solve is skipped, dist unchanged
    Wb = synth.single_int32(n, p=0.05, seed=14)
    Wb[5, 5] = 3
    d = torch.from_numpy(Wb.copy()).cuda()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, status=st, validate=True, schedule=3)
    torch.cuda.synchronize()
    assert int(st.item()) == apsp.INVALID_VALUE
    assert np.array_equal(d.cpu().numpy(), Wb)


def test_single_launch_rejected_where_it_does_not_apply():
    import torch

    import paper_1811_01201_amd as apsp
    describe("single launch: option checks")
    d = torch.zeros((100, 100), dtype=torch.int32, device="cuda")
    p = torch.zeros((100, 100), dtype=torch.int32, device="cuda")
    bad = [dict(schedule=3, block_size=128), dict(schedule=3, thread_tile=8), dict(schedule=3, arith=2),
           dict(schedule=4)]
    for kw in bad:
        assert apsp.solve(d, check=False, **kw) == apsp.INVALID_ARGUMENT, kw
    assert apsp.solve(d, p, check=False, schedule=3) == apsp.INVALID_ARGUMENT


@pytest.mark.parametrize("n,schedule,dtype", [(1024, 0, "int"), (300, 3, "int"), (1000, 3, "f32"), (2500, 3, "int")])
def test_single_launch_in_a_graph_replayed(orc, n, schedule, dtype):
    """The single launch recorded into a hipGraph (its work memory made before
    the capture) and replayed several times, with other work on the device
    between the replays: every replay exact."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"single launch: hipGraph replays n={n} schedule={schedule} {dtype}")
    W = _graph(dtype, n)
    D0, _, _ = oracle_expect(orc, W)
    s = torch.cuda.Stream()
    w = torch.from_numpy(W).cuda()
    d = torch.empty_like(w)  # one buffer set: the first call captures, the others replay
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for rep in range(3):
        d.copy_(w)
        st.fill_(-1)
        torch.cuda.synchronize()
        apsp.solve(d, status=st, stream=s, use_graph=True, schedule=schedule)
        s.synchronize()
        junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
        torch.cuda.synchronize()
        del junk
        assert int(st.item()) == 0, rep
        assert first_mismatch(d.cpu().numpy(), D0) is None, rep
