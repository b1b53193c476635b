"""The seeded generator: compiled code == its pure-Python definition, which is
itself pinned to the published SplitMix64 output sequence; workload shapes."""
import math

import numpy as np

import synth


def test_splitmix64_published_sequence():
    # SplitMix64 with state 0: the first two outputs of the reference sequence
    assert synth._mix64_py(synth.GOLDEN) == 0xE220A8397B1DCDAF
    assert synth._mix64_py((2 * synth.GOLDEN) & synth.MASK64) == 0x6E789E6AA1B965F4


def test_compiled_matches_definition():
    for (seed, g, i, j, s) in [(0, 0, 0, 0, 0), (1, 2, 3, 4, 1), (synth.BASE_SEED, 4095, 511, 7, 2),
                               (2**63 + 5, 1, 32767, 32766, 0)]:
        assert synth.u64(seed, g, i, j, s) == synth.u64_py(seed, g, i, j, s)
        assert synth.u01(seed, g, i, j, s) == (synth.u64_py(seed, g, i, j, s) >> 11) * 2.0 ** -53


def test_matrix_cells_follow_definition():
    n, p, seed = 37, 0.4, 12345
    W = synth.single_int32(n, p=p, lo=1, hi=1000, seed=seed)
    for i in range(n):
        for j in range(n):
            if i == j:
                assert W[i, j] == 0
                continue
            pres = (synth.u64_py(seed, 0, i, j, 0) >> 11) * 2.0 ** -53 < p
            if pres:
                assert W[i, j] == 1 + synth.u64_py(seed, 0, i, j, 1) % 1000
            else:
                assert W[i, j] == synth.INF32


def test_rows_are_slices_and_dtypes_agree():
    n = 300
    full = synth.potential_int32(n, p=0.1, seed=3)
    part = synth.potential_int32(n, p=0.1, seed=3, r0=100, r1=150)
    assert np.array_equal(full[100:150], part)
    Wi = synth.single_int32(n, p=0.3, seed=8)
    Wf = synth.single_f32int(n, p=0.3, seed=8)
    assert np.array_equal(np.where(Wi == synth.INF32, np.inf, Wi).astype(np.float32), Wf)


def test_potential_workload_shape():
    n = 1000
    W = synth.potential_int32(n, p=0.1, seed=1)
    fin = (W != synth.INF32) & ~np.eye(n, dtype=bool)
    frac = fin.sum() / (n * (n - 1))
    assert abs(frac - 0.1) < 0.005
    w = W[fin]
    assert w.min() >= -99 and w.max() <= 1100
    i, j = np.nonzero(fin & (W < 0))
    assert len(i) > 0 and (i < j).all()


def test_batch_and_requests_shape():
    b = synth.batch(count=256)
    assert b.ns.min() >= 16 and b.ns.max() <= 512
    assert (b.ps >= 0.05).all() and (b.ps <= 0.9).all()
    assert (b.offsets % 4 == 0).all()
    ends = b.offsets + b.ns.astype(np.int64) ** 2
    assert (ends[:-1] <= b.offsets[1:]).all() and ends[-1] <= b.total
    reqs = synth.requests(2000, rate_per_s=100.0)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 8192
    # log-uniform: the median of n is near sqrt(32*8192) = 512
    assert 400 < np.median(ns) < 650
    gaps = np.diff([0.0] + [r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 0.01) < 0.001
    assert 0.45 < np.mean([r.dtype == "int32" for r in reqs]) < 0.55
    assert 0.25 < np.mean([r.want_pred for r in reqs]) < 0.35
    assert math.isclose(reqs[5].arrival_s, synth.requests(6, 100.0)[5].arrival_s)
