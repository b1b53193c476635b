"""Seeded random configurations of apsp_solve_ex (size, graph kind,
predecessors, arithmetic, block size, register tile, schedule, graph
replay) against the oracle, element by element.  Each case is fixed by its
seed, so a failure names a reproducible configuration."""
import numpy as np
import pytest

import pins
import synth
from gpu_util import describe, first_mismatch, gpu_solve, oracle_expect

pytestmark = pytest.mark.gpu


def _case(seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.choice([1, 2, 5, 31, 64, 65, 100, 129, 200, 255, 256, 257, 333, 500, 640, 777, 1000, 1100]))
    kind = str(rng.choice(["int", "sparse", "pot", "f32", "ties"]))
    pred = bool(rng.random() < 0.5)
    arith = int(rng.choice([0, 1, 2]))
    bs, tt = [(0, 0), (64, 4), (64, 8), (128, 8), (256, 8)][int(rng.integers(0, 5))]
    if pred and bs == 256:
        bs, tt = 128, 8
    schedule = int(rng.integers(0, 2))
    use_graph = bool(rng.random() < 0.2)
    p = float(rng.choice([0.02, 0.1, 0.3, 0.7]))
    gseed = int(rng.integers(0, 1 << 30))
    if kind == "int":
        W = synth.single_int32(n, p=p, seed=gseed)
    elif kind == "sparse":
        W = synth.single_int32(n, p=min(1.0, 3.0 / max(n, 1)), seed=gseed)
    elif kind == "pot":
        W = synth.potential_int32(n, p=p, seed=gseed)
    elif kind == "f32":
        W = synth.single_f32int(n, p=p, seed=gseed)
    else:  # weights 1..3: many equal-length paths (ties for the predecessor rule)
        W = pins.random_graph(np.random.default_rng(gseed), n, p, 1, 3)
    return W, pred, dict(arith=arith, block_size=bs, thread_tile=tt, schedule=schedule, use_graph=use_graph)


@pytest.mark.parametrize("seed", range(160))
def test_random_configuration(orc, seed):
    W, pred, kw = _case(seed)
    describe(f"random seed={seed} n={W.shape[0]} dtype={W.dtype} pred={pred} {kw}")
    D0, P0, st0 = oracle_expect(orc, W, pred)
    assert st0 == 0
    if kw["use_graph"]:
        import torch
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            D, P, st = gpu_solve(W, pred, **kw)
    else:
        D, P, st = gpu_solve(W, pred, **kw)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    if pred:
        assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
