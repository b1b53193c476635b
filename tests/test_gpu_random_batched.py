"""Seeded random batches for the fused batched launch: mixed sizes 1..700,
weight regimes that select each arithmetic (small integers -> float32,
large or negative int32 weights -> int32, non-integer float32 weights with
predecessors -> (distance, predecessor) pairs), predecessors or not, and
automatic or forced team configurations; every graph against the oracle."""
import numpy as np
import pytest

import pins
import synth
from gpu_util import describe, first_mismatch

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _batch(seed):
    rng = np.random.default_rng(9000 + seed)
    dtype = np.int32 if rng.random() < 0.6 else np.float32
    pred = bool(rng.random() < 0.5)
    count = int(rng.integers(3, 14))
    graphs = []
    for g in range(count):
        n = int(rng.choice([1, 2, 7, 33, 64, 65, 100, 128, 129, 190, 256, 257, 300, 400, 511, 512, 513, 700]))
        regime = int(rng.integers(0, 4))
        p = float(rng.uniform(0.05, 0.8))
        gr = np.random.default_rng(int(rng.integers(0, 1 << 30)))
        if dtype == np.int32:
            if regime == 0:
                W = pins.random_graph(gr, n, p, 1, 1000)
            elif regime == 1:   # weights too large for float32 arithmetic at this size
                bound = (2 ** 28 - 1) // max(1, n - 1)
                W = pins.random_graph(gr, n, p, max(1, bound // 2), max(1, bound))
            elif regime == 2:   # negative weights, no negative cycle
                W = pins.random_graph(gr, n, p, 1, 500, potential=True)
            else:
                W = pins.random_graph(gr, n, p, 1, 3)
        else:
            W = pins.random_graph(gr, n, p, 1, 1000 if regime < 2 else 3, dtype=np.float32)
            if regime == 3:     # half-integers: pairs with predecessors, exact sums
                fin = np.isfinite(W) & ~np.eye(n, dtype=bool)
                W[fin] += 0.5
        graphs.append(W)
    cfg = None if rng.random() < 0.5 else int(rng.integers(0, 3))
    return graphs, dtype, pred, cfg


def _pack(graphs, dtype):
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    sizes = ns.astype(np.int64) ** 2
    offsets = np.zeros(len(graphs), dtype=np.int64)
    offsets[1:] = np.cumsum((sizes + 3) // 4 * 4)[:-1]
    total = int(offsets[-1] + sizes[-1])
    buf = np.full(max(total, 4), INF32 if dtype == np.int32 else np.inf, dtype=dtype)
    for g, o in zip(graphs, offsets):
        buf[o:o + g.size] = g.ravel()
    return buf, ns, offsets


@pytest.mark.parametrize("seed", range(40))
def test_random_batch(orc, seed):
    import torch

    import paper_1811_01201_amd as apsp
    graphs, dtype, pred, cfg = _batch(seed)
    describe(f"random batch seed={seed} B={len(graphs)} dtype={dtype.__name__} pred={pred} cfg={cfg}")
    buf, ns, offs = _pack(graphs, dtype)
    plan = apsp.BatchPlan(ns, offs, "int32" if dtype == np.int32 else "float32", want_pred=pred, team_config=cfg)
    d = torch.from_numpy(buf.copy()).cuda()
    p = torch.full(d.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((len(graphs),), -1, dtype=torch.int32, device="cuda")
    plan.execute(d, p, st)
    torch.cuda.synchronize()
    plan.destroy()
    D, S = d.cpu().numpy(), st.cpu().numpy()
    P = p.cpu().numpy() if pred else None
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        D0, P0, s0 = orc.fw(W, pred=pred)
        assert s0 == 0 and S[b] == 0, (b, n)
        if dtype == np.float32:
            D0 = D0.astype(np.float32)
        got = D[o:o + n * n].reshape(n, n)
        assert first_mismatch(got, D0) is None, (b, n, first_mismatch(got, D0))
        if pred:
            gp = P[o:o + n * n].reshape(n, n)
            assert first_mismatch(gp, P0) is None, (b, n, first_mismatch(gp, P0))
