"""GPU parity of predecessor solves on the float32 route (arith=2): exact
float32 distances, then the canonical predecessors read off the float32
key product, with the device falling back to the fp64-key recurrence
whenever a key could be inexact.  Distances and predecessors must match the
oracle bit for bit either way; the device reports which route held."""
import numpy as np
import pytest

import oracle
import pins
import synth
from gpu_util import describe, first_mismatch, oracle_expect

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _solve(W, arith=2, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, p, status=st, arith=arith, arith_used=used, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), p.cpu().numpy(), int(st.item()), int(used.item())


def _graph(kind, n, seed):
    if kind == "int":
        return synth.single_int32(n, p=0.3, seed=seed)
    if kind == "sparse":
        return synth.single_int32(n, p=min(1.0, 2.0 / max(n, 1)), seed=seed)
    if kind == "pot":
        return synth.potential_int32(n, p=0.1, seed=seed)
    if kind == "f32":
        return synth.single_f32int(n, p=0.3, seed=seed)
    raise ValueError(kind)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 127, 129, 255, 257, 383, 513, 1000])
@pytest.mark.parametrize("kind", ["int", "sparse", "pot", "f32"])
def test_float32_route_parity(orc, n, kind):
    describe(f"pred product n={n} kind={kind}")
    W = _graph(kind, n, seed=4000 + n)
    D0, P0, st0 = oracle_expect(orc, W, True)
    D, P, st, used = _solve(W)
    assert st == 0 and st0 == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    if kind in ("int", "f32", "pot"):
        assert used == 1  # short distances, small weights: the product held
    assert used in (0, 1)


@pytest.mark.parametrize("bs,tt", [(64, 4), (64, 8), (128, 8)])
@pytest.mark.parametrize("n,kind", [(130, "int"), (300, "pot"), (700, "f32")])
def test_float32_route_block_sizes(orc, bs, tt, n, kind):
    describe(f"pred product bs={bs} tt={tt} n={n} kind={kind}")
    W = _graph(kind, n, seed=91 + n)
    D0, P0, _ = oracle_expect(orc, W, True)
    D, P, st, used = _solve(W, block_size=bs, thread_tile=tt)
    assert st == 0 and used == 1
    assert first_mismatch(D, D0) is None
    assert first_mismatch(P, P0) is None


@pytest.mark.parametrize("case", ["big_weights", "long_paths", "big_negative", "half_integer", "key_bound"])
def test_float32_route_falls_back(orc, case):
    """Inputs whose keys cannot be exact in float32: the device runs the
    recurrence instead (reported as 0) and the result is still exact."""
    describe(f"pred product fallback {case}")
    rng = np.random.default_rng(7)
    n = 150
    bound = (2 ** 28 - 1) // (n - 1)
    if case == "big_weights":      # weights of 2^23 and more: float32 distances not watched-exact
        n = 12
        W = pins.random_graph(rng, n, 0.4, 2 ** 23, 2 ** 23 + 1000)
    elif case == "long_paths":     # distances beyond 2^(24-S): keys out of range, after dist was written
        W = pins.random_graph(rng, n, 0.03, 20000, 30000)
    elif case == "big_negative":   # negative weights with large distances elsewhere
        pot = np.arange(n, dtype=np.int64) * (bound // 4) // (n - 1)
        B = pins.random_graph(rng, n, 0.2, 1, 100)
        fin = B != INF32
        W = np.where(fin, B + pot[:, None] - pot[None, :], INF32)
        np.fill_diagonal(W, 0)
        W = W.astype(np.int32)
    elif case == "half_integer":   # float32 weights that are not integers: (distance, predecessor) pairs
        W = pins.random_graph(rng, n, 0.3, 0, 2, dtype=np.float32)
        fin = np.isfinite(W) & ~np.eye(n, dtype=bool)
        W[fin] += 0.5
    else:                          # an integer float32 weight above the key-mode bound: pairs
        W = synth.single_f32int(n, p=0.2, seed=12)
        W[3, 7] = 1.0e7
    D0, P0, st0 = oracle_expect(orc, W, True)
    assert st0 == oracle.OK
    D, P, st, used = _solve(W)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)
    assert used == 0


def test_float32_route_nonzero_diagonal_matches_recurrence():
    """Unvalidated input with a positive diagonal entry: the product's
    closed form assumes a zero diagonal, so the device takes the
    recurrence; the result equals the recurrence's own."""
    describe("pred product nonzero diagonal")
    W = synth.single_int32(200, p=0.2, seed=3)
    W[5, 5] = 7
    D, P, st, used = _solve(W, arith=2)
    D1, P1, st1, used1 = _solve(W, arith=1)
    assert used == 0 and used1 == 0 and st == st1 == 0
    assert np.array_equal(D, D1) and np.array_equal(P, P1)


@pytest.mark.parametrize("dtype", ["int", "f32"])
def test_float32_route_negative_cycle(dtype):
    describe(f"pred product negative cycle {dtype}")
    n = 400
    W = synth.single_int32(n, p=0.05, seed=21) if dtype == "int" else synth.single_f32int(n, p=0.05, seed=21)
    W[10, 150], W[150, 10] = 5, -9
    _, _, st, _ = _solve(W)
    assert st == 3


def test_float32_route_validate_rejects_and_leaves_input():
    import torch

    import paper_1811_01201_amd as apsp
    describe("pred product validate")
    W = synth.single_int32(300, p=0.2, seed=4)
    W[3, 3] = 1  # non-zero diagonal: invalid
    d = torch.from_numpy(W.copy()).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, p, validate=True, status=st, arith=2)
    torch.cuda.synchronize()
    assert int(st.item()) == apsp.INVALID_VALUE
    assert np.array_equal(d.cpu().numpy(), W)
    assert (p.cpu().numpy() == -7).all()


def test_float32_route_equals_recurrence_mid_size(orc):
    """n = 4500 (automatic choice: the float32 route) against the recurrence,
    bit for bit, plus sampled rows against the row oracle."""
    describe("pred product n=4500 vs recurrence")
    n = 4500
    W = synth.single_f32int(n, p=0.3, seed=synth.BASE_SEED + 9)
    D, P, st, used = _solve(W, arith=0)
    D1, P1, st1, used1 = _solve(W, arith=1)
    assert st == st1 == 0 and used == 1 and used1 == 0
    assert np.array_equal(D, D1) and np.array_equal(P, P1)
    for src in (0, 2777, n - 1):
        dr, pr, s = orc.row(W, src, pred=True)
        assert s == 0
        assert np.array_equal(D[src], dr.astype(np.float32)) and np.array_equal(P[src], pr)


def test_float32_route_graph_replays(orc):
    import torch

    import paper_1811_01201_amd as apsp
    describe("pred product graph replays")
    n = 600
    W = synth.single_int32(n, p=0.3, seed=31)
    D0, P0, _ = orc.fw(W, pred=True)
    d = torch.from_numpy(W.copy()).cuda()
    w0 = d.clone()
    p = torch.empty((n, n), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            d.copy_(w0)
            p.fill_(-7)
            apsp.solve(d, p, use_graph=True, arith=2)
            torch.cuda.current_stream().synchronize()
            assert np.array_equal(d.cpu().numpy(), D0)
            assert np.array_equal(p.cpu().numpy(), P0)
