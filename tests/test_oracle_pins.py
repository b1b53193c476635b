"""Pins for the CPU oracle: every check here compares the oracle with
something other than itself (path enumeration, Dijkstra, Bellman–Ford,
scipy's shortest-path routines, closed forms, invariants)."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csg

import oracle
import pins
import synth

INF32 = pins.INF32


def _as_lists(D, inf):
    return [[None if x == inf else x.item() for x in r] for r in D]


# ------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_bruteforce_int(orc, n, seed):
    rng = np.random.default_rng(1000 * n + seed)
    p = [0.2, 0.5, 0.9][seed % 3]
    W = pins.random_graph(rng, n, p, 1, 9 if seed % 2 else 1000, potential=(seed % 4 == 3))
    D, P, st = orc.fw(W, pred=True)
    assert st == oracle.OK
    bd, bp = pins.brute_force(W)
    assert _as_lists(D, INF32) == bd
    assert P.tolist() == bp


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_float_real(orc, seed):
    rng = np.random.default_rng(77 + seed)
    n = 6
    W = pins.random_graph(rng, n, 0.6, 1, 100, dtype=np.float32)
    W[W != np.inf] += rng.random(np.count_nonzero(W != np.inf)).astype(np.float32)
    np.fill_diagonal(W, 0)
    D, P, st = orc.fw(W, pred=True)
    bd, bp = pins.brute_force(W.astype(np.float64))
    for i in range(n):
        for j in range(n):
            if bd[i][j] is None:
                assert D[i, j] == np.inf and P[i, j] == -1
            else:
                assert D[i, j] == pytest.approx(bd[i][j], rel=1e-12)
    # real weights: shortest paths unique with probability 1, so P is too
    assert P.tolist() == bp


def test_ties_pick_smallest_predecessor(orc):
    # 0->1->3 and 0->2->3 both weigh 2: the predecessor of 3 must be 1
    W = np.full((4, 4), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    W[0, 1] = W[1, 3] = W[0, 2] = W[2, 3] = 1
    D, P, _ = orc.fw(W, pred=True)
    assert D[0, 3] == 2 and P[0, 3] == 1
    # reverse the labels of the middle vertices: still the smaller one wins
    W[0, 1] = 5
    W[0, 2] = 1
    W[2, 3] = 1
    W[1, 3] = 1
    D, P, _ = orc.fw(W, pred=True)
    assert D[0, 3] == 2 and P[0, 3] == 2


# --------------------------------------------------------------- Dijkstra
@pytest.mark.parametrize("n,p,seed", [(40, 0.1, 1), (64, 0.5, 2), (97, 0.05, 3), (120, 0.9, 4)])
def test_dijkstra_int(orc, n, p, seed):
    rng = np.random.default_rng(seed)
    W = pins.random_graph(rng, n, p, 1, 1000)
    D, P, st = orc.fw(W, pred=True)
    assert st == oracle.OK
    for i in range(0, n, max(1, n // 12)):
        dr = pins.dijkstra_row(W, i)
        assert _as_lists(D[i:i + 1], INF32)[0] == dr
        assert P[i].tolist() == pins.canonical_pred_row(W, dr, i)


@pytest.mark.parametrize("n,seed", [(50, 5), (80, 6)])
def test_bellman_ford_negative(orc, n, seed):
    rng = np.random.default_rng(seed)
    W = pins.random_graph(rng, n, 0.15, 1, 30, potential=True)
    assert (W[W != INF32] < 0).any()
    D, P, st = orc.fw(W, pred=True)
    assert st == oracle.OK
    for i in range(0, n, 7):
        dr, neg = pins.bellman_ford_row(W, i)
        assert not neg
        assert _as_lists(D[i:i + 1], INF32)[0] == dr
        assert P[i].tolist() == pins.canonical_pred_row(W, dr, i)


# ------------------------------------------------------------------ scipy
def _scipy(W, method):
    A = W.astype(np.float64)
    absent = (W == INF32) | np.isinf(A) | np.eye(W.shape[0], dtype=bool)
    G = csg.csgraph_from_masked(np.ma.masked_array(A, mask=absent))  # keeps 0-weight edges
    return csg.shortest_path(G, method=method, directed=True)


@pytest.mark.parametrize("n,p,seed,method", [(300, 0.3, 11, "D"), (257, 0.05, 12, "D"),
                                             (200, 0.2, 13, "J")])
def test_scipy_int(orc, n, p, seed, method):
    rng = np.random.default_rng(seed)
    W = pins.random_graph(rng, n, p, 1, 1000, potential=(method == "J"))
    D, _, st = orc.fw(W)
    ref = _scipy(W, method)
    got = np.where(D == INF32, np.inf, D.astype(np.float64))
    assert np.array_equal(got, ref)


def test_scipy_float_real(orc):
    rng = np.random.default_rng(21)
    n = 180
    W = pins.random_graph(rng, n, 0.2, 1, 1000, dtype=np.float32)
    fin = np.isfinite(W) & ~np.eye(n, dtype=bool)
    W[fin] = (W[fin] * rng.random(np.count_nonzero(fin))).astype(np.float32) + 0.5
    D, _, _ = orc.fw(W)
    ref = _scipy(W, "D")
    assert np.allclose(D, ref, rtol=1e-12, atol=0)
    assert np.array_equal(np.isinf(D), np.isinf(ref))


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("n,w", [(1, 3), (2, 5), (17, 3), (64, 1)])
def test_directed_cycle(orc, n, w):
    W = np.full((n, n), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    for i in range(n):
        if n > 1:
            W[i, (i + 1) % n] = w
    D, P, _ = orc.fw(W, pred=True)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(D, w * ((j - i) % n))
    expP = (j - 1) % n
    expP[i == j] = -1
    assert np.array_equal(P, expP)


@pytest.mark.parametrize("n,w", [(5, 7), (33, 1)])
def test_complete_uniform(orc, n, w):
    W = np.full((n, n), w, dtype=np.int32)
    np.fill_diagonal(W, 0)
    D, P, _ = orc.fw(W, pred=True)
    assert np.array_equal(D, W)
    expP = np.repeat(np.arange(n)[:, None], n, axis=1).astype(np.int32)
    np.fill_diagonal(expP, -1)
    assert np.array_equal(P, expP)


def test_empty_graph(orc):
    n = 9
    W = np.full((n, n), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    D, P, _ = orc.fw(W, pred=True)
    assert np.array_equal(D, W) and (P == -1).all()
    Wf = np.where(W == INF32, np.inf, 0).astype(np.float32)
    Df, Pf, _ = orc.fw(Wf, pred=True)
    assert np.array_equal(Df, Wf.astype(np.float64)) and (Pf == -1).all()


def test_chain_prefix_sums(orc):
    n = 30
    rng = np.random.default_rng(3)
    w = rng.integers(-50, 100, size=n - 1)
    W = np.full((n, n), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    for i in range(n - 1):
        W[i, i + 1] = w[i]
    D, P, st = orc.fw(W, pred=True)
    assert st == oracle.OK
    c = np.concatenate([[0], np.cumsum(w)])
    for i in range(n):
        for j in range(n):
            if j >= i:
                assert D[i, j] == c[j] - c[i]
                assert P[i, j] == (j - 1 if j > i else -1)
            else:
                assert D[i, j] == INF32 and P[i, j] == -1


@pytest.mark.parametrize("seed", [1, 2])
def test_uniform_weight_is_bfs(orc, seed):
    rng = np.random.default_rng(seed)
    n, w = 70, 13
    W = pins.random_graph(rng, n, 0.05, w, w)
    D, _, _ = orc.fw(W)
    for i in range(0, n, 9):
        h = pins.bfs_hops(W, i)
        assert [None if x == INF32 else x for x in D[i].tolist()] == \
               [None if x is None else w * x for x in h]


# ------------------------------------------------------------- invariants
def test_invariants_and_pred_chains(orc):
    rng = np.random.default_rng(5)
    n = 150
    W = pins.random_graph(rng, n, 0.08, 1, 1000)
    D, P, _ = orc.fw(W, pred=True)
    assert (np.diag(D) == 0).all()
    fin = W != INF32
    assert (D[fin] <= W[fin]).all()
    for _ in range(3000):
        i, j, k = rng.integers(0, n, 3)
        if D[i, k] != INF32 and D[k, j] != INF32:
            assert D[i, j] <= D[i, k] + D[k, j]
    # INF pattern equals reachability
    reach = np.array([[h is not None for h in pins.bfs_hops(W, i)] for i in range(n)])
    assert np.array_equal(D != INF32, reach)
    for i in range(0, n, 11):
        for j in range(n):
            assert pins.walk_pred_chain(W, D, P, i, j)


def test_negative_cycle(orc):
    W = np.full((4, 4), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    W[0, 1], W[1, 2], W[2, 0], W[2, 3] = 2, -5, 1, 1
    assert pins.has_negative_cycle_bruteforce(W)
    _, _, st = orc.fw(W, pred=True)
    assert st == oracle.NEGATIVE_CYCLE
    _, _, st = orc.fw(W.astype(np.float32))
    assert st == oracle.NEGATIVE_CYCLE
    _, _, st = orc.row(W, 0)
    assert st == oracle.NEGATIVE_CYCLE
    W[1, 2] = -2  # cycle weight +1
    assert not pins.has_negative_cycle_bruteforce(W)
    _, _, st = orc.fw(W, pred=True)
    assert st == oracle.OK


def test_input_checks(orc):
    n = 5
    W = np.full((n, n), 3, dtype=np.int32)
    np.fill_diagonal(W, 0)
    assert orc.check(W) == oracle.OK
    W[2, 2] = 1
    assert orc.check(W) == oracle.INVALID_VALUE
    W[2, 2] = 0
    W[1, 3] = orc.weight_bound(n) + 1
    assert orc.check(W) == oracle.INVALID_VALUE
    W[1, 3] = -orc.weight_bound(n)
    assert orc.check(W) == oracle.OK
    assert orc.weight_bound(32769) == (2 ** 28 - 1) // 32768
    F = np.zeros((3, 3), dtype=np.float32)
    F[0, 1] = np.nan
    assert orc.check(F) == oracle.INVALID_VALUE
    F[0, 1] = -np.inf
    assert orc.check(F) == oracle.INVALID_VALUE
    F[0, 1] = np.inf
    assert orc.check(F) == oracle.OK


# -------------------------------------------------- dtype consistency
def test_float_integer_valued_equals_int(orc):
    n = 200
    Wi = synth.single_int32(n, p=0.3, seed=99)
    Wf = synth.single_f32int(n, p=0.3, seed=99)
    assert np.array_equal(np.where(Wi == INF32, np.inf, Wi).astype(np.float32), Wf)
    Di, Pi, _ = orc.fw(Wi, pred=True)
    Df, Pf, _ = orc.fw(Wf, pred=True)
    assert np.array_equal(np.where(Di == INF32, np.inf, Di.astype(np.float64)), Df)
    assert np.array_equal(Pi, Pf)


def test_steps_compose(orc):
    n = 90
    W = synth.single_int32(n, p=0.2, seed=7)
    D1, P1, _ = orc.fw(W, pred=True)
    D2 = W.copy()
    P2 = np.empty_like(D2)
    orc.L.oracle_pred_init_i32(D2.ctypes.data, P2.ctypes.data, n)
    assert orc.fw_steps(D2, 0, 37, P2) == 0
    assert orc.fw_steps(D2, 37, n, P2) == 0
    orc.L.oracle_finalize_i32(D2.ctypes.data, P2.ctypes.data, n)
    assert np.array_equal(D1, D2) and np.array_equal(P1, P2)


# ----------------------------------------------------------- row oracle
@pytest.mark.parametrize("kind", ["int", "pot", "f32", "f32real"])
def test_row_matches_full_and_dijkstra(orc, kind):
    n = 160
    if kind == "int":
        W = synth.single_int32(n, p=0.1, seed=31)
    elif kind == "pot":
        W = synth.potential_int32(n, p=0.1, seed=32)
    elif kind == "f32":
        W = synth.single_f32int(n, p=0.1, seed=33)
    else:
        W = synth.single_f32real(n, p=0.1, seed=34)
    D, P, _ = orc.fw(W, pred=True)
    for src in [0, 1, n // 2, n - 1]:
        dr, pr, st = orc.row(W, src, pred=True)
        assert st == oracle.OK
        if kind == "f32real":
            assert np.allclose(dr, D[src], rtol=1e-12)
        else:
            assert np.array_equal(dr, D[src])
            assert np.array_equal(pr, P[src])
        if kind in ("int", "f32"):
            ref = pins.dijkstra_row(W, src)
            assert [None if (x == INF32 or x == np.inf) else x for x in dr.tolist()] == ref


@pytest.mark.parametrize("n,p,seed", [(160, 0.1, 34), (90, 0.3, 35), (200, 0.03, 36)])
def test_row_real_valued_predecessors_pinned(orc, n, p, seed):
    """Real-valued float32 weights: the row oracle's predecessors equal the
    closed form of the canonical rule evaluated on distances from an
    independent binary-heap Dijkstra (both sides add the float32 weights in
    double precision along the path, so the distances agree exactly), and
    every predecessor chain reproduces its distance."""
    W = synth.single_f32real(n, p=p, lo=0.5, hi=100.0, seed=seed)
    D, _, _ = orc.fw(W)
    for src in [0, 1, n // 3, n - 1]:
        dr, pr, st = orc.row(W, src, pred=True)
        assert st == oracle.OK
        ref = pins.dijkstra_row(W, src)
        assert [None if x == np.inf else x for x in dr.tolist()] == ref
        assert pr.tolist() == pins.canonical_pred_row(W, ref, src)
        P = np.broadcast_to(pr, (n, n))
        for j in range(n):
            assert pins.walk_pred_chain(W, D, P, src, j, tol=1e-9), (src, j)


def test_potential_graph_johnson_identity(orc):
    """Weights b + pi(i) - pi(j): D_w(i,j) = D_b(i,j) + pi(i) - pi(j)."""
    n = 220
    Ww = synth.potential_int32(n, p=0.1, seed=41)
    Wb = synth.single_int32(n, p=0.1, lo=1, hi=1000, seed=41)
    pi = synth.potential(n).astype(np.int64)
    assert (Ww[Ww < 0] > -100).all() and (Ww < 0).any()
    neg_i, neg_j = np.nonzero((Ww < 0))
    assert (neg_i < neg_j).all()
    Dw, _, st = orc.fw(Ww)
    assert st == oracle.OK
    for i in range(0, n, 17):
        db = pins.dijkstra_row(Wb, i)
        for j in range(n):
            if db[j] is None:
                assert Dw[i, j] == INF32
            else:
                assert Dw[i, j] == db[j] + pi[i] - pi[j]
