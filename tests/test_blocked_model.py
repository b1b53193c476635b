"""CPU model of the GPU schedule (test code only, not the oracle).

The GPU library reaches the oracle's result in a different order:
* blocked rounds over k-blocks of size BS (the paper's Section on data
  locality: diagonal block, then its row and column, then the rest);
* phase 2 written as a min-plus product against the already closed
  diagonal block instead of an in-place k-sequential sweep;
* phase 3 as a min-plus product of the column and row panels;
* int32 sums formed by plain addition, with every value that ends at or
  above 2^29 mapped back to INF afterwards; in 32-bit wrapping arithmetic
  a negative cycle is still reported (a negative diagonal, or a value below
  -2^29, without which no sum can wrap).

These tests check, on small graphs, that each of those choices gives
exactly the oracle's distances and canonical predecessors, for many block
sizes, ragged n and shuffled tile orders."""
import numpy as np
import pytest

import oracle
import pins
import synth

INF32 = pins.INF32
NONE = np.iinfo(np.int32).max


def lexmin_update(D, P, S, C, sat_inf):
    """D,P <- lexmin((D,P), (S,C)); C is ignored where S is 'infinite'."""
    better = (S < D) | ((S == D) & ~sat_inf & (C < P))
    D[better] = S[better]
    P[better] = C[better]


def add_sat(a, b, saturating):
    s = a.astype(np.int64) + b.astype(np.int64)
    if saturating:
        s = np.where((a == INF32) | (b == INF32), INF32, s)
    return s


def product_update(D, P, A, B, PB, saturating):
    """D,P <- lexmin(D,P, min_k (A[:,k] + B[k,:], PB[k,:]))."""
    for k in range(A.shape[1]):
        S = add_sat(A[:, k:k + 1], B[k:k + 1, :], saturating)
        C = np.broadcast_to(PB[k:k + 1, :], S.shape)
        inf = S >= INF32 if saturating else S >= (1 << 29)
        lexmin_update(D, P, S, C, inf)


def close_tile(D, P, saturating):
    """Sequential FW on a square tile, in place (phase 1)."""
    m = D.shape[0]
    for k in range(m):
        a = D[:, k:k + 1].copy()
        b = D[k:k + 1, :].copy()
        pb = P[k:k + 1, :].copy()
        S = add_sat(a, b, saturating)
        inf = S >= INF32 if saturating else S >= (1 << 29)
        lexmin_update(D, P, S, np.broadcast_to(pb, S.shape), inf)


def blocked(W, bs, rng, saturating=True, phase2_product=True):
    n = W.shape[0]
    D = W.astype(np.int64)
    P = np.where((W != INF32) & ~np.eye(n, dtype=bool),
                 np.arange(n)[:, None], NONE).astype(np.int64)
    R = (n + bs - 1) // bs
    blk = [slice(r * bs, min(n, (r + 1) * bs)) for r in range(R)]
    for r in range(R):
        K = blk[r]
        close_tile(D[K, K], P[K, K], saturating)
        others = [q for q in range(R) if q != r]
        rng.shuffle(others)
        for q in others:
            J = blk[q]
            if phase2_product:
                Bold, PBold = D[K, J].copy(), P[K, J].copy()
                product_update(D[K, J], P[K, J], D[K, K], Bold, PBold, saturating)
                Aold = D[J, K].copy()
                product_update(D[J, K], P[J, K], Aold, D[K, K], P[K, K], saturating)
            else:  # the paper's in-place k-sequential block update
                for k in range(K.stop - K.start):
                    kk = K.start + k
                    S = add_sat(D[K, kk:kk + 1], D[kk:kk + 1, J], saturating)
                    C = np.broadcast_to(P[kk:kk + 1, J], S.shape).copy()
                    inf = S >= INF32 if saturating else S >= (1 << 29)
                    lexmin_update(D[K, J], P[K, J], S, C, inf)
                for k in range(K.stop - K.start):
                    kk = K.start + k
                    S = add_sat(D[J, kk:kk + 1], D[kk:kk + 1, K], saturating)
                    C = np.broadcast_to(P[kk:kk + 1, K], S.shape).copy()
                    inf = S >= INF32 if saturating else S >= (1 << 29)
                    lexmin_update(D[J, K], P[J, K], S, C, inf)
        tiles = [(a, b) for a in others for b in others]
        rng.shuffle(tiles)
        for a, b in tiles:
            I, J = blk[a], blk[b]
            product_update(D[I, J], P[I, J], D[I, K], D[K, J], P[K, J], saturating)
    if not saturating:
        D = np.where(D >= (1 << 29), INF32, D)
    P = np.where((P == NONE) | (D == INF32) | np.eye(n, dtype=bool), -1, P)
    return D.astype(np.int32), P.astype(np.int32)


@pytest.mark.parametrize("n,bs", [(1, 4), (2, 1), (7, 3), (23, 5), (40, 8), (41, 16), (37, 37), (50, 64)])
@pytest.mark.parametrize("kind", ["dense", "sparse", "potential", "ties"])
def test_blocked_matches_oracle(orc, n, bs, kind):
    rng = np.random.default_rng(n * 131 + bs)
    if kind == "dense":
        W = pins.random_graph(rng, n, 0.5, 1, 1000)
    elif kind == "sparse":
        W = pins.random_graph(rng, n, 0.06, 1, 1000)
    elif kind == "ties":
        W = pins.random_graph(rng, n, 0.3, 1, 2)
    else:
        W = synth.potential_int32(n, p=0.15, seed=n + bs)
    D0, P0, st = orc.fw(W, pred=True)
    assert st == oracle.OK
    for sat in (True, False):
        D, P = blocked(W, bs, rng, saturating=sat)
        assert np.array_equal(D, D0)
        assert np.array_equal(P, P0)


@pytest.mark.parametrize("n,bs", [(30, 7), (33, 8)])
def test_paper_phase2_equals_product_phase2(orc, n, bs):
    rng = np.random.default_rng(9)
    W = pins.random_graph(rng, n, 0.2, 1, 5)
    D1, P1 = blocked(W, bs, rng, phase2_product=True)
    D2, P2 = blocked(W, bs, rng, phase2_product=False)
    assert np.array_equal(D1, D2) and np.array_equal(P1, P2)
    D0, P0, _ = orc.fw(W, pred=True)
    assert np.array_equal(D1, D0) and np.array_equal(P1, P0)


def test_plain_add_threshold_large_potential(orc):
    """Negative weights, plain addition plus the 2^29 threshold == saturating."""
    n = 120
    W = synth.potential_int32(n, p=0.012, seed=5)
    D0, _, _ = orc.fw(W)
    rng = np.random.default_rng(0)
    D, _ = blocked(W, 32, rng, saturating=False)
    assert np.array_equal(D, D0)
    assert (D0 == INF32).any()


def blocked_wrapping(W, bs, rng):
    """Distances-only blocked schedule in wrapping int32 arithmetic on a
    matrix padded to a multiple of bs with isolated vertices, as the GPU
    runs it.  Returns (D padded, negative-cycle flag as the GPU's wrap-up
    computes it, whether any sum wrapped)."""
    n = W.shape[0]
    ld = (n + bs - 1) // bs * bs
    D = np.full((ld, ld), INF32, dtype=np.int32)
    np.fill_diagonal(D, 0)
    D[:n, :n] = W
    wrapped = False

    def upd(C, A, B):
        nonlocal wrapped
        for k in range(A.shape[1]):
            with np.errstate(over="ignore"):
                S = A[:, k:k + 1] + B[k:k + 1, :]          # int32, wraps
            exact = A[:, k:k + 1].astype(np.int64) + B[k:k + 1, :].astype(np.int64)
            wrapped |= bool((S.astype(np.int64) != exact).any())
            np.minimum(C, S, out=C)

    R = ld // bs
    blk = [slice(r * bs, (r + 1) * bs) for r in range(R)]
    for r in range(R):
        K = blk[r]
        for k in range(bs):  # phase 1, k sequential
            kk = K.start + k
            upd(D[K, K], D[K, kk:kk + 1].copy(), D[kk:kk + 1, K].copy())
        others = [q for q in range(R) if q != r]
        rng.shuffle(others)
        for q in others:
            J = blk[q]
            upd(D[K, J], D[K, K], D[K, J].copy())
            upd(D[J, K], D[J, K].copy(), D[K, K])
        for a in others:
            for b in others:
                upd(D[blk[a], blk[b]], D[blk[a], K], D[K, blk[b]])
    real = D[:n, :n]
    neg = bool((np.diag(real) < 0).any() or (real < -(1 << 29)).any())
    return D, neg, wrapped


@pytest.mark.parametrize("seed", range(12))
def test_wrapping_adds_detect_every_negative_cycle(orc, seed):
    """Plain wrapping int32 adds: within the weight bound every result equals
    the oracle; with negative cycles (also ones deep enough to wrap) the
    wrap-up still reports them: a negative diagonal, or a value below
    -2^29, which a wrap cannot happen without."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    bs = int(rng.integers(2, 9))
    bound = (2 ** 28 - 1) // (n - 1)
    kind = seed % 3
    if kind == 0:    # within the bound, negative weights, no negative cycle
        W = synth.potential_int32(n, p=0.3, seed=seed)
    elif kind == 1:  # one shallow negative cycle
        W = pins.random_graph(rng, n, 0.3, 1, 50)
        W[0, 1], W[1, 0] = 3, -4
    else:            # dense weights at the bound, many deep negative cycles
        W = rng.integers(-bound, bound + 1, size=(n, n)).astype(np.int32)
        np.fill_diagonal(W, 0)
    D0, _, st = orc.fw(W)
    D, neg, wrapped = blocked_wrapping(W, bs, rng)
    assert neg == (st == oracle.NEGATIVE_CYCLE)
    if st == oracle.OK:
        out = np.where(D[:n, :n] >= (1 << 29), INF32, D[:n, :n])
        assert np.array_equal(out, D0)
        assert not wrapped
    if kind == 2:
        assert neg


def test_wrapping_model_does_wrap():
    """The deep negative-cycle case above really exercises wrapping."""
    rng = np.random.default_rng(3)
    n, bs = 32, 4
    bound = (2 ** 28 - 1) // (n - 1)
    W = np.full((n, n), -bound, dtype=np.int32)
    np.fill_diagonal(W, 0)
    _, neg, wrapped = blocked_wrapping(W, bs, rng)
    assert wrapped and neg


def test_float32_eligibility_as_one_unsigned_compare():
    """The batched launches test int32 weights for float32 arithmetic as
    (unsigned)w >= ceil(2^23/(n-1)) and w != INF (2^31 for n <= 1): the same
    predicate as "finite and (negative, or w (n-1) >= 2^23)", on edge values
    of every size class and beyond."""
    rng = np.random.default_rng(3)
    for n in list(range(1, 70)) + [127, 128, 129, 511, 512, 513, 1024, 4097, 65536]:
        lim = 2 ** 31 if n <= 1 else (2 ** 23 + n - 2) // (n - 1)
        near = [lim - 1, lim, lim + 1] if lim < 2 ** 31 else []
        ws = np.array([0, 1, -1, -(2 ** 31), 2 ** 31 - 1, INF32, INF32 - 1, INF32 + 1, 2 ** 23, 2 ** 22] + near +
                      list(rng.integers(-(2 ** 31), 2 ** 31, size=200)), dtype=np.int64)
        ws = ws[(ws >= -(2 ** 31)) & (ws < 2 ** 31)]
        for w in ws.tolist():
            plain = w != INF32 and (w < 0 or w * (n - 1) >= 2 ** 23)
            fast = (w % 2 ** 32) >= lim and w != INF32
            assert plain == fast, (n, w)
