"""CPU model of the predecessor key product (test code only, not the oracle).

Given exact distances D, the canonical predecessor is the smallest v != j
with W(v,j) finite and D(i,v) + W(v,j) = D(i,j).  With S bits for a vertex,
    D(i,j) * 2^S + P(i,j) = min over v != j of (D(i,v) 2^S + v) + W(v,j) 2^S,
so one min-plus product of A(i,v) = D(i,v) 2^S + v with B(v,j) = W(v,j) 2^S
(B(j,j) = +inf) yields both.  The library forms it in float32 and accepts
it only under the exactness rule modelled here (numpy float32 adds round to
nearest like v_add_f32):
* every finite weight is an integer below 2^23 in magnitude (B exact),
* no A entry is at or below -2^24, and A entries at or above 2^24 only
  when every weight is non-negative (they then never win),
* each winning key lies below 2^24 in magnitude and decodes to D(i,j).
The tests check that whenever the rule accepts, the decoded predecessors
are the oracle's, and that it does accept the ordinary workloads."""
import math

import numpy as np
import pytest

import oracle
import pins

INF32 = pins.INF32


def key_product_model(W, D):
    """Returns (P, accepted) as the library would: P valid only if accepted."""
    n = W.shape[0]
    S = max(1, math.ceil(math.log2(n))) if n > 1 else 1
    isf = W.dtype == np.float32
    finW = np.isfinite(W) if isf else (W != INF32)
    off = ~np.eye(n, dtype=bool)
    w64 = W.astype(np.float64)
    if (np.abs(w64[finW & off]) >= 2 ** 23).any():
        return None, False
    B = np.where(finW & off, w64 * 2.0 ** S, np.inf).astype(np.float32)
    finD = np.isfinite(D) if D.dtype.kind == "f" else (D != INF32)
    Akey = D.astype(np.float64) * 2.0 ** S + np.arange(n)[None, :]
    Akey = np.where(finD, Akey, np.inf)
    negw = (w64[finW & off] < 0).any()
    if (Akey[finD] <= -2.0 ** 24).any() or ((Akey[finD] >= 2.0 ** 24).any() and negw):
        return None, False
    A = Akey.astype(np.float32)
    C = np.min(A[:, :, None] + B[None, :, :], axis=1)  # float32 sums, then min over v
    P = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        for j in range(n):
            if i == j or not finD[i, j]:
                continue
            key = float(C[i, j])
            if not abs(key) < 2.0 ** 24:
                return None, False
            d = math.floor(key / 2.0 ** S)
            if d != float(D[i, j]):
                return None, False
            P[i, j] = int(key - d * 2.0 ** S)
    return P, True


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("n,p,lo,hi,pot", [(7, 0.5, 1, 9, False), (33, 0.3, 1, 1000, False),
                                           (64, 0.1, 0, 3, False), (65, 0.2, 1, 1000, True),
                                           (90, 0.05, 1, 100, False)])
def test_product_gives_canonical_predecessors(seed, n, p, lo, hi, pot):
    rng = np.random.default_rng(seed * 1000 + n)
    W = pins.random_graph(rng, n, p, lo, hi, potential=pot)
    D, P0, st = oracle.fw(W, pred=True)
    assert st == oracle.OK
    P, ok = key_product_model(W, D)
    assert ok  # small weights and distances: the float32 keys are exact
    assert np.array_equal(P, P0)


def test_product_float32_integer_weights():
    rng = np.random.default_rng(5)
    W = pins.random_graph(rng, 80, 0.3, 1, 1000, dtype=np.float32)
    D, P0, _ = oracle.fw(W, pred=True)
    P, ok = key_product_model(W, D)
    assert ok and np.array_equal(P, P0)


@pytest.mark.parametrize("seed", range(40))
def test_rule_never_accepts_a_wrong_answer(seed):
    """Weights and path lengths straddling the 2^(24-S) limit, with and
    without negative weights: the rule may decline, but what it accepts is
    exact."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 70))
    S = max(1, math.ceil(math.log2(n)))
    lim = 2 ** (24 - S)
    hi = int(rng.choice([lim // 8, lim // 2, lim, 2 * lim, 2 ** 22]))
    pot = bool(seed % 3 == 0)
    W = pins.random_graph(rng, n, float(rng.choice([0.05, 0.2, 0.6])), max(1, hi // 4), hi, potential=pot)
    if pot:  # stretch the potential so that some weights are large and negative
        pi = rng.integers(0, hi, size=n)
        fin = (W != INF32) & ~np.eye(n, dtype=bool)
        W = np.where(fin, W.astype(np.int64) + pi[:, None] - pi[None, :], W).astype(np.int32)
    D, P0, st = oracle.fw(W, pred=True)
    assert st == oracle.OK
    P, ok = key_product_model(W, D)
    if ok:
        assert np.array_equal(P, P0)


def test_rule_declines_long_distances():
    """A path longer than 2^(24-S) cannot be keyed exactly: declined."""
    n = 16  # S = 4, keys hold distances below 2^20
    W = np.full((n, n), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    for v in range(n - 1):
        W[v, v + 1] = 2 ** 19
    D, _, _ = oracle.fw(W, pred=True)
    _, ok = key_product_model(W, D)
    assert not ok
