"""Independent reference computations used to pin the oracle (and, through it,
the GPU library).  None of these share code with ``oracle/``: they are other
algorithms (path enumeration, Dijkstra, Bellman–Ford, BFS) or closed forms
that the shortest-path definition fixes.

Conventions match the library's output: int32 "no path" is INF32, float is
+inf; predecessors are the canonical ones (smallest vertex just before j on
a shortest i->j path), -1 on the diagonal and for unreachable pairs.
"""
from __future__ import annotations

import heapq
import itertools

import numpy as np

INF32 = 1073741823


def _is_inf(x) -> bool:
    return x == INF32 or x == float("inf")


def edges_of(W):
    n = W.shape[0]
    out = []
    for u in range(n):
        for v in range(n):
            if u != v and not _is_inf(W[u, v]):
                out.append((u, v, W[u, v].item()))
    return out


# ------------------------------------------------------------ brute force
def brute_force(W):
    """Enumerate every simple path (n <= 7).  Returns (D, P) with D as Python
    numbers (None = unreachable) and the canonical predecessor."""
    n = W.shape[0]
    D = [[None] * n for _ in range(n)]
    P = [[-1] * n for _ in range(n)]
    for i in range(n):
        D[i][i] = 0
        # DFS over simple paths from i
        stack = [(i, 0, (i,))]
        best = {}
        while stack:
            u, w, path = stack.pop()
            for v in range(n):
                if v in path or _is_inf(W[u, v]):
                    continue
                wv = w + W[u, v].item()
                key = (wv, u)
                if v not in best or key < best[v]:
                    best[v] = key
                stack.append((v, wv, path + (v,)))
        for v, (wv, pv) in best.items():
            D[i][v] = wv
            P[i][v] = pv
    return D, P


def has_negative_cycle_bruteforce(W) -> bool:
    n = W.shape[0]
    for r in range(1, n + 1):
        for cyc in itertools.permutations(range(n), r):
            if cyc[0] != min(cyc):
                continue
            tot = 0
            ok = True
            for a, b in zip(cyc, cyc[1:] + cyc[:1]):
                if a == b:
                    ok = ok and True
                    continue
                if _is_inf(W[a, b]):
                    ok = False
                    break
                tot += W[a, b].item()
            if ok and r > 1 and tot < 0:
                return True
    return False


# --------------------------------------------------------------- Dijkstra
def dijkstra_row(W, src):
    """Binary-heap Dijkstra on non-negative weights; returns python list with
    None for unreachable."""
    n = W.shape[0]
    dist = [None] * n
    dist_tent = {src: 0}
    heap = [(0, src)]
    done = [False] * n
    while heap:
        d, u = heapq.heappop(heap)
        if done[u]:
            continue
        done[u] = True
        dist[u] = d
        row = W[u]
        for v in range(n):
            if v == u or done[v] or _is_inf(row[v]):
                continue
            nd = d + row[v].item()
            if v not in dist_tent or nd < dist_tent[v]:
                dist_tent[v] = nd
                heapq.heappush(heap, (nd, v))
    return dist


def bellman_ford_row(W, src):
    """Bellman–Ford over the edge list; returns (dist list with None, neg_cycle)."""
    n = W.shape[0]
    E = edges_of(W)
    dist = [None] * n
    dist[src] = 0
    for _ in range(n - 1):
        changed = False
        for u, v, w in E:
            if dist[u] is not None and (dist[v] is None or dist[u] + w < dist[v]):
                dist[v] = dist[u] + w
                changed = True
        if not changed:
            break
    neg = any(dist[u] is not None and (dist[v] is None or dist[u] + w < dist[v]) for u, v, w in E)
    return dist, neg


def canonical_pred_row(W, drow, src):
    """P(src,j) = min{v != j : W(v,j) finite, d(src,v) + W(v,j) == d(src,j)}."""
    n = W.shape[0]
    prow = [-1] * n
    for j in range(n):
        if j == src or drow[j] is None:
            continue
        for v in range(n):
            if v == j or drow[v] is None or _is_inf(W[v, j]):
                continue
            if drow[v] + W[v, j].item() == drow[j]:
                prow[j] = v
                break
    return prow


def bfs_hops(W, src):
    n = W.shape[0]
    hops = [None] * n
    hops[src] = 0
    frontier = [src]
    while frontier:
        nxt = []
        for u in frontier:
            for v in range(n):
                if v != u and hops[v] is None and not _is_inf(W[u, v]):
                    hops[v] = hops[u] + 1
                    nxt.append(v)
        frontier = nxt
    return hops


def to_matrix(rows, dtype):
    """List-of-lists with None -> numpy with INF32 / +inf."""
    n = len(rows)
    if dtype == np.int32:
        A = np.full((n, n), INF32, dtype=np.int64)
    else:
        A = np.full((n, n), np.inf, dtype=np.float64)
    for i, r in enumerate(rows):
        for j, x in enumerate(r):
            if x is not None:
                A[i, j] = x
    return A


# ------------------------------------------------------------ invariants
def walk_pred_chain(W, D, P, i, j, tol=0.0):
    """Follow P from j back to i; check it reaches i in <= n-1 hops, that every
    hop is an edge, and that the edge weights add up to D[i,j]."""
    n = W.shape[0]
    if i == j:
        return P[i, j] == -1
    if _is_inf(D[i, j]):
        return P[i, j] == -1
    total = 0.0 if W.dtype != np.int32 else 0
    v = j
    for _ in range(n):
        u = int(P[i, v])
        if u < 0 or _is_inf(W[u, v]):
            return False
        total += W[u, v].item()
        v = u
        if v == i:
            if tol == 0.0:
                return total == D[i, j].item()
            return abs(total - D[i, j].item()) <= tol * max(1.0, abs(D[i, j].item()))
    return False


# ------------------------------------------------------------ small graphs
def random_graph(rng, n, p, lo, hi, dtype=np.int32, potential=False):
    W = np.full((n, n), INF32 if dtype == np.int32 else np.inf,
                dtype=np.int32 if dtype == np.int32 else np.float32)
    mask = rng.random((n, n)) < p
    w = rng.integers(lo, hi + 1, size=(n, n))
    if potential:
        pi = rng.integers(0, 50, size=n)
        w = w + pi[:, None] - pi[None, :]
    W[mask] = w[mask]
    np.fill_diagonal(W, 0)
    return W
