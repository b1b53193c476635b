"""GPU tests of path reconstruction (apsp_paths) from the canonical
predecessor matrix: every path is the CPU walk of the same matrix, starts at
the source, ends at the target, uses only edges and adds up to the distance
the oracle gives; unreachable pairs, trivial paths, short buffers, bad
queries and a matrix that was not produced by a solve are reported."""
import numpy as np
import pytest

import synth
from gpu_util import describe

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _cpu_walk(P, s, d, n, max_len):
    if not (0 <= s < n and 0 <= d < n):
        return None, -2
    if s != d and P[s, d] < 0:
        return None, 0
    out, v = [], d
    for step in range(n + 1):
        if len(out) >= max_len:
            return None, -1
        out.append(v)
        if v == s:
            return out[::-1], len(out)
        u = int(P[s, v])
        if u < 0 or u >= n or step + 1 >= n:
            return None, -3
        v = u
    return None, -3


@pytest.mark.parametrize("kind", ["int", "f32", "pot"])
def test_paths_match_cpu_walk_and_distances(orc, kind):
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"paths {kind}")
    n = 300
    if kind == "int":
        W = synth.single_int32(n, p=0.02, seed=41)
    elif kind == "pot":
        W = synth.potential_int32(n, p=0.02, seed=42)
    else:
        W = synth.single_f32int(n, p=0.02, seed=43)
    d = torch.from_numpy(W).cuda()
    p = torch.empty((n, n), dtype=torch.int32, device="cuda")
    apsp.solve(d, p)
    D0, P0, _ = orc.fw(W, pred=True)
    rng = np.random.default_rng(7)
    q = 2000
    src = rng.integers(0, n, q).astype(np.int32)
    dst = rng.integers(0, n, q).astype(np.int32)
    src[:5] = dst[:5]  # trivial paths
    src[5], dst[5] = -1, 3  # bad query
    dst[6] = n
    for max_len in (n, 4):
        paths, lengths = apsp.paths(p, torch.from_numpy(src), torch.from_numpy(dst), max_len)
        torch.cuda.synchronize()
        paths, lengths = paths.cpu().numpy(), lengths.cpu().numpy()
        for t in range(q):
            ref, ln = _cpu_walk(P0, int(src[t]), int(dst[t]), n, max_len)
            assert lengths[t] == ln, (t, src[t], dst[t], lengths[t], ln)
            if ln > 0:
                path = paths[t, :ln]
                assert list(path) == ref
                total = sum(W[path[h], path[h + 1]].item() for h in range(ln - 1))
                assert total == D0[src[t], dst[t]]
        if max_len == n:
            reach = (D0[src[7:], dst[7:]] < (INF32 if kind != "f32" else np.inf))
            assert (lengths[7:][reach] > 0).all() and (lengths[7:][~reach] == 0).all()


def test_paths_broken_matrix_is_reported():
    """A matrix with a predecessor cycle: every walk stops within n steps."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("paths broken matrix")
    n = 50
    P = np.full((n, n), -1, dtype=np.int32)
    P[0, 5], P[0, 6] = 6, 5  # 5 <- 6 <- 5 ... never reaches 0
    P[0, 7] = 99             # out of range
    p = torch.from_numpy(P).cuda()
    src = torch.tensor([0, 0, 0], dtype=torch.int32)
    dst = torch.tensor([5, 7, 8], dtype=torch.int32)
    paths, lengths = apsp.paths(p, src, dst, n)
    torch.cuda.synchronize()
    assert lengths.cpu().tolist() == [apsp.PATH_BROKEN, apsp.PATH_BROKEN, 0]


def _rebuild(Pm, i, j, calls):
    """Recursive rebuild from an intermediate-vertex matrix (the paper's form)."""
    calls[0] += 1
    assert calls[0] <= 2 * Pm.shape[0]
    m = int(Pm[i, j])
    if m < 0:
        return [i, j]
    left = _rebuild(Pm, i, m, calls)
    right = _rebuild(Pm, m, j, calls)
    return left + right[1:]


@pytest.mark.parametrize("kind", ["int", "pot"])
def test_intermediate_vertex_matrix_rebuilds_shortest_paths(orc, kind):
    """The paper's form of P: recursive rebuilding terminates within 2n - 3
    calls and gives a path of edges whose weights add up to the oracle's
    distance, ending with the same last hop as the canonical predecessor."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"paths intermediate matrix {kind}")
    n = 200
    W = synth.single_int32(n, p=0.03, seed=51) if kind == "int" else synth.potential_int32(n, p=0.03, seed=52)
    d = torch.from_numpy(W).cuda()
    p = torch.empty((n, n), dtype=torch.int32, device="cuda")
    apsp.solve(d, p)
    Pm = apsp.pred_to_intermediate(p).cpu().numpy()
    D0, P0, _ = orc.fw(W, pred=True)
    rng = np.random.default_rng(3)
    src = rng.integers(0, n, 500).astype(np.int32)
    dst = rng.integers(0, n, 500).astype(np.int32)
    paths, lengths = apsp.paths(p, torch.from_numpy(src), torch.from_numpy(dst), n)
    paths, lengths = paths.cpu().numpy(), lengths.cpu().numpy()
    for t in range(500):
        i, j = int(src[t]), int(dst[t])
        if i == j or D0[i, j] >= INF32:
            assert Pm[i, j] == -1
            continue
        rebuilt = _rebuild(Pm, i, j, [0])
        assert rebuilt[0] == i and rebuilt[-1] == j
        assert all(W[rebuilt[h], rebuilt[h + 1]] != INF32 for h in range(len(rebuilt) - 1))
        assert sum(W[rebuilt[h], rebuilt[h + 1]] for h in range(len(rebuilt) - 1)) == D0[i, j]
        assert rebuilt[-2] == paths[t, lengths[t] - 2]  # the canonical last hop
    assert np.array_equal(Pm, np.where((P0 < 0) | (P0 == np.arange(n)[:, None]), -1, P0))
