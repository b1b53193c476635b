"""GPU parity of apsp_solve against the CPU oracle (element by element).

Bit-exact for int32 weights and integer-valued float32 weights, distances
and canonical predecessors; relative 1e-6 for real-valued float32 with
predecessor chains checked for validity.  Sizes span one to many tiles with
ragged tails, every block size, both dtypes, negative weights (potential
graphs), unreachable pairs, validation failures and negative cycles."""
import numpy as np
import pytest

import oracle
import pins
import synth
from gpu_util import describe, first_mismatch, gpu_solve, oracle_expect

pytestmark = pytest.mark.gpu
INF32 = synth.INF32

SIZES = [1, 2, 3, 17, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 383, 513, 1000]


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


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["int", "sparse", "pot", "f32"])
@pytest.mark.parametrize("pred", [False, True])
def test_parity_auto_block(orc, n, kind, pred):
    describe(f"single auto n={n} kind={kind} pred={pred}")
    W = _graph(kind, n, seed=1000 + n)
    D0, P0, st0 = oracle_expect(orc, W, pred)
    D, P, st = gpu_solve(W, pred)
    assert st == 0 and st0 == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    if pred:
        assert first_mismatch(P, P0) is None, first_mismatch(P, P0)


# predecessor solves use blocks of at most 128 (8-byte keys); block size 256
# with predecessors is rejected on the host (test_abi_cpu)
@pytest.mark.parametrize("bs,tt,pred", [(64, 4, False), (64, 8, False), (128, 8, False), (256, 8, False),
                                        (64, 4, True), (64, 8, True), (128, 8, True)])
@pytest.mark.parametrize("n,kind", [(130, "int"), (300, "pot"), (512, "f32"), (700, "sparse")])
def test_parity_every_block_size(orc, bs, tt, pred, n, kind):
    describe(f"single bs={bs} tt={tt} n={n} kind={kind} pred={pred}")
    W = _graph(kind, n, seed=77 + n)
    D0, P0, _ = oracle_expect(orc, W, pred)
    D, P, st = gpu_solve(W, pred, block_size=bs, thread_tile=tt)
    assert st == 0
    assert first_mismatch(D, D0) is None, first_mismatch(D, D0)
    if pred:
        assert first_mismatch(P, P0) is None, first_mismatch(P, P0)


def test_config_n1024_dense_int32(orc):
    """n=1024, p=0.5, weights 1..1000, distances only (the small single-graph workload)."""
    describe("single n=1024 p=0.5 int32")
    W = synth.single_int32(1024, p=0.5, seed=synth.BASE_SEED + 0)
    D0, _, _ = orc.fw(W)
    D, _, st = gpu_solve(W)
    assert st == 0 and np.array_equal(D, D0)


def test_real_valued_float32_tolerance(orc):
    describe("single real f32 n=400 pred")
    n = 400
    W = synth.single_f32real(n, p=0.05, lo=0.5, hi=100.0, seed=5)
    D0, _, _ = orc.fw(W)
    D, P, st = gpu_solve(W, pred=False)
    assert st == 0
    fin = np.isfinite(D0)
    assert np.array_equal(np.isfinite(D), fin)
    rel = np.abs(D[fin].astype(np.float64) - D0[fin]) / np.maximum(1.0, np.abs(D0[fin]))
    assert rel.max() <= 1e-6, rel.max()


def test_empty_and_degenerate():
    import torch

    import paper_1811_01201_amd as apsp
    describe("single degenerate")
    d = torch.empty((0, 0), dtype=torch.int32, device="cuda")
    assert apsp.solve(d) == apsp.SUCCESS
    W = np.zeros((1, 1), dtype=np.int32)
    D, P, st = gpu_solve(W, pred=True)
    assert D[0, 0] == 0 and P[0, 0] == -1 and st == 0
    n = 150
    W = np.full((n, n), INF32, dtype=np.int32)
    np.fill_diagonal(W, 0)
    D, P, st = gpu_solve(W, pred=True)
    assert np.array_equal(D, W) and (P == -1).all()


def test_validate_rejects_and_leaves_input():
    describe("single validate")
    n = 90
    W = synth.single_int32(n, p=0.2, seed=3)
    W[5, 5] = 1
    D, _, st = gpu_solve(W, validate=True)
    assert st == 2 and np.array_equal(D, W)
    W = synth.single_int32(n, p=0.2, seed=3)
    W[1, 2] = 10 ** 7  # beyond the weight bound for n=90
    D, _, st = gpu_solve(W, validate=True)
    assert st == 2 and np.array_equal(D, W)
    F = synth.single_f32int(n, p=0.2, seed=3)
    F[3, 4] = np.nan
    D, _, st = gpu_solve(F, validate=True)
    assert st == 2
    W = synth.single_int32(n, p=0.2, seed=3)
    D, _, st = gpu_solve(W, validate=True)
    assert st == 0


@pytest.mark.parametrize("pred", [False, True])
@pytest.mark.parametrize("dtype", ["int", "f32"])
def test_negative_cycle_reported(orc, pred, dtype):
    describe(f"single negative cycle pred={pred} {dtype}")
    n = 200
    W = synth.single_int32(n, p=0.05, seed=11)
    W[10, 150], W[150, 10] = 5, -9
    if dtype == "f32":
        W = np.where(W == INF32, np.inf, W).astype(np.float32)
    _, _, st0 = orc.fw(W)
    assert st0 == oracle.NEGATIVE_CYCLE
    _, _, st = gpu_solve(W, pred=pred)
    assert st == 3


@pytest.mark.parametrize("n", [256, 1024, 4160, 5120])
def test_float32_in_place_negative_cycle_and_clean_diagonal(orc, n):
    """Float32 distances solved in the caller's own buffer (n a multiple of
    the block size) are checked on the diagonal only: a negative cycle
    through two vertices is reported, a graph without one ends with status 0
    and a zero diagonal (and, where the oracle is quick, every distance)."""
    describe(f"float32 in place: negative cycle n={n}")
    W = synth.single_f32int(n, p=0.05, seed=31 + n)
    _, _, st = gpu_solve(W)
    assert st == 0
    a, b = 7, n - 3
    Wn = W.copy()
    Wn[a, b], Wn[b, a] = 5.0, -9.0
    D, _, st = gpu_solve(Wn)
    assert st == 3
    assert D[a, a] < 0 and D[b, b] < 0
    if n <= 1024:
        D0, _, st0 = orc.fw(W)
        D, _, st = gpu_solve(W)
        assert st == 0 and st0 == oracle.OK
        assert np.array_equal(D, D0.astype(np.float32))
    else:
        D, _, st = gpu_solve(W)
        assert st == 0 and np.all(np.diag(D) == 0.0)


def _deep_negative(n):
    """Every off-diagonal weight at minus the bound: negative cycles deep
    enough that plain 32-bit sums wrap long before the solve ends."""
    W = np.full((n, n), -synth_weight_bound(n), dtype=np.int32)
    np.fill_diagonal(W, 0)
    return W


def synth_weight_bound(n):
    return (2 ** 28 - 1) // (n - 1)


@pytest.mark.parametrize("n,bs,tt", [(300, 64, 4), (300, 64, 8), (300, 128, 8), (520, 256, 8), (4096, 0, 0)])
def test_deep_negative_cycle_with_wrapping_sums_reported(n, bs, tt):
    describe(f"single deep negative cycle n={n} bs={bs} tt={tt}")
    W = _deep_negative(n)
    _, _, st = gpu_solve(W, block_size=bs, thread_tile=tt)
    assert st == 3


def _solve_arith(W, arith, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, status=st, arith=arith, arith_used=used, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), int(st.item()), int(used.item())


@pytest.mark.parametrize("n,bs,tt", [(1, 0, 0), (63, 64, 4), (200, 64, 8), (257, 128, 8), (600, 256, 8),
                                     (1000, 0, 0), (5000, 0, 0)])
@pytest.mark.parametrize("kind", ["int", "sparse", "pot"])
def test_float32_arithmetic_exact_for_int32(orc, n, bs, tt, kind):
    """int32 distances computed in float32 arithmetic: bit-exact, and the
    device reports that the float32 result was used."""
    describe(f"single f32 arithmetic n={n} bs={bs} tt={tt} {kind}")
    W = _graph(kind, n, seed=n + 17)
    D, st, used = _solve_arith(W, 2, block_size=bs, thread_tile=tt)
    assert st == 0 and used == 1
    if n <= 1000:
        D0, _, _ = orc.fw(W)
        assert first_mismatch(D, D0) is None
    else:
        for src in (0, n // 2, n - 1):
            dr, _, s = orc.row(W, src)
            assert s == 0 and np.array_equal(D[src], dr)
    D1, _, used1 = _solve_arith(W, 1, block_size=bs, thread_tile=tt)
    assert used1 == 0 and np.array_equal(D, D1)


@pytest.mark.parametrize("case", ["big_weights", "long_paths", "big_negative"])
@pytest.mark.parametrize("n,bs", [(20, 64), (150, 64), (700, 256)])
def test_float32_arithmetic_falls_back_to_int32(orc, case, n, bs):
    """Operands that reach 2^23 make the device redo the solve in int32:
    still exact, and reported as int32 arithmetic."""
    describe(f"single f32 fallback {case} n={n} bs={bs}")
    rng = np.random.default_rng(n)
    bound = (2 ** 28 - 1) // (n - 1)
    if case == "big_weights":      # some single weights above 2^23 (only possible for small n)
        lo = min(bound, 2 ** 23 + 5)
        W = pins.random_graph(rng, n, 0.3, max(1, lo - 1000), max(lo, bound))
    elif case == "long_paths":     # weights below 2^23, path lengths above it
        W = pins.random_graph(rng, n, 0.05, max(1, bound // 2), bound)
    else:                          # negative weights below -2^22, no negative cycle (potentials)
        pot = (np.arange(n, dtype=np.int64) * (bound // 3) // max(1, n - 1))
        B = pins.random_graph(rng, n, 0.2, 1, max(2, bound // 3))
        fin = B != INF32
        W = np.where(fin, B + pot[:, None] - pot[None, :], INF32)
        np.fill_diagonal(W, 0)
        W = W.astype(np.int32)
    D0, _, st0 = orc.fw(W)
    assert st0 == oracle.OK
    D, st, used = _solve_arith(W, 2, block_size=bs)
    assert st == 0
    assert first_mismatch(D, D0) is None
    if case == "big_weights" and (np.abs(W[W != INF32]) >= 2 ** 23).any():
        assert used == 0


@pytest.mark.parametrize("deep", [False, True])
def test_float32_arithmetic_negative_cycle(deep):
    describe(f"single f32 arithmetic negative cycle deep={deep}")
    n = 600
    if deep:
        W = _deep_negative(n)
    else:
        W = synth.single_int32(n, p=0.05, seed=12)
        W[10, 150], W[150, 10] = 5, -9
    _, st, used = _solve_arith(W, 2, block_size=256)
    assert st == 3
    if deep:
        assert used == 0


def test_pred_chains_reproduce_distances():
    describe("single pred chains n=333")
    n = 333
    W = synth.single_int32(n, p=0.02, seed=8)
    D, P, st = gpu_solve(W, pred=True)
    for i in range(0, n, 37):
        for j in range(n):
            assert pins.walk_pred_chain(W, D, P, i, j)


def test_full_size_n8192_f32_pred_sampled_rows(orc):
    """The n=8192 float32 (integer weights 1..1000, p=0.3) distances + predecessors
    workload at full size: sampled rows against the row oracle, exactly."""
    describe("single n=8192 f32 pred sampled")
    n = 8192
    W = synth.single_f32int(n, p=0.3, seed=synth.BASE_SEED + 1)
    D, P, st = gpu_solve(W, pred=True)
    assert st == 0
    for src in [0, 1, 4095, 5000, 8190, 8191]:
        dr, pr, s = orc.row(W, src, pred=True)
        assert s == 0
        assert np.array_equal(D[src], dr.astype(np.float32)), src
        assert np.array_equal(P[src], pr), src
    assert (np.diag(D) == 0).all()


@pytest.mark.parametrize("half", [0, 1])
def test_full_size_n32768_potential_sampled_rows(orc, half):
    """The n=32768 int32 potential-weight workload (negative weights, no
    negative cycle) in the launch configuration the benchmark times
    (automatic block size 256, two-stream schedule, phase 1 as the dataflow
    closure over 32-wide sub-blocks, one kRest launch per round): two rows
    in every other block row (the two halves together cover all 128 block
    rows with 256 rows, at varying offsets inside the block) against the row oracle
    exactly, and properties that hold at any size checked on every element:
    zero diagonal, D <= W, and D(i,j) <= D(i,k) + D(k,j) for 32 values of k
    spread over the block rows."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"single n=32768 int32 potential full size, block rows = {half} mod 2")
    n = 32768
    W = synth.potential_int32(n, p=0.1, seed=synth.BASE_SEED + 2)
    d = torch.from_numpy(W).cuda()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.profile_begin()
    apsp.solve(d, status=st, arith_used=used)
    torch.cuda.synchronize()
    prof = apsp.profile_end()
    assert int(st.item()) == 0
    assert int(used.item()) == 1  # the float32 arithmetic held (exact)
    assert prof["phase1_flow"]["launches"] == n // 256 and prof["phase3_cross"]["launches"] == n // 256 - 1
    srcs = [256 * r + (37 * r + 11 * half + 128 * e) % 256 for r in range(half, n // 256, 2) for e in (0, 1)]
    got = d[torch.tensor(srcs, device="cuda")].cpu().numpy()
    for src, g, (dr, _, s) in zip(srcs, got, orc.rows(W, srcs)):
        assert s == 0
        assert np.array_equal(g, dr), (src, first_mismatch(g[None], dr[None]))
    assert bool((torch.diagonal(d) == 0).all())
    w = torch.from_numpy(W).cuda()
    ks = [1024 * q + (97 * q + half) % 1024 for q in range(32)]
    dk_rows = {k: d[k].long() for k in ks}
    for r0 in range(0, n, 2048):
        blk = d[r0:r0 + 2048]
        assert bool((blk <= w[r0:r0 + 2048]).all()), r0
        b64 = blk.long()
        for k in ks:
            bound = b64[:, k][:, None] + dk_rows[k][None, :]
            assert bool((b64 <= bound).all()), (r0, k)
    del d, w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,rows", [(16384, 48), (32768, 32)])
def test_paper_configuration_float32_pred_large_sampled_rows(orc, n, rows):
    """The paper's configuration (float32 distances plus the path matrix) at
    its larger sizes, integer weights 1..1000 with p = 0.3, in the automatic
    launch configuration (float32 route: 256-wide distance rounds on two
    streams with the blocked phase 1, then the key product): sampled rows
    spread over all block rows against the row oracle, distances and
    canonical predecessors exactly."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"single n={n} float32 + predecessors sampled rows")
    W = synth.single_f32int(n, p=0.3, seed=synth.BASE_SEED + 1 + n)
    d = torch.from_numpy(W).cuda()
    p = torch.full((n, n), -7, dtype=torch.int32, device="cuda")
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, p, status=st, arith_used=used)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(used.item()) == 1
    step = n // rows
    srcs = [step * q + (53 * q) % step for q in range(rows)]
    idx = torch.tensor(srcs, device="cuda")
    gd, gp = d[idx].cpu().numpy(), p[idx].cpu().numpy()
    for src, g, gq, (dr, pr, s) in zip(srcs, gd, gp, orc.rows(W, srcs, pred=True)):
        assert s == 0
        assert np.array_equal(g, dr.astype(np.float32)), (src, first_mismatch(g[None], dr[None]))
        assert np.array_equal(gq, pr), (src, first_mismatch(gq[None], pr[None]))
    assert bool((torch.diagonal(d) == 0).all()) and bool((torch.diagonal(p) == -1).all())
    del d, p
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,kind,pred,alt_bs", [
    (3500, "f32", True, 128), (4096, "int", True, 128), (5000, "int", False, 128), (5700, "pot", False, 256), (5000, "f32", True, 128),
    (6300, "pot", False, 64), (6144, "f32", True, 64),
    (10300, "pot", False, 128), (12288, "int", False, 128), (10240, "f32", True, 128)])
def test_auto_configuration_mid_sizes(orc, n, kind, pred, alt_bs):
    """Sizes around the automatic configuration's switches: the fp64-key
    recurrence on two streams from ld = 3072, predecessors
    by the float32 key product from n = 4096, distance rounds in 64-wide
    blocks with 4 x 4 register blocks up to n = 4864 and 256-wide above (the
    float32 predecessor route: 64-wide to 5888, 128-wide below 7168, 256-wide
    above), phase 1 as the dataflow closure of 128- and 256-wide diagonal
    blocks (n = 10300 pads to ld = 10496).  The automatic route against an
    independent configuration (another block size, int32 or fp64-key
    arithmetic, rounds in order) on every element, and sampled rows against
    the row oracle."""
    describe(f"single auto configuration n={n} {kind} pred={pred}")
    W = _graph(kind, n, seed=n + 17)
    D, P, st = gpu_solve(W, pred)
    D1, P1, st1 = gpu_solve(W, pred, block_size=alt_bs, schedule=1, arith=1)
    assert st == 0 and st1 == 0
    assert first_mismatch(D, D1) is None, first_mismatch(D, D1)
    if pred:
        assert first_mismatch(P, P1) is None, first_mismatch(P, P1)
    for src in (0, n // 2 + 3, n - 1):
        dr, pr, s = orc.row(W, src, pred=pred)
        assert s == 0
        assert np.array_equal(D[src], dr.astype(D.dtype)), src
        if pred:
            assert np.array_equal(P[src], pr), src


def test_maximum_size_n65536(orc):
    """n = 65536, the largest size the library accepts (the paper's largest),
    potential weights with negative edges: one sampled row against the row
    oracle exactly, plus the zero diagonal and D <= W on every element."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("single n=65536 maximum size")
    n = 65536
    W = synth.potential_int32(n, p=0.05, seed=synth.BASE_SEED + 7)
    d = torch.from_numpy(W).cuda()
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    src = 40000
    dr, _, s = orc.row(W, src)
    assert s == 0
    got = d[src].cpu().numpy()
    assert np.array_equal(got, dr), first_mismatch(got[None], dr[None])
    assert bool((torch.diagonal(d) == 0).all())
    for r0 in range(0, n, 4096):
        w = torch.from_numpy(W[r0:r0 + 4096]).cuda()
        assert bool((d[r0:r0 + 4096] <= w).all()), r0
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [100, 257])
def test_half_integer_float32_pred_exact(orc, n):
    """Non-integer weights switch predecessor solves to (distance, predecessor)
    pairs; half-integers keep every float32 sum exact, so distances and the
    canonical predecessors (with many ties) must still match bit for bit."""
    describe(f"single half-integer f32 pred n={n}")
    rng = np.random.default_rng(n)
    W = pins.random_graph(rng, n, 0.3, 0, 2, dtype=np.float32)
    fin = np.isfinite(W) & ~np.eye(n, dtype=bool)
    W[fin] += 0.5
    D0, P0, _ = orc.fw(W, pred=True)
    D, P, st = gpu_solve(W, pred=True)
    assert st == 0
    assert first_mismatch(D, D0.astype(np.float32)) is None
    assert first_mismatch(P, P0) is None, first_mismatch(P, P0)


def test_float32_pred_weight_beyond_key_bound(orc):
    """An integer weight above the key-mode bound also takes the pair path."""
    describe("single f32 pred big weight")
    n = 200
    W = synth.single_f32int(n, p=0.2, seed=12)
    W[3, 7] = 1.0e7
    D0, P0, _ = orc.fw(W, pred=True)
    D, P, st = gpu_solve(W, pred=True)
    assert st == 0
    assert first_mismatch(D, D0.astype(np.float32)) is None
    assert first_mismatch(P, P0) is None


def test_real_valued_float32_pred_chains(orc):
    describe("single real f32 pred n=300")
    n = 300
    W = synth.single_f32real(n, p=0.05, lo=0.5, hi=100.0, seed=6)
    D0, _, _ = orc.fw(W)
    D, P, st = gpu_solve(W, pred=True)
    assert st == 0
    fin = np.isfinite(D0)
    assert np.array_equal(np.isfinite(D), fin)
    rel = np.abs(D[fin].astype(np.float64) - D0[fin]) / np.maximum(1.0, np.abs(D0[fin]))
    assert rel.max() <= 1e-6
    for i in range(0, n, 23):
        for j in range(n):
            assert pins.walk_pred_chain(W, D, P, i, j, tol=1e-5), (i, j)


@pytest.mark.parametrize("n,bs,kind,pred", [(700, 64, "pot", False), (1000, 128, "int", True),
                                            (1536, 256, "f32", False), (1300, 128, "sparse", False),
                                            (900, 64, "f32", True)])
def test_lookahead_schedule_matches_in_order(orc, n, bs, kind, pred):
    """The two-stream lookahead (forced at these sizes with schedule=2; the
    profile shows its next-round panel launches ran) == one stream in round
    order == oracle."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"single schedules n={n} bs={bs} {kind} pred={pred}")
    W = _graph(kind, n, seed=n + bs)
    D0, P0, _ = oracle_expect(orc, W, pred)
    torch.cuda.synchronize()
    apsp.profile_begin()
    Da, Pa, sa = gpu_solve(W, pred, block_size=bs, schedule=2, arith=1)
    prof = apsp.profile_end()
    assert prof["phase3_cross"]["launches"] == (n + bs - 1) // bs - 1, prof["phase3_cross"]
    Db, Pb, sb = gpu_solve(W, pred, block_size=bs, schedule=1, arith=1)
    assert sa == 0 and sb == 0
    assert first_mismatch(Da, D0) is None and first_mismatch(Db, D0) is None
    if pred:
        assert first_mismatch(Pa, P0) is None and first_mismatch(Pb, P0) is None


def test_release_workspace_then_solve_again(orc):
    """apsp_release_workspace frees the work matrices, cached graphs, second
    streams and closure scratch; solves after it make them again and give
    the same result (two-stream split with the closure at n = 5000, on a
    side stream, the default stream and replayed from a captured graph)."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("release_workspace, then solve again")
    n = 5000
    W = _graph("int", n, seed=5000)
    w = torch.from_numpy(W).cuda()
    s = torch.cuda.Stream()

    def solve(stream, **kw):
        d = w.clone()
        st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        apsp.solve(d, status=st, stream=stream, **kw)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        return d.cpu().numpy()

    D1 = solve(s)
    apsp.release_workspace()
    for D in (solve(s), solve(None), solve(s, use_graph=True), solve(s, use_graph=True)):
        assert first_mismatch(D, D1) is None, first_mismatch(D, D1)
    apsp.release_workspace()
    assert first_mismatch(solve(s), D1) is None
    for src in (0, n // 2, n - 1):
        dr, _, st = orc.row(W, src)
        assert st == 0 and np.array_equal(D1[src], dr.astype(D1.dtype)), src


def test_concurrent_solves_on_streams(orc):
    """Solves enqueued on different streams at once (each with its own
    auxiliary stream and work memory) all match the oracle."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("single concurrent streams")
    graphs = [_graph(k, n, seed=5 + n) for k, n in [("int", 900), ("pot", 777), ("f32", 1030), ("int", 513)]]
    streams = [torch.cuda.Stream() for _ in graphs]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    preds = [torch.empty(W.shape, dtype=torch.int32, device="cuda") for W in graphs]
    torch.cuda.synchronize()
    for d, p, s in zip(dev, preds, streams):
        apsp.solve(d, p, stream=s)
    torch.cuda.synchronize()
    for W, d, p in zip(graphs, dev, preds):
        D0, P0, _ = oracle_expect(orc, W, True)
        assert first_mismatch(d.cpu().numpy(), D0) is None
        assert first_mismatch(p.cpu().numpy(), P0) is None


@pytest.mark.parametrize("n,kind,pred", [(1000, "int", False), (600, "f32", True), (4096, "pot", False)])
def test_graph_replays_match_eager(orc, n, kind, pred):
    """use_graph records the launch sequence once and replays it; every replay
    (with other eager work and synchronisations in between) equals the eager
    solve, and the eager solve equals the oracle where the oracle is cheap."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"single graph replays n={n} {kind} pred={pred}")
    W = _graph(kind, n, seed=31 + n)
    De, Pe, se = gpu_solve(W, pred)
    assert se == 0
    if n <= 1024:
        D0, P0, _ = oracle_expect(orc, W, pred)
        assert first_mismatch(De, D0) is None
    stream = torch.cuda.Stream()
    pristine = torch.from_numpy(W).cuda()
    d = torch.empty_like(pristine)
    p = torch.empty(W.shape, dtype=torch.int32, device="cuda") if pred else None
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    other = torch.from_numpy(_graph("int", 300, seed=3)).cuda()
    for rep in range(4):
        with torch.cuda.stream(stream):
            d.copy_(pristine)
            apsp.solve(d, p, status=st, use_graph=True, stream=stream)
        stream.synchronize()
        assert int(st.item()) == 0
        assert first_mismatch(d.cpu().numpy(), De) is None, rep
        if pred:
            assert first_mismatch(p.cpu().numpy(), Pe) is None, rep
        apsp.solve(other.clone())  # eager work between replays
        torch.cuda.synchronize()
