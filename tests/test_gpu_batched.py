"""GPU parity of the batched fused launch: every graph of a packed ragged
batch against the oracle (and against apsp_solve on the same graph)."""
import numpy as np
import pytest

import pins
import synth
from gpu_util import describe, first_mismatch, gpu_solve

pytestmark = pytest.mark.gpu
INF32 = synth.INF32


def _pack(graphs, dtype):
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    sizes = ns.astype(np.int64) ** 2
    offsets = np.zeros(len(graphs), dtype=np.int64)
    offsets[1:] = np.cumsum((sizes + 3) // 4 * 4)[:-1]
    total = int(offsets[-1] + sizes[-1]) if len(graphs) else 0
    fill = INF32 if dtype == np.int32 else np.inf
    buf = np.full(max(total, 4), fill, dtype=dtype)
    for g, o in zip(graphs, offsets):
        buf[o:o + g.size] = g.ravel()
    return buf, ns, offsets


def _run(graphs, dtype, pred, reps=1, team_config=None):
    import torch

    import paper_1811_01201_amd as apsp
    buf, ns, offs = _pack(graphs, dtype)
    plan = apsp.BatchPlan(ns, offs, "int32" if dtype == np.int32 else "float32", want_pred=pred,
                          team_config=team_config)
    outs = []
    for _ in range(reps):
        d = torch.from_numpy(buf.copy()).cuda()
        p = torch.full(d.shape, -7, dtype=torch.int32, device="cuda") if pred else None
        st = torch.full((len(graphs),), -1, dtype=torch.int32, device="cuda")
        plan.execute(d, p, st)
        torch.cuda.synchronize()
        outs.append((d.cpu().numpy(), p.cpu().numpy() if pred else None, st.cpu().numpy()))
    plan.destroy()
    return outs, ns, offs


def _graphs(kind, sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for b, n in enumerate(sizes):
        p = float(rng.uniform(0.05, 0.9))
        if kind == "int":
            out.append(synth.int32_rows(n, p, 1, 1000, seed, g=b))
        elif kind == "f32":
            out.append(synth.single_f32int(n, p, seed=seed, g=b))
        elif kind == "half":
            W = pins.random_graph(rng, n, p, 0, 3, dtype=np.float32)
            fin = np.isfinite(W) & ~np.eye(n, dtype=bool)
            W[fin] += 0.5
            out.append(W)
        elif kind == "pot":
            out.append(synth.potential_int32(n, p=0.1, seed=seed, g=b))
    return out


SIZES = [1, 2, 5, 16, 17, 33, 63, 64, 65, 100, 127, 128, 129, 190, 255, 256, 257, 300, 511, 512, 513,
         700, 1024, 40, 3, 64, 200]


@pytest.mark.parametrize("kind,pred", [("int", False), ("int", True), ("f32", False), ("f32", True),
                                       ("half", True), ("pot", False), ("pot", True)])
def test_batched_matches_oracle(orc, kind, pred):
    describe(f"batched kind={kind} pred={pred}")
    graphs = _graphs(kind, SIZES, seed=100 + len(kind))
    dtype = np.int32 if kind in ("int", "pot") else np.float32
    (out,), ns, offs = _run(graphs, dtype, pred)
    D, P, st = out
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        D0, P0, s0 = orc.fw(W, pred=pred)
        if dtype == np.float32:
            D0 = D0.astype(np.float32)
        got = D[o:o + n * n].reshape(n, n)
        assert first_mismatch(got, D0) is None, (b, n, first_mismatch(got, D0))
        if pred:
            gp = P[o:o + n * n].reshape(n, n)
            assert first_mismatch(gp, P0) is None, (b, n, first_mismatch(gp, P0))
        assert st[b] == 0


def test_batched_replay_and_negative_cycle_status(orc):
    describe("batched replay + status")
    graphs = _graphs("int", [70, 10, 300, 64, 129], seed=7)
    graphs[1] = graphs[1].copy()
    graphs[1][2, 3], graphs[1][3, 2] = 4, -9
    graphs[2] = graphs[2].copy()
    graphs[2][5, 200], graphs[2][200, 5] = 1, -3
    outs, ns, offs = _run(graphs, np.int32, False, reps=3)
    for D, _, st in outs:
        assert list(st) == [0, 3, 3, 0, 0]
        assert np.array_equal(D, outs[0][0])
    D = outs[0][0]
    for b in (0, 3, 4):
        n = graphs[b].shape[0]
        o = int(offs[b])
        D0, _, _ = orc.fw(graphs[b])
        assert np.array_equal(D[o:o + n * n].reshape(n, n), D0)


def test_batched_deep_negative_cycle_reported():
    """Negative cycles deep enough to wrap 32-bit sums, next to normal graphs."""
    describe("batched deep negative cycle")
    graphs = _graphs("int", [40, 300, 90, 500], seed=9)
    for b in (0, 1, 3):
        n = graphs[b].shape[0]
        W = np.full((n, n), -((2 ** 28 - 1) // (n - 1)), dtype=np.int32)
        np.fill_diagonal(W, 0)
        graphs[b] = W
    outs, ns, offs = _run(graphs, np.int32, False)
    assert list(outs[0][2]) == [3, 3, 0, 3]


@pytest.mark.parametrize("cfg", [None, 0, 1, 2])
def test_batched_large_weights_exact(orc, cfg):
    """Weights near the int32 bound, long paths and large negative weights
    (potentials), mixed with ordinary graphs, in every team configuration:
    every graph exact."""
    describe(f"batched large weights cfg={cfg}")
    rng = np.random.default_rng(21)
    graphs = []
    for n, case in [(20, "big"), (40, "plain"), (150, "long"), (300, "plain"), (70, "neg"), (33, "long"),
                    (129, "big"), (500, "plain")]:
        bound = (2 ** 28 - 1) // (n - 1)
        if case == "plain":
            W = synth.int32_rows(n, 0.3, 1, 1000, 5, g=n)
        elif case == "big":
            W = pins.random_graph(rng, n, 0.3, max(1, bound - 1000), bound)
        elif case == "long":
            W = pins.random_graph(rng, n, 0.08, bound // 2, bound)
        else:
            pot = np.arange(n, dtype=np.int64) * (bound // 3) // (n - 1)
            B = pins.random_graph(rng, n, 0.2, 1, bound // 3)
            W = np.where(B != INF32, B + pot[:, None] - pot[None, :], INF32).astype(np.int32)
            np.fill_diagonal(W, 0)
        graphs.append(W)
    team = None if cfg is None else [cfg] * len(graphs)
    outs, ns, offs = _run(graphs, np.int32, False, team_config=team)
    D, _, st = outs[0]
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        D0, _, st0 = orc.fw(W)
        assert st0 == 0 and st[b] == 0
        assert first_mismatch(D[o:o + n * n].reshape(n, n), D0) is None, (b, n)


def test_batched_equals_single_and_one_shot():
    import torch

    import paper_1811_01201_amd as apsp
    describe("batched == single")
    graphs = _graphs("int", [300, 64, 17, 129], seed=9)
    (out,), ns, offs = _run(graphs, np.int32, True)
    D, P, _ = out
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        Ds, Ps, _ = gpu_solve(W, pred=True)
        assert np.array_equal(D[o:o + n * n].reshape(n, n), Ds)
        assert np.array_equal(P[o:o + n * n].reshape(n, n), Ps)
    buf, ns, offs = _pack(graphs, np.int32)
    d = torch.from_numpy(buf.copy()).cuda()
    apsp.solve_batched(d, ns, offs)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        assert np.array_equal(got[o:o + n * n], D[o:o + n * n])


def test_batched_full_workload_all_graphs(orc):
    """The 4096-graph batch (n uniform in [16, 512], p uniform in [0.05, 0.9],
    int32 weights 1..1000) at full size, in the launch configuration the
    benchmark times: every graph compared with the oracle (one graph per
    host thread)."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("batched full 4096, every graph against the oracle")
    bt = synth.batch()
    buf = bt.pack_int32()
    plan = apsp.BatchPlan(bt.ns, bt.offsets, "int32")
    d = torch.from_numpy(buf).cuda()
    st = torch.full((len(bt.ns),), -1, dtype=torch.int32, device="cuda")
    plan.execute(d, status=st)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    plan.destroy()
    expect = orc.fw_many([bt.graph(b) for b in range(len(bt.ns))])
    for b, (D0, _, s0) in enumerate(expect):
        n = int(bt.ns[b])
        o = int(bt.offsets[b])
        assert s0 == 0
        got = D[o:o + n * n].reshape(n, n)
        assert np.array_equal(got, D0), (b, n, first_mismatch(got, D0))


@pytest.mark.parametrize("cfg", [0, 1, 2])
@pytest.mark.parametrize("kind,pred", [("int", False), ("f32", True), ("pot", True), ("half", True)])
def test_every_team_configuration_matches_oracle(orc, cfg, kind, pred):
    """Each team configuration (tile size / register block) forced for every
    graph gives the oracle's result."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"batched cfg={cfg} kind={kind} pred={pred}")
    sizes = [65, 100, 128, 129, 200, 256, 257, 300, 383, 512, 600, 1024, 30]
    graphs = _graphs(kind, sizes, seed=500 + cfg)
    dtype = np.int32 if kind in ("int", "pot") else np.float32
    buf, ns, offs = _pack(graphs, dtype)
    plan = apsp.BatchPlan(ns, offs, "int32" if dtype == np.int32 else "float32", want_pred=pred,
                          team_config=cfg)
    d = torch.from_numpy(buf.copy()).cuda()
    p = torch.full(d.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    plan.execute(d, p)
    torch.cuda.synchronize()
    D = d.cpu().numpy()
    P = p.cpu().numpy() if pred else None
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        D0, P0, _ = orc.fw(W, pred=pred)
        if dtype == np.float32:
            D0 = D0.astype(np.float32)
        assert first_mismatch(D[o:o + n * n].reshape(n, n), D0) is None, (cfg, n)
        if pred:
            assert first_mismatch(P[o:o + n * n].reshape(n, n), P0) is None, (cfg, n)
    plan.destroy()


def test_autotune_fills_table():
    import paper_1811_01201_amd as apsp
    describe("batched autotune")
    rep = apsp.batch_autotune("int32", False, graphs_per_class=16, reps=1)
    assert sorted(rep) == list(apsp.SIZE_CLASSES)
    for hi, row in rep.items():
        times = [row[c] for c in apsp.TEAM_CONFIGS]
        assert all(t > 0 for t in times)
        # coordinate descent: the kept choice is the fastest trial for its class
        assert row["best"] == apsp.TEAM_CONFIGS[int(np.argmin(times))]


def test_autotune_on_workload_sizes(orc, tmp_path):
    """Tuning on the caller's sizes times only the classes present, keeps the
    fastest trial for each, and leaves results exact."""
    import paper_1811_01201_amd as apsp
    describe("batched autotune on sizes")
    saved = tmp_path / "before.json"
    apsp.tune_save(str(saved))
    try:
        sizes = [70, 100, 300, 310, 40, 20]
        rep = apsp.batch_autotune("int32", False, reps=1, ns=sizes)
        for hi, row in rep.items():
            times = [row[c] for c in apsp.TEAM_CONFIGS]
            if hi in (128, 320):
                assert all(t > 0 for t in times)
                assert row["best"] == apsp.TEAM_CONFIGS[int(np.argmin(times))]
            else:
                assert all(t == 0 for t in times)
        graphs = _graphs("int", sizes, seed=31)
        outs, ns, offs = _run(graphs, np.int32, False)
        D, _, st = outs[0]
        for b, W in enumerate(graphs):
            n = W.shape[0]
            o = int(offs[b])
            D0, _, _ = orc.fw(W)
            assert st[b] == 0 and np.array_equal(D[o:o + n * n].reshape(n, n), D0)
    finally:
        apsp.tune_load(str(saved))


@pytest.mark.parametrize("kind,pred", [("int", False), ("f32", True)])
def test_batched_plan_in_captured_hipgraph(orc, kind, pred):
    """The plan's launches captured once into a hipGraph (torch.cuda.graph)
    and replayed several times, with eager work and synchronizations between
    the replays; every replay equals the eager result and the oracle.  The
    int32 batch holds a graph whose weights rule float32 arithmetic out, so
    both of its launches solve graphs."""
    import torch

    import paper_1811_01201_amd as apsp
    describe(f"batched hipGraph replays {kind} pred={pred}")
    sizes = [300, 17, 129, 64, 513, 200, 5, 256]
    graphs = _graphs(kind, sizes, seed=23)
    if kind == "int":
        n = graphs[2].shape[0]
        graphs[2] = graphs[2].copy()
        graphs[2][4, 9] = (2 ** 23) // (n - 1) + 5  # float32 ruled out for this graph only
    dtype = np.int32 if kind == "int" else np.float32
    buf, ns, offs = _pack(graphs, dtype)
    plan = apsp.BatchPlan(ns, offs, "int32" if kind == "int" else "float32", want_pred=pred)
    pristine = torch.from_numpy(buf).cuda()
    d = pristine.clone()
    p = torch.full(d.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((len(graphs),), -1, dtype=torch.int32, device="cuda")
    plan.execute(d, p, st)
    torch.cuda.synchronize()
    D_e = d.cpu().numpy()
    P_e = p.cpu().numpy() if pred else None
    assert (st.cpu().numpy() == 0).all()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(d, p, st)
    for rep in range(3):
        d.copy_(pristine)
        if pred:
            p.fill_(-7)
        st.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), D_e), rep
        if pred:
            assert np.array_equal(p.cpu().numpy(), P_e), rep
        assert (st.cpu().numpy() == 0).all(), rep
    for b, W in enumerate(graphs):
        n = W.shape[0]
        o = int(offs[b])
        D0, P0, _ = orc.fw(W, pred=pred)
        assert first_mismatch(D_e[o:o + n * n].reshape(n, n), D0) is None, (b, n)
        if pred:
            assert first_mismatch(P_e[o:o + n * n].reshape(n, n), P0) is None, (b, n)
    del g
    plan.destroy()
