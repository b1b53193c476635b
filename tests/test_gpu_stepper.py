"""GPU parity of stepped solves (apsp_stepper_*): a solve recorded once and
issued a few rounds at a time, interleaved with other work, must end with
exactly what apsp_solve gives in one go (and the oracle)."""
import numpy as np
import pytest

import synth
from gpu_util import describe, first_mismatch, oracle_expect

pytestmark = pytest.mark.gpu


def _one_shot(W, pred, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, p, status=st, arith_used=used, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (p.cpu().numpy() if pred else None), int(st.item()), int(used.item())


def _stepped(W, pred, rounds_per_step, interleave=False, **kw):
    import torch

    import paper_1811_01201_amd as apsp
    n = W.shape[0]
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    s = apsp.Stepper(n, "int32" if W.dtype == np.int32 else "float32", pred, status=st, arith_used=used, **kw)
    s.begin(d, p)
    total = s.rounds
    other = torch.zeros(1 << 20, device="cuda")
    steps = 0
    while not s.step(rounds_per_step):
        steps += 1
        if interleave:  # unrelated work on the same stream between slices
            other.add_(1.0)
        assert steps <= total + 2
    torch.cuda.synchronize()
    s.destroy()
    return d.cpu().numpy(), (p.cpu().numpy() if pred else None), int(st.item()), int(used.item()), total


CASES = [
    # (n, kind, pred, options)
    (1, "int", False, {}),
    (300, "int", False, {}),
    (700, "f32", False, {"block_size": 256}),
    (1000, "int", True, {}),
    (4200, "int", False, {"arith": 1}),          # int32 arithmetic, two-stream schedule
    (5000, "pot", False, {}),                    # float32 pass + skipped int32 pass
    (4500, "f32", True, {}),                     # float32 distances + key product + skipped recurrence
    (600, "int", True, {"arith": 2, "block_size": 64, "thread_tile": 4}),
]


def _graph(kind, n, seed):
    if kind == "int":
        return synth.single_int32(n, p=0.3, seed=seed)
    if kind == "pot":
        return synth.potential_int32(n, p=0.1, seed=seed)
    return synth.single_f32int(n, p=0.3, seed=seed)


@pytest.mark.parametrize("rps", [1, 3])
@pytest.mark.parametrize("n,kind,pred,opts", CASES)
def test_stepped_equals_one_shot(orc, n, kind, pred, opts, rps):
    describe(f"stepper n={n} {kind} pred={pred} {opts} rounds/step={rps}")
    W = _graph(kind, n, seed=900 + n)
    D1, P1, st1, used1 = _one_shot(W, pred, **opts)
    D, P, st, used, total = _stepped(W, pred, rps, interleave=(rps == 3), **opts)
    assert total >= 1 or n == 0
    assert st == st1 == 0 and used == used1
    assert np.array_equal(D, D1)
    if pred:
        assert np.array_equal(P, P1)
    if n <= 1000:
        D0, P0, _ = oracle_expect(orc, W, pred)
        assert first_mismatch(D, D0) is None
        if pred:
            assert first_mismatch(P, P0) is None


def test_two_steppers_interleaved_on_one_stream(orc):
    import torch

    import paper_1811_01201_amd as apsp
    describe("stepper two interleaved")
    Ws = [synth.single_int32(4200, p=0.2, seed=5), synth.single_f32int(4300, p=0.2, seed=6)]
    outs = []
    steppers = []
    for W in Ws:
        d = torch.from_numpy(W.copy()).cuda()
        s = apsp.Stepper(W.shape[0], "int32" if W.dtype == np.int32 else "float32", False, arith=1)
        s.begin(d)
        steppers.append(s)
        outs.append(d)
    done = [False, False]
    while not all(done):
        for i, s in enumerate(steppers):
            if not done[i]:
                done[i] = s.step(2)
    torch.cuda.synchronize()
    for W, d, s in zip(Ws, outs, steppers):
        s.destroy()
        D1, _, st1, _ = _one_shot(W, False, arith=1)
        assert np.array_equal(d.cpu().numpy(), D1)


def test_stepper_negative_cycle_and_validation():
    import torch

    import paper_1811_01201_amd as apsp
    describe("stepper status")
    n = 500
    W = synth.single_int32(n, p=0.05, seed=21)
    W[10, 150], W[150, 10] = 5, -9
    _, _, st, _, _ = _stepped(W, False, 2)
    assert st == 3
    W2 = synth.single_int32(300, p=0.2, seed=4)
    W2[3, 3] = 1
    d = torch.from_numpy(W2.copy()).cuda()
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    s = apsp.Stepper(300, "int32", False, validate=True, status=status)
    s.begin(d)
    while not s.step(1):
        pass
    torch.cuda.synchronize()
    s.destroy()
    assert int(status.item()) == apsp.INVALID_VALUE and np.array_equal(d.cpu().numpy(), W2)


def test_stepper_begin_while_unfinished_is_refused():
    import torch

    import paper_1811_01201_amd as apsp
    describe("stepper begin refused")
    W = synth.single_int32(400, p=0.3, seed=2)
    d = torch.from_numpy(W.copy()).cuda()
    s = apsp.Stepper(400, "int32", False)
    s.begin(d)
    s.step(1)
    with pytest.raises(apsp.APSPError):
        s.begin(d)
    while not s.step(0):
        pass
    torch.cuda.synchronize()
    D1, _, _, _ = _one_shot(W, False)
    assert np.array_equal(d.cpu().numpy(), D1)
    s.destroy()


def test_stepper_empty_and_reuse():
    """n = 0 records nothing and is done at once; a stepper solves several
    graphs in turn (begin again after the last step)."""
    import torch

    import paper_1811_01201_amd as apsp
    describe("stepper empty and reuse")
    s0 = apsp.Stepper(0, "int32")
    s0.begin(torch.empty((0, 0), dtype=torch.int32, device="cuda"))
    assert s0.rounds == 0 and s0.step(1)
    s0.destroy()
    s = apsp.Stepper(700, "float32", True)
    for seed in (1, 2):
        W = synth.single_f32int(700, p=0.2, seed=seed)
        d = torch.from_numpy(W.copy()).cuda()
        p = torch.empty((700, 700), dtype=torch.int32, device="cuda")
        s.begin(d, p)
        while not s.step(2):
            pass
        torch.cuda.synchronize()
        D1, P1, _, _ = _one_shot(W, True)
        assert np.array_equal(d.cpu().numpy(), D1) and np.array_equal(p.cpu().numpy(), P1)
    s.destroy()
