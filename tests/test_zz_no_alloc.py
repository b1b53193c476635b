"""apsp_solve_noalloc (the entry point for callers that cannot allocate)
against apsp_solve_ex on the same inputs, bit for bit, through the C ABI:
two calls in a row on one device (the second on a smaller graph, so it runs
on what the first left in the shared static array), every work-memory route
(in-place distances, padded work matrix, float32 arithmetic with its int32
redo words, fp64 predecessor keys, the float32 predecessor route), the
status and arithmetic words, and that the call leaves device memory use
unchanged."""
import numpy as np
import pytest

import paper_1811_01201_amd as apsp
import synth
from gpu_util import describe, first_mismatch

pytestmark = pytest.mark.gpu


def _graph(kind, n, seed):
    if kind == "int":
        return synth.single_int32(n, p=0.3, seed=seed)
    if kind == "pot":
        return synth.potential_int32(n, p=0.1, seed=seed)
    return synth.single_f32int(n, p=0.3, seed=seed)


def _run(fn, W, pred, **kw):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    used = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    fn(d, p, status=st, arith_used=used, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (p.cpu().numpy() if pred else None), int(st.item()), int(used.item())


# (kind, first n, second n, predecessors, options): the second call is smaller
CASES = [
    ("int", 2048, 1000, False, dict(arith=1)),            # in place, then a padded work matrix
    ("pot", 2000, 777, False, dict(arith=2)),             # float32 watch words + int32 redo matrix
    ("f32", 1536, 300, False, dict()),                    # float32 weights
    ("int", 2048, 513, True, dict(arith=1)),              # fp64 predecessor keys
    ("f32", 2048, 1000, True, dict(arith=2)),             # float32 predecessor route
    ("pot", 1800, 640, True, dict(arith=2, block_size=256, phase1=2)),  # route falls back or holds
]


@pytest.mark.parametrize("kind,n1,n2,pred,kw", CASES)
def test_noalloc_equals_solve_ex_two_calls(kind, n1, n2, pred, kw):
    for n in (n1, n2):
        describe(f"noalloc kind={kind} n={n} pred={pred} {kw}")
        W = _graph(kind, n, seed=900 + n)
        Dn, Pn, sn, un = _run(apsp.solve_noalloc, W, pred, **kw)
        De, Pe, se, ue = _run(apsp.solve, W, pred, schedule=1, **kw)
        assert sn == se == 0 and un == ue
        assert first_mismatch(Dn, De) is None, first_mismatch(Dn, De)
        if pred:
            assert first_mismatch(Pn, Pe) is None, first_mismatch(Pn, Pe)


def test_noalloc_status_words_and_validation():
    describe("noalloc status words")
    n = 700
    W = synth.single_int32(n, p=0.05, seed=12)
    W[10, 150], W[150, 10] = 5, -9                         # a negative cycle
    _, _, st, _ = _run(apsp.solve_noalloc, W, False, arith=2)
    assert st == 3
    W = synth.single_int32(n, p=0.2, seed=3)
    W[5, 5] = 1                                            # invalid diagonal: input untouched
    D, _, st, _ = _run(apsp.solve_noalloc, W, True, validate=True)
    assert st == 2 and np.array_equal(D, W)


def test_noalloc_leaves_device_memory_unchanged():
    import torch
    describe("noalloc device memory")
    W1 = synth.single_f32int(1900, p=0.3, seed=1)
    W2 = synth.single_int32(1111, p=0.3, seed=2)
    d1 = torch.from_numpy(W1).cuda()
    d2 = torch.from_numpy(W2).cuda()
    p1 = torch.empty(W1.shape, dtype=torch.int32, device="cuda")
    apsp.solve_noalloc(d1, p1)  # first call on the device looks the array up
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    apsp.solve_noalloc(d2, None, arith=2)
    apsp.solve_noalloc(d1, p1, arith=2)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_noalloc_rejects_beyond_scratch_and_unsupported_options():
    import torch
    describe("noalloc rejections")
    assert apsp.noalloc_scratch_bytes() >= 2048 * 2048 * 8
    big = torch.zeros((2600, 2600), dtype=torch.int32, device="cuda")
    pb = torch.empty_like(big)
    assert apsp.solve_noalloc(big, pb, arith=1, check=False) == apsp.INVALID_ARGUMENT
    small = torch.zeros((100, 100), dtype=torch.int32, device="cuda")
    L = apsp.lib()
    import ctypes
    for field, value in (("schedule", 2), ("use_graph", 1)):
        opt = apsp.Options()
        setattr(opt, field, value)
        assert L.apsp_solve_noalloc(small.data_ptr(), None, 100, apsp.INT32, None, ctypes.byref(opt)) == \
            apsp.INVALID_ARGUMENT
