"""Helpers for the GPU parity tests: run the library through its C ABI on
torch device memory and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

INF32 = 1073741823


def gpu_solve(W: np.ndarray, pred: bool = False, **kw):
    """Copy W to the GPU, solve in place through apsp_solve_ex, copy back.
    Returns (D, P or None, device status)."""
    import torch

    import paper_1811_01201_amd as apsp

    d = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    p = torch.full(W.shape, -7, dtype=torch.int32, device="cuda") if pred else None
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    apsp.solve(d, p, status=st, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), (p.cpu().numpy() if pred else None), int(st.item())


def oracle_expect(orc, W: np.ndarray, pred: bool = False):
    """Oracle result in the library's output dtype (float64 -> float32 is
    exact for integer-valued inputs)."""
    D, P, st = orc.fw(W, pred=pred)
    if W.dtype == np.float32:
        D = D.astype(np.float32)
    return D, P, st


def describe(tag: str):
    print(f"[gpu-case] {tag}", flush=True)
    sys.stdout.flush()


def first_mismatch(A, B):
    idx = np.argwhere(A != B)
    if len(idx) == 0:
        return None
    i, j = idx[0]
    return (int(i), int(j), A[i, j].item(), B[i, j].item(), len(idx))
