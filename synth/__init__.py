"""Seeded synthetic inputs for the APSP tests and benchmark.

This module only generates graphs (adjacency matrices with edge weights);
it contains no shortest-path arithmetic and is imported both by the oracle's
tests and by the GPU tests/benchmark.  The counter-based definition lives in
``synth/gen.c`` (SplitMix64 finaliser over a (seed, graph, row, column,
stream) counter); ``u64_py`` restates it in pure Python so tests can pin the
compiled generator to the published SplitMix64 definition.

Workload recipes (shapes, densities and weight ranges of the benchmark
configurations):

* ``single_int32``    dense directed graph, int32 weights, absent = INF32.
* ``single_f32int``   same pattern, float32 holding integers, absent = +inf.
* ``single_f32real``  real-valued float32 weights, absent = +inf.
* ``potential_int32`` integer weights b + pi(i) - pi(j) with
  pi(v) = floor(100 v / (n-1)): negative weights only on i<j edges and no
  negative cycles (every cycle weighs the sum of its b > 0).
* ``batch``           many small graphs of uneven n, packed ragged.
* ``requests``        a Poisson stream of mixed-size solve requests.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

INF32 = 1073741823  # "no edge" for int32 weights (INT32_MAX // 2)
GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
BASE_SEED = 18110120100  # per-configuration seed = BASE_SEED + config index

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "gen.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u64, i64, dbl, vp, i32 = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_int32)
        L.synth_u64.restype = u64
        L.synth_u64.argtypes = [u64] * 5
        L.synth_u01.restype = dbl
        L.synth_u01.argtypes = [u64] * 5
        L.synth_int_rows.restype = None
        L.synth_int_rows.argtypes = [vp, i64, u64, u64, i64, i64, i64, dbl, i64, i64, i32, vp]
        L.synth_intf32_rows.restype = None
        L.synth_intf32_rows.argtypes = [vp, i64, u64, u64, i64, i64, i64, dbl, i64, i64]
        L.synth_realf32_rows.restype = None
        L.synth_realf32_rows.argtypes = [vp, i64, u64, u64, i64, i64, i64, dbl, dbl, dbl]
        _lib = L
    return _lib


# ----------------------------------------------------------------- definition
def _mix64_py(z: int) -> int:
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK64
    z ^= z >> 31
    return z


def u64_py(seed: int, g: int, i: int, j: int, s: int) -> int:
    """Pure-Python restatement of the counter-based generator."""
    h = _mix64_py((seed + GOLDEN * (s + 1)) & MASK64)
    h = _mix64_py((h + GOLDEN * (g + 1)) & MASK64)
    h = _mix64_py((h + GOLDEN * (i + 1)) & MASK64)
    return _mix64_py((h + GOLDEN * (j + 1)) & MASK64)


def u64(seed: int, g: int, i: int, j: int, s: int) -> int:
    return int(lib().synth_u64(seed, g, i, j, s))


def u01(seed: int, g: int, i: int, j: int, s: int) -> float:
    return float(lib().synth_u01(seed, g, i, j, s))


# ------------------------------------------------------------- single graphs
def potential(n: int) -> np.ndarray:
    """pi(v) = floor(100 v / (n-1)): the vertex potential of the
    negative-weight workload."""
    if n <= 1:
        return np.zeros(max(n, 0), dtype=np.int32)
    v = np.arange(n, dtype=np.int64)
    return ((100 * v) // (n - 1)).astype(np.int32)


def int32_rows(n, p, lo, hi, seed, r0=0, r1=None, g=0, absent=INF32, pot=None, out=None):
    r1 = n if r1 is None else r1
    if out is None:
        out = np.empty((r1 - r0, n), dtype=np.int32)
    assert out.dtype == np.int32 and out.flags.c_contiguous and out.shape == (r1 - r0, n)
    potp = None
    if pot is not None:
        pot = np.ascontiguousarray(pot, dtype=np.int32)
        assert pot.shape == (n,)
        potp = pot.ctypes.data
    if r1 > r0 and n > 0:
        lib().synth_int_rows(out.ctypes.data, n, seed, g, n, r0, r1, float(p), int(lo), int(hi),
                             int(absent), potp)
    return out


def single_int32(n, p=0.5, lo=1, hi=1000, seed=BASE_SEED, g=0, out=None):
    return int32_rows(n, p, lo, hi, seed, g=g, out=out)


def potential_int32(n, p=0.1, seed=BASE_SEED + 2, g=0, r0=0, r1=None, out=None):
    """Integer weights b + pi(i) - pi(j), b uniform in [1, 1000]."""
    return int32_rows(n, p, 1, 1000, seed, r0=r0, r1=r1, g=g, pot=potential(n), out=out)


def single_f32int(n, p=0.3, lo=1, hi=1000, seed=BASE_SEED + 1, g=0, r0=0, r1=None, out=None):
    r1 = n if r1 is None else r1
    if out is None:
        out = np.empty((r1 - r0, n), dtype=np.float32)
    assert out.dtype == np.float32 and out.flags.c_contiguous and out.shape == (r1 - r0, n)
    if r1 > r0 and n > 0:
        lib().synth_intf32_rows(out.ctypes.data, n, seed, g, n, r0, r1, float(p), int(lo), int(hi))
    return out


def single_f32real(n, p=0.3, lo=1.0, hi=1000.0, seed=BASE_SEED + 1, g=0, r0=0, r1=None, out=None):
    r1 = n if r1 is None else r1
    if out is None:
        out = np.empty((r1 - r0, n), dtype=np.float32)
    if r1 > r0 and n > 0:
        lib().synth_realf32_rows(out.ctypes.data, n, seed, g, n, r0, r1, float(p), float(lo), float(hi))
    return out


# ------------------------------------------------------------------- batches
@dataclass
class Batch:
    ns: np.ndarray        # int32 [B]
    ps: np.ndarray        # float64 [B]
    offsets: np.ndarray   # int64 [B], element offsets, multiples of 4
    total: int            # elements in the packed buffer
    seed: int

    def graph(self, b: int, absent=INF32) -> np.ndarray:
        n = int(self.ns[b])
        return int32_rows(n, float(self.ps[b]), 1, 1000, self.seed, g=b, absent=absent)

    def pack_int32(self) -> np.ndarray:
        buf = np.full(self.total, INF32, dtype=np.int32)
        for b in range(len(self.ns)):
            n = int(self.ns[b])
            o = int(self.offsets[b])
            view = buf[o:o + n * n].reshape(n, n)
            int32_rows(n, float(self.ps[b]), 1, 1000, self.seed, g=b, out=view)
        return buf


def batch(count=4096, n_lo=16, n_hi=512, p_lo=0.05, p_hi=0.9, seed=BASE_SEED + 3) -> Batch:
    """Graph b: n = n_lo + u64(s=2) mod (n_hi-n_lo+1), p = p_lo + u01(s=3)(p_hi-p_lo)."""
    L = lib()
    ns = np.empty(count, dtype=np.int32)
    ps = np.empty(count, dtype=np.float64)
    span = n_hi - n_lo + 1
    for b in range(count):
        ns[b] = n_lo + L.synth_u64(seed, b, 0, 0, 2) % span
        ps[b] = p_lo + L.synth_u01(seed, b, 0, 0, 3) * (p_hi - p_lo)
    sizes = ns.astype(np.int64) ** 2
    padded = (sizes + 3) // 4 * 4
    offsets = np.zeros(count, dtype=np.int64)
    if count > 1:
        offsets[1:] = np.cumsum(padded)[:-1]
    total = int(padded.sum())
    return Batch(ns=ns, ps=ps, offsets=offsets, total=total, seed=seed)


# ------------------------------------------------------------------ requests
@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    dtype: str        # "int32" | "float32"
    want_pred: bool
    seed: int

    def weights(self) -> np.ndarray:
        if self.dtype == "int32":
            return int32_rows(self.n, 0.2, 1, 1000, self.seed, g=self.rid)
        return single_f32int(self.n, 0.2, 1, 1000, self.seed, g=self.rid)


def requests(count, rate_per_s, n_lo=32, n_hi=8192, seed=BASE_SEED + 4):
    """Poisson arrivals (exponential gaps, s=4), n = round(exp U[ln n_lo, ln n_hi]) (s=5),
    dtype int32/float32 with probability 1/2 (s=6), predecessors with probability 0.3 (s=7)."""
    L = lib()
    out = []
    t = 0.0
    a, b = math.log(n_lo), math.log(n_hi)
    for r in range(count):
        t += -math.log(1.0 - L.synth_u01(seed, r, 0, 0, 4)) / rate_per_s
        n = int(round(math.exp(a + (b - a) * L.synth_u01(seed, r, 0, 0, 5))))
        dt = "int32" if L.synth_u01(seed, r, 0, 0, 6) < 0.5 else "float32"
        wp = L.synth_u01(seed, r, 0, 0, 7) < 0.3
        out.append(Request(r, t, n, dt, wp, seed))
    return out
