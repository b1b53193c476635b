"""Floyd–Warshall oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library: the two share no code.

``oracle_fw.c`` is the plain triple-loop recurrence of the paper's Section
"Floyd-Warshall Algorithm" (see the header of that file for every reading
taken where the paper is silent).  This module only marshals numpy arrays
to it:

* int32 weights are solved in int32 storage with int64 sums saturating at
  INF = 1073741823;
* float weights are widened to float64 and solved in float64 (exact for
  integer-valued float32 inputs, the reference value for real-valued ones).

Status codes: 0 ok, 2 invalid value, 3 negative cycle, 4 out of memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

INF32 = 1073741823
OK, INVALID_VALUE, NEGATIVE_CYCLE, NOMEM = 0, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle_fw.c")
_lib = None


def build(verbose: bool = False, src: str = SRC_PATH, out: str = LIB_PATH) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP over rows)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build_native(out_dir: str) -> str:
    """The same source built for the host it runs on (gcc -O3 -march=native,
    OpenMP over rows), for the benchmark's CPU baseline; tests use build()."""
    out = os.path.join(out_dir, "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-fopenmp", "-o", out,
                           SRC_PATH, "-lm"])
    return out


def load(path: str = LIB_PATH):
    L = ctypes.CDLL(path)
    vp, i64, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    for name, args in [
        ("oracle_check_i32", [vp, i64]),
        ("oracle_check_f32", [vp, i64]),
        ("oracle_fw_i32", [vp, vp, i64, c_int]),
        ("oracle_fw_f64", [vp, vp, i64, c_int]),
        ("oracle_fw_i32_steps", [vp, vp, i64, i64, i64, c_int]),
        ("oracle_fw_f64_steps", [vp, vp, i64, i64, i64, c_int]),
        ("oracle_pred_init_i32", [vp, vp, i64]),
        ("oracle_pred_init_f64", [vp, vp, i64]),
        ("oracle_finalize_i32", [vp, vp, i64]),
        ("oracle_finalize_f64", [vp, vp, i64]),
        ("oracle_row_i32", [vp, i64, i64, vp, vp]),
        ("oracle_row_f64", [vp, i64, i64, vp, vp]),
    ]:
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int
    L.oracle_weight_bound.argtypes = [i64]
    L.oracle_weight_bound.restype = i64
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = load(LIB_PATH)
    return _lib


def default_threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _ptr(a):
    return None if a is None else a.ctypes.data


class Oracle:
    """Thin wrapper over one loaded oracle library (tests may load a variant)."""

    def __init__(self, L=None):
        self.L = L if L is not None else lib()

    def weight_bound(self, n: int) -> int:
        return int(self.L.oracle_weight_bound(n))

    def check(self, W: np.ndarray) -> int:
        n = W.shape[0]
        if W.dtype == np.int32:
            return self.L.oracle_check_i32(_ptr(np.ascontiguousarray(W)), n)
        return self.L.oracle_check_f32(_ptr(np.ascontiguousarray(W, dtype=np.float32)), n)

    def fw(self, W: np.ndarray, pred: bool = False, threads: int | None = None):
        """Solve APSP on a square matrix.  Returns (D, P or None, status).

        int32 input -> int32 D; float input -> float64 D."""
        threads = threads or default_threads()
        W = np.asarray(W)
        assert W.ndim == 2 and W.shape[0] == W.shape[1]
        n = W.shape[0]
        P = np.empty((n, n), dtype=np.int32) if pred else None
        if W.dtype == np.int32:
            D = np.array(W, dtype=np.int32, order="C", copy=True)
            st = self.L.oracle_fw_i32(_ptr(D), _ptr(P), n, threads)
        else:
            D = np.array(W, dtype=np.float64, order="C", copy=True)
            st = self.L.oracle_fw_f64(_ptr(D), _ptr(P), n, threads)
        return D, P, int(st)

    def fw_steps(self, D: np.ndarray, k0: int, k1: int, P: np.ndarray | None = None,
                 threads: int | None = None) -> int:
        """Run iterations k0..k1-1 of the recurrence in place (no init/finalize)."""
        threads = threads or default_threads()
        n = D.shape[0]
        assert D.flags.c_contiguous
        if D.dtype == np.int32:
            return int(self.L.oracle_fw_i32_steps(_ptr(D), _ptr(P), n, k0, k1, threads))
        assert D.dtype == np.float64
        return int(self.L.oracle_fw_f64_steps(_ptr(D), _ptr(P), n, k0, k1, threads))

    def row(self, W: np.ndarray, src: int, pred: bool = False):
        """Row src of the APSP result by single-source label correcting.
        Returns (drow, prow or None, status); float input gives float64 drow."""
        n = W.shape[0]
        prow = np.empty(n, dtype=np.int32) if pred else None
        if W.dtype == np.int32:
            W = np.ascontiguousarray(W)
            drow = np.empty(n, dtype=np.int32)
            st = self.L.oracle_row_i32(_ptr(W), n, src, _ptr(drow), _ptr(prow))
        else:
            W = np.ascontiguousarray(W, dtype=np.float32)
            drow = np.empty(n, dtype=np.float64)
            st = self.L.oracle_row_f64(_ptr(W), n, src, _ptr(drow), _ptr(prow))
        return drow, prow, int(st)

    def rows(self, W: np.ndarray, srcs, pred: bool = False, workers: int | None = None):
        """row() for several sources at once, one source per host thread (the
        C routine runs without the GIL).  Returns a list of (drow, prow, status)
        in the order of srcs."""
        from concurrent.futures import ThreadPoolExecutor
        W = np.ascontiguousarray(W) if W.dtype == np.int32 else np.ascontiguousarray(W, dtype=np.float32)
        workers = workers or default_threads()
        with ThreadPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(lambda s: self.row(W, int(s), pred=pred), list(srcs)))

    def fw_many(self, graphs, pred: bool = False, workers: int | None = None):
        """fw() for many independent graphs, one graph per host thread (each
        solve single-threaded).  Returns a list of (D, P or None, status)."""
        from concurrent.futures import ThreadPoolExecutor
        workers = workers or default_threads()
        with ThreadPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(lambda W: self.fw(W, pred=pred, threads=1), list(graphs)))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def fw(W, pred=False, threads=None):
    return default().fw(W, pred=pred, threads=threads)


def row(W, src, pred=False):
    return default().row(W, src, pred=pred)


def check(W):
    return default().check(W)
