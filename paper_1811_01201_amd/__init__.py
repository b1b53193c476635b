"""MI355X-native blocked Floyd–Warshall all-pairs shortest paths.

Thin ctypes binding over ``libapsp.so`` (C ABI declared in
``include/apsp.h``).  Every step of a solve runs in the library's HIP
kernels; this module only turns torch tensors into device pointers and the
current torch stream into a ``hipStream_t``.  There is no fallback: if the
library is missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libapsp.so")

INF_INT32 = 1073741823
NO_PRED = -1
INT32, FLOAT32 = 0, 1

STATUS = {
    0: "SUCCESS", 1: "INVALID_ARGUMENT", 2: "INVALID_VALUE", 3: "NEGATIVE_CYCLE",
    4: "OUT_OF_MEMORY", 5: "HIP", 6: "QUEUE_FULL", 7: "NOT_READY", 8: "CANCELLED",
    9: "TIMEOUT", 10: "UNKNOWN_TICKET",
}
SUCCESS, INVALID_ARGUMENT, INVALID_VALUE, NEGATIVE_CYCLE, OUT_OF_MEMORY, HIP_ERROR, \
    QUEUE_FULL, NOT_READY, CANCELLED, TIMEOUT, UNKNOWN_TICKET = range(11)


class APSPError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        msg = f"{where}: {STATUS.get(status, status)}"
        if status == HIP_ERROR and _lib is not None:
            msg += f" (hipError {_lib.apsp_last_hip_error()})"
        super().__init__(msg)


class KernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("updates", ctypes.c_double)]


class Profile(ctypes.Structure):
    _fields_ = [("phase1", KernelTime), ("phase2", KernelTime), ("phase3", KernelTime),
                ("other", KernelTime), ("phase3_cross", KernelTime), ("pred_product", KernelTime),
                ("phase1_blocked", KernelTime), ("single_launch", KernelTime), ("phase1_flow", KernelTime)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            k = getattr(self, name)
            out[name] = {"launches": int(k.launches), "total_ms": k.total_ms, "max_ms": k.max_ms,
                         "updates": k.updates}
        return out


class Options(ctypes.Structure):
    _fields_ = [("validate", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("thread_tile", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("arith", ctypes.c_int32),
                ("d_status", ctypes.c_void_p), ("d_arith", ctypes.c_void_p),
                ("phase1", ctypes.c_int32)]


_lib = None


def lib():
    """Load libapsp.so (built by ``python -m paper_1811_01201_amd._build``)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime: load it first so libapsp.so binds to the
        # same libamdhip64 instance (two runtimes in one process cannot share a GPU)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1811_01201_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        L.apsp_solve.argtypes = [vp, vp, i64, c_int, vp]
        L.apsp_solve.restype = c_int
        L.apsp_solve_ex.argtypes = [vp, vp, i64, c_int, vp, ctypes.POINTER(Options)]
        L.apsp_solve_ex.restype = c_int
        L.apsp_status_string.argtypes = [c_int]
        L.apsp_status_string.restype = ctypes.c_char_p
        L.apsp_last_hip_error.restype = c_int
        L.apsp_version.restype = c_int
        L.apsp_weight_bound.argtypes = [i64]
        L.apsp_weight_bound.restype = i64
        L.apsp_release_workspace.restype = c_int
        L.apsp_solve_noalloc.argtypes = [vp, vp, i64, c_int, vp, ctypes.POINTER(Options)]
        L.apsp_solve_noalloc.restype = c_int
        L.apsp_noalloc_scratch_bytes.restype = i64
        L.apsp_profile_begin.restype = c_int
        L.apsp_profile_end.argtypes = [ctypes.POINTER(Profile)]
        L.apsp_profile_end.restype = c_int
        _bind_optional(L)
        _lib = L
    return _lib


def _bind_optional(L):
    """Signatures of the batched and server entry points."""
    vp, i64, i32, c_int, u64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                ctypes.c_uint64)
    table = {
        "apsp_batch_plan_create": ([vp, vp, i32, c_int, i32, ctypes.POINTER(vp)], c_int),
        "apsp_batch_plan_execute": ([vp, vp, vp, vp, vp], c_int),
        "apsp_batch_plan_destroy": ([vp], c_int),
        "apsp_solve_batched": ([vp, vp, vp, vp, i32, c_int, vp], c_int),
        "apsp_server_create": ([vp, ctypes.POINTER(vp)], c_int),
        "apsp_server_submit": ([vp, vp, ctypes.POINTER(u64)], c_int),
        "apsp_server_poll": ([vp, u64], c_int),
        "apsp_server_wait": ([vp, u64, i64], c_int),
        "apsp_server_result": ([vp, u64, ctypes.POINTER(vp), ctypes.POINTER(vp)], c_int),
        "apsp_server_copy_result": ([vp, u64, vp, vp], c_int),
        "apsp_server_release": ([vp, u64], c_int),
        "apsp_server_stats": ([vp, vp], c_int),
        "apsp_server_destroy": ([vp], c_int),
        "apsp_probe_valu": ([i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], c_int),
        "apsp_batch_plan_create_ex": ([vp, vp, i32, c_int, i32, vp, ctypes.POINTER(vp)], c_int),
        "apsp_batch_autotune": ([c_int, i32, i32, i32, ctypes.POINTER(ctypes.c_double)], c_int),
        "apsp_batch_autotune_sizes": ([vp, i32, c_int, i32, i32, ctypes.POINTER(ctypes.c_double)], c_int),
        "apsp_paths": ([vp, i64, vp, vp, i32, vp, i32, vp, vp], c_int),
        "apsp_pred_to_intermediate": ([vp, i64, vp, vp], c_int),
        "apsp_batch_config": ([i64, c_int, i32], i32),
        "apsp_tune_save": ([ctypes.c_char_p], c_int),
        "apsp_tune_load": ([ctypes.c_char_p], c_int),
        "apsp_stepper_create": ([i64, c_int, i32, ctypes.POINTER(Options), ctypes.POINTER(vp)], c_int),
        "apsp_stepper_begin": ([vp, vp, vp, vp], c_int),
        "apsp_stepper_step": ([vp, i32, ctypes.POINTER(i32)], c_int),
        "apsp_stepper_rounds": ([vp], i64),
        "apsp_stepper_destroy": ([vp], c_int),
    }
    for name, (args, res) in table.items():
        f = getattr(L, name, None)
        if f is not None:
            f.argtypes = args
            f.restype = res


def status_string(st: int) -> str:
    return lib().apsp_status_string(st).decode()


def weight_bound(n: int) -> int:
    return int(lib().apsp_weight_bound(n))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.int32:
        return INT32
    if t.dtype == torch.float32:
        return FLOAT32
    raise TypeError(f"dist must be int32 or float32, got {t.dtype}")


def solve(dist, pred=None, *, validate=False, block_size=0, use_graph=False, status=None,
          stream=None, check=True, schedule=0, thread_tile=0, arith=0, arith_used=None,
          phase1=0) -> int:
    """Solve APSP in place on a square device tensor.

    dist   : torch.Tensor [n, n] int32/float32 on the GPU, contiguous (weights in,
             distances out).
    pred   : optional torch.Tensor [n, n] int32 on the same device (output).
    status : optional torch.Tensor [1] int32 on the device, receives the
             data-dependent status (required with validate=True).
    arith  : int32 distance solves: 0 automatic, 1 int32 arithmetic, 2 float32
             arithmetic (exact, checked, int32 redo when needed).  With pred
             (either dtype): 0 automatic, 1 the fp64-key recurrence, 2 float32
             distances + the predecessor key product (exact, checked, the
             recurrence when needed).
    arith_used : optional torch.Tensor [1] int32 on the device, receives 1 if the
             result came from float32 arithmetic (with pred: the product held),
             else 0.
    schedule : 0 automatic, 1 rounds in order on one stream, 2 the two-stream
             split at any size with three rounds or more, 3 all rounds in one
             task-graph launch (distances; 32- or 64-wide blocks; int32 in
             int32 arithmetic, or float32; automatic for distance solves up
             to a padded order of 4096).
    phase1 : 0 automatic (the dataflow closure for 4-byte distances in 128-
             and 256-wide blocks, else the stepwise kernel), 1 the stepwise
             diagonal kernel, 2 the blocked
             closure of the diagonal block (block_size=256), 3 the dataflow
             closure over 32-wide sub-blocks (block_size 128 or 256; 4-byte
             distance rounds, the stepwise kernel for the fp64-key recurrence).
    Returns the host status of the enqueue (raises APSPError unless check=False).
    """
    assert dist.dim() == 2 and dist.shape[0] == dist.shape[1], "dist must be square"
    assert dist.is_cuda and dist.is_contiguous()
    n = dist.shape[0]
    pp = None
    if pred is not None:
        import torch
        assert pred.dtype == torch.int32 and pred.is_cuda and pred.is_contiguous()
        assert tuple(pred.shape) == (n, n)
        pp = pred.data_ptr()
    opt = Options(int(validate), int(block_size), int(thread_tile), int(schedule), int(use_graph), int(arith),
                  status.data_ptr() if status is not None else None,
                  arith_used.data_ptr() if arith_used is not None else None, int(phase1))
    st = lib().apsp_solve_ex(dist.data_ptr(), pp, n, _dtype_code(dist), _stream_ptr(stream),
                             ctypes.byref(opt))
    if check and st != SUCCESS:
        raise APSPError(st, "apsp_solve_ex")
    return st


def solve_noalloc(dist, pred=None, *, validate=False, block_size=0, status=None, stream=None, check=True,
                  thread_tile=0, arith=0, arith_used=None, phase1=0) -> int:
    """solve() through apsp_solve_noalloc: the library allocates nothing (its
    work memory is a static per-device array, see noalloc_scratch_bytes());
    rounds in order on the stream.  Same arguments and results as solve()."""
    assert dist.dim() == 2 and dist.shape[0] == dist.shape[1], "dist must be square"
    assert dist.is_cuda and dist.is_contiguous()
    n = dist.shape[0]
    pp = None
    if pred is not None:
        assert pred.is_cuda and pred.is_contiguous() and tuple(pred.shape) == (n, n)
        pp = pred.data_ptr()
    opt = Options(int(validate), int(block_size), int(thread_tile), 1, 0, int(arith),
                  status.data_ptr() if status is not None else None,
                  arith_used.data_ptr() if arith_used is not None else None, int(phase1))
    st = lib().apsp_solve_noalloc(dist.data_ptr(), pp, n, _dtype_code(dist), _stream_ptr(stream),
                                  ctypes.byref(opt))
    if check and st != SUCCESS:
        raise APSPError(st, "apsp_solve_noalloc")
    return st


def noalloc_scratch_bytes() -> int:
    return int(lib().apsp_noalloc_scratch_bytes())


class Stepper:
    """A solve issued a few rounds at a time (apsp_stepper_*): begin() records
    the launch sequence of solve() for these tensors on a stream, step(k)
    issues the next k rounds (k <= 0: all that is left) and returns True once
    everything is issued.  The final result equals solve()'s bit for bit."""

    def __init__(self, n: int, dtype: str = "int32", want_pred: bool = False, *, validate=False, block_size=0,
                 thread_tile=0, schedule=0, arith=0, status=None, arith_used=None, phase1=0):
        self.n = int(n)
        self.want_pred = bool(want_pred)
        opt = Options(int(validate), int(block_size), int(thread_tile), int(schedule), 0, int(arith),
                      status.data_ptr() if status is not None else None,
                      arith_used.data_ptr() if arith_used is not None else None, int(phase1))
        self._s = ctypes.c_void_p()
        st = lib().apsp_stepper_create(self.n, INT32 if dtype in ("int32", INT32) else FLOAT32,
                                       int(self.want_pred), ctypes.byref(opt), ctypes.byref(self._s))
        if st != SUCCESS:
            raise APSPError(st, "apsp_stepper_create")

    def begin(self, dist, pred=None, stream=None) -> None:
        assert dist.is_cuda and dist.is_contiguous() and tuple(dist.shape) == (self.n, self.n)
        st = lib().apsp_stepper_begin(self._s, dist.data_ptr(), pred.data_ptr() if pred is not None else None,
                                      _stream_ptr(stream))
        if st != SUCCESS:
            raise APSPError(st, "apsp_stepper_begin")

    def step(self, rounds: int = 1) -> bool:
        done = ctypes.c_int32(0)
        st = lib().apsp_stepper_step(self._s, int(rounds), ctypes.byref(done))
        if st != SUCCESS:
            raise APSPError(st, "apsp_stepper_step")
        return bool(done.value)

    @property
    def rounds(self) -> int:
        return int(lib().apsp_stepper_rounds(self._s))

    def destroy(self) -> None:
        if self._s:
            lib().apsp_stepper_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


PATH_TOO_LONG, PATH_BAD_QUERY, PATH_BROKEN = -1, -2, -3


def paths(pred, src, dst, max_len: int, stream=None, check=True):
    """Shortest paths read from a predecessor matrix (apsp_paths).

    pred : torch.Tensor [n, n] int32 on the GPU (from solve(..., pred)).
    src, dst : torch.Tensor [q] int32 on the same device.
    Returns (paths [q, max_len] int32, lengths [q] int32), device tensors:
    lengths[t] vertices, 0 unreachable, PATH_TOO_LONG / PATH_BAD_QUERY /
    PATH_BROKEN otherwise."""
    import torch
    assert pred.dim() == 2 and pred.shape[0] == pred.shape[1] and pred.dtype == torch.int32
    assert pred.is_cuda and pred.is_contiguous()
    src = src.to(device=pred.device, dtype=torch.int32).contiguous()
    dst = dst.to(device=pred.device, dtype=torch.int32).contiguous()
    q = src.numel()
    assert dst.numel() == q
    out = torch.full((q, max(1, int(max_len))), -1, dtype=torch.int32, device=pred.device)
    lengths = torch.empty(q, dtype=torch.int32, device=pred.device)
    st = lib().apsp_paths(pred.data_ptr(), pred.shape[0], src.data_ptr(), dst.data_ptr(), q, out.data_ptr(),
                          int(max_len), lengths.data_ptr(), _stream_ptr(stream))
    if check and st != SUCCESS:
        raise APSPError(st, "apsp_paths")
    return out, lengths


def pred_to_intermediate(pred, out=None, stream=None, check=True):
    """The paper's intermediate-vertex path matrix from a canonical
    predecessor matrix (device tensors; see apsp_pred_to_intermediate)."""
    import torch
    assert pred.dim() == 2 and pred.shape[0] == pred.shape[1] and pred.dtype == torch.int32
    assert pred.is_cuda and pred.is_contiguous()
    if out is None:
        out = torch.empty_like(pred)
    st = lib().apsp_pred_to_intermediate(pred.data_ptr(), pred.shape[0], out.data_ptr(), _stream_ptr(stream))
    if check and st != SUCCESS:
        raise APSPError(st, "apsp_pred_to_intermediate")
    return out


def solve_raw(dist_ptr, pred_ptr, n, dtype_code, stream_ptr, options: Options | None = None) -> int:
    """Direct call with raw integers (used by the ABI tests)."""
    L = lib()
    if options is None:
        return L.apsp_solve(dist_ptr, pred_ptr, n, dtype_code, stream_ptr)
    return L.apsp_solve_ex(dist_ptr, pred_ptr, n, dtype_code, stream_ptr, ctypes.byref(options))


def profile_begin() -> None:
    lib().apsp_profile_begin()


def profile_end() -> dict:
    """Stop per-kernel timing; returns {phase: {launches, total_ms, max_ms, updates}}."""
    prof = Profile()
    st = lib().apsp_profile_end(ctypes.byref(prof))
    if st != SUCCESS:
        raise APSPError(st, "apsp_profile_end")
    return prof.as_dict()


PROBE_KINDS = ("mix_f32", "add_f32", "min3_f32", "add_u32", "min_f32", "mix_i32")


def probe_valu(kind="mix_f32") -> dict:
    """Measured VALU lane-instructions per second of one instruction kind
    (see PROBE_KINDS and apsp_probe_valu; synchronises the device)."""
    r = ctypes.c_double()
    ms = ctypes.c_double()
    st = lib().apsp_probe_valu(PROBE_KINDS.index(kind), ctypes.byref(r), ctypes.byref(ms))
    if st != SUCCESS:
        raise APSPError(st, "apsp_probe_valu")
    return {"lane_instr_per_s": r.value, "elapsed_ms": ms.value}


def release_workspace() -> None:
    st = lib().apsp_release_workspace()
    if st != SUCCESS:
        raise APSPError(st, "apsp_release_workspace")


class BatchPlan:
    """A reusable plan for solving many graphs of uneven size in one launch.

    ns / offsets: host sequences (graph sizes, element offsets of each graph
    in the packed buffers; offsets multiples of 4)."""

    def __init__(self, ns, offsets, dtype: str = "int32", want_pred: bool = False, team_config=None):
        import numpy as np
        self._ns = np.ascontiguousarray(ns, dtype=np.int32)
        self._offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        assert self._ns.shape == self._offsets.shape
        self.batch = int(self._ns.shape[0])
        self.dtype = INT32 if dtype in ("int32", INT32) else FLOAT32
        self.want_pred = bool(want_pred)
        self._plan = ctypes.c_void_p()
        cfg = None
        if team_config is not None:
            self._cfg = np.ascontiguousarray(np.broadcast_to(team_config, self._ns.shape), dtype=np.int8)
            cfg = self._cfg.ctypes.data
        st = lib().apsp_batch_plan_create_ex(self._ns.ctypes.data, self._offsets.ctypes.data, self.batch,
                                             self.dtype, int(self.want_pred), cfg,
                                             ctypes.byref(self._plan))
        if st != SUCCESS:
            raise APSPError(st, "apsp_batch_plan_create")

    def execute(self, packed_dist, packed_pred=None, status=None, stream=None, check=True) -> int:
        st = lib().apsp_batch_plan_execute(
            self._plan, packed_dist.data_ptr(),
            packed_pred.data_ptr() if packed_pred is not None else None,
            status.data_ptr() if status is not None else None, _stream_ptr(stream))
        if check and st != SUCCESS:
            raise APSPError(st, "apsp_batch_plan_execute")
        return st

    def destroy(self) -> None:
        if self._plan:
            lib().apsp_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def solve_batched(packed_dist, ns, offsets, packed_pred=None, stream=None) -> None:
    """One-shot batched solve (plan created, executed and retired by the library)."""
    import numpy as np
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    st = lib().apsp_solve_batched(packed_dist.data_ptr(),
                                  packed_pred.data_ptr() if packed_pred is not None else None,
                                  ns.ctypes.data, offsets.ctypes.data, int(ns.shape[0]),
                                  _dtype_code(packed_dist), _stream_ptr(stream))
    if st != SUCCESS:
        raise APSPError(st, "apsp_solve_batched")


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("batch_max_n", ctypes.c_int32), ("slice_rounds", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("weights", ctypes.c_void_p), ("n", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("dtype", ctypes.c_int), ("want_pred", ctypes.c_int32), ("borrow", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("inflight", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("p50_latency_ms", ctypes.c_double),
                ("p99_latency_ms", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("p50_small_ms", ctypes.c_double), ("p99_small_ms", ctypes.c_double),
                ("p50_large_ms", ctypes.c_double), ("p99_large_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Server:
    """Request loop with continuous batching on the current device (see
    include/apsp.h).  Weights are numpy arrays (copied at submit) or, with
    borrow=True, pinned host tensors that stay alive until completion."""

    def __init__(self, hbm_budget_bytes=0, max_inflight=0, n_streams=0, max_queue=0, batch_max_n=0,
                 slice_rounds=0):
        self._h = ctypes.c_void_p()
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_inflight), int(n_streams), int(max_queue),
                           int(batch_max_n), int(slice_rounds))
        st = lib().apsp_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if st != SUCCESS:
            raise APSPError(st, "apsp_server_create")
        self._dtypes = {}

    def submit(self, weights, want_pred=False, n=None, ld=None, borrow=False, check=True):
        """weights: numpy int32/float32 [n, >=n] C-contiguous rows, or (borrow=True) a
        pinned torch CPU tensor.  Returns the ticket (or the status if check=False)."""
        import numpy as np
        if hasattr(weights, "data_ptr"):
            ptr = weights.data_ptr()
            rows, cols = weights.shape
            dt = INT32 if str(weights.dtype).endswith("int32") else FLOAT32
            stride = weights.stride(0)
        else:
            assert weights.flags.c_contiguous
            ptr = weights.ctypes.data
            rows, cols = weights.shape
            dt = INT32 if weights.dtype == np.int32 else FLOAT32
            stride = cols
        n = rows if n is None else n
        req = Request(ptr, int(n), int(ld if ld is not None else stride), dt, int(want_pred),
                      int(borrow))
        t = ctypes.c_uint64()
        st = lib().apsp_server_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st != SUCCESS:
            if check:
                raise APSPError(st, "apsp_server_submit")
            return st
        self._dtypes[t.value] = (dt, int(n), bool(want_pred))
        return t.value

    def poll(self, ticket) -> int:
        return lib().apsp_server_poll(self._h, ticket)

    def wait(self, ticket, timeout_us=-1) -> int:
        return lib().apsp_server_wait(self._h, ticket, int(timeout_us))

    def device_result(self, ticket):
        d = ctypes.c_void_p()
        p = ctypes.c_void_p()
        st = lib().apsp_server_result(self._h, ticket, ctypes.byref(d), ctypes.byref(p))
        if st != SUCCESS:
            raise APSPError(st, "apsp_server_result")
        return d.value, p.value

    def result(self, ticket):
        """Copy a finished request's (distances, predecessors or None) to numpy."""
        import numpy as np
        dt, n, wp = self._dtypes[ticket]
        D = np.empty((n, n), dtype=np.int32 if dt == INT32 else np.float32)
        P = np.empty((n, n), dtype=np.int32) if wp else None
        st = lib().apsp_server_copy_result(self._h, ticket, D.ctypes.data,
                                           P.ctypes.data if P is not None else None)
        if st != SUCCESS:
            raise APSPError(st, "apsp_server_copy_result")
        return D, P

    def release(self, ticket) -> int:
        st = lib().apsp_server_release(self._h, ticket)
        self._dtypes.pop(ticket, None)
        return st

    def stats(self) -> dict:
        s = ServerStats()
        st = lib().apsp_server_stats(self._h, ctypes.byref(s))
        if st != SUCCESS:
            raise APSPError(st, "apsp_server_stats")
        return s.as_dict()

    def destroy(self) -> None:
        if self._h:
            lib().apsp_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


TEAM_CONFIGS = ("wave_tiles_64", "group_tiles_64", "group_tiles_128", "mixed_128")
SIZE_CLASSES = (128, 192, 256, 320, 384, 448, 512, 1024)


def batch_autotune(dtype="int32", want_pred=False, graphs_per_class=0, reps=0, ns=None) -> dict:
    """Time every batched team configuration per size class on the current
    device and keep the fastest in the library's table.  With ns (graph
    sizes of the intended workload) the synthetic batch has exactly those
    sizes.  Returns {class_upper_bound: {config_name: ms, ..., "best": name}}
    (ms 0 for classes that were not timed)."""
    ms = (ctypes.c_double * (len(SIZE_CLASSES) * len(TEAM_CONFIGS)))()
    dt = INT32 if dtype in ("int32", INT32) else FLOAT32
    if ns is None:
        st = lib().apsp_batch_autotune(dt, int(want_pred), int(graphs_per_class), int(reps), ms)
    else:
        import numpy as np
        arr = np.ascontiguousarray(ns, dtype=np.int32)
        st = lib().apsp_batch_autotune_sizes(arr.ctypes.data, int(arr.size), dt, int(want_pred), int(reps), ms)
    if st != SUCCESS:
        raise APSPError(st, "apsp_batch_autotune")
    out = {}
    for c, hi in enumerate(SIZE_CLASSES):
        row = {TEAM_CONFIGS[k]: ms[c * len(TEAM_CONFIGS) + k] for k in range(len(TEAM_CONFIGS))}
        row["best"] = TEAM_CONFIGS[lib().apsp_batch_config(hi, dt, int(want_pred))]
        out[hi] = row
    return out


def batch_config(n, dtype="int32", want_pred=False) -> int:
    dt = INT32 if dtype in ("int32", INT32) else FLOAT32
    return int(lib().apsp_batch_config(int(n), dt, int(want_pred)))


def tune_save(path: str) -> None:
    st = lib().apsp_tune_save(path.encode())
    if st != SUCCESS:
        raise APSPError(st, "apsp_tune_save")


def tune_load(path: str) -> None:
    st = lib().apsp_tune_load(path.encode())
    if st != SUCCESS:
        raise APSPError(st, "apsp_tune_load")
