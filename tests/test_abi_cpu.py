"""CPU-only checks of the C ABI: the library loads, exports every function
include/apsp.h declares, and rejects bad arguments on the host before
touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1811_01201_amd as apsp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apsp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(apsp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["apsp_solve", "apsp_solve_ex", "apsp_solve_batched", "apsp_batch_plan_create",
                 "apsp_batch_plan_execute", "apsp_batch_plan_destroy", "apsp_server_create",
                 "apsp_server_submit", "apsp_server_wait", "apsp_server_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = apsp.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert missing == []
    out = subprocess.run(["nm", "-D", "--defined-only", apsp.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (apsp_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared_functions()) <= exported


def test_host_side_argument_errors():
    L = apsp.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails before any HIP call
    assert apsp.solve_raw(fake, None, -1, apsp.INT32, None) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(fake, None, 65537, apsp.INT32, None) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(fake, None, 10, 7, None) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(None, None, 10, apsp.INT32, None) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(ctypes.c_void_p(0x1002), None, 10, apsp.INT32, None) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(fake, None, 0, apsp.INT32, None) == apsp.SUCCESS  # n = 0: nothing to do
    bad_bs = apsp.Options(0, 96, 0, 0, 0, 0, None)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, bad_bs) == apsp.INVALID_ARGUMENT
    no_status = apsp.Options(1, 0, 0, 0, 0, 0, None)  # validate needs a status word
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, no_status) == apsp.INVALID_ARGUMENT
    pred256 = apsp.Options(0, 256, 0, 0, 0, 0, None)
    assert apsp.solve_raw(fake, fake, 10, apsp.INT32, None, pred256) == apsp.INVALID_ARGUMENT
    bad_tile = apsp.Options(0, 0, 6, 0, 0, 0, None)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, bad_tile) == apsp.INVALID_ARGUMENT
    tile4_bs128 = apsp.Options(0, 128, 4, 0, 0, 0, None)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, tile4_bs128) == apsp.INVALID_ARGUMENT
    bad_arith = apsp.Options(0, 0, 0, 0, 0, 3, None)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, bad_arith) == apsp.INVALID_ARGUMENT
    bad_schedule = apsp.Options(0, 0, 0, 4, 0, 0, None)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, bad_schedule) == apsp.INVALID_ARGUMENT
    # the single-launch schedule (3): distances, 64-wide blocks, 4 x 4 thread
    # tiles, int32 arithmetic for int32 weights
    for kw in (dict(block_size=128), dict(thread_tile=8), dict(arith=2)):
        o = apsp.Options(0, kw.get("block_size", 0), kw.get("thread_tile", 0), 3, kw.get("use_graph", 0),
                         kw.get("arith", 0), None)
        assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, o) == apsp.INVALID_ARGUMENT, kw
    single = apsp.Options(0, 0, 0, 3, 0, 0, None)
    assert apsp.solve_raw(fake, None, 16385, apsp.INT32, None, single) == apsp.INVALID_ARGUMENT
    assert apsp.solve_raw(fake, fake, 10, apsp.INT32, None, single) == apsp.INVALID_ARGUMENT
    float_arith2 = apsp.Options(0, 0, 0, 3, 0, 2, None)  # arith is ignored for float32 weights
    assert apsp.solve_raw(fake, fake, 10, apsp.FLOAT32, None, float_arith2) == apsp.INVALID_ARGUMENT
    L.apsp_stepper_create.restype = ctypes.c_int
    stp = ctypes.c_void_p()
    assert L.apsp_stepper_create(100, apsp.INT32, 0, ctypes.byref(single), ctypes.byref(stp)) == \
        apsp.INVALID_ARGUMENT
    bad_phase1 = apsp.Options(0, 256, 0, 0, 0, 0, None, None, 4)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, bad_phase1) == apsp.INVALID_ARGUMENT
    # the dataflow closure needs 128- or 256-wide blocks
    for bs in (0, 64):
        flow_bs = apsp.Options(0, bs, 0, 0, 0, 0, None, None, 3)
        assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, flow_bs) == apsp.INVALID_ARGUMENT
    # the blocked diagonal closure needs 256-wide blocks
    blocked_bs128 = apsp.Options(0, 128, 0, 0, 0, 0, None, None, 2)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, blocked_bs128) == apsp.INVALID_ARGUMENT
    blocked_auto = apsp.Options(0, 0, 0, 0, 0, 0, None, None, 2)
    assert apsp.solve_raw(fake, None, 10, apsp.INT32, None, blocked_auto) == apsp.INVALID_ARGUMENT
    # 256-wide blocks with predecessors only on the float32 route (arith 2, or
    # automatically from n = 4096): the fp64-key recurrence holds 8-byte keys
    pred256_keys = apsp.Options(0, 256, 0, 0, 0, 1, None)
    assert apsp.solve_raw(fake, fake, 5000, apsp.INT32, None, pred256_keys) == apsp.INVALID_ARGUMENT
    # the no-allocation entry point: sizes beyond its static array, the
    # two-stream split and graph replay are refused before any HIP call
    L.apsp_solve_noalloc.restype = ctypes.c_int
    assert L.apsp_solve_noalloc(fake, fake, 4000, apsp.INT32, None, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_solve_noalloc(fake, None, 100, apsp.INT32, None, ctypes.byref(bad_schedule)) == \
        apsp.INVALID_ARGUMENT
    split = apsp.Options(0, 0, 0, 2, 0, 0, None)
    assert L.apsp_solve_noalloc(fake, None, 100, apsp.INT32, None, ctypes.byref(split)) == apsp.INVALID_ARGUMENT
    assert L.apsp_solve_noalloc(fake, None, 100, apsp.INT32, None, ctypes.byref(single)) == apsp.INVALID_ARGUMENT
    graph = apsp.Options(0, 0, 0, 0, 1, 0, None)
    assert L.apsp_solve_noalloc(fake, None, 100, apsp.INT32, None, ctypes.byref(graph)) == apsp.INVALID_ARGUMENT
    assert L.apsp_solve_noalloc(fake, None, 0, apsp.INT32, None, None) == apsp.SUCCESS
    assert L.apsp_noalloc_scratch_bytes() >= 2048 * 2048 * 8
    assert L.apsp_status_string(3) == b"negative cycle"
    assert L.apsp_version() >= 100


def test_weight_bound_matches_definition():
    for n in [1, 2, 3, 1024, 8192, 32768, 65536]:
        expect = (2 ** 28 - 1) if n <= 1 else (2 ** 28 - 1) // (n - 1)
        assert apsp.weight_bound(n) == expect


def test_server_host_argument_errors():
    L = apsp.lib()
    t = ctypes.c_uint64()
    req = apsp.Request(None, 10, 0, apsp.INT32, 0, 0)
    assert L.apsp_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == apsp.INVALID_ARGUMENT
    assert L.apsp_server_poll(None, 1) == apsp.INVALID_ARGUMENT
    assert L.apsp_server_wait(None, 1, 0) == apsp.INVALID_ARGUMENT
    assert L.apsp_server_release(None, 1) == apsp.INVALID_ARGUMENT
    assert L.apsp_server_destroy(None) == apsp.INVALID_ARGUMENT
    assert L.apsp_server_create(None, None) == apsp.INVALID_ARGUMENT
    bad = apsp.ServerConfig(-1, 0, 0, 0, 0)
    out = ctypes.c_void_p()
    assert L.apsp_server_create(ctypes.byref(bad), ctypes.byref(out)) == apsp.INVALID_ARGUMENT
    bad = apsp.ServerConfig(0, 0, 0, 0, 2048)
    assert L.apsp_server_create(ctypes.byref(bad), ctypes.byref(out)) == apsp.INVALID_ARGUMENT
    bad = apsp.ServerConfig(0, 0, 0, 0, 0, -1)  # negative slice length
    assert L.apsp_server_create(ctypes.byref(bad), ctypes.byref(out)) == apsp.INVALID_ARGUMENT


def test_batch_plan_host_argument_errors():
    import numpy as np
    L = apsp.lib()
    plan = ctypes.c_void_p()
    ns = np.array([10, 20], dtype=np.int32)
    offs = np.array([0, 100], dtype=np.int64)
    assert L.apsp_batch_plan_create(ns.ctypes.data, offs.ctypes.data, 2, 0, 0, None) == apsp.INVALID_ARGUMENT
    bad = np.array([0, 96], dtype=np.int64)   # 10*10 = 100 > 96: overlapping graphs
    assert L.apsp_batch_plan_create(ns.ctypes.data, bad.ctypes.data, 2, 0, 0,
                                    ctypes.byref(plan)) == apsp.INVALID_ARGUMENT
    bad = np.array([0, 102], dtype=np.int64)  # not a multiple of 4
    assert L.apsp_batch_plan_create(ns.ctypes.data, bad.ctypes.data, 2, 0, 0,
                                    ctypes.byref(plan)) == apsp.INVALID_ARGUMENT
    big = np.array([10, 1025], dtype=np.int32)
    assert L.apsp_batch_plan_create(big.ctypes.data, offs.ctypes.data, 2, 0, 0,
                                    ctypes.byref(plan)) == apsp.INVALID_ARGUMENT
    assert L.apsp_batch_plan_create(ns.ctypes.data, offs.ctypes.data, 2, 5, 0,
                                    ctypes.byref(plan)) == apsp.INVALID_ARGUMENT
    assert L.apsp_batch_plan_execute(None, None, None, None, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_batch_autotune_sizes(None, 3, 0, 0, 0, None) == apsp.INVALID_ARGUMENT
    too_big = np.array([100, 2000], dtype=np.int32)
    assert L.apsp_batch_autotune_sizes(too_big.ctypes.data, 2, 0, 0, 0, None) == apsp.INVALID_ARGUMENT


def test_tuning_table_roundtrip(tmp_path):
    """The batched tuning table saves to JSON and loads back (host only)."""
    p = tmp_path / "t.json"
    apsp.tune_save(str(p))
    text = p.read_text()
    import json
    doc = json.loads(text)
    assert doc["classes"] == [128, 192, 256, 320, 384, 448, 512, 1024]
    assert set(doc["table"]) == {"int32", "float32"}
    doc["table"]["float32"]["pred"] = [2, 1, 0, 2, 1, 0, 2, 1]
    p.write_text(json.dumps(doc))
    apsp.tune_load(str(p))
    assert [apsp.batch_config(n, "float32", True) for n in (100, 150, 200, 300, 350, 400, 500, 900)] == \
        [2, 1, 0, 2, 1, 0, 2, 1]
    assert apsp.batch_config(64, "int32") == -1
    bad = tmp_path / "bad.json"
    bad.write_text('{"table": {"int32": {"dist": [0, 7, 0, 0, 0, 0, 0, 0]}}}')
    with pytest.raises(apsp.APSPError):
        apsp.tune_load(str(bad))
    with pytest.raises(apsp.APSPError):
        apsp.tune_load(str(tmp_path / "missing.json"))
    apsp.tune_load(str(p))  # a valid table stays in force after failed loads
    assert apsp.batch_config(500, "float32", True) == 2


def test_paths_host_argument_errors():
    L = apsp.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.apsp_paths(fake, 10, fake, fake, -1, fake, 4, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_paths(fake, 10, fake, fake, 3, fake, 0, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_paths(None, 10, fake, fake, 3, fake, 4, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_paths(fake, 70000, fake, fake, 3, fake, 4, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_paths(None, 10, None, None, 0, None, 4, None, None) == apsp.SUCCESS  # nothing to do


def test_pred_to_intermediate_host_argument_errors():
    L = apsp.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.apsp_pred_to_intermediate(None, 10, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_pred_to_intermediate(fake, -1, fake, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_pred_to_intermediate(None, 0, None, None) == apsp.SUCCESS


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "single GPU" in r.stderr


def test_stepper_host_argument_errors():
    L = apsp.lib()
    out = ctypes.c_void_p()
    bad = apsp.Options(0, 256, 0, 0, 0, 0, None)  # block 256 with predecessors
    assert L.apsp_stepper_create(100, apsp.INT32, 1, ctypes.byref(bad), ctypes.byref(out)) == apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_create(-1, apsp.INT32, 0, None, ctypes.byref(out)) == apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_create(10, 5, 0, None, ctypes.byref(out)) == apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_create(10, apsp.INT32, 0, None, None) == apsp.INVALID_ARGUMENT
    bad_arith = apsp.Options(0, 0, 0, 0, 0, 4, None)
    assert L.apsp_stepper_create(10, apsp.INT32, 0, ctypes.byref(bad_arith), ctypes.byref(out)) == \
        apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_begin(None, None, None, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_step(None, 1, None) == apsp.INVALID_ARGUMENT
    assert L.apsp_stepper_rounds(None) == -1
    assert L.apsp_stepper_destroy(None) == apsp.INVALID_ARGUMENT
