"""Host-only C++ parts of the library under sanitizers (CPU, no GPU).

* tests/cpp/test_server_core.cpp: the serving core (admission by
  device-memory budget, arrival order, coalescing, completion, waits, pinned
  results racing with release, cancellation) with a fake executor, built
  with ThreadSanitizer and, separately, AddressSanitizer.
* tests/cpp/test_batch_host.cpp: the batched plans' argument checks,
  ordering and metadata image over seeded random batches, with a bounds
  model of every index the batched kernels compute, built with
  AddressSanitizer + UndefinedBehaviorSanitizer.

Each is compiled with g++ from the host-only headers (apsp_server_core.h,
apsp_batch_host.h) the library itself includes; the HIP runtime header is
used for its type declarations only."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = [f"-I{ROOT}/include", f"-I{ROOT}/paper_1811_01201_amd/csrc", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]


def _build_and_run(src, sanitize, tmp_path, timeout=600):
    exe = str(tmp_path / (os.path.basename(src) + "." + sanitize.replace(",", "_")))
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-pthread", *INC, os.path.join(ROOT, "tests", "cpp", src), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]


@pytest.mark.parametrize("sanitize", ["thread", "address,undefined"])
def test_server_core_with_fake_executor(sanitize, tmp_path):
    _build_and_run("test_server_core.cpp", sanitize, tmp_path)


def test_batch_plans_and_kernel_bounds_model(tmp_path):
    _build_and_run("test_batch_host.cpp", "address,undefined", tmp_path)
