"""The host runtime and the request scheduler of libhawkes, built for the CPU against a test double
of the device (tests/mock_hip): admission under a tiny HBM budget (requests queue rather than fail),
the size and carving of one evaluation's scratch by precision (binary32 column partials for FP32C)
with a budget for four FP32C requests admitting four at once,
a request that can never fit failing alone, invalid requests failing alone, a busy dataset, eight
threads submitting and polling at once, a device failure that fails its requests and makes the
context unusable, and teardown with requests pending and in flight (tests/mock_hip/sched_test.cpp).

Built three ways: plain (g++), under ThreadSanitizer and under AddressSanitizer with
UndefinedBehaviorSanitizer and leak detection (ROCm's clang; GCC 11's ThreadSanitizer does not
follow the timed condition-variable waits of its own libstdc++).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_10123_amd", "csrc")
MOCK = os.path.join(ROOT, "tests", "mock_hip")
CLANG = "/opt/rocm/llvm/bin/clang++"
SCENARIOS = ["basic_mix", "blocking_beside_serving", "shared_passes", "tiny_budget_queues", "column_scratch_by_precision",
             "too_large_fails_alone",
             "invalid_requests_fail_alone", "busy_dataset", "many_threads", "device_failure_poisons",
             "destroy_in_flight"]
BUILDS = {
    "plain": ("g++", ["-O2", "-Wno-subobject-linkage"]),
    "thread": (CLANG, ["-O1", "-fsanitize=thread"]),
    "address": (CLANG, ["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer"]),
}


@pytest.mark.parametrize("build", list(BUILDS))
def test_scheduler_scenarios(tmp_path, build):
    compiler, flags = BUILDS[build]
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    # One translation unit per library source, including it by path: with the test double's
    # hip/hip_runtime.h first on the include path, their host code is plain C++.
    units = []
    for name in ("hawkes_runtime", "hawkes_serving"):
        unit = tmp_path / f"{name}_host.cpp"
        unit.write_text(f'#include "{os.path.join(CSRC, name)}.hip"\n')
        units.append(str(unit))
    exe = str(tmp_path / "sched_test")
    cmd = [compiler, "-std=c++17", "-g", "-pthread", *flags, "-I", MOCK, "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), *units, os.path.join(MOCK, "mock_device.cpp"),
           os.path.join(MOCK, "sched_test.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-6000:]
    for name in SCENARIOS:
        assert f"PASS {name}" in r.stdout, r.stdout
