"""Compile the HIP sources under csrc/ into the in-tree shared library libhawkes.so (gfx950), and
the instruction-rate microbenchmark csrc/rates_probe.hip into the executable rates_probe (the
measured rates behind the pairwise pass's roofline; not part of the library).

Run as ``python -m paper_2005_10123_amd.build`` or through ``__graft_entry__.build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBRARY = os.path.join(HERE, "libhawkes.so")
RATES_PROBE = os.path.join(HERE, "rates_probe")
SOURCES = ["hawkes_kernels.hip", "hawkes_runtime.hip", "hawkes_serving.hip", "hawkes_multi.hip", "hawkes_shard.hip", "hawkes_epilogue.hip", "hawkes_host.hip", "hawkes_noalloc.hip"]
ARCH = "gfx950"
# Packed FP32 VALU forms are switched off for all device code on this target.
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(output: str = LIBRARY, extra_flags=()) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        _run(["hipcc", *FLAGS, *extra_flags, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    def probe():
        if output != LIBRARY:
            return
        tmp_exe = RATES_PROBE + ".tmp"
        _run(["hipcc", *FLAGS, *extra_flags, os.path.join(CSRC, "rates_probe.hip"), "-o", tmp_exe])
        os.replace(tmp_exe, RATES_PROBE)

    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        probe_job = ex.submit(probe)
        objs = list(ex.map(compile_one, SOURCES))
        probe_job.result()
    tmp = output + ".tmp"
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, output)
    return output


if __name__ == "__main__":
    print(build())
