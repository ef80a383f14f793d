"""Host-side pieces of bench.py: the provenance of the reported HBM traffic (a profile record counts
only while the kernel code it was taken on is unchanged) and the refusal of several GPUs.  CPU only."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORD = os.path.join(ROOT, "profiles", "pair_sym_fp32c_grad_city85k.json")


def test_committed_traffic_record_is_used_only_for_its_kernel_code():
    rec = json.load(open(RECORD))
    if rec["kernel_source_sha256"] == bench.kernel_source_sha256():
        assert bench.measured_traffic(RECORD) == rec["fetch_bytes"] + rec["write_bytes"] > 0
    else:  # kernels changed since the counters were taken: the bench reports no traffic
        assert bench.measured_traffic(RECORD) is None


def test_traffic_is_dropped_when_the_code_changes(tmp_path):
    rec = json.load(open(RECORD))
    rec["kernel_source_sha256"] = "0" * 64
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps(rec))
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.json")) is None


def test_hash_ignores_comments_only(tmp_path, monkeypatch):
    """Editing a comment keeps the hash; editing code changes it."""
    src = os.path.join(ROOT, "paper_2005_10123_amd", "csrc")
    for name in bench.KERNEL_SOURCES:
        (tmp_path / name).write_text(open(os.path.join(src, name)).read())
    fake_root = tmp_path / "root"
    (fake_root / "paper_2005_10123_amd").mkdir(parents=True)
    os.symlink(tmp_path, fake_root / "paper_2005_10123_amd" / "csrc")
    monkeypatch.setattr(bench, "ROOT", str(fake_root))
    base = bench.kernel_source_sha256()
    k = tmp_path / bench.KERNEL_SOURCES[0]
    k.write_text(k.read_text() + "\n// a trailing comment\n/* and a block\n   comment */\n")
    assert bench.kernel_source_sha256() == base
    k.write_text(k.read_text() + "\nstatic int extra_symbol = 1;\n")
    assert bench.kernel_source_sha256() != base


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_gfx_clock_parsing(monkeypatch):
    """amd-smi's per-XCD graphics clocks (MHz) are read per listed GPU; other clocks are ignored,
    and a missing or failing amd-smi gives None."""
    import subprocess

    fake = {"gpu_data": [
        {"gpu": 0, "clock": {"gfx_0": {"clk": {"value": 2390, "unit": "MHz"}, "min_clk": {"value": 500}},
                             "gfx_1": {"clk": {"value": 2370, "unit": "MHz"}},
                             "mem_0": {"clk": {"value": 2000, "unit": "MHz"}}}},
        {"gpu": 1, "clock": {"gfx_0": {"clk": {"value": 95, "unit": "MHz"}}}},
    ]}

    class Done:
        stdout = json.dumps(fake)

    monkeypatch.setattr(subprocess, "run", lambda *a, **k: Done())
    assert bench.gfx_clocks_ghz() == {0: [2.39, 2.37], 1: [0.095]}

    def missing(*a, **k):
        raise FileNotFoundError("amd-smi")

    monkeypatch.setattr(subprocess, "run", missing)
    assert bench.gfx_clocks_ghz() is None


def test_engine_clock_samples_under_load(monkeypatch):
    """The clock is read while evaluations run back to back (a worker thread), from the loaded GPU
    (highest mean clock), averaged per XCD over the samples; the worker stops afterwards.  None
    when amd-smi gives nothing."""
    import threading

    calls = []
    running = threading.Event()

    class FakeCtx:
        def grad(self, ds, theta, precision):
            running.set()
            calls.append(precision)

    readings = iter([{0: [2.38, 2.36], 1: [0.1, 0.1]}, {0: [2.40, 2.34], 1: [0.1, 0.1]}])
    monkeypatch.setattr(bench.time, "sleep", lambda s: running.wait(5.0))
    monkeypatch.setattr(bench, "gfx_clocks_ghz", lambda: next(readings))
    clk = bench.engine_clock(FakeCtx(), None, None, nsamples=2)
    assert clk["samples"] == 2
    assert all(abs(a - b) < 1e-12 for a, b in zip(clk["per_xcd_ghz"], [2.39, 2.35]))
    assert abs(clk["measured_ghz"] - 2.37) < 1e-12
    assert clk["evaluations_meanwhile"] >= 1 and set(calls) == {"fp32c"}
    n = len(calls)
    threading.Event().wait(0.05)
    assert len(calls) == n  # the worker has stopped
    monkeypatch.setattr(bench, "gfx_clocks_ghz", lambda: None)
    assert bench.engine_clock(FakeCtx(), None, None) is None
