"""Host logic of bench.py (no GPU): the measured HBM traffic goes into a bench
line only while the kernel sources hash to the value its counter summary
records (and, for the batched kernel, while the launch runs the profiled
variant); the committed summaries are consistent with their counters; the
bench refuses more than one GPU."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_traffic_summaries(bench):
    """Each summary's bytes follow from its counters; the bench uses them
    exactly while the sources hash to the recorded value."""
    for tag, sources in (("ttm_slab_c3_bf16x3", bench.CHAIN_SOURCES), ("ttm_batched_c4", bench.BATCHED_SOURCES)):
        with open(os.path.join(ROOT, "profiles", f"{tag}_traffic.json")) as f:
            t = json.load(f)
        # HBM bytes = scaled FETCH + scaled WRITE counters; the scales make the
        # 1 GiB copy read 1048576 KiB each way
        expect = (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024
        assert abs(t["bytes_per_launch"] - expect) <= 1e-6 * expect
        assert t["copy_fetch_kib"] * t["fetch_scale"] == pytest.approx(1048576.0)
        assert t["copy_write_kib"] * t["write_scale"] == pytest.approx(1048576.0)
        got = bench.measured_traffic(tag, sources=sources)
        if t["kernel_src_sha"] == bench.kernel_src_sha(sources):
            assert got == pytest.approx(t["bytes_per_launch"])
        else:
            assert got is None, tag


def test_traffic_dropped_when_sources_or_variant_differ(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", "ttm_batched_c4_traffic.json"), prof)
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    with open(prof / "ttm_batched_c4_traffic.json") as f:
        t = json.load(f)
    assert bench.c4_traffic(t["variant"]) == pytest.approx(t["bytes_per_launch"])
    assert bench.c4_traffic(t["variant"] + 1) is None
    t["kernel_src_sha"] = "0" * 16
    with open(prof / "ttm_batched_c4_traffic.json", "w") as f:
        json.dump(t, f)
    assert bench.c4_traffic(t["variant"]) is None
    assert bench.measured_traffic("no_such_kernel") is None


def test_sources_hash_covers_every_listed_file(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2411_13532_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in set(bench.CHAIN_SOURCES) | set(bench.BATCHED_SOURCES):
        shutil.copy(os.path.join(ROOT, "paper_2411_13532_amd", "csrc", name), csrc)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    ref = {s: bench.kernel_src_sha(s) for s in (bench.CHAIN_SOURCES, bench.BATCHED_SOURCES)}
    for name in bench.BATCHED_SOURCES:
        with open(csrc / name, "ab") as f:
            f.write(b"\n")
        assert bench.kernel_src_sha(bench.BATCHED_SOURCES) != ref[bench.BATCHED_SOURCES], name
        ref[bench.BATCHED_SOURCES] = bench.kernel_src_sha(bench.BATCHED_SOURCES)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
