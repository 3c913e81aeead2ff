"""CPU checks of the benchmark's bookkeeping: the measured-traffic figure of
the bench line comes from the committed counter summary only while the kernel
sources still hash as they did when the counters were taken, and is null
(with the reason) otherwise; `--gpus` above 1 is refused before anything
touches a GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

bench = pytest.importorskip("bench")


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.md"
    good.write_text(f"traffic_bytes_per_product: 123456\nkernel_sources_sha256_16: {bench.kernel_sources_hash()}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(good))
    assert bench.measured_traffic()[0] == 123456
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_product: 123456\nkernel_sources_sha256_16: 0000000000000000\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    value, why = bench.measured_traffic()
    assert value is None and "changed" in why
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic()[0] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stdout
