"""Host-side contract of bench.py (no GPU): the one-GPU rule and the binding of the
measured HBM traffic to the kernel source it was measured on."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_table_is_tied_to_its_source(tmp_path, monkeypatch):
    import bench
    m = bench.MEASURED_TRAFFIC["slab_hv"]
    src = os.path.join(ROOT, m["source"])
    with open(src, "rb") as f:
        current = hashlib.sha1(f.read()).hexdigest()
    got = bench.measured_traffic("slab_hv", "medium")
    if current == m["sha1"]:
        want = 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])
        assert got == pytest.approx(want)
    else:
        assert got is None          # a changed kernel source reports no measured traffic
    # another workload, or a source that differs from the measured one, reports none
    assert bench.measured_traffic("slab_hv", "small") is None
    fake = tmp_path / "fft.hip"
    fake.write_bytes(b"// not the measured source\n")
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "slab_hv", dict(m, source=str(fake)))
    monkeypatch.setattr(bench, "ROOT", "/")
    assert bench.measured_traffic("slab_hv", "medium") is None
