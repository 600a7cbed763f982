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
    alg = m["algorithmic_bytes"]
    got = bench.measured_traffic("slab_hv", "medium", alg)
    if current == m["sha1"]:
        want = 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])
        assert got == pytest.approx(want)
        # launches of another chain block keep the measured-to-algorithmic ratio
        assert bench.measured_traffic("slab_hv", "medium", 1.5 * alg) == pytest.approx(1.5 * want)
    else:
        assert got is None          # a changed kernel source reports no measured traffic
    # another workload, or a source that differs from the measured one, reports none
    assert bench.measured_traffic("slab_hv", "small", alg) is None
    fake = tmp_path / "fft.hip"
    fake.write_bytes(b"// not the measured source\n")
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "slab_hv", dict(m, source=str(fake)))
    monkeypatch.setattr(bench, "ROOT", "/")
    assert bench.measured_traffic("slab_hv", "medium", alg) is None


def test_roofline_bound_is_the_larger_floor():
    """The bound is the larger of the two algorithmic floors at published peaks: the FP32
    slab pass of the medium step (0.2562 GB and 4.55 GFLOP per launch, 137.3 us) is
    HBM-bound at 1.87 TB/s; the same bytes with 30x the flops would be ALU-bound."""
    import bench
    prof = {"slab_hv": {"ms": 137.3, "launches": 1000, "bytes": 0.2562e9 * 1000, "flops": 4.55e9 * 1000}}
    name, r = bench.dominant_roofline(prof, "bf16")
    assert name == "slab_hv" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(0.2562e9 / 137.3e-6 / 8e12, rel=1e-3)
    prof["slab_hv"]["flops"] *= 30
    _, r = bench.dominant_roofline(prof, "bf16")
    assert r["bound"] == "alu" and r["peak"] == 157.3
    # a matrix-core class in BF16x3 mode is priced at a third of the bf16 peak
    prof = {"gemm_ahb": {"ms": 1.0, "launches": 1, "bytes": 1e3, "flops": 1e12}}
    _, r = bench.dominant_roofline(prof, "bf16")
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(2500.0 / 3, rel=1e-3)
