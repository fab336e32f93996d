"""Host-side logic of bench.py (no GPU): the roofline arithmetic, the gating of
the committed PMC summary on source hash and scheme, and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def fake_run(ms_per_step=2.0, launches=60):
    # per-kernel (total ms, launches) as rh_kernel_times returns them
    return {"kernels": {"sweep_x": (12.0, launches), "sweep_y": (13.0, launches),
                        "sweep_z": (15.0, launches)}, "ms_per_step": ms_per_step}


def test_roofline_arithmetic_without_profile(monkeypatch):
    monkeypatch.setattr(bench, "load_profile", lambda precision, order=5: {})
    n = 256 ** 3
    dom, roof, hbm = bench.roofline(fake_run(), "fp32", 5, n)
    assert dom == "sweep_z" and roof["kernel"] == "sweep_z"
    avg_s = 15.0 / 60 * 1e-3
    flops = bench.sweep_flops_per_cell(5) * n
    assert roof["achieved"] == pytest.approx(flops / avg_s / 1e12, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 157.3, rel=1e-3)
    assert roof["bound"] == "alu" and roof["traffic"] is None and roof["valu"] is None
    # algorithmic bytes of the z sweep: (15 + 20 + 20) / 3 values of 4 B per cell
    assert hbm["design_bytes_per_launch"] == pytest.approx(55.0 / 3.0 * 4 * n)
    # whole step: 40 values per cell-update
    assert hbm["step_alg"]["bytes"] == 160.0 * n
    assert hbm["step_alg"]["GBps"] == pytest.approx(160.0 * n / 2.0e-3 / 1e9, rel=1e-3)
    assert "step_counted" not in hbm


def test_roofline_uses_profile_counters(monkeypatch):
    prof = {k: {"bytes_per_launch": b, "SQ_INSTS_VALU": 1.0e8}
            for k, b in (("sweep_x", 1.0e9), ("sweep_y", 1.1e9), ("sweep_z", 1.3e9))}
    monkeypatch.setattr(bench, "load_profile", lambda precision, order=5: prof)
    n = 256 ** 3
    _, roof, hbm = bench.roofline(fake_run(), "fp32", 5, n)
    avg_s = 15.0 / 60 * 1e-3
    assert roof["traffic"] == 1.3e9
    assert hbm["counted_GBps"] == pytest.approx(1.3e9 / avg_s / 1e9, rel=1e-3)
    assert hbm["step_counted"]["bytes"] == pytest.approx(3 * 3.4e9)
    rate = 1.0e8 / avg_s / (256 * 2.4e9)
    assert roof["valu"]["wave_instr_per_cu_cycle"] == pytest.approx(rate, rel=1e-3)
    assert roof["valu"]["frac_of_peak"] == pytest.approx(rate / 2, rel=1e-3)
    assert roof["valu"]["instr_per_cell"] == pytest.approx(1.0e8 * 64 / n, rel=1e-3)


def test_profile_gated_on_hash_and_scheme(tmp_path, monkeypatch):
    prof = {"source_hash": bench.source_hash(), "order": 5,
            "kernels": {"fp32": {"sweep_z": {"bytes_per_launch": 5.0}}}}
    os.makedirs(tmp_path / "profiles")
    path = tmp_path / "profiles" / "pmc_traffic_blob256.json"
    path.write_text(json.dumps(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: prof["source_hash"])
    assert bench.load_traffic("sweep_z", "fp32", 5) == 5.0
    assert bench.load_traffic("sweep_z", "fp32", 7) is None
    assert bench.load_traffic("sweep_z", "fp64", 5) is None
    path.write_text(json.dumps(dict(prof, source_hash="0" * 16)))
    assert bench.load_traffic("sweep_z", "fp32", 5) is None


def test_roofline_of_the_fused_sweep(monkeypatch):
    monkeypatch.setattr(bench, "load_profile", lambda precision, order=5: {})
    n = 256 ** 3
    run = {"kernels": {"sweep_x": (0.0, 0), "sweep_y": (0.0, 0), "sweep_xy": (18.0, 60),
                       "sweep_z": (15.0, 60)}, "ms_per_step": 2.0}
    dom, roof, hbm = bench.roofline(run, "fp32", 5, n)
    assert dom == "sweep_xy"
    # two directional sweeps per launch; reads u and writes L (10 values per cell)
    assert roof["flops_per_cell"] == 2 * bench.sweep_flops_per_cell(5)
    assert roof["achieved"] == pytest.approx(2 * bench.sweep_flops_per_cell(5) * n / (18.0 / 60 * 1e-3) / 1e12,
                                             rel=1e-3)
    assert hbm["design_bytes_per_launch"] == 10.0 * 4 * n


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
