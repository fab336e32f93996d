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
    monkeypatch.setattr(bench, "load_trace_avg", lambda kernel, precision, order=5: None)
    n = 256 ** 3
    dom, roof, hbm = bench.roofline(fake_run(), "fp32", 5, n)
    assert dom == "sweep_z" and roof["kernel"] == "sweep_z"
    avg_s = 15.0 / 60 * 1e-3
    flops = bench.sweep_flops_per_cell(5) * n
    assert roof["achieved"] == pytest.approx(flops / avg_s / 1e12, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 157.3, rel=1e-3)
    assert roof["bound"] == "alu" and roof["traffic"] is None and roof["valu"] is None
    assert "frac_trace" not in roof
    # algorithmic bytes of the z sweep: (15 + 20 + 20) / 3 values of 4 B per cell
    assert hbm["design_bytes_per_launch"] == pytest.approx(55.0 / 3.0 * 4 * n)
    # whole step: 40 values per cell-update
    assert hbm["step_alg"]["bytes"] == 160.0 * n
    assert hbm["step_alg"]["GBps"] == pytest.approx(160.0 * n / 2.0e-3 / 1e9, rel=1e-3)
    assert "step_counted" not in hbm


def test_roofline_uses_profile_counters(monkeypatch):
    # the counter pass's own dispatch duration (2.6e-4 s) is the time base of the
    # issue rate, not the live event time (2.5e-4 s per launch)
    prof = {k: {"bytes_per_launch": b, "SQ_INSTS_VALU": 1.0e8, "_dur_valu_run": 2.6e-4,
                "clock_ghz": 2.2, "valu_busy": 0.93}
            for k, b in (("sweep_x", 1.0e9), ("sweep_y", 1.1e9), ("sweep_z", 1.3e9))}
    monkeypatch.setattr(bench, "load_profile", lambda precision, order=5: prof)
    monkeypatch.setattr(bench, "load_trace_avg", lambda kernel, precision, order=5: 0.255)
    n = 256 ** 3
    _, roof, hbm = bench.roofline(fake_run(), "fp32", 5, n, copy_GBps=5000.0)
    avg_s = 15.0 / 60 * 1e-3
    assert roof["traffic"] == 1.3e9
    assert hbm["counted_GBps"] == pytest.approx(1.3e9 / avg_s / 1e9, rel=1e-3)
    assert hbm["step_counted"]["bytes"] == pytest.approx(3 * 3.4e9)
    # every sweep class against the peak and the plain copy's rate
    assert hbm["copy_GBps"] == 5000.0 and hbm["copy_frac_of_peak"] == pytest.approx(0.625)
    y = hbm["sweeps"]["sweep_y"]
    assert y["ms_per_launch"] == pytest.approx(13.0 / 60, rel=1e-3)
    assert y["counted_GBps"] == pytest.approx(1.1e9 / (13.0 / 60 * 1e-3) / 1e9, rel=1e-3)
    assert y["of_copy_rate"] == pytest.approx(y["counted_GBps"] / 5000.0, rel=1e-3)
    assert set(hbm["sweeps"]) == {"sweep_x", "sweep_y", "sweep_z"}
    assert roof["valu"]["wave_instr_per_cu_cycle_at_2.4GHz"] == pytest.approx(1.0e8 / 2.6e-4 / (256 * 2.4e9),
                                                                             rel=1e-3)
    assert roof["valu"]["wave_instr_per_cu_cycle"] == pytest.approx(1.0e8 / 2.6e-4 / (256 * 2.2e9), rel=1e-3)
    assert roof["valu"]["valu_busy"] == 0.93
    assert roof["valu"]["instr_per_cell"] == pytest.approx(1.0e8 * 64 / n, rel=1e-3)
    # the trace-based fraction uses the committed trace's average launch time
    flops = bench.sweep_flops_per_cell(5) * n
    assert roof["frac_trace"] == pytest.approx(flops / 0.255e-3 / 1e12 / 157.3, rel=1e-3)


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
    monkeypatch.setattr(bench, "load_trace_avg", lambda kernel, precision, order=5: None)
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


def test_autotune_cache_round_trip(tmp_path):
    """The tuned launch shape of an ensemble is stored under a key of its path,
    scheme, precision and size multiset, independent of the order of the grids."""
    from paper_1604_03360_amd import rh
    a = rh.make_desc((64, 64, 64), (0.1,) * 3, (0, 0, 0), 5, rh.RH_PREC_FP32)
    b = rh.make_desc((96, 96, 96), (0.1,) * 3, (0, 0, 0), 5, rh.RH_PREC_FP32)
    k1 = rh.autotune_key([a, b, a], rh.RH_PATH_STAGE, "dev")
    k2 = rh.autotune_key([b, a, a], rh.RH_PATH_STAGE, "dev")
    assert k1 == k2 and "64x64x64*2" in k1 and "96x96x96*1" in k1
    assert k1 != rh.autotune_key([a, b, a], rh.RH_PATH_SWEEPS, "dev")
    assert k1 != rh.autotune_key([a, b], rh.RH_PATH_STAGE, "dev")
    c = rh.make_desc((64, 64, 64), (0.1,) * 3, (0, 0, 0), 5, rh.RH_PREC_FP64)
    assert k1 != rh.autotune_key([c, b, c], rh.RH_PATH_STAGE, "dev")
    path = str(tmp_path / "tune.json")
    assert rh.load_autotune_cache(path) == {}
    rh.store_autotune_cache(path, k1, (16, 32))
    rh.store_autotune_cache(path, "other", (32, 24))
    assert rh.load_autotune_cache(path)[k1] == [16, 32]
    assert rh.load_autotune_cache(path)["other"] == [32, 24]
