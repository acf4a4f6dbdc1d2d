"""Host-side logic of the benchmark and of the profile summaries (no GPU)."""
import os
import subprocess
import sys

import numpy as np


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2307_06471_amd import profsummary as PS  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_fused_step():
    S, N = 160, 1000
    assert bench.algorithmic_bytes("fused", S * N, S * N, N, 2) == 2 * S * N


def test_algorithmic_bytes_of_the_step_kernels():
    S, N = 160, 1000  # FP32-bulk Q2 state bytes per cell x cells
    state = S * N
    # scheme (eq:3): final-stage states u^n and u^(3); the stored stage has the state's layout
    assert bench.algorithmic_bytes("inner", state, state, N, 2) == 2 * state
    assert bench.algorithmic_bytes("final", state, state, N, 2) == 3 * state
    assert bench.algorithmic_bytes("limit", state, state, N, 2) == state + N
    assert bench.algorithmic_bytes("dt", state, state, N, 2) == ((N + 255) // 256) * 8
    assert bench.algorithmic_bytes("other", state, state, N, 2) is None


def test_traffic_summary_round_trip_and_source_gate(tmp_path):
    p = tmp_path / "k_final2_fp32_traffic.txt"
    p.write_text("# HBM traffic per launch of k\n\n  a command line: with colons\n"
                 f"kernel source hash: {PS.kernel_source_hash()}\n"
                 "traffic_bytes_per_launch: 123456\n")
    d = PS.read_traffic(str(p))
    assert d["traffic_bytes_per_launch"] == "123456"
    assert d["kernel source hash"] == PS.kernel_source_hash()
    assert PS.read_traffic(str(tmp_path / "missing.txt")) is None
    h = PS.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0 and h == PS.kernel_source_hash()


def test_committed_traffic_summaries_parse():
    import glob
    files = glob.glob(os.path.join(ROOT, "profiles", "k_*_traffic.txt"))
    assert any(f.endswith("k_fused2_fp32_traffic.txt") for f in files)
    for f in files:
        d = PS.read_traffic(f)
        assert d is not None
        assert float(d["traffic_bytes_per_launch"]) > 0
        assert float(d["fetch_factor"]) > 0 and float(d["write_factor"]) > 0
        assert d["fetch_dispatches"] == d["write_dispatches"]


def test_indicator_file_round_trip(tmp_path):
    rng = np.random.default_rng(3)
    P = rng.standard_normal(1505).astype(np.float32)
    info = {"tau_lo": 0.2, "validation": {"fn_rate": 0.01}}
    f = str(tmp_path / "ind.npz")
    bench.save_indicator(f, P, 0.2, 0.9, info)
    P2, lo, hi, info2 = bench.load_indicator(f)
    assert np.array_equal(P, P2) and P2.dtype == np.float32
    assert (lo, hi) == (0.2, 0.9)
    assert info2["validation"] == info["validation"] and info2["loaded_from"] == "ind.npz"


def test_algorithmic_bytes_of_the_original_rkdg():
    S, N = 288, 1000
    assert bench.algorithmic_bytes("final", S * N, S * N, N, 2, "rkdg3") == 8 * S * N / 3
    assert bench.algorithmic_bytes("limit", S * N, S * N, N, 2, "rkdg3") == S * N
    assert bench.algorithmic_bytes("dt", S * N, S * N, N, 2, "rkdg3") is None


def test_traffic_calibration_arithmetic(tmp_path):
    """profsummary.traffic: per-dispatch mean of the kernel's counter, scaled
    by (copy bytes) / (counter of the largest copy dispatch)"""
    def csv(path, counter, rows):
        with open(path, "w") as f:
            f.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
            for name, grid, val in rows:
                f.write(f'"{name}",{grid},{counter},{val}\n')
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    copy = 256 << 20
    csv(fetch, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 512, 3.0),
                              ("__amd_rocclr_copyBuffer", 131072, copy / 1024 / 2),
                              ("void k_final2<A, 2, 1, false, false>(x)", 64, 1000.0),
                              ("void k_final2<A, 2, 1, false, false>(x)", 64, 1200.0),
                              ("void k_final2<A, 2, 1, true, false>(x)", 64, 9999.0)])
    csv(write, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 131072, copy / 1024),
                              ("void k_final2<A, 2, 1, false, false>(x)", 64, 500.0)])
    out = tmp_path / "t.txt"
    PS.traffic(str(fetch), str(write), "k_final2<A, 2, 1, false, false>", copy, str(out), "cmd")
    d = PS.read_traffic(str(out))
    assert float(d["fetch_factor"]) == 2.0 and float(d["write_factor"]) == 1.0
    assert float(d["fetch_bytes_per_launch"]) == 1100.0 * 1024 * 2
    assert float(d["write_bytes_per_launch"]) == 500.0 * 1024
    assert float(d["traffic_bytes_per_launch"]) == 1100.0 * 2048 + 500.0 * 1024
    assert d["fetch_dispatches"] == "2"


def test_traffic_refuses_a_name_matching_several_kernels(tmp_path):
    import pytest
    f = tmp_path / "f.csv"
    with open(f, "w") as fh:
        fh.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        fh.write('"void k_final2<A, 2, 1, false, false>(x)",64,FETCH_SIZE,1\n')
        fh.write('"void k_final2<A, 2, 0, false, false>(x)",64,FETCH_SIZE,1\n')
    with pytest.raises(SystemExit):
        PS.traffic(str(f), str(f), "k_final2<A", 1 << 20, str(tmp_path / "o.txt"), "cmd")


def test_counter_summary_ratios(tmp_path):
    f = tmp_path / "c.csv"
    with open(f, "w") as fh:
        fh.write("Kernel_Name,Counter_Name,Counter_Value\n")
        for c, v in (("SQ_WAVES", 100), ("SQ_INSTS_VALU", 50000), ("SQ_ACTIVE_INST_VALU", 2560),
                     ("GRBM_GUI_ACTIVE", 80), ("SQ_WAIT_INST_ANY", 30), ("SQ_WAVE_CYCLES", 120)):
            fh.write(f'"void crk::k_final2<A, 2, 1, false, false>(x, y)",{c},{v}\n')
            fh.write(f'"void crk::k_final2<A, 2, 1, true, false>(x, y)",{c},{2 * v}\n')
    out = tmp_path / "o.txt"
    PS.counters(str(f), ["k_final2<A, 2, 1, false, false>"], str(out), "cmd", simds=16, xcds=8)
    d = dict(l.strip().split(": ", 1) for l in open(out) if l.startswith("  ") and ": " in l)
    assert float(d["valu_insts_per_wave"]) == 500.0
    assert float(d["valu_busy"]) == 4 * 2560 / (16 * 80 / 8)
    assert float(d["wait_fraction"]) == 0.25
