"""Host-side parts of bench.py that need no GPU: the multi-GPU refusal, the
recovery curve, the traffic record's validity rules and the instruction
models used for the roofline's issue fraction."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_recovery_curve():
    p_rot = np.array([10.0, 20.0, 30.0, 40.0])
    p_lc_days = np.array([5.0, 10.04, 15.2, 20.0]) / 24.0  # doubled: 10, 20.08, 30.4, 40 h
    n_t = np.array([10, 60, 200, 600])
    frac, curve, ok = bench.recovery_curve(p_rot, p_lc_days, n_t)
    assert list(ok) == [True, True, False, True]
    assert frac == 0.75
    by = {c["cutoff"]: c for c in curve}
    assert by[0]["objects"] == 4 and by[50]["objects"] == 3 and by[550]["objects"] == 1
    assert abs(by[50]["matched"] - 2 / 3) < 1e-12 and by[550]["matched"] == 1.0


def test_traffic_record_rules(tmp_path, monkeypatch):
    rec = {"kernel_hash": bench.kernel_hash("standard"), "workload_name": "single_4096",
           "bytes_per_launch": 123}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "standard", str(f))
    assert bench.measured_traffic("standard", "single_4096") == 123
    assert bench.measured_traffic("standard", "learned_100k") is None  # other workload
    # a workload with a record of its own reads that record while it was taken
    # on the current kernel source
    own = json.load(open(bench.TRAFFIC_FILES[("standard", "batch_10k")]))
    expect = own["bytes_per_launch"] if own["kernel_hash"] == bench.kernel_hash("standard") \
        else None
    assert bench.measured_traffic("standard", "batch_10k") == expect
    rec["kernel_hash"] = "0" * 16  # taken on another kernel source
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("standard", "single_4096") is None


def test_instruction_models():
    # the K = 16 loop models: 106 instructions per observation and lane for
    # the standard form (6.625 per evaluation; SQ_INSTS_VALU reads 6.72 with
    # the loop overhead) and 140 for the generalized one (8.75; reads 8.88)
    assert abs(bench.valu_ops_per_eval("chebyshev", 16) - 106 / 16) < 1e-12
    assert abs(bench.valu_ops_per_eval_gen(16) - 140 / 16) < 1e-12
    assert bench.FLOPS_PER_EVAL["chebyshev"] == 12 and bench.FLOPS_PER_EVAL_GEN == 16
    assert abs(bench.PEAK_FP32_TFLOPS - 157.3) < 0.1


def test_committed_traffic_records_are_consistent():
    """Each committed counter record's bytes follow from its KiB counters and
    copy-calibration scales, and its commands name its kernel and workload."""
    import glob
    import os
    files = sorted(glob.glob(os.path.join(bench.ROOT, "profiles", "*_traffic.json")))
    assert len(files) >= 4
    for path in files:
        rec = json.load(open(path))
        for side in ("fetch", "write"):
            got = rec[f"{side}_bytes_per_launch"]
            want = rec[f"{side}_size_kib"] * 1024 * rec[f"{side}_scale"]
            assert abs(got - want) <= 2e-3 * want + 1024, (path, side)
        assert rec["bytes_per_launch"] == rec["fetch_bytes_per_launch"] + \
            rec["write_bytes_per_launch"]
        assert 1.99 < rec["fetch_scale"] < 2.01 and 0.99 < rec["write_scale"] < 1.01
        assert len(rec["kernel_hash"]) == 16
        kernel = rec["kernel"].split("<")[0]
        assert kernel in ("fp32p_kernel", "gen_fp32p_kernel")
        runs = [c for c in rec["commands"] if "--mode copy" not in c]
        assert runs and all(kernel in c for c in runs), path
        if rec["workload_name"] != "lsst_200k":  # the bench's default workload
            assert all(f"--workload {rec['workload_name']}" in c for c in runs), path
