"""bench.py's contract on the host: more than one GPU is refused with a
message, before anything touches a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_modes_are_listed_in_help():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ("--config", "--dag", "--learners", "--ablation", "--warmstart", "--steps", "--warmup"):
        assert flag in r.stdout


def test_new_modes_are_listed_in_help():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for flag in ("--peaks", "--products", "--orth", "--traffic-from", "--bf16-steps", "--oracle-runs",
                 "--calibrate-copy", "--start-study"):
        assert flag in r.stdout


def _counter_csv(path, counter, rows):
    import csv
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (kname, v) in enumerate(rows):
            # two rows per dispatch (counters summed over instances)
            w.writerow([i, i, kname, counter, v / 2])
            w.writerow([i, i, kname, counter, v / 2])


def test_traffic_summary_scales_counters_by_the_copy_kernel(tmp_path):
    """The counter summary: each pass's FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch) times the factor that maps the copy kernel's reading onto its
    known 1 GiB."""
    import json
    cp = "isvd::(anonymous namespace)::peak_copy_kernel(uint4 const*, uint4*, long)"
    f32 = "void isvd::(anonymous namespace)::spmm_pass_kernel<float, float, 64, 2, true>(isvd::SpmmPass)"
    b16 = "void isvd::(anonymous namespace)::spmm_pass_kernel<isvd::bf16, float, 64, 1, true>(isvd::SpmmPass)"
    gib_kib = float(1 << 20)
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(cp, gib_kib / 2), (f32, 1000.0), (f32, 3000.0), (b16, 500.0)])
    _counter_csv(write, "WRITE_SIZE", [(cp, gib_kib), (f32, 100.0), (f32, 100.0), (b16, 50.0)])
    out = tmp_path / "t.json"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--config", "c4", "--traffic-from",
                        str(fetch), str(write), "--traffic-json", str(out)], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    tj = json.loads(out.read_text())
    assert tj["workload"] == "c4_chunglu2m_bf16"
    assert abs(tj["fetch_scale"] - 2.0) < 1e-9 and abs(tj["write_scale"] - 1.0) < 1e-9
    assert tj["passes"]["fp32"]["dispatches"] == 2
    assert tj["passes"]["fp32"]["bytes_per_launch"] == round(2000.0 * 1024 * 2 + 100.0 * 1024)
    assert tj["passes"]["bf16"]["bytes_per_launch"] == round(500.0 * 1024 * 2 + 50.0 * 1024)


def test_gapped_k_and_subspace_helpers():
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch

    import bench
    s = np.array([10.0, 5.0, 4.9999, 4.0, 3.0])
    assert bench.gapped_k(s, 2) == 1          # s_2 and s_3 are within 1e-3 of each other
    assert bench.gapped_k(s, 3) == 3
    assert bench.gapped_k(s, 4) == 4
    # the helper's principal angle against a rotation by a known angle (on the CPU)
    th = 1e-3
    a = torch.zeros((6, 2), dtype=torch.float64)
    a[0, 0] = a[1, 1] = 1.0
    b = a.clone()
    b[1, 1], b[2, 1] = np.cos(th), np.sin(th)
    assert abs(bench.subspace_angle(torch, a, b, 2) - th) < 1e-12


def test_phase_summary_per_step_and_remainder():
    sys.path.insert(0, ROOT)
    import bench

    class FakeLib:
        @staticmethod
        def profile_phases_read():
            return {"products": (8000.0, 390), "orthonormalisation": (1200.0, 388), "rayleigh_ritz": (50.0, 14),
                    "residual_checks": (80.0, 14), "output_products": (10.0, 2)}

    out = bench.phase_summary(FakeLib, 2, 4.8)
    assert out["products"] == 4.0 and out["orthonormalisation"] == 0.6
    assert out["occurrences_per_step"]["products"] == 195
    # the rest of the step: 4.8 - (4.0 + 0.6 + 0.025 + 0.04 + 0.005)
    assert abs(out["between_phases"] - 0.13) < 1e-9
