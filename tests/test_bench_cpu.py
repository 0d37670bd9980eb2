"""bench.py contract checks that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_flop_model_matches_kernel_structure():
    sys.path.insert(0, ROOT)
    import bench

    # 25 setup operations, 6 per order, the closing sums per layer mask
    assert bench.flops_per_pair(16, 1) == 5 * 16 + 25
    assert bench.flops_per_pair(16, 2) == 6 * 16 + 37
    assert bench.flops_per_pair(16, 3) == 6 * 16 + 48
    assert bench.flops_per_pair(0, 3) == bench.flops_per_pair(1, 3)
    assert bench.flops_per_pair(0, 1) == 28
    # S': alone, beside the single layer, beside the double layer, all three
    assert bench.flops_per_pair(16, 4) == 6 * 16 + 29
    assert bench.flops_per_pair(16, 5) == 6 * 16 + 44
    assert bench.flops_per_pair(16, 6) == 6 * 16 + 50
    assert bench.flops_per_pair(16, 7) == 6 * 16 + 60


def test_traffic_record_is_ignored_after_a_kernel_change(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    rec = tmp_path / "t.json"
    rec.write_text(json.dumps({"kernel_source_sha256": "0" * 64, "hbm_bytes_per_launch": 1.0}))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec))
    assert bench.measured_traffic() is None


def test_traffic_record_is_used_while_the_kernel_is_unchanged(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    rec = tmp_path / "t.json"
    rec.write_text(json.dumps({"kernel_source_sha256": bench.kernel_source_sha256(),
                               "hbm_bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec))
    assert bench.measured_traffic() == 123.0


def test_helmholtz_flop_model():
    sys.path.insert(0, ROOT)
    import bench

    S = bench.HELM_SINCOS_FLOPS
    # setup 27 + sincos + h_0, h_1 8 + n = 0 2 + n = 1 5 + 14 per further order + 8
    assert bench.helm_flops_per_pair(16, 1) == 27 + S + 8 + 2 + 5 + 15 * 14 + 8
    # the double layer: 5 + 8 + 13 + 17 per further order + 30
    assert bench.helm_flops_per_pair(16, 3) == bench.helm_flops_per_pair(16, 1) + 5 + 8 + 13 + 15 * 17 + 30
    assert bench.helm_flops_per_pair(0, 1) == 27 + S + 8 + 2 + 8
    # S': P_n' 3 per further order, nu_t . d 5, n = 0 2, n = 1 9, 11 per further order, 17
    assert bench.helm_flops_per_pair(16, 4) == 27 + S + 8 + 15 * 8 + 15 * 3 + 5 + 2 + 9 + 15 * 11 + 17
    assert (bench.helm_flops_per_pair(16, 7)
            == bench.helm_flops_per_pair(16, 3) + 5 + 2 + 9 + 15 * 11 + 17)
    assert bench.helm_flops_per_pair(0, 4) == 27 + S + 8 + 5 + 2 + 17


def test_separate_recurrence_figure():
    sys.path.insert(0, ROOT)
    import bench

    assert bench.separate_recurrence_flops_per_pair(16, 3) == (6 * 16 + 20) + (11 * 16 + 36) == 328
    assert bench.separate_recurrence_flops_per_pair(16, 1) == 116
    assert bench.separate_recurrence_flops_per_pair(24, 2) == 300
