"""Host-side logic of bench.py (no GPU): the one-GPU contract, the kernel source hashes that tie
committed counter summaries to the sources they were taken from, and the counting formulas."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr


def test_source_hash_covers_the_inlined_raster_headers():
    csrc = os.path.join(ROOT, "paper_2407_01866_amd", "csrc")
    for kernel, src in bench.KERNEL_SOURCES.items():
        h = hashlib.sha256()
        for name in (src,) + bench.KERNEL_HEADERS:
            h.update(open(os.path.join(csrc, name), "rb").read())
        assert bench.kernel_source_hash(kernel) == h.hexdigest()[:16]
    assert "raster_tile.hpp" in bench.KERNEL_HEADERS


@pytest.mark.parametrize("matching", [True, False])
def test_counters_are_used_only_for_the_source_they_were_taken_from(tmp_path, monkeypatch,
                                                                    matching):
    sha = bench.kernel_source_hash("raster_fit") if matching else "0123456789abcdef"
    traffic = tmp_path / "traffic.txt"
    traffic.write_text("# header\n"
                       f"kernel raster_fit source_sha256 {sha} fetch_kib 1 write_kib 1 "
                       "read_bytes 4e8 write_bytes 7e7 traffic_bytes 4.7e+08\n")
    valu = tmp_path / "valu.txt"
    valu.write_text(f"kernel raster_fit_kernel<9,10,false> family raster_fit source_sha256 {sha} "
                    "dispatches 8 valu_insts 2.2e+08 lds_insts 2.6e+07 cycles_per_xcd 1.2e+06 "
                    "issue_busy 0.703 active_lanes 0.823 executed_lane_slots 1.412e+10\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    monkeypatch.setattr(bench, "VALU_FILE", str(valu))
    t = bench.measured_traffic("raster_fit")
    v = bench.measured_valu("raster_fit")
    if matching:
        assert t == pytest.approx(4.7e8)
        assert v == {"issue_busy": 0.703, "active_lanes": 0.823, "executed_lane_slots": 1.412e10}
    else:
        assert t is None and v is None


def test_single_pass_work_is_the_sum_of_both_passes():
    e_fwd, e_bwd, hw, n = 3.9e8, 4.2e7, 2048 * 2048, 9
    # per (pixel, candidate) 9 lane-ops, per pixel 60 + 18 n; per retained pair 35 + 3 n
    assert bench.fwd_valu_ops(e_fwd, hw, n) == pytest.approx(9 * e_fwd + (60 + 18 * n) * hw)
    assert bench.bwd_valu_ops(e_bwd, n) == pytest.approx((35 + 3 * n) * e_bwd)


def test_cpu_baseline_reports_model_median_of_three_and_one_thread():
    import numpy as np
    from paper_2407_01866_amd import synth
    H, W, n = 64, 48, 3
    p = synth.gen_gaussians(3, H, W, 100, n)
    g = synth.gen_grad_image(4, n, H, W).astype(np.float64)
    r = bench.cpu_baseline(p, H, W, 10, g, budget_s=1.0)
    assert r["kind"] == "oracle" and r["cores"] >= 1 and r["cpu_model"]
    assert len(r["runs"]) == 3 and r["runs"][0] <= r["value"] <= r["runs"][2]
    assert r["one_core"]["cores"] == 1 and r["one_core"]["value"] > 0
    assert "tiles" in r["one_core"]["sample"]
