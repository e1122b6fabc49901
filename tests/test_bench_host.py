"""Host-side logic of bench.py (no GPU): the one-GPU contract, the algorithmic
flop counts the rooflines use, and the rule that a stored traffic figure is
used only while the kernel sources still hash to the recorded value."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_fx16_executes_six_products_per_fp32_one():
    for tr in (5, 21, 41):
        assert bench.mfma_flops_per_cell("fx16", tr) == 6 * bench.mfma_flops_per_cell("fp32", tr)
        assert bench.mfma_flops_per_cell("fx16", tr, 64) == 4 * bench.mfma_flops_per_cell("fx16", tr, 32)


def test_flop_counts_from_the_pass_structure():
    # one complex 32-point pass over a 32 x 32 tile: M = 32, K = 64, N = 64
    full = 2 * 32 * 64 * 64
    tr = 21
    want = full / 2 + full + (tr - 1) * 2 * full + full + full / 2
    assert bench.mfma_flops_per_cell("fp32", tr) == want
    assert abs(bench.mfma_flops_per_cell("fx16", tr) - 67.6e6) < 0.05e6
    # 3D: 32 tiles x 16 steps x 4 MFMAs of 4096 flops per pass, 2.5 + 3 x 33 passes
    assert bench.mfma_flops_per_cell_3d(32, 33) == (2.5 + 3 * 33) * 32 * 16 * 4 * 4096
    n = 16 * 16
    assert bench.classical_flops_per_cell(16) == 10 * n * n + 24 * n * 16


def test_stored_traffic_only_for_the_recorded_sources(monkeypatch, tmp_path):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_hs2d_32.md").write_text(
        "text\n- source_sha256: abc123\n- hbm_bytes_per_launch: 12345\n- read_scale: 2.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda w: "abc123")
    assert bench.measured_traffic("hs2d_32") == 12345.0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda w: "changed")
    assert bench.measured_traffic("hs2d_32") is None
    assert bench.measured_traffic("hs3d") is None          # no summary at all


@pytest.mark.parametrize("w", sorted(bench.KERNEL_SOURCE))
def test_every_workload_names_an_existing_kernel_source(w):
    assert os.path.exists(os.path.join(ROOT, "paper_2103_14890_amd", "csrc", bench.KERNEL_SOURCE[w]))
    assert len(bench.kernel_source_hash(w)) == 64
