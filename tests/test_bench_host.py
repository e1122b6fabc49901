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


def test_algorithmic_flops_match_the_scope_table():
    # alg flops per cell: HS-2D 32^2 (20 packed gain transforms) 1.29 M, Maxwell 32^2
    # (4) 0.32 M, HS-2D 64^2 (40) 11.7 M, HS-3D 32^3 and 16^3 (32) 91.9 M and 9.4 M
    # (each within half a unit of the last printed digit)
    for (d, N, P), want, step in (((2, 32, 20), 1.29e6, 0.01e6), ((2, 32, 4), 0.32e6, 0.01e6),
                                  ((2, 64, 40), 11.7e6, 0.1e6), ((3, 32, 32), 91.9e6, 0.1e6),
                                  ((3, 16, 32), 9.4e6, 0.1e6)):
        got = bench.alg_flops_per_cell(d, N, P)
        assert abs(got - want) <= 0.5 * step, (d, N, P, got)
    # exact form: FFTs (real forward + P + 1 complex inverse) and pointwise work
    assert bench.alg_flops_per_cell(2, 32, 20) == 2.5 * 1024 * 10 + 21 * 5 * 1024 * 10 + (9 * 20 + 4) * 1024


def test_roofline_conventions_scale_with_the_counting_basis():
    main, conv = bench.roofline_2d(4096, 2.7e-4, 21, 32, "fx16", None)
    assert main["flops_per_cell"] == bench.alg_flops_per_cell(2, 32, 20)
    assert main["peak"] == 2500.0 and abs(main["frac"] - main["achieved"] / 2500.0) < 1e-12
    g = conv["gemm_fp32_equiv"]["flops_per_cell"]
    assert conv["gemm_x3"]["flops_per_cell"] == 3 * g and conv["executed_fx16_x6"]["flops_per_cell"] == 6 * g
    assert abs(conv["executed_fx16_x6"]["frac"] - 2 * conv["gemm_x3"]["frac"]) < 1e-12
    m32, c32 = bench.roofline_2d(4096, 3.7e-4, 21, 32, "fp32", None)
    assert m32["peak"] == 157.3 and "gemm_x3" not in c32


def test_cpu_oracle_baseline_runs_the_oracle_on_worker_processes():
    import numpy as np
    import workloads as wl
    from oracle import spectral as sp
    f = wl.mixture_cells(2, 16, 8.0, 12, 5)
    items = bench.chunks(f, 3)
    b = bench.cpu_oracle_baseline("q_fast", dict(d=2, N=16, L=8.0, kernel="hard_sphere", M=8), items, len, 0.5)
    assert b["value"] > 0 and 1 <= b["cores"] <= 16 and len(b["runs_s"]) == 3
    assert b["units"] == sum(len(c) for c in items[:b["items"]])
    s = sp.Setup(d=2, N=16, L=8.0, kernel="hard_sphere", M=8)
    want = sp.project_conservative(sp.q_fast(f[:b["units"]], s), 2, 8.0)
    assert np.allclose(np.concatenate(b["outputs"]), want, rtol=0, atol=1e-14 * np.abs(want).max())
    assert b["median_s"] == sorted(b["runs_s"])[1] or abs(b["median_s"] - sorted(b["runs_s"])[1]) < 1e-3
