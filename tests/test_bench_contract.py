"""Host-side contract of bench.py (no GPU): one GPU only, argument checks,
and the algorithmic work it prices each phase at."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


@pytest.mark.parametrize("gpus", ["2", "8"])
def test_more_than_one_gpu_exits_with_a_message(gpus):
    r = _run("--gpus", gpus)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_step_count_is_bounded():
    r = _run("--steps", "0")
    assert r.returncode == 2 and "--steps" in r.stderr


def test_phase_work_counts_the_products_of_the_method():
    sys.path.insert(0, ROOT)
    import bench

    m, n, k, l = 8192, 8192, 200, 210
    w = bench.phase_work(m, n, k, l, 8.0, 8.0)
    # the two products with A: 2 m n (l + k) flops, A read once by each
    assert w["sketch_gemm"][0] + w["project_gemm"][0] == 2.0 * m * n * (l + k)
    assert w["sketch_gemm"][1] >= 8.0 * m * n and w["project_gemm"][1] >= 8.0 * m * n
    # partial pivoting of the m x l sketch: m l^2 - l^3 / 3
    assert w["panel_lu_y"][0] == pytest.approx(m * l * l - l ** 3 / 3.0)
    # T_roof at the FP64 peak: the products are MFMA-bound at this size
    r = bench.step_roofline(w, 3.0)
    gem = sum(v[0] for key, v in w.items() if key.endswith("gemm"))
    assert r["t_roof_ms"] >= gem / bench.PEAK["f64"] * 1e3
    assert 0.0 < r["frac"] < 1.0


def test_mixed_step_roofline_prices_the_fp64_products_at_the_fp64_peak():
    sys.path.insert(0, ROOT)
    import bench

    m, n, k, l = 16384, 16384, 500, 520
    w = bench.phase_work(m, n, k, l, 4.0, 4.0, "bf16")
    # only the two products with A run on BF16 matrix cores
    assert w["sketch_gemm"][2] == "bf16" and w["project_gemm"][2] == "bf16"
    for key in ("gram_gemm", "solve_gemm", "form_l_gemm", "panel_lu_y", "panel_lu_bt",
                "gram_inverse"):
        assert w[key][2] == "f64", key
    r = bench.step_roofline(w, 10.0)
    f64_tail = sum(w[key][0] for key in ("gram_gemm", "solve_gemm", "form_l_gemm", "panel_lu_y",
                                         "panel_lu_bt", "gram_inverse"))
    a_bytes = w["sketch_gemm"][1] + w["project_gemm"][1]
    want = max((w["sketch_gemm"][0] + w["project_gemm"][0]) / bench.PEAK["bf16"],
               a_bytes / bench.PEAK["hbm"]) + f64_tail / bench.PEAK["f64"]
    assert r["t_roof_ms"] == pytest.approx(want * 1e3)
    # about 0.30 ms of HBM time for the two passes over A plus 0.32 ms of FP64 tail
    assert 0.6 < r["t_roof_ms"] < 0.8


def test_dominant_roofline_picks_the_slowest_kernel():
    sys.path.insert(0, ROOT)
    import bench

    m, n, k, l = 16384, 16384, 500, 520
    w = bench.phase_work(m, n, k, l, 4.0, 4.0, "bf16")
    names = bench.KERNEL_NAMES["bf16"]
    kern = {"sketch_ms": 0.4, "panel_ms_per_launch": 1.5, "panel_launches_per_call": 4,
            "panel_ms_per_call": 6.0}
    r = bench.dominant_roofline(m, n, k, l, w, {"project_gemm": 0.5}, kern, names, {})
    assert r["kernel"] == names["panel_lu_kernel"] and r["bound"] == "alu"
    fl = (w["panel_lu_y"][0] + w["panel_lu_bt"][0]) / 4
    assert r["achieved"] == pytest.approx(fl / 1.5e-3 / 1e12)
    assert r["frac"] == pytest.approx(fl / 1.5e-3 / bench.PEAK["f64"])
    assert r["us_per_pivot_step"] == pytest.approx(6.0e3 / (l + k))
    kern = {"sketch_ms": 2.0, "panel_ms_per_launch": 0.1, "panel_launches_per_call": 4,
            "panel_ms_per_call": 0.4}
    r = bench.dominant_roofline(m, n, k, l, w, {"project_gemm": 0.5}, kern, names, {})
    assert r["kernel"] == names["sketch_gemm"] and r["bound"] == "hbm"
    assert r["achieved"] == pytest.approx(w["sketch_gemm"][1] / 2.0e-3 / 1e9)
