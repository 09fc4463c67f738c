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
    r = bench.step_roofline(w, bench.PEAK["f64"], 3.0)
    gem = sum(v[0] for key, v in w.items() if key.endswith("gemm"))
    assert r["t_roof_ms"] >= gem / bench.PEAK["f64"] * 1e3
    assert 0.0 < r["frac"] < 1.0
