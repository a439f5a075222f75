"""Host-side logic of bench.py (no GPU): the per-cell byte counts behind the roofline,
the source-hash guard on the committed counter summaries, and the one-GPU limit."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bytes_per_cell():
    """FP64 3D: 11 values at 27 points (2376 B), 24 unique velocity dofs read and written
    (384 B), 27 int32 node indices (108 B) = 2868 B; the A-only kernel reads one value per
    point less (2652 B); FP32: 1188 + 192 + 108 = 1488 B."""
    b = _bench()
    assert b.algorithmic_bytes_per_cell(3, 8) == 2868
    assert b.kernel_bytes_per_cell(3, 8) == 2652
    assert b.algorithmic_bytes_per_cell(3, 4) == 1488
    # 2D: 6 values at 9 points, 8 unique dofs, 9 indices
    assert b.algorithmic_bytes_per_cell(2, 8) == 6 * 9 * 8 + 2 * 4 * 2 * 8 + 4 * 9


def test_counter_profiles_follow_the_kernel_source():
    """The committed counter summaries are used only while their source hash matches
    the cell-kernel source; a changed source gives no traffic figure."""
    b = _bench()
    for form, prec, var in (("phased", "fp64", 0), ("atomic", "fp64", 16), ("atomic", "fp64", 21),
                            ("atomic", "fp32", 20), ("atomic", "fp32", 17)):
        prof = b.load_counter_profile("C3", form, prec, var)
        assert prof is not None, (form, prec, var)
        assert prof["variant"] == var and prof["hbm_bytes_per_launch"] > 0
    assert b.load_counter_profile("C3", "atomic", "fp32")["fp32_flops_per_launch"] > 0
    # a variant with no summary of its own gives no traffic figure
    assert b.load_counter_profile("C3", "atomic", "fp64", 18) is None
    b.cell_kernel_source_hash = lambda: "0" * 16
    assert b.load_counter_profile("C3") is None
    assert b.load_counter_profile("C3", "atomic") is None
    assert b.load_counter_profile("C3", "atomic", "fp32") is None
    assert b.load_counter_profile("no-such-workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
