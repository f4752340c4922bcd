"""bench.py's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    """The library drives one GPU: --gpus above 1 exits with a message
    instead of reporting a figure."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench():
    import importlib
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    return importlib.import_module("bench")


def test_birthday_fit_reproduces_its_own_input():
    """alpha fitted at N=4096, k=64 and used at k = sqrt(N) predicts the same
    probability for every N (Sec. 3.4: constant for k ~ sqrt(N))."""
    import math
    b = _bench()
    p = 0.3
    out = b.birthday({"legs": 40, "N4096": {"8": p}, "N65536": {"8": 0.31}, "N1048576": {"8": 0.29}})
    row = out["by_T"]["8"]
    assert math.isclose(row["alpha"], -2 * 4096 * math.log(1 - p) / 64 ** 2)
    assert math.isclose(row["N65536_predicted"], p) and math.isclose(row["N1048576_predicted"], p)
    assert not row["alpha_is_bound"]
    # a saturated measurement is clipped and marked as a bound
    sat = b.birthday({"legs": 40, "N4096": {"34": 1.0}})["by_T"]["34"]
    assert sat["alpha_is_bound"] and math.isfinite(sat["alpha"])


def test_cpu_oracle_on_all_cores_reports_its_cores():
    b = _bench()
    r = b.cpu_baseline_batch(4, 200, max_procs=2)
    assert r["kind"] == "oracle" and r["cores"] in (1, 2) and r["value"] > 0
    assert r["cpu_model"]
