"""bench.py's command line on the CPU: the one-GPU rule (no compute)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""          # no JSON line


def test_bench_help_lists_the_contract_flags():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup"):
        assert flag in r.stdout


def test_cpu_baseline_fills_its_budget_with_whole_runs():
    """The oracle leg of the bench line: a run that fits the time budget is
    repeated, a larger one is scaled down; both report the oracle kind."""
    sys.path.insert(0, ROOT)
    import bench
    small = bench.cpu_baseline({"N": [4000, 400, 100]}, 4, 0.3)
    assert small["kind"] == "oracle" and small["cores"] >= 1 and small["value"] > 0
    assert "pass(es)" in small["sample"] and not small["sample"].startswith("1 pass")
    big = bench.cpu_baseline({"N": [10**10, 10**9, 10**8]}, 4, 0.3)
    assert "scaled by" in big["sample"] and big["value"] > 0
