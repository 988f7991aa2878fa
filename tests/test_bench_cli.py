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


def test_cpu_baseline_uses_its_budget():
    """The oracle leg of the bench line: passes over the run's levels, sized
    from the measured rate, until most of the time budget is used -- both for
    a run that fits the budget many times and for one far too large for it
    (scaled down); the host threads, one thread, the CPU model and nproc are
    reported."""
    import time
    sys.path.insert(0, ROOT)
    import bench
    for N, budget in (([4000, 400, 100], 1.0), ([10**10, 10**9, 10**8], 1.0)):
        t0 = time.perf_counter()
        r = bench.cpu_baseline({"N": N}, 4, budget)
        wall = time.perf_counter() - t0
        assert r["kind"] == "oracle" and r["cores"] >= 1 and r["value"] > 0
        assert r["single_thread"]["value"] > 0 and r["nproc"] >= 1 and r["cpu_model"]
        # both legs spend most of their share of the budget sampling
        spent = r["single_thread"]["seconds"] + float(r["sample"].split(" in ")[1].split(" s")[0])
        assert spent >= 0.8 * budget, (N, spent)
        assert wall <= budget + 6.0, (N, wall)   # warm-up calls and probes
        if N[0] == 4000:
            assert r["single_thread"]["passes"] > 1
        else:
            assert r["scales"][0] < 0.1
