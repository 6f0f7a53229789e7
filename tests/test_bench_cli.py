"""The benchmark script's command line on the CPU: one GPU only, and the option set parses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_options_parse():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--workload", "--tile", "--convergence", "--modes", "--repeats"):
        assert opt in r.stdout


def test_cpu_baseline_waits_for_the_gpu_measurements():
    """The oracle baseline process does nothing until released (so it never overlaps the GPU timing),
    then reports its time per iteration and the threads it used."""
    import multiprocessing as mp
    import queue as q

    sys.path.insert(0, ROOT)
    import bench
    ctx = mp.get_context("spawn")
    res, go = ctx.Queue(), ctx.Event()
    p = ctx.Process(target=bench.cpu_baseline_worker, args=(res, go, "c0", 8, 2), daemon=True)
    p.start()
    try:
        try:
            res.get(timeout=3.0)
            raise AssertionError("the worker ran before it was released")
        except q.Empty:
            pass
        go.set()
        out = res.get(timeout=240)
        assert out["ok"], out
        assert out["threads"] == 2 and out["sec_per_iter"] > 0
    finally:
        p.join(timeout=30)
        if p.is_alive():
            p.kill()
    hc = bench.host_cpu()
    assert hc["nproc"] >= 1
