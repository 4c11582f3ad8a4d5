"""bench.py's contract on a machine without a GPU: more than one GPU is refused
with a message, and without a visible GPU the run fails loudly instead of
printing a result line (there is no CPU fallback)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    env = dict(os.environ, HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, cwd=ROOT, env=env, timeout=600)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_no_gpu_fails_without_a_result_line():
    r = run("--steps", "2", "--warmup", "1", "--no-cpu-baseline", "--no-batch", "--no-serve")
    assert r.returncode != 0
    assert '"metric"' not in r.stdout
