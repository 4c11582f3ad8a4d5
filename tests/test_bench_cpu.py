"""bench.py's contract on a machine without a GPU: more than one GPU is refused
with a message, and without a visible GPU the run fails loudly instead of
printing a result line (there is no CPU fallback).  The roofline's measured
traffic comes from the committed counter record only while the kernel sources
hash to the ones it was taken on."""
import json
import os
import shutil
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


def test_traffic_record_is_keyed_to_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_step_tgv256_traffic.json")))
    val = bench.measured_traffic()
    if val is not None:
        # 140 B read and 140 B written per cell update, 256^3 cells per launch
        assert val == rec["traffic_bytes_per_launch"]
        assert abs(val / (16777216 * 280) - 1) < 1e-3
    # a copy of the tree whose kernel source differs by one byte gets no traffic
    for rel in ["profiles/k_step_tgv256_traffic.json"] + rec["sources"]:
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    with open(tmp_path / rec["sources"][0], "a") as fh:
        fh.write("\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic() is None
