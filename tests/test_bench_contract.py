"""The bench script's command-line contract, checked without a GPU: more than
one GPU is refused with a message before any device work, and the metric
metadata it prints is the fixed one."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_refused_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    msg = r.stdout + r.stderr
    assert "one GPU" in msg
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def test_metric_metadata_in_source():
    src = open(os.path.join(ROOT, "bench.py")).read()
    for field in ('"metric"', '"value"', '"unit"', '"n_gpus"', '"steps"', '"warmup"',
                  '"ms_per_step"', '"higher_is_better"', '"scaling"', '"vs_baseline"',
                  '"dtype"', '"data"', '"config"', '"roofline"', '"cpu_baseline"'):
        assert field in src, field
