"""The benchmark's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, env=env)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""


def test_a_distributed_launch_is_refused_too():
    env = dict(os.environ, WORLD_SIZE="4")
    r = _bench(env=env)
    assert r.returncode == 2
    assert "single GPU" in r.stderr


def test_help_lists_the_modes():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--batched-only", "--serving-only", "--streaming-only",
                 "--copy-probe", "--placement-probe"):
        assert flag in r.stdout
