"""The benchmark's one-GPU contract, checked on the CPU: asked for more than
one GPU (by flag or by a launcher's WORLD_SIZE), bench.py exits with status 2
and a message before importing torch or touching a device; --help lists the
flags the records name."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env_extra=None):
    env = dict(os.environ)
    env.pop("WORLD_SIZE", None)
    if env_extra:
        env.update(env_extra)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                          capture_output=True, text=True, env=env, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    r = run([], {"WORLD_SIZE": "8"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_help_lists_the_measurement_flags():
    r = run(["--help"])
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--workload", "--approx-rate", "--fp64-ceiling",
                 "--copy-calibration", "--precision", "--pair-cache"):
        assert flag in r.stdout, flag
