"""bench.py's command line on the CPU: more than one GPU is refused with a message (the
library has no multi-GPU path), before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = run(["--gpus", n])
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_a_distributed_launch_is_refused():
    env = dict(os.environ, WORLD_SIZE="4", RANK="0", LOCAL_RANK="0")
    r = run(["--gpus", "1"], env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr
