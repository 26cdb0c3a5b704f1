"""bench.py's command line on a machine without a GPU: a run on more than
one GPU is refused with a message before anything touches a device, and the
workloads the harness knows are all offered.  No device work here."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = run("--gpus", n)
        assert r.returncode != 0
        out = r.stdout + r.stderr
        assert "exactly one GPU" in out and f"asked for {n}" in out
        assert not any(line.startswith("{") for line in r.stdout.splitlines())  # no result line


def test_workloads_offered():
    r = run("--help")
    assert r.returncode == 0
    for w in ("rmat16", "batched", "serve", "forms"):
        assert w in r.stdout
