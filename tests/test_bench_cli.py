"""The benchmark's command-line contract, checked on the CPU: one GPU only, and the options that the profiles'
commands use exist."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_options_used_by_profile_commands_exist():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--only", "--extra-steps", "--tune-cache", "--copy-calibration",
                "--stream-bandwidth", "--no-cpu", "--no-extra"):
        assert opt in r.stdout, opt
