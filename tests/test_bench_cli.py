"""Command-line contract of bench.py that holds without a GPU.

The benchmark measures one GPU: asked for more (flag or a launcher's
WORLD_SIZE) it exits with status 2 and says why, before touching any device.
"""
import os
import subprocess
import sys

import pytest

from conftest import ROOT


def run_bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          env=env, capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None),
                                      (["--gpus", "8", "--steps", "1"], None),
                                      (["--gpus", "1"], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = run_bench(args, env)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""          # no JSON line for a configuration it does not run


def test_help_lists_the_run_flags():
    r = run_bench(["--help"])
    assert r.returncode == 0
    for flag in ["--gpus", "--steps", "--warmup"]:
        assert flag in r.stdout
