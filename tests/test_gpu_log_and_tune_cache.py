"""DDM_LOG and the on-disk autotune cache (DDM_TUNE_CACHE), in child
processes (the library reads DDM_LOG once per process): the first process
times and appends its results, the second reads them back instead of timing,
for both step-two methods of an automatic plan."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
sys.path.insert(0, %r)
import torch
from paper_2012_05695_amd import api, synth
plan = api.Plan(128, 128, 256, max_lag=16, method="auto")
plan.allocate_workspace()
E, q, ms = plan.autotune()
fr = synth.uniform_stack(128, 128, 256, seed=1).cuda()
plan.structure_function(fr)
torch.cuda.synchronize()
print("RESULT", E, q, "%%.6f" %% ms, plan.method, flush=True)
""" % ROOT


def run(env):
    r = subprocess.run([sys.executable, "-c", SCRIPT], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    res = [line for line in r.stdout.splitlines() if line.startswith("RESULT")]
    return res[0].split()[1:], r.stderr


def test_log_and_autotune_cache_across_processes(gpu, tmp_path):
    print("case: DDM_LOG and DDM_TUNE_CACHE, 128x128x256 auto, two child processes", flush=True)
    cache = str(tmp_path / "tune.txt")
    env = dict(os.environ, DDM_LOG="1", DDM_TUNE_CACHE=cache)
    first, log1 = run(env)
    assert "[ddm] plan" in log1 and "step two" in log1 and "[ddm] autotune plan" in log1
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and " fourier " in lines[0] and " direct " in lines[1]
    assert lines[0].split()[0].startswith("gfx")
    second, log2 = run(env)
    assert "2 result(s)" in log2 and log2.count("(cached)") == 2
    assert second == first  # the same shape, time and method from the file
    assert len(open(cache).read().splitlines()) == 2  # nothing timed, nothing appended
    # without DDM_LOG nothing is printed
    quiet = dict(os.environ, DDM_TUNE_CACHE=cache)
    quiet.pop("DDM_LOG", None)
    _, log3 = run(quiet)
    assert "[ddm]" not in log3
