"""The single-launch step one at other pipeline depths (DDM_STEP1_LAG column
items behind their rows, DDM_STEP1_BUFS frame buffers per XCD; read once per
process, so each depth runs in a child process): the same bits as the default
depth, for square frames of 128, 256 and 512 pixels."""

import os
import subprocess
import sys

import pytest
import torch

from paper_2012_05695_amd import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHAPES = [(128, 128, 500, "u8"), (256, 256, 200, "u16"), (512, 512, 64, "u16")]

CHILD = r"""
import sys
sys.path.insert(0, %r)
import torch
from paper_2012_05695_amd import api
data = torch.load(sys.argv[1], weights_only=True)
out = {}
for key, frames in data.items():
    W, H, N, pixel = key.split("_")
    plan = api.Plan(int(W), int(H), int(N), pixel=pixel)
    out[key] = plan.structure_function(frames.cuda()).cpu()
    assert plan.status() == 0
torch.save(out, sys.argv[2])
print("child done", flush=True)
""" % ROOT


def test_step_one_pipeline_depths_give_the_same_bits(gpu, tmp_path):
    print("case: step-one pipeline depths (lag, buffers) 1/2, 2/3, 4/8 against the default", flush=True)
    frames = {"%d_%d_%d_%s" % s: synth.brownian_stack(s[0], s[1], s[2], max(4, s[0] * s[1] // 60), 1.5, 40.0,
                                                       300.0, 0.3, seed=s[2], pixel=s[3]) for s in SHAPES}
    ref = {}
    for key, fr in frames.items():
        W, H, N, pixel = key.split("_")
        ref[key] = gpu.Plan(int(W), int(H), int(N), pixel=pixel).structure_function(fr.cuda()).cpu()
    torch.cuda.synchronize()
    src = str(tmp_path / "frames.pt")
    torch.save(frames, src)
    for lag, bufs in [(1, 2), (2, 3), (4, 8)]:
        dst = str(tmp_path / ("D_%d_%d.pt" % (lag, bufs)))
        env = dict(os.environ, DDM_STEP1_LAG=str(lag), DDM_STEP1_BUFS=str(bufs))
        r = subprocess.run([sys.executable, "-c", CHILD, src, dst], capture_output=True, text=True, env=env,
                           timeout=240)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
        got = torch.load(dst, weights_only=True)
        for key in frames:
            assert torch.equal(got[key], ref[key]), (lag, bufs, key)
        print("lag %d, %d buffers: identical" % (lag, bufs), flush=True)
