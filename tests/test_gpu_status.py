"""Device-side outcomes come back to the caller: the single-launch step one's
error flag (forced from the host: the plan starts that kernel with its flag
raised, so every bounded wait gives up at once and the kernel exits normally)
and the FP16 saturation warning, for one plan and per stack of a batch."""

import os

import pytest
import torch

from paper_2012_05695_amd import _lib as L
from paper_2012_05695_amd import synth

pytestmark = pytest.mark.gpu


def forced(make):
    os.environ["DDM_STEP1_FAIL"] = "1"
    try:
        return make()
    finally:
        del os.environ["DDM_STEP1_FAIL"]


def test_plan_status_reports_forced_step_one_failure(gpu):
    print("case: plan status, forced step-one failure 256x256x64", flush=True)
    frames = synth.brownian_stack(256, 256, 64, 300, 1.5, 40.0, 300.0, 0.3, seed=1).cuda()
    plan = forced(lambda: gpu.Plan(256, 256, 64))
    plan.structure_function(frames)
    with pytest.raises(gpu.DdmError) as ei:
        plan.status()
    assert ei.value.status == L.DDM_ERR_HIP
    assert "not valid" in str(ei.value)
    assert plan.status() == L.DDM_OK  # reported once, then cleared
    # the asynchronous path: a later call takes in the earlier call's outcome
    plan.structure_function(frames)
    torch.cuda.synchronize()
    with pytest.raises(gpu.DdmError) as ei:
        plan.structure_function(frames)
    assert ei.value.status == L.DDM_ERR_HIP
    plan.close()
    # an ordinary plan on the same frames reports nothing
    ok = gpu.Plan(256, 256, 64)
    ok.structure_function(frames)
    assert ok.status() == L.DDM_OK


def test_plan_status_reports_saturation_once(gpu):
    print("case: plan status, FP16 saturation", flush=True)
    frames = synth.uniform_stack(64, 64, 1, seed=2).repeat(64, 1, 1)
    frames[5] = 4095
    plan = gpu.Plan(64, 64, 64, spectrum="f16")
    plan.structure_function(frames.cuda())
    assert plan.status() == L.DDM_WARN_FP16_SATURATED
    assert plan.status() == L.DDM_OK


def test_batch_status_per_stack(gpu):
    print("case: batch status, forced step-one failure in the single-launch stacks", flush=True)
    shapes = [(128, 128, 64), (96, 64, 40), (1024, 1024, 8), (256, 256, 33)]
    fr = [synth.brownian_stack(w, h, n, max(4, w * h // 100), 1.5, 40.0, 300.0, 0.3, seed=i, pixel="u16").cuda()
          for i, (w, h, n) in enumerate(shapes)]
    batch = forced(lambda: gpu.Batch(shapes, lanes=2))
    batch.structure_function(fr)
    # square stacks up to 512 x 512 run the single-launch step one; the others do not
    expect = [L.DDM_ERR_HIP, L.DDM_OK, L.DDM_OK, L.DDM_ERR_HIP]
    assert batch.status() == expect
    assert batch.status() == [L.DDM_OK] * 4
    batch.structure_function(fr)                 # graph replay
    torch.cuda.synchronize()
    with pytest.raises(gpu.DdmError) as ei:      # the replay's outcome comes back on the next call
        batch.structure_function(fr)
    assert ei.value.status == L.DDM_ERR_HIP and "stack(s) 0, 3" in str(ei.value)
    batch.close()
    ok = gpu.Batch(shapes, lanes=2)
    Db = ok.structure_function(fr)
    assert ok.status() == [L.DDM_OK] * 4
    for i, (w, h, n) in enumerate(shapes):
        assert torch.equal(Db[i], gpu.Plan(w, h, n).structure_function(fr[i]))
