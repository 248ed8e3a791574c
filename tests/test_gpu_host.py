"""Frames resident in host memory: copies through a small device staging
buffer overlap the two-kernel step one; the result equals the device-resident
path bit for bit (the single-launch step one equals the two-kernel one)."""

import numpy as np
import pytest
import torch

from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,H,N,pixel,batch_frames,kw", [(256, 256, 300, "u16", 3, {}), (96, 64, 77, "u8", 5, {}),
                                                        (64, 64, 128, "u8", 1, {"k2_max": 300, "max_lag": 60}),
                                                        (512, 512, 200, "u16", 16, {}),
                                                        (96, 64, 77, "u16", 4, {"method": "direct", "max_lag": 20})])
def test_host_frames_match_device_frames(gpu, W, H, N, pixel, batch_frames, kw):
    print("case: host frames", W, H, N, pixel, batch_frames, kw, flush=True)
    frames = synth.brownian_stack(W, H, N, max(4, W * H // 50), 1.5, 40.0, 300.0, 0.3, seed=N, pixel=pixel)
    plan = gpu.Plan(W, H, N, pixel=pixel, **kw)
    ref = plan.structure_function(frames.cuda()).clone()
    fb = W * H * (1 if pixel == "u8" else 2)
    staging = torch.empty(((fb + 255) // 256) * 256 + 2 * batch_frames * fb + 512, dtype=torch.uint8, device="cuda")
    pinned = frames.pin_memory()
    out = plan.structure_function_host(pinned, staging)
    out2 = plan.structure_function_host(pinned, staging)      # the staging memory reused
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(out2, ref)
    if W * H <= 96 * 64:
        Do, _ = oracle_D(frames.numpy(), k2_max=kw.get("k2_max", -1), max_lag=kw.get("max_lag"))
        e = per_q_error(out.cpu().numpy(), Do)
        print("host frames:", describe(e), flush=True)
        assert e.max() <= TOL_F32


def test_host_frames_group_execution(gpu):
    print("case: host frames, minimum workspace (every group copies the frames again)", flush=True)
    frames = synth.brownian_stack(128, 96, 150, 300, 1.5, 40.0, 500.0, 0.2, seed=9)
    plan = gpu.Plan(128, 96, 150)
    ref = plan.structure_function(frames.cuda()).clone()
    mn, full = plan.workspace_size()
    plan.allocate_workspace(mn + (full - mn) // 5)
    staging = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    out = plan.structure_function_host(frames.pin_memory(), staging)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_host_frames_rejects_small_staging(gpu):
    from paper_2012_05695_amd import _lib as L
    plan = gpu.Plan(64, 64, 16)
    staging = torch.empty(64 * 64 * 2 * 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu.DdmError) as ei:
        plan.structure_function_host(torch.zeros((16, 64, 64), dtype=torch.uint16), staging)
    assert ei.value.status == L.DDM_ERR_OUT_OF_MEMORY
