"""The no-allocation entry point (static device scratch as the workspace)
against the ordinary entry point, through the C ABI: two calls in a row, the
second on a smaller stack, then the first again (the scratch keeps the last
call's contents; nothing may depend on them)."""

import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(api, frames, **kw):
    N, H, W = frames.shape
    pixel = "u8" if frames.dtype == torch.uint8 else "u16"
    plan = api.Plan(W, H, N, pixel=pixel, **kw)
    ref = plan.structure_function(frames).clone()
    out = torch.full_like(ref, float("nan"))
    plan.structure_function_noalloc(frames, out=out)
    torch.cuda.synchronize()
    return plan, ref, out


def test_noalloc_matches_workspace_entry_point(gpu):
    # 512 x 512 x 1024 needs more than the scratch for one group: several groups
    say("case: noalloc 512x512x1024 u16 (grouped on the scratch)")
    big = synth.make(synth.PAPER, device="cuda")
    plan, ref, out = run_pair(gpu, big)
    mn, full = plan.workspace_size()
    assert full > gpu.NOALLOC_SCRATCH_BYTES >= mn
    assert torch.equal(ref, out)
    say("case: noalloc 96x64x200 u8 (smaller, after the larger call)")
    small = synth.brownian_stack(96, 64, 200, 150, 1.5, 40.0, 100.0, 0.4, seed=11, pixel="u8")
    plan2, ref2, out2 = run_pair(gpu, small.cuda())
    assert torch.equal(ref2, out2)
    Do, _ = oracle_D(small.numpy())
    e = per_q_error(out2.cpu().numpy(), Do)
    say("noalloc small:", describe(e))
    assert e.max() <= TOL_F32
    # FP16 store and the larger stack again on the same scratch
    say("case: noalloc FP16 store 128x128x300, then 512x512x1024 again")
    f16 = synth.brownian_stack(128, 128, 300, 300, 1.5, 40.0, 400.0, 0.3, seed=12, pixel="u16").cuda()
    _, ref3, out3 = run_pair(gpu, f16, spectrum="f16")
    assert torch.equal(ref3, out3)
    out4 = torch.full_like(ref, float("nan"))
    plan.structure_function_noalloc(big, out=out4)
    torch.cuda.synchronize()
    assert torch.equal(ref, out4)


def test_noalloc_rejects_plans_beyond_the_scratch(gpu):
    say("case: noalloc size limit")
    from paper_2012_05695_amd import _lib as L
    from paper_2012_05695_amd.api import _lib as lib
    # FP16 store at 4096 x 4096: its per-q pilot spectra alone exceed the scratch
    plan = gpu.Plan(4096, 4096, 64, spectrum="f16")
    mn, _ = plan.workspace_size()
    assert mn > gpu.NOALLOC_SCRATCH_BYTES
    frames = torch.zeros((64, 16, 16), dtype=torch.uint16, device="cuda")  # never read
    D = torch.full((4, 4), float("nan"), device="cuda")
    st = lib.ddm_structure_function_noalloc(plan.handle, ctypes.c_void_p(frames.data_ptr()),
                                           ctypes.c_void_p(D.data_ptr()))
    assert st == L.DDM_ERR_UNSUPPORTED
    assert b"scratch" in lib.ddm_last_error()
    torch.cuda.synchronize()
    assert torch.isnan(D).all()
