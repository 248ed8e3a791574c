"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Error metric per wave vector q: max_m |D_gpu - D_oracle| / max_m D_oracle(q),
bound 1e-4 for FP32 spectra.  Integer results (bin indices, counts) must be
bit-exact.
"""

import ctypes
import os
import sys

import numpy as np
import pytest
import torch

from oracle import dft, radial, structure
from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_full(api, frames_cpu, **kw):
    N, H, W = frames_cpu.shape
    pixel = "u8" if frames_cpu.dtype == torch.uint8 else "u16"
    plan = api.Plan(W, H, N, pixel=pixel, **kw)
    D = plan.structure_function(frames_cpu.cuda())
    torch.cuda.synchronize()
    return plan, D.cpu().numpy()


def test_plain_config(gpu):
    say("case: plain 64x64x128 u8 seed 0")
    frames = synth.make(synth.PLAIN)
    plan, Dg = run_full(gpu, frames)
    Do, _ = oracle_D(frames.numpy())
    e = per_q_error(Dg, Do)
    say("plain:", describe(e))
    assert np.all(Dg[:, 0] == 0.0)
    assert e.max() <= TOL_F32


@pytest.mark.parametrize("W,H,N,pixel", [
    (48, 96, 64, "u16"), (96, 48, 33, "u8"), (128, 64, 200, "u16"), (384, 16, 20, "u16"),
    (16, 16, 5, "u8"), (64, 32, 2, "u16"), (32, 64, 1000, "u8")])
def test_shapes(gpu, W, H, N, pixel):
    say("case: shape", W, H, N, pixel)
    frames = synth.brownian_stack(W, H, N, n_spots=max(4, W * H // 40), sigma=1.5, amplitude=40.0,
                                  background=200.0, D0=0.3, seed=W + H + N, pixel=pixel)
    plan, Dg = run_full(gpu, frames)
    Do, _ = oracle_D(frames.numpy())
    e = per_q_error(Dg, Do)
    say("shape", W, H, N, describe(e))
    assert e.max() <= TOL_F32


@pytest.mark.parametrize("precondition", [True, False])
def test_step_one_spectra(gpu, precondition):
    say("case: step one, precondition", precondition)
    frames = synth.uniform_stack(96, 64, 9, seed=3, pixel="u16")
    N, H, W = frames.shape
    plan = gpu.Plan(W, H, N, pixel="u16", precondition=precondition)
    Fg = plan.image_spectra(frames.cuda()).cpu().numpy()
    fr = frames.numpy().astype(np.int64)
    if precondition:
        fr = fr - fr[:1]
    kx, ky, _ = dft.q_list(W, H)
    Fo = dft.dft_half_plane(fr)[:, ky, kx].T
    err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    say("step one rel err %.3e" % err)
    assert err < 2e-6


@pytest.mark.parametrize("padding", ["pow2", "minimal"])
@pytest.mark.parametrize("N", [2, 3, 5, 17, 100, 150, 192, 300, 384, 700, 768, 1000, 1200, 1536, 1537, 2048, 2500,
                               3000, 3072, 4096, 5000, 8192])
def test_step_two_from_spectra(gpu, N, padding):
    say("case: step two N =", N, padding)
    r = np.random.default_rng(N)
    Q = 37
    F = (r.standard_normal((Q, N)) + 1j * r.standard_normal((Q, N))).astype(np.complex64)
    F += np.complex64(20 + 5j)  # a static offset per q
    plan = gpu.Plan(16, 16, N, k2_max=40, padding=padding)  # step two only uses the plan's n_q and N
    nq = plan.n_q
    Fx = np.resize(F, (nq, N)).astype(np.complex64)
    Dg = plan.structure_from_spectra(torch.from_numpy(Fx).cuda()).cpu().numpy()
    Do = structure.structure_function_direct(Fx.astype(np.complex128))
    e = per_q_error(Dg, Do)
    say("N", N, padding, describe(e))
    assert e.max() <= TOL_F32


def test_k2_max_and_max_lag(gpu):
    say("case: k2_max 150, max_lag 40")
    frames = synth.brownian_stack(64, 64, 96, 100, 1.5, 40.0, 100.0, 0.5, seed=5, pixel="u8")
    plan, Dg = run_full(gpu, frames, k2_max=150, max_lag=40)
    kx, ky = plan.q_index()
    kxo, _, kyso = dft.q_list(64, 64, 150)
    np.testing.assert_array_equal(kx, kxo)
    np.testing.assert_array_equal(ky, kyso)
    assert Dg.shape == (len(kxo), 40)
    Do, _ = oracle_D(frames.numpy(), k2_max=150, max_lag=40)
    e = per_q_error(Dg, Do)
    say("k2_max:", describe(e))
    assert e.max() <= TOL_F32


def test_group_execution_bit_identical(gpu):
    say("case: group execution (minimum workspace)")
    frames = synth.brownian_stack(128, 96, 150, 300, 1.5, 40.0, 500.0, 0.2, seed=9).cuda()
    plan = gpu.Plan(128, 96, 150)
    mn, full = plan.workspace_size()
    plan.allocate_workspace(full)
    D_full = plan.structure_function(frames).clone()
    plan.allocate_workspace(mn)
    D_min = plan.structure_function(frames).clone()
    plan.allocate_workspace(mn + 3 * (full - mn) // 7)
    D_mid = plan.structure_function(frames).clone()
    torch.cuda.synchronize()
    assert torch.equal(D_full, D_min)
    assert torch.equal(D_full, D_mid)


def test_deterministic(gpu):
    say("case: determinism")
    frames = synth.brownian_stack(96, 96, 70, 200, 1.5, 40.0, 500.0, 0.2, seed=2).cuda()
    plan = gpu.Plan(96, 96, 70)
    a = plan.structure_function(frames).clone()
    b = plan.structure_function(frames).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("W,H", [(64, 64), (96, 48)])
def test_radial_average(gpu, W, H):
    say("case: radial", W, H)
    frames = synth.brownian_stack(W, H, 40, 100, 1.5, 40.0, 100.0, 0.5, seed=4, pixel="u8")
    plan, Dg = run_full(gpu, frames)
    kx, ky = plan.q_index()
    k2 = dft.k2_of(kx, ky, W, H)
    T = gpu.integer_bin_thresholds(int(np.sqrt(k2.max())) + 1)
    if (W, H) != (64, 64):
        T = np.unique(np.concatenate([[0], np.geomspace(1, k2.max() + 1, 25).astype(np.int64)]))
    Dbar, counts, boq = plan.radial_average(torch.from_numpy(Dg).cuda(), T)
    torch.cuda.synchronize()
    Do_bar, Do_counts, Do_b = radial.radial_average(Dg.astype(np.float64), kx, ky, W, H, T)
    np.testing.assert_array_equal(boq.cpu().numpy(), Do_b)
    np.testing.assert_array_equal(counts.cpu().numpy(), Do_counts)
    np.testing.assert_allclose(Dbar.cpu().numpy(), Do_bar, rtol=1e-12, atol=0)
    # and against the oracle's D end to end
    Do, _ = oracle_D(frames.numpy())
    Do_bar2, _, _ = radial.radial_average(Do, kx, ky, W, H, T)
    rel = np.abs(Dbar.cpu().numpy() - Do_bar2).max(axis=1) / np.maximum(Do_bar2.max(axis=1), 1e-300)
    assert rel[counts.cpu().numpy() > 0].max() <= TOL_F32


def test_radial_wide_bins_and_threshold_reuse(gpu):
    """384x384 (two 256-row chunks), 70 lags (a partial second lag tile), a bin
    with ~70k members (many list windows), an empty bin; the same thresholds
    again (no new copy) and then new ones; reruns are bit-identical."""
    say("case: radial wide bins 384x384x70")
    W = H = 384
    frames = synth.uniform_stack(W, H, 70, seed=9, pixel="u8")
    plan, Dg = run_full(gpu, frames)
    kx, ky = plan.q_index()
    k2max = int(dft.k2_of(kx, ky, W, H).max())
    D = torch.from_numpy(Dg).cuda()
    Ts = [np.array([0, 10, 10, 1000, k2max + 1], dtype=np.int64),
          np.array([0, 10, 10, 1000, k2max + 1], dtype=np.int64),
          np.array([3, 4000, 4001, 90000], dtype=np.int64)]
    first = None
    for i, T in enumerate(Ts):
        Dbar, counts, boq = plan.radial_average(D, T)
        torch.cuda.synchronize()
        Do_bar, Do_counts, Do_b = radial.radial_average(Dg.astype(np.float64), kx, ky, W, H, T)
        np.testing.assert_array_equal(boq.cpu().numpy(), Do_b)
        np.testing.assert_array_equal(counts.cpu().numpy(), Do_counts)
        np.testing.assert_allclose(Dbar.cpu().numpy(), Do_bar, rtol=1e-12, atol=0)
        if i == 0:
            assert Do_counts[1] == 0 and Do_counts[3] > 4 * 4096
            first = Dbar.clone()
        if i == 1:
            assert torch.equal(Dbar, first)


def test_radial_four_lag_lanes_match_one_lag_lanes(gpu):
    """Rows of D 16-byte aligned with M % 4 == 0 take four lags per lane; the
    same values one float off that alignment take one lag per lane: the
    summation order is the same, so the results are bit-identical."""
    say("case: radial lanes of 4 vs 1 lag, 96x96x64")
    W = H = 96
    frames = synth.uniform_stack(W, H, 64, seed=13, pixel="u8")
    plan, Dg = run_full(gpu, frames)
    kx, ky = plan.q_index()
    k2max = int(dft.k2_of(kx, ky, W, H).max())
    T = np.array([0, 1, 50, 51, 700, k2max + 1], dtype=np.int64)
    D = torch.from_numpy(Dg).cuda()
    buf = torch.empty(D.numel() + 1, dtype=torch.float32, device=D.device)
    Dmis = buf[1:].view(D.shape)
    Dmis.copy_(D)
    assert D.data_ptr() % 16 == 0 and Dmis.data_ptr() % 16 == 4
    a = plan.radial_average(D, T)
    b = plan.radial_average(Dmis, T)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    Do_bar, Do_counts, _ = radial.radial_average(Dg.astype(np.float64), kx, ky, W, H, T)
    np.testing.assert_array_equal(a[1].cpu().numpy(), Do_counts)
    np.testing.assert_allclose(a[0].cpu().numpy(), Do_bar, rtol=1e-12, atol=0)


@pytest.mark.parametrize("W,N,pixel,kw", [(64, 200, "u8", {}), (256, 96, "u16", {}), (512, 40, "u16", {}),
                                          (128, 64, "u16", {"k2_max": 900}),
                                          (256, 48, "u16", {"spectrum": "f16"})])
def test_fused_step_one_matches_split(gpu, W, N, pixel, kw):
    """Step one in one launch (square frames up to 512) gives the same bits as
    the separate row and column kernels."""
    say("case: fused vs split step one", W, N, pixel, kw)
    frames = synth.brownian_stack(W, W, N, max(4, W * W // 80), 1.5, 40.0, 300.0, 0.3, seed=21, pixel=pixel).cuda()
    a = gpu.Plan(W, W, N, pixel=pixel, **kw).structure_function(frames)
    os.environ["DDM_STEP1"] = "split"
    try:
        b = gpu.Plan(W, W, N, pixel=pixel, **kw).structure_function(frames)
    finally:
        del os.environ["DDM_STEP1"]
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_error_paths_leave_outputs_untouched(gpu):
    say("case: error paths")
    from paper_2012_05695_amd import _lib as L
    from paper_2012_05695_amd.api import _lib as lib
    plan = gpu.Plan(64, 64, 16)
    D = torch.full((plan.n_q, plan.max_lag), float("nan"), device="cuda")
    frames = torch.zeros((16, 64, 64), dtype=torch.uint16, device="cuda")
    h = plan.handle
    assert lib.ddm_structure_function(h, None, ctypes.c_void_p(D.data_ptr())) == L.DDM_ERR_INVALID_ARGUMENT
    # no workspace attached yet
    assert lib.ddm_structure_function(h, ctypes.c_void_p(frames.data_ptr()),
                                      ctypes.c_void_p(D.data_ptr())) == L.DDM_ERR_OUT_OF_MEMORY
    mn, _ = plan.workspace_size()
    small = torch.empty(mn - 256, dtype=torch.uint8, device="cuda")
    assert lib.ddm_plan_set_workspace(h, ctypes.c_void_p(small.data_ptr()), mn - 256) == L.DDM_ERR_OUT_OF_MEMORY
    thr = np.array([0, 5, 4], dtype=np.int64)  # decreasing: invalid
    out = torch.full((2, plan.max_lag), float("nan"), dtype=torch.float64, device="cuda")
    cnt = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    assert lib.ddm_radial_average(h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(thr.ctypes.data), 2,
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                  None) == L.DDM_ERR_INVALID_ARGUMENT
    torch.cuda.synchronize()
    assert torch.isnan(D).all() and torch.isnan(out).all() and (cnt == -7).all()


def test_static_stack_gives_zero(gpu):
    say("case: static stack")
    f0 = synth.uniform_stack(64, 48, 1, seed=1)
    frames = f0.repeat(50, 1, 1)
    plan, Dg = run_full(gpu, frames)
    assert np.all(Dg == 0.0)


def test_paper_config_sampled(gpu):
    """512x512x1024 uint16 (12-bit), oracle on the kx columns {0,1,7,128,256} x all ky."""
    say("case: paper-shaped 512x512x1024, sampled columns")
    frames = synth.make(synth.PAPER, device="cuda")
    plan = gpu.Plan(512, 512, 1024)
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    Dg = D.cpu().numpy()
    cols = [0, 1, 7, 128, 256]
    Do, rows = oracle_D(frames.cpu().numpy(), kx_subset=cols)
    e = per_q_error(Dg[rows], Do)
    say("paper sampled:", describe(e))
    assert e.max() <= TOL_F32


# ---- FP16 per-q-scaled spectrum store: bound 5e-3 ----
TOL_F16 = 5e-3


def test_fp16_plain_config(gpu):
    say("case: FP16 store, plain 64x64x128 u8")
    frames = synth.make(synth.PLAIN)
    plan, Dg = run_full(gpu, frames, spectrum="f16")
    Do, _ = oracle_D(frames.numpy())
    e = per_q_error(Dg, Do)
    say("plain f16:", describe(e))
    assert e.max() <= TOL_F16
    assert plan.fp16_saturations() == 0


def test_fp16_group_execution_bit_identical(gpu):
    say("case: FP16 store, group execution")
    frames = synth.brownian_stack(128, 96, 150, 300, 1.5, 40.0, 500.0, 0.2, seed=9).cuda()
    plan = gpu.Plan(128, 96, 150, spectrum="f16")
    mn, full = plan.workspace_size()
    plan.allocate_workspace(full)
    a = plan.structure_function(frames).clone()
    plan.allocate_workspace(mn)
    b = plan.structure_function(frames).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_fp16_saturation_is_reported(gpu):
    say("case: FP16 saturation warning")
    from paper_2012_05695_amd import _lib as L
    # static frames: the pilot frames see no change, so every scale is 2^0;
    # a bright non-pilot frame then exceeds the FP16 range
    frames = synth.uniform_stack(64, 64, 1, seed=2).repeat(64, 1, 1)
    frames[5] = 4095
    plan = gpu.Plan(64, 64, 64, spectrum="f16")
    plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    assert plan.fp16_saturations() > 0
    plan.structure_function(frames.cuda())
    assert plan.last_status == L.DDM_WARN_FP16_SATURATED


def test_fp16_paper_config_sampled(gpu):
    """512x512x1024 uint16, FP16 spectra, oracle on kx columns {0,1,7,128,256}."""
    say("case: FP16 store, paper-shaped 512x512x1024, sampled columns")
    frames = synth.make(synth.PAPER, device="cuda")
    plan = gpu.Plan(512, 512, 1024, spectrum="f16")
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    Dg = D.cpu().numpy()
    Do, rows = oracle_D(frames.cpu().numpy(), kx_subset=[0, 1, 7, 128, 256])
    e = per_q_error(Dg[rows], Do)
    say("paper f16 sampled:", describe(e))
    assert e.max() <= TOL_F16
    assert plan.fp16_saturations() == 0


def test_fp16_saturation_count_over_many_calls(gpu):
    say("case: FP16 saturation counts of calls in flight")
    # more calls than the host keeps in flight before it waits: every call's
    # count is folded in exactly once
    frames = synth.uniform_stack(64, 64, 1, seed=2).repeat(64, 1, 1)
    frames[5] = 4095
    frames = frames.cuda()
    plan = gpu.Plan(64, 64, 64, spectrum="f16")
    plan.structure_function(frames)
    one = plan.fp16_saturations()
    assert one > 0
    for _ in range(9):
        plan.structure_function(frames)
    assert plan.fp16_saturations() == 10 * one
