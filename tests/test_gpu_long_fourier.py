"""Step two by the Fourier route at the time-transform length L = 16384
(8192 < N <= 16384, N2 = 32768 in Eq. (B4)).

Each case is compared with the oracle (FP64 direct differences, Eq. (1), of a
naive DFT) on every ky and every lag of a subset of kx columns:
  * N = L = 16384, all lags (the 16 largest lags summed directly);
  * N = 12000 with max_lag 6000 (a zero-padded tail, truncated output);
  * the FP16 per-q-scaled store at N = 9000;
  * the plain [q][N] layout (the step-two-only call) at N = 8193, 9000 and 16384;
  * the same D bit for bit on a second call (fixed-order sums, no atomics);
  * a batch (captured graph) holding such a stack, bit-identical to single plans;
  * holes of a low-q cut in the blocked store, with the minimum workspace
    (several groups of wave vectors).
"""

import sys

import numpy as np
import pytest
import torch

from oracle import structure
from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_sampled(D_dev, frames_dev, cols, label, max_lag=None, tol=TOL_F32):
    Dg = D_dev.cpu().numpy()
    Do, rows = oracle_D(frames_dev.cpu().numpy(), kx_subset=cols, max_lag=max_lag)
    e = per_q_error(Dg[rows], Do)
    say(label, "(%d q):" % len(rows), describe(e))
    assert e.max() <= tol
    assert np.all(Dg[:, 0] == 0.0)
    assert np.all(np.isfinite(Dg))


def test_fourier_64x64x16384(gpu):
    say("case: fourier 64x64x16384 u16 (N = L), kx columns {0, 5, 32}")
    frames = synth.brownian_stack(64, 64, 16384, 40, 1.5, 40.0, 800.0, 0.1, seed=16385, pixel="u16", device="cuda")
    plan = gpu.Plan(64, 64, 16384)
    assert plan.method == "fourier"
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    assert plan.status() == 0
    D2 = plan.structure_function(frames)
    torch.cuda.synchronize()
    assert torch.equal(D, D2)
    check_sampled(D, frames, [0, 5, 32], "64x64x16384 fourier")


def test_fourier_32x32x12000_truncated(gpu):
    say("case: fourier 32x32x12000 u8, max_lag 6000, kx columns {0, 7, 16}")
    frames = synth.brownian_stack(32, 32, 12000, 12, 1.5, 40.0, 200.0, 0.3, seed=12000, pixel="u8", device="cuda")
    plan = gpu.Plan(32, 32, 12000, pixel="u8", max_lag=6000, method="fourier")
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    assert D.shape[1] == 6000
    check_sampled(D, frames, [0, 7, 16], "32x32x12000 fourier, 6000 lags", max_lag=6000)


def test_fourier_f16_32x32x9000(gpu):
    say("case: fourier 32x32x9000 u16, FP16 store, kx columns {0, 3}")
    frames = synth.brownian_stack(32, 32, 9000, 12, 1.5, 40.0, 400.0, 0.3, seed=9001, pixel="u16", device="cuda")
    plan = gpu.Plan(32, 32, 9000, spectrum="f16", method="fourier")
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    check_sampled(D, frames, [0, 3], "32x32x9000 fourier FP16 store", tol=5e-3)


@pytest.mark.parametrize("N", [8193, 9000, 16384])
def test_fourier_plain_layout(gpu, N):
    say("case: step two from [q][N] spectra, N =", N)
    r = np.random.default_rng(N)
    plan = gpu.Plan(16, 16, N, k2_max=12, method="fourier")
    nq = plan.n_q
    F = (r.standard_normal((nq, N)) + 1j * r.standard_normal((nq, N))).astype(np.complex64)
    F += np.complex64(20 + 5j)  # a static offset per q
    Dg = plan.structure_from_spectra(torch.from_numpy(F).cuda()).cpu().numpy()
    Do = structure.structure_function_direct(F.astype(np.complex128))
    e = per_q_error(Dg, Do)
    say("N", N, "(%d q)" % nq, describe(e))
    assert e.max() <= TOL_F32


def test_method_choice_at_16384(gpu):
    """DDM_METHOD_AUTO at N = 16384: the cost model takes direct differences
    below the measured crossover (about 224 lags at 512x512) and the transform
    above it; ddm_plan_autotune times both and reports the length-16384
    kernel's single launch shape."""
    say("case: method choice at N = 16384")
    for M, want in ((192, "direct"), (256, "fourier")):
        plan = gpu.Plan(64, 64, 16384, max_lag=M, method="auto")
        assert plan.method == want, (M, plan.method)
        plan.close()
    plan = gpu.Plan(64, 64, 16384, max_lag=192, method="auto")
    E, qpw, ms = plan.autotune()
    say("autotune 64x64x16384, 192 lags:", plan.method, E, qpw, "%.3f ms" % ms)
    assert (E, qpw) == (16, 1) and ms > 0
    assert plan.method in ("direct", "fourier")
    plan.close()


def test_batch_with_long_stack(gpu):
    """A batch (one captured graph over two lanes) holding a stack on the
    length-16384 transform: D bit-identical to single plans, on the first
    capture and on a replay."""
    say("case: batch of 32x32x9000 and 64x64x300 on two lanes")
    shapes = [(32, 32, 9000), (64, 64, 300)]
    fr = [synth.brownian_stack(W, H, N, 12, 1.5, 40.0, 400.0, 0.2, seed=9100 + i, pixel="u16", device="cuda")
          for i, (W, H, N) in enumerate(shapes)]
    batch = gpu.Batch(shapes, lanes=2)
    Db = [d.clone() for d in batch.structure_function(fr)]
    Db2 = batch.structure_function(fr)  # graph replay
    torch.cuda.synchronize()
    for i, (W, H, N) in enumerate(shapes):
        plan = gpu.Plan(W, H, N)
        Ds = plan.structure_function(fr[i])
        torch.cuda.synchronize()
        assert torch.equal(Db[i], Ds), i
        assert torch.equal(Db2[i], Ds), i
        plan.close()


def test_fourier_long_holes_and_groups(gpu):
    """Length-16384 transform on the blocked store with holes (a low-q cut)
    and the minimum workspace (several groups of wave vectors, every frame
    transformed per group); every q against the oracle."""
    say("case: fourier 32x32x9000 u8, k2_max 60, minimum workspace")
    frames = synth.brownian_stack(32, 32, 9000, 12, 1.5, 40.0, 200.0, 0.3, seed=9060, pixel="u8")
    plan = gpu.Plan(32, 32, 9000, pixel="u8", k2_max=60, method="fourier")
    mn, full = plan.workspace_size()
    plan.allocate_workspace(mn)
    D = plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    assert plan.status() == 0
    Do, _ = oracle_D(frames.numpy(), k2_max=60)
    e = per_q_error(D.cpu().numpy(), Do)
    say("32x32x9000 k2_max 60, min workspace (%d q):" % D.shape[0], describe(e), "(full ws %d, min %d)" % (full, mn))
    assert e.max() <= TOL_F32
    assert np.all(D[:, 0].cpu().numpy() == 0.0)
