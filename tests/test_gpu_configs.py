"""Parity at the shapes the measured workloads run through.

Each case names the kernel instances it reaches:
  * 1024 x 1024 frames: the two-kernel step one (row and column transforms of
    length 1024, the column workgroup of 1024 threads);
  * N = 2048: the time transform of length L = 2048 with N = L (no padding);
  * minimal padding: transform lengths 3 * 2^k (N = 700, 1536, 2049, 3000,
    3072, ...), with and without a zero-padded tail, max_lag < N and the FP16
    store;
  * a batch with a 1024 x 1024 stack and a 512 x 512 stack of 2500 frames on
    two lanes.
The oracle (FP64 direct differences of a naive DFT) covers every ky, every
lag and a subset of kx columns where the full set would take minutes.
"""

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


def check_sampled(D_dev, frames_dev, cols, label):
    Dg = D_dev.cpu().numpy()
    Do, rows = oracle_D(frames_dev.cpu().numpy(), kx_subset=cols)
    e = per_q_error(Dg[rows], Do)
    say(label, "(%d q):" % len(rows), describe(e))
    assert e.max() <= TOL_F32
    assert np.all(Dg[:, 0] == 0.0)
    return e


def test_learned_shape_1024x1024x2048(gpu):
    """1024 x 1024 u16 x 2048 frames (the fit workload's stack): step one in two
    kernels of length 1024, the time transform at L = N = 2048."""
    say("case: 1024x1024x2048 u16, kx columns {0,1,5,300,511,512}")
    frames = synth.brownian_stack(1024, 1024, 2048, 8000, 1.5, 40.0, 800.0, 0.75, seed=7, pixel="u16",
                                  device="cuda")
    plan = gpu.Plan(1024, 1024, 2048)
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    check_sampled(D, frames, [0, 1, 5, 300, 511, 512], "1024x1024x2048")


MIN = {"padding": "minimal"}


@pytest.mark.parametrize("W,H,N,pixel,kw", [(16, 16, 2048, "u8", {}), (32, 32, 3000, "u8", {}),
                                             (16, 32, 2049, "u16", {}), (32, 32, 3000, "u8", MIN),
                                             (16, 32, 2049, "u16", MIN), (32, 32, 700, "u8", MIN),
                                             (64, 48, 1536, "u16", dict(MIN, max_lag=1000)),
                                             (16, 16, 150, "u8", MIN), (32, 16, 3072, "u16", MIN),
                                             (48, 48, 400, "u16", dict(MIN, max_lag=37)),
                                             (64, 64, 700, "u16", dict(MIN, spectrum="f16")),
                                             (16, 16, 8192, "u8", {}), (16, 16, 5000, "u16", {})])
def test_long_time_series_full_oracle(gpu, W, H, N, pixel, kw):
    """Full pipeline (blocked spectra store) at transform lengths L = 2^k and
    (minimal padding) 3 * 2^k, N = L without padding and with padded tails,
    max_lag < N and the FP16 store; every q against the oracle."""
    say("case: long series", W, H, N, pixel, kw)
    frames = synth.brownian_stack(W, H, N, max(4, W * H // 30), 1.5, 40.0, 200.0, 0.2, seed=N, pixel=pixel)
    plan = gpu.Plan(W, H, N, pixel=pixel, **kw)
    D = plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    Do, _ = oracle_D(frames.numpy(), max_lag=kw.get("max_lag"))
    e = per_q_error(D.cpu().numpy(), Do)
    say("long", W, H, N, kw, describe(e))
    assert e.max() <= (5e-3 if kw.get("spectrum") == "f16" else TOL_F32)


def test_batch_1024_and_long_512(gpu):
    """Two lanes: a 1024 x 1024 stack, a 512 x 512 stack of 2500 frames (L = 4096)
    and a small stack, each against the oracle on sampled columns; the graph
    replay gives the same bits."""
    say("case: batch 1024x1024x300 + 512x512x2500 + 128x128x700, lanes 2")
    shapes = [(1024, 1024, 300), (512, 512, 2500), (128, 128, 700)]
    fr = [synth.brownian_stack(w, h, n, max(4, 2000 * w * h // (512 * 512)), 1.5, 40.0, 800.0, d0, seed=900 + i,
                               pixel="u16", device="cuda")
          for i, ((w, h, n), d0) in enumerate(zip(shapes, [0.05, 1.0, 3.0]))]
    batch = gpu.Batch(shapes, lanes=2)
    assert len(set(batch.lane)) == 2
    Db = [d.clone() for d in batch.structure_function(fr)]
    Db2 = batch.structure_function(fr)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(Db[i], Db2[i]), i
    check_sampled(Db[0], fr[0], [0, 2, 511, 512], "batch 1024x1024x300")
    check_sampled(Db[1], fr[1], [0, 3, 256], "batch 512x512x2500")
    check_sampled(Db[2], fr[2], [0, 1, 17, 64], "batch 128x128x700")


def test_long_stack_256x256x8192(gpu):
    """256 x 256 u16 x 8192 frames: the time transform of length 8192 (one wave
    vector per workgroup of 512 threads) behind the single-launch step one."""
    say("case: 256x256x8192 u16, kx columns {0, 3, 128}")
    frames = synth.brownian_stack(256, 256, 8192, 500, 1.5, 40.0, 800.0, 0.1, seed=8192, pixel="u16", device="cuda")
    plan = gpu.Plan(256, 256, 8192)
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    check_sampled(D, frames, [0, 3, 128], "256x256x8192")
    assert plan.status() == 0
