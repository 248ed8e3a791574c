"""The host Fourier method of bench.py (the paper's CPU WITH_FT mode, a
second host baseline beside the oracle) against the FP64 oracle."""

import numpy as np
import pytest

import bench
from paper_2012_05695_amd import synth

from helpers import TOL_F32, oracle_D, per_q_error


@pytest.mark.parametrize("W,H,N,M", [(32, 32, 100, 0), (48, 32, 77, 20), (16, 16, 2, 0), (16, 16, 129, 64)])
def test_cpu_fourier_matches_oracle(W, H, N, M):
    frames = synth.brownian_stack(W, H, N, max(4, W * H // 30), 1.5, 40.0, 200.0, 0.4, seed=N, pixel="u16").numpy()
    D = bench.cpu_fourier(frames, max_lag=M, workers=2, chunk=100)
    Do, _ = oracle_D(frames, max_lag=M or None)
    assert D.shape == Do.shape
    assert np.all(D[:, 0] == 0.0)
    assert per_q_error(D, Do).max() <= TOL_F32


def test_cpu_fourier_leg_reports_whole_workload():
    import torch
    frames = synth.uniform_stack(32, 32, 40, seed=3)
    thr = np.array([0, 1, 3, 7, 13], dtype=np.int64)
    r = bench.cpu_fourier_leg(torch.as_tensor(frames), thr, 4)
    assert r["unit"] == "frames/s" and r["value"] > 0 and r["cores"] >= 1
    assert "all 544 q" in r["sample"]
