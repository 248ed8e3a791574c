"""2048 x 2048 uint16 x 4096 frames (30000 spots, D0 0.05): the full-size case.

D is computed with a workspace that holds only part of the spectra, so the
wave vectors run in several groups (the paper's group execution, Appendix C).
The FP64 oracle covers a subset of wave vectors (kx in {0, 1, 5, 100, 1024},
every 32nd ky): their transforms are accumulated over frame chunks copied to
the host.  The 200 logarithmic |q| bins are checked bit-exactly on all q.
"""

import numpy as np
import pytest
import torch

from oracle import dft, radial, structure
from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, per_q_error

pytestmark = pytest.mark.gpu

KX = [0, 1, 5, 100, 1024]


def test_large_config_sampled_and_binned(gpu):
    print("case: 2048x2048x4096 u16, grouped workspace, sampled oracle", flush=True)
    W = H = 2048
    N = 4096
    frames = synth.make(synth.LARGE, device="cuda")
    torch.cuda.synchronize()
    plan = gpu.Plan(W, H, N)
    mn, full = plan.workspace_size()
    plan.allocate_workspace(mn + (full - mn) // 3)      # about three groups
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    print("D computed", flush=True)
    kx, ky = plan.q_index()
    ky_u = np.where(ky < 0, ky + H, ky)
    KY = np.arange(0, H, 32)
    rows = np.flatnonzero(np.isin(kx, KX) & np.isin(ky_u, KY))
    Dg = D[torch.from_numpy(rows).cuda()].cpu().numpy()
    # oracle transforms at the sampled (kx, ky), accumulated over frame chunks
    F = np.empty((N, len(KY), len(KX)), dtype=np.complex128)
    for t0 in range(0, N, 128):
        F[t0:t0 + 128] = dft.dft_columns(frames[t0:t0 + 128].cpu().numpy(), KX, KY, chunk=8)
    col = {k: i for i, k in enumerate(KX)}
    rowi = {k: i for i, k in enumerate(KY)}
    Fq = np.stack([F[:, rowi[ky_u[r]], col[kx[r]]] for r in rows])
    Do = structure.structure_function_direct(Fq)
    e = per_q_error(Dg, Do)
    print("large sampled (%d q):" % len(rows), describe(e), flush=True)
    assert e.max() <= TOL_F32
    # 200 logarithmic |q| bins, edges geomspace(1, k_max), on all q
    T = gpu.log_bin_thresholds(200, 1.0, float(np.sqrt(2.0) * 1024))
    Dbar, counts, boq = plan.radial_average(D, T)
    torch.cuda.synchronize()
    b_o = radial.bin_index(dft.k2_of(kx, ky, W, H), T)
    np.testing.assert_array_equal(boq.cpu().numpy(), b_o)
    w = radial.weights(kx, W)
    c_o = np.bincount(b_o[b_o >= 0], weights=w[b_o >= 0], minlength=200).astype(np.int64)
    np.testing.assert_array_equal(counts.cpu().numpy(), c_o)
