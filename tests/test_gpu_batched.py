"""Batched stacks of uneven sizes in one graph launch; autotuned launch shapes."""

import numpy as np
import pytest
import torch

from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64, 300), (128, 128, 257), (96, 96, 1000), (48, 96, 77), (256, 256, 129), (384, 48, 40),
          (64, 64, 2), (128, 64, 700), (32, 32, 1537), (256, 128, 64)]


def stacks():
    out = []
    for i, (W, H, N) in enumerate(SHAPES):
        out.append(synth.brownian_stack(W, H, N, max(4, W * H // 60), 1.5, 40.0, 600.0, 0.05 * (i + 1),
                                        seed=100 + i, pixel="u16").cuda())
    return out


def test_batch_equals_single_plans(gpu):
    print("case: batched stacks vs single plans", flush=True)
    fr = stacks()
    batch = gpu.Batch(SHAPES, lanes=4)
    Db = [d.clone() for d in batch.structure_function(fr)]
    Db2 = batch.structure_function(fr)            # graph replay
    torch.cuda.synchronize()
    for i, (W, H, N) in enumerate(SHAPES):
        plan = gpu.Plan(W, H, N)
        Ds = plan.structure_function(fr[i])
        torch.cuda.synchronize()
        assert torch.equal(Db[i], Ds), i
        assert torch.equal(Db2[i], Ds), i
    # new output buffers: a new capture, same results
    outs = [torch.empty_like(d) for d in Db]
    Db3 = batch.structure_function(fr, outs)
    torch.cuda.synchronize()
    for i in range(len(SHAPES)):
        assert torch.equal(Db3[i], Db[i])


def test_batch_against_oracle(gpu):
    print("case: batched stacks vs oracle", flush=True)
    fr = stacks()
    batch = gpu.Batch(SHAPES, lanes=3)
    Db = batch.structure_function(fr)
    torch.cuda.synchronize()
    for i in [0, 3, 5, 6, 9]:
        Do, _ = oracle_D(fr[i].cpu().numpy())
        e = per_q_error(Db[i].cpu().numpy(), Do)
        print(SHAPES[i], describe(e), flush=True)
        assert e.max() <= TOL_F32


def test_autotune_keeps_parity(gpu):
    print("case: autotune", flush=True)
    frames = synth.brownian_stack(128, 128, 1024, 300, 1.5, 40.0, 600.0, 0.3, seed=3)
    plan = gpu.Plan(128, 128, 1024)
    E, qpw, ms = plan.autotune()
    print("autotuned E=%d qpw=%d (%.3f ms)" % (E, qpw, ms), flush=True)
    assert E in (8, 16) and qpw >= 1
    D = plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    Do, _ = oracle_D(frames.numpy(), kx_subset=[0, 3, 64])
    kx, _ = plan.q_index()
    rows = np.flatnonzero(np.isin(kx, [0, 3, 64]))
    e = per_q_error(D.cpu().numpy()[rows], Do)
    assert e.max() <= TOL_F32


def test_batch_bins_match_radial_average(gpu):
    """|q| bins inside the batch graph equal ddm_radial_average on the batch's
    D bit for bit; counts equal the full-plane lattice counts of the oracle."""
    print("case: batch with bins on stacks 0, 2 and 4", flush=True)
    from oracle import dft, radial
    fr = stacks()
    batch = gpu.Batch(SHAPES, lanes=3)
    thr = {0: gpu.integer_bin_thresholds(40), 2: gpu.integer_bin_thresholds(60),
           4: np.array([0, 3, 50, 400, 3000, 40000], dtype=np.int64)}
    for i, t in thr.items():
        batch.set_bins(i, t)
    D, Dbar, cnt = batch.structure_function_binned(fr)
    D2, Dbar2, cnt2 = batch.structure_function_binned(fr)      # a second capture (new outputs)
    torch.cuda.synchronize()
    for i, (W, H, N) in enumerate(SHAPES):
        if i not in thr:
            assert Dbar[i] is None
            continue
        plan = gpu.Plan(W, H, N)
        ref, rc, _ = plan.radial_average(D[i], thr[i], bin_of_q=False)
        torch.cuda.synchronize()
        assert torch.equal(Dbar[i], ref) and torch.equal(cnt[i], rc), i
        assert torch.equal(Dbar2[i], ref) and torch.equal(cnt2[i], rc), i
        kx, ky = plan.q_index()
        b = radial.bin_index(dft.k2_of(kx, ky, W, H), thr[i])
        w = radial.weights(kx, W)
        c_o = np.bincount(b[b >= 0], weights=w[b >= 0], minlength=len(thr[i]) - 1).astype(np.int64)
        np.testing.assert_array_equal(cnt[i].cpu().numpy(), c_o)
    assert batch.status() == [0] * len(SHAPES)


def test_batch_graph_cache_alternating_outputs(gpu):
    """Output buffers alternated between calls replay their own captured graphs;
    more pointer sets than the batch keeps replace the least recently launched
    graph. Every call's results equal the first call's bit for bit."""
    print("case: batch graph cache, alternating and evicted output sets", flush=True)
    shapes = [(64, 64, 100), (96, 48, 60), (128, 128, 40)]
    fr = [synth.uniform_stack(w, h, n, seed=40 + i).cuda() for i, (w, h, n) in enumerate(shapes)]
    batch = gpu.Batch(shapes, lanes=2)
    ref = [d.clone() for d in batch.structure_function(fr)]
    sets = [[torch.full_like(d, float("nan")) for d in ref] for _ in range(6)]
    order = [0, 1, 0, 1, 2, 3, 4, 5, 0, 1, 5]  # sets 0 and 1 are evicted by 2..5, then captured again
    for k in order:
        for d in sets[k]:
            d.fill_(float("nan"))
        out = batch.structure_function(fr, sets[k])
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            assert torch.equal(out[i], ref[i]), (k, i)
    assert batch.status() == [0] * len(shapes)
