"""GPU curve sampling and Levenberg-Marquardt fit against the FP64 oracle."""

import sys

import numpy as np
import pytest
import torch

from oracle import lm
from paper_2012_05695_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_sample_curves(gpu):
    say("case: sample curves")
    r = np.random.default_rng(0)
    D = np.abs(r.standard_normal((300, 500))).astype(np.float32) * 10
    D[7] = 0.0
    lags = lm.log_lags(500)
    cg, sg = gpu.sample_curves(torch.from_numpy(D).cuda(), lags)
    co, so = lm.sample_curves(D, lags)
    np.testing.assert_allclose(sg.cpu().numpy(), so, rtol=1e-6)
    np.testing.assert_allclose(cg.cpu().numpy(), co, rtol=2e-6, atol=1e-7)


def synth_curves(n, K=64, N=2048, noise=0.0, seed=0):
    r = np.random.default_rng(seed)
    m = lm.log_lags(N, K).astype(np.float64)
    A = r.uniform(0.3, 1.0, n)
    B = r.uniform(0.0, 0.5, n)
    tau = np.exp(r.uniform(np.log(2.0), np.log(0.5 * N), n))
    Y = A[:, None] * (1 - np.exp(-m[None, :] / tau[:, None])) + B[:, None]
    Y = Y * (1 + noise * r.standard_normal(Y.shape))
    return Y.astype(np.float32), np.stack([A, B, tau], 1), m.astype(np.float32)


def test_lm_noise_free_recovery(gpu):
    say("case: LM noise-free")
    Y, P, m = synth_curves(2000)
    params, iters, flags = gpu.fit(torch.from_numpy(Y).cuda(), m)
    params, flags = params.cpu().numpy(), flags.cpu().numpy()
    conv = (flags & 1) != 0
    say("converged %.4f, median iters %d" % (conv.mean(), np.median(iters.cpu().numpy())))
    assert conv.mean() >= 0.995
    rel = np.abs(params[conv] - P[conv]) / np.abs(P[conv]).clip(1e-3)
    assert np.percentile(rel, 99) < 1e-3


def test_lm_matches_oracle_on_noisy_curves(gpu):
    say("case: LM noisy vs oracle")
    Y, P, m = synth_curves(400, noise=0.02, seed=3)
    params, iters, flags = gpu.fit(torch.from_numpy(Y).cuda(), m)
    params, flags = params.cpu().numpy(), flags.cpu().numpy()
    Po, Co, Io, Fo = lm.lm_fit_many(Y.astype(np.float64), m.astype(np.float64))
    mm = m.astype(np.float64)
    cost_g = np.array([np.sum((lm.model((p[0], p[1], np.log(p[2])), mm) - y) ** 2)
                       for p, y in zip(params.astype(np.float64), Y.astype(np.float64))])
    both = ((flags & 1) != 0) & ((Fo & 1) != 0)
    say("both converged %.4f" % both.mean())
    assert both.mean() >= 0.98
    excess = (cost_g[both] - Co[both]) / Co[both]
    say("cost excess max %.3e" % excess.max())
    assert excess.max() < 1e-4
    tau_o = np.exp(Po[both, 2])
    assert np.percentile(np.abs(params[both, 2] - tau_o) / tau_o, 95) < 1e-2


def test_fit_init_and_fallback(gpu):
    say("case: LM init + fallback")
    Y, P, m = synth_curves(256, noise=0.01, seed=5)
    good = torch.from_numpy(np.stack([P[:, 0], P[:, 1], np.log(P[:, 2])], 1).astype(np.float32)).cuda()
    pa, ia, fa = gpu.fit(torch.from_numpy(Y).cuda(), m, init=good)
    pd, id_, fd = gpu.fit(torch.from_numpy(Y).cuda(), m)
    assert ia.float().mean() < id_.float().mean()      # a good start saves iterations
    bad = good.clone()
    bad[:10] = float("nan")                              # poisoned starts -> default-start refit
    pb, ib, fb = gpu.fit(torch.from_numpy(Y).cuda(), m, init=bad)
    fb = fb.cpu().numpy()
    assert np.all(fb[:10] & 16) and np.all(fb[:10] & 1)
    assert not np.any(fb[10:] & 16)


def test_fit_best_start(gpu):
    """fallback="best": each curve starts from the lower-cost of the given and the
    default start (flag 32 when the default wins), then one fit; results match
    the FP64 oracle fitted from the same start."""
    say("case: LM best start")
    Y, P, m = synth_curves(256, noise=0.01, seed=6)
    good = np.stack([P[:, 0], P[:, 1], np.log(P[:, 2])], 1).astype(np.float32)
    start = good.copy()
    start[::2, 2] += 6.0                                # every other start is far off in tau
    pb, ib, fb = gpu.fit(torch.from_numpy(Y).cuda(), m, init=torch.from_numpy(start).cuda(), fallback="best")
    pb, fb = pb.cpu().numpy(), fb.cpu().numpy()
    mm = m.astype(np.float64)
    chose_default = (fb & 32) != 0
    assert not np.any(fb & 16)
    for i in range(0, 256, 17):
        # the choice itself: the lower of the two initial costs (FP64 here)
        d0 = lm.default_init(Y[i].astype(np.float64), mm)
        ci = np.sum((lm.model(start[i].astype(np.float64), mm) - Y[i]) ** 2)
        cd = np.sum((lm.model(d0, mm) - Y[i]) ** 2)
        if abs(ci - cd) > 1e-3 * max(ci, cd):
            assert chose_default[i] == (cd < ci), i
        p0 = d0 if chose_default[i] else start[i].astype(np.float64)
        po, co, io, fo = lm.lm_fit(Y[i].astype(np.float64), mm, p0)
        cg = np.sum((lm.model((pb[i, 0], pb[i, 1], np.log(pb[i, 2])), mm) - Y[i]) ** 2)
        assert cg <= co * (1 + 1e-4) + 1e-10, (i, cg, co)


def test_lm_many_curves_per_lane(gpu):
    """250,000 curves (more than one per lane of the resident waves, so lanes
    take further curves as theirs finish), mixed clean, noisy and flat so that
    the lanes of a wave finish at different iterations: every curve gets the
    same bits as in a call of 2,000 curves (one curve per lane), from the
    default start and with a start plus the refit pass, and sampled curves
    reach the FP64 oracle's cost."""
    say("case: LM 250000 curves, several per lane")
    n = 250_000
    Y, P, m = synth_curves(n, noise=0.0, seed=11)
    r = np.random.default_rng(12)
    kind = r.integers(0, 3, n)
    Y[kind == 1] *= (1 + 0.05 * r.standard_normal((int((kind == 1).sum()), Y.shape[1]))).astype(np.float32)
    Y[kind == 2] = (0.5 + 0.05 * r.standard_normal((int((kind == 2).sum()), Y.shape[1]))).astype(np.float32)
    Yd = torch.from_numpy(Y).cuda()
    pick = np.sort(r.choice(n, 2000, replace=False))
    pick_d = torch.from_numpy(pick).cuda()
    start = torch.from_numpy(np.stack([P[:, 0] * 0.8, P[:, 1] + 0.05, np.log(P[:, 2]) + 0.7], 1)
                             .astype(np.float32)).cuda()
    first = None
    for init, fb in ((None, True), (start, True)):
        big = gpu.fit(Yd, m, init=init, fallback=fb)
        first = first or big
        small = gpu.fit(Yd[pick_d].contiguous(), m, init=None if init is None else init[pick_d].contiguous(),
                        fallback=fb)
        torch.cuda.synchronize()
        for a, b, what in zip(big, small, ("params", "iters", "flags")):
            assert torch.equal(a[pick_d], b), (what, init is None)
        fl = big[2].cpu().numpy()
        say("init" if init is not None else "default", "converged %.4f, mean iters %.1f" %
            (((fl & 1) != 0).mean(), big[1].float().mean().item()))
    # the default-start fit of the noisy curves against the oracle's (clean ones fit to
    # rounding, where a relative cost excess means nothing)
    params, flags = first[0].cpu().numpy(), first[2].cpu().numpy()
    sub = pick[kind[pick] == 1][:300]
    Po, Co, Io, Fo = lm.lm_fit_many(Y[sub].astype(np.float64), m.astype(np.float64))
    mm = m.astype(np.float64)
    cost_g = np.array([np.sum((lm.model((p[0], p[1], np.log(p[2])), mm) - y) ** 2)
                       for p, y in zip(params[sub].astype(np.float64), Y[sub].astype(np.float64))])
    both = ((flags[sub] & 1) != 0) & ((Fo & 1) != 0)
    say("both converged %.4f of %d" % (both.mean(), len(sub)))
    assert both.mean() >= 0.9
    excess = (cost_g[both] - Co[both]) / np.maximum(Co[both], 1e-30)
    say("cost excess max %.3e" % excess.max())
    assert excess.max() < 1e-4
