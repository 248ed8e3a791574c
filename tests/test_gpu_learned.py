"""The learned start: trained on curves this pipeline computes from synthetic
Brownian stacks, it must beat the default start of the plain fit (fewer
iterations, no loss of convergence or of final cost) on the wave vectors
whose relaxation time is measurable from the sampled lags, and the gated
start must cost no iterations on the whole stack.  Reduced sizes
(128 x 128 x 512 stacks, ~100k training curves) keep the test short."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_learned_start_beats_default(gpu):
    from paper_2012_05695_amd import learn
    print("case: learned start, 128x128x512 stacks", flush=True)
    X, T, lags = learn.make_training_set(100_000, W=128, H=128, N=512, seed0=1000,
                                         log=lambda s: print(s, flush=True))
    init, losses = learn.train(X, T, epochs=20, batch=4096, lr=2e-3, log=lambda s: print(s, flush=True))
    assert losses[-1] < 0.5  # standardised targets: 1.0 is the mean predictor
    rng = np.random.default_rng(7)
    D0, snr, n_spots, a = learn.draw_stack_params(rng, 128, 128)
    curves, scale, (A, B, tau) = learn.stack_curves(128, 128, 512, D0, n_spots, a, 7, lags)
    res = learn.compare(curves, lags, init, truth_tau=tau, tau_window=(2.0, 128.0))
    print(res, flush=True)
    m, a = res["measurable"], res["all"]
    for key in ("learned", "learned_refit", "learned_gated"):
        assert m[key]["mean_iters"] < 0.9 * m["default"]["mean_iters"]
        assert m[key]["converged"] >= m["default"]["converged"] - 0.005
        assert m[key]["cost_not_worse"] >= 0.97
    # refitting the failures keeps every curve the default start converges, and
    # so does the gated start (the default start wherever tau is not resolvable)
    assert a["learned_refit"]["converged"] >= a["default"]["converged"] - 0.005
    assert a["learned_gated"]["converged"] >= a["default"]["converged"] - 0.005
    # over all curves the gated start needs no more iterations on average than
    # the default start (41.9 against 42.5 per curve on this stack) and ends at a
    # cost no worse on almost every curve (99.5%)
    assert a["learned_gated"]["mean_iters"] <= a["default"]["mean_iters"]
    assert a["learned_gated"]["cost_not_worse"] >= 0.98
    # the lower-cost start with one fit costs about one fit more than the network
    assert res["learned_ms"] < res["learned_refit_ms"]
