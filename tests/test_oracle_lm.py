"""Pins of the LM oracle: exact recovery, a library minimiser, stationarity."""

import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import lm

M = lm.log_lags(2048).astype(np.float64)


@pytest.mark.parametrize("A,B,tau", [(1.0, 0.05, 30.0), (7.5, 0.3, 2.5), (0.2, 1.0, 900.0),
                                     (3.0, 0.0, 120.0), (1.0, 2.0, 8.0)])
def test_noise_free_recovery(A, B, tau):
    y = lm.model((A, B, np.log(tau)), M)
    p, cost, it, flags = lm.lm_fit(y, M)
    assert flags & lm.FLAG_CONVERGED
    np.testing.assert_allclose(p, [A, B, np.log(tau)], rtol=1e-7, atol=1e-9)
    assert cost < 1e-18 * (y @ y)


def test_matches_minpack_on_noisy_curves():
    r = np.random.default_rng(0)
    for i in range(20):
        A, B, tau = r.uniform(0.5, 5), r.uniform(0.01, 1), np.exp(r.uniform(np.log(2), np.log(1500)))
        y = lm.model((A, B, np.log(tau)), M) * (1 + 0.03 * r.standard_normal(len(M)))
        p, cost, it, flags = lm.lm_fit(y, M)
        assert flags & lm.FLAG_CONVERGED
        ref = least_squares(lambda q: lm.model(q, M) - y, lm.default_init(y, M), method="lm",
                            xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
        cref = float(ref.fun @ ref.fun)
        assert cost <= cref * (1 + 1e-8) + 1e-300
        np.testing.assert_allclose(p, ref.x, rtol=1e-5, atol=1e-7)


def test_gradient_vanishes_at_solution():
    r = np.random.default_rng(1)
    y = lm.model((2.0, 0.4, np.log(60.0)), M) + 0.05 * r.standard_normal(len(M))
    p, _, _, _ = lm.lm_fit(y, M)
    J = lm.jacobian(p, M)
    g = J.T @ (lm.model(p, M) - y)
    assert np.linalg.norm(g) <= 1e-7 * np.linalg.norm(J.T @ y)


def test_nonfinite_flag():
    y = lm.model((1.0, 0.1, 3.0), M)
    y[5] = np.nan
    _, _, _, flags = lm.lm_fit(y, M)
    assert flags & lm.FLAG_NONFINITE


def test_sample_curves_interpolates_linearly():
    D = np.zeros((3, 100))
    D[0] = np.arange(100) * 2.0 + 1.0            # linear: reproduced exactly
    D[1] = np.arange(100) ** 2                   # integer lags hit the table exactly
    D[2] = 0.0                                   # all zero: scale 1
    lags = np.array([1.0, 2.5, 7.25, 50.0, 99.0])
    Y, c = lm.sample_curves(D, lags)
    np.testing.assert_allclose(Y[0] * c[0], 2 * lags + 1, rtol=1e-15)
    np.testing.assert_allclose(Y[1, [0, 3, 4]] * c[1], lags[[0, 3, 4]] ** 2, rtol=1e-15)
    assert c[2] == 1.0 and np.all(Y[2] == 0)
    assert np.isclose(Y[0].max(), 1.0)


@pytest.mark.parametrize("A,B,tau,noise", [(1.0, 0.05, 30.0, 0.0), (7.5, 0.3, 2.5, 0.02), (0.2, 1.0, 900.0, 0.05)])
def test_default_start_properties(A, B, tau, noise):
    """The default start (the reading of the fit start: B0 = y_1 / c, A0 = 1 - B0 on the curve
    scaled by its maximum c, tau0 = sqrt(m_1 m_K)) checked through the model it starts: at lag 0
    it takes the first sample's value, for large lags it plateaus at the curve's maximum, and
    its relaxation time lies halfway between the first and last lags on the log axis."""
    r = np.random.default_rng(3)
    y = lm.model((A, B, np.log(tau)), M) * (1 + noise * r.standard_normal(len(M)))
    p0 = lm.default_init(y, M)
    start = lambda m: lm.model(p0, np.asarray(m, dtype=np.float64))
    assert start([0.0])[0] == pytest.approx(y[0], rel=1e-12)
    assert start([1e9 * M[-1]])[0] == pytest.approx(y.max(), rel=1e-12)
    assert np.exp(2 * p0[2]) == pytest.approx(M[0] * M[-1], rel=1e-12)
    # a curve of zeros, and one with a non-finite maximum, take the scale 1
    z = lm.default_init(np.zeros(len(M)), M)
    assert z[0] == 1.0 and z[1] == 0.0
    bad = y.copy()
    bad[-1] = np.inf
    assert lm.default_init(bad, M)[0] == pytest.approx(1.0 - y[0])
