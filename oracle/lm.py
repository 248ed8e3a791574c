"""Levenberg-Marquardt fit of the DDM model, FP64 (oracle; test only).

Model of one structure-function curve (standard DDM form; the paper computes
D and leaves the fit to the analysis):

    D(m) = A (1 - exp(-m / tau)) + B,   parameters p = (A, B, theta = log tau),

fitted by least squares over K lags m_j.  Marquardt's damped Gauss-Newton
step with the damping scaled by diag(J^T J):

    (J^T J + lambda diag(J^T J)) delta = -J^T r,

lambda starts at 1e-3, is divided by 10 after an accepted step (cost
decreased) and multiplied by 10 after a rejected one.  One iteration is one
Jacobian evaluation followed by trial steps until one is accepted.  Stops when
an accepted step lowers the cost by at most 1e-12 of it, or moves p by at most
1e-12 (|delta| <= 1e-12 (|p| + 1e-12)), after 200 iterations, or when lambda
exceeds 1e16 without an accepted step (a stall; at a cost below 1e-20 of
sum y^2 the fit is exact to rounding and counts as converged).

Default initialisation on a curve normalised by c = max_j y_j:
B0 = y_1 / c (the smallest lag), A0 = 1 - B0, tau0 = sqrt(m_1 m_K) (the
geometric middle of the lag range), all expressed back in units of c.

Flags: 1 converged, 2 iteration limit, 4 non-finite data or parameters,
8 damping overflow (no decreasing step found).
"""

import numpy as np

LAM0 = 1e-3
MAX_ITER = 200
FTOL = 1e-12
XTOL = 1e-12
LAM_MAX = 1e16
EXACT_FIT = 1e-20  # relative cost below which a stall is an exact fit (FP64)

FLAG_CONVERGED = 1
FLAG_MAXITER = 2
FLAG_NONFINITE = 4
FLAG_STALLED = 8


def model(p, m):
    A, B, th = p
    return A * (1.0 - np.exp(-m / np.exp(th))) + B


def jacobian(p, m):
    A, _, th = p
    tau = np.exp(th)
    e = np.exp(-m / tau)
    return np.stack([1.0 - e, np.ones_like(m), -A * e * m / tau], axis=1)


def default_init(y, m):
    c = float(np.max(y))
    if not np.isfinite(c) or c <= 0:
        c = 1.0
    B0 = y[0] / c
    A0 = 1.0 - B0
    return np.array([A0 * c, B0 * c, 0.5 * (np.log(m[0]) + np.log(m[-1]))])


def lm_fit(y, m, p0=None):
    """Fit one curve.  Returns (p, cost, iterations, flags)."""
    y = np.asarray(y, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    p = default_init(y, m) if p0 is None else np.asarray(p0, dtype=np.float64).copy()
    if not (np.all(np.isfinite(y)) and np.all(np.isfinite(p))):
        return p, np.inf, 0, FLAG_NONFINITE
    r = model(p, m) - y
    cost = float(r @ r)
    lam = LAM0
    it = 0
    flags = 0
    while True:
        if it >= MAX_ITER:
            flags |= FLAG_MAXITER
            break
        J = jacobian(p, m)
        g = J.T @ r
        Hm = J.T @ J
        it += 1
        accepted = False
        while lam <= LAM_MAX:
            Ad = Hm + lam * np.diag(np.diag(Hm))
            try:
                delta = np.linalg.solve(Ad, -g)
            except np.linalg.LinAlgError:
                lam *= 10.0
                continue
            pn = p + delta
            rn = model(pn, m) - y
            cn = float(rn @ rn)
            if np.isfinite(cn) and cn < cost:
                small_f = (cost - cn) <= FTOL * cost
                small_x = np.linalg.norm(delta) <= XTOL * (np.linalg.norm(p) + XTOL)
                p, r, cost = pn, rn, cn
                lam /= 10.0
                accepted = True
                break
            lam *= 10.0
        if not accepted:
            # no decreasing step at any damping: a stationary point to rounding;
            # an exact fit (cost at the FP64 rounding floor) counts as converged
            flags |= FLAG_CONVERGED if cost <= EXACT_FIT * float(y @ y) else FLAG_STALLED
            break
        if small_f or small_x:
            flags |= FLAG_CONVERGED
            break
    if not np.all(np.isfinite(p)):
        flags |= FLAG_NONFINITE
    return p, cost, it, flags


def lm_fit_many(Y, m, P0=None):
    n = Y.shape[0]
    P = np.zeros((n, 3))
    C = np.zeros(n)
    I = np.zeros(n, dtype=np.int64)
    F = np.zeros(n, dtype=np.int64)
    for i in range(n):
        P[i], C[i], I[i], F[i] = lm_fit(Y[i], m, None if P0 is None else P0[i])
    return P, C, I, F


def log_lags(n_frames, K=64):
    """K log-spaced fractional lags from 1 to N-1 (FP32, as both sides use them)."""
    return np.geomspace(1.0, float(n_frames - 1), K).astype(np.float32)


def sample_curves(D, lags):
    """Linear interpolation of each row of D [Q, M] at fractional lags.

    Returns (curves [Q, K] normalised by c = max_j curve_j, c [Q]).  A row whose
    maximum is not positive keeps c = 1.
    """
    D = np.asarray(D, dtype=np.float64)
    m = np.asarray(lags, dtype=np.float64)
    i0 = np.floor(m).astype(np.int64)
    i1 = np.minimum(i0 + 1, D.shape[1] - 1)
    f = m - i0
    Y = D[:, i0] + f[None, :] * (D[:, i1] - D[:, i0])
    c = Y.max(axis=1)
    c = np.where(np.isfinite(c) & (c > 0), c, 1.0)
    return Y / c[:, None], c
