"""Shared test helpers: oracle evaluations on given frames and error metrics."""

import numpy as np

from oracle import dft, structure

# Tolerance of the FP32 path: per wave vector, max over lags of |D_gpu - D_oracle|
# divided by max over lags of D_oracle(q).
TOL_F32 = 1e-4


def oracle_D(frames, k2_max=-1, max_lag=None, kx_subset=None):
    """FP64 oracle D [Q, M] in q order (optionally only the q with kx in kx_subset).

    Returns (D, q_rows) where q_rows are the row indices of the returned
    wave vectors in the full kept-q order.
    """
    frames = np.asarray(frames)
    N, H, W = frames.shape
    kx, ky, _ = dft.q_list(W, H, k2_max)
    rows = np.arange(len(kx))
    if kx_subset is not None:
        sel = np.isin(kx, np.asarray(kx_subset))
        kx, ky, rows = kx[sel], ky[sel], rows[sel]
    ukx = np.unique(kx)
    F = dft.dft_columns(frames, ukx, np.arange(H))          # [N, H, len(ukx)]
    col = np.searchsorted(ukx, kx)
    Fq = F[:, ky, col].T                                     # [Q, N]
    return structure.structure_function_direct(Fq, max_lag), rows


def per_q_error(D_gpu, D_ora):
    D_gpu = np.asarray(D_gpu, dtype=np.float64)
    num = np.abs(D_gpu - D_ora).max(axis=1)
    den = D_ora.max(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(den > 0, num / np.where(den > 0, den, 1.0), num)
    return e


def describe(e):
    return "max %.3e (q=%d)  p99 %.3e  median %.3e" % (
        e.max(), int(e.argmax()), np.percentile(e, 99), np.median(e))
