"""Azimuthal |q| averaging of the structure function, FP64 (oracle; test only).

The paper computes D for every wave vector and does not bin; binning is the
standard DDM reduction of D(q, m) to D(|q|, m).  Reading used here:

* a wave vector belongs to bin b when T[b] <= k2 < T[b+1], with k2 the exact
  integer squared magnitude of ``dft.k2_of`` and T a given increasing integer
  threshold array (n_bins + 1 entries); wave vectors outside every bin are
  dropped (bin -1);
* the half plane stands for the full plane: a wave vector with 0 < kx < W/2
  also represents its mirror -q, so it carries weight 2, the kx = 0 and
  kx = W/2 columns weight 1;
* Dbar[b, m] = sum_{q in b} w(q) D(q, m) / sum_{q in b} w(q), in FP64;
  counts[b] = sum_{q in b} w(q), the number of full-plane lattice points.
"""

import numpy as np

from .dft import k2_of


def bin_index(k2, thresholds):
    """b with T[b] <= k2 < T[b+1], or -1.  Pure integer comparisons."""
    T = np.asarray(thresholds, dtype=np.int64)
    k2 = np.asarray(k2, dtype=np.int64)
    b = np.searchsorted(T, k2, side="right") - 1
    b[(k2 < T[0]) | (k2 >= T[-1])] = -1
    return b.astype(np.int64)


def weights(kx, W):
    kx = np.asarray(kx, dtype=np.int64)
    return np.where((kx > 0) & (kx < W // 2), 2, 1).astype(np.int64)


def radial_average(D, kx, ky_s, W, H, thresholds):
    """Returns (Dbar [n_bins, M] float64, counts [n_bins] int64, bin_of_q [Q] int64)."""
    D = np.asarray(D, dtype=np.float64)
    T = np.asarray(thresholds, dtype=np.int64)
    nb = len(T) - 1
    b = bin_index(k2_of(kx, ky_s, W, H), T)
    w = weights(kx, W)
    Dbar = np.zeros((nb, D.shape[1]), dtype=np.float64)
    counts = np.zeros(nb, dtype=np.int64)
    for i in range(nb):
        sel = b == i
        if not sel.any():
            continue
        ws = w[sel]
        counts[i] = int(ws.sum())
        Dbar[i] = (ws[:, None].astype(np.float64) * D[sel]).sum(axis=0) / float(counts[i])
    return Dbar, counts, b
