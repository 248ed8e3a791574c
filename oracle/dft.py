"""Naive 2-D DFT of image frames, FP64 (oracle; test infrastructure only).

The paper applies an unnormalised "bi-dimensional FFT" F_xy to every image
(section "The algorithm", Eq. (1)) but states neither the sign nor the
normalisation.  Reading used here: the forward transform with kernel
exp(-2*pi*i*(kx*x/W + ky*y/H)) and no scale factor, the default of the FFT
libraries the paper names.  D is invariant under the sign choice and scales
with the square of the normalisation, so this fixes the units of D.

Frames are real, so F(-q) = conj(F(q)) and D(-q) = D(q): the half plane
kx in [0, W/2], ky in [0, H) holds every distinct value.

The transform is written as its definition: a sum over x, then a sum over y,
each as a dense matrix product with explicitly tabulated phase factors.  The
phase index (k*x) mod L is reduced in exact integer arithmetic before the
cosine/sine, so every factor is correct to FP64 rounding.  No FFT is used.
"""

from math import gcd

import numpy as np


def _phase_matrix(L, k_values):
    """M[x, j] = exp(-2*pi*i * ((k_j * x) mod L) / L) for x in [0, L)."""
    x = np.arange(L, dtype=np.int64)
    k = np.asarray(k_values, dtype=np.int64)
    r = np.outer(x, k) % L                      # exact integer reduction
    ang = (-2.0 * np.pi / L) * r.astype(np.float64)
    return np.cos(ang) + 1j * np.sin(ang)


def k2_of(kx, ky_s, W, H):
    """Integer squared wave-vector magnitude on the frame's lattice.

    |q|^2 is proportional to (kx/W)^2 + (ky/H)^2.  Multiplying by (W*H/g)^2,
    g = gcd(W, H), gives the exact integer kx^2 (H/g)^2 + ky^2 (W/g)^2,
    which for square frames is kx^2 + ky^2.
    """
    g = gcd(int(W), int(H))
    a = (int(H) // g) ** 2
    c = (int(W) // g) ** 2
    kx = np.asarray(kx, dtype=np.int64)
    ky_s = np.asarray(ky_s, dtype=np.int64)
    return kx * kx * a + ky_s * ky_s * c


def q_list(W, H, k2_max=-1):
    """Kept wave vectors in output-row order.

    Order: ky ascending over [0, H), then kx ascending over [0, W/2], keeping
    those with k2 <= k2_max (all when k2_max < 0).  ky is the unsigned DFT
    index; its signed frequency is ky for ky <= H/2 and ky - H above.
    The optional cut is the paper's restriction to low-frequency wave vectors
    (section "Conclusion").

    Returns (kx, ky, ky_signed) as int64 arrays.
    """
    W = int(W)
    H = int(H)
    kxs, kys = np.meshgrid(np.arange(W // 2 + 1), np.arange(H), indexing="xy")
    kx = kxs.ravel().astype(np.int64)
    ky = kys.ravel().astype(np.int64)
    ky_s = np.where(ky <= H // 2, ky, ky - H)
    if k2_max is not None and k2_max >= 0:
        keep = k2_of(kx, ky_s, W, H) <= int(k2_max)
        kx, ky, ky_s = kx[keep], ky[keep], ky_s[keep]
    return kx, ky, ky_s


def dft_columns(frames, kx_list, ky_list, chunk=64):
    """F[t, i, j] = sum_y sum_x I_t[y, x] exp(-2 pi i (kx_j x / W + ky_i y / H)).

    frames: integer or float array [N, H, W].  Returns complex128 [N, len(ky), len(kx)].
    """
    frames = np.asarray(frames)
    N, H, W = frames.shape
    Tx = _phase_matrix(W, kx_list)              # [W, nkx]
    Ty = _phase_matrix(H, ky_list).T            # [nky, H]
    out = np.empty((N, len(ky_list), len(kx_list)), dtype=np.complex128)
    for t0 in range(0, N, chunk):
        blk = frames[t0:t0 + chunk].astype(np.float64)
        rows = blk @ Tx                          # sum over x: [c, H, nkx]
        out[t0:t0 + chunk] = Ty @ rows           # sum over y: [c, nky, nkx]
    return out


def dft_half_plane(frames, chunk=64):
    """F[t, ky, kx] on the full half plane kx in [0, W/2], ky in [0, H)."""
    frames = np.asarray(frames)
    _, H, W = frames.shape
    return dft_columns(frames, np.arange(W // 2 + 1), np.arange(H), chunk=chunk)
