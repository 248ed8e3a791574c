"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties an oracle function to something other than itself: brute force
on tiny inputs, a library routine it does not use, closed forms of D for
stacks whose dynamics are known exactly, an exact integer sum rule, and the
paper's own FFT-in-time method (Appendix B) written independently here.
A plausible slip in the oracle (a dropped term, a wrong sign or lag index, a
transposed operand, a wrong weight) fails at least one of them.
"""

import math
import os

import numpy as np
import pytest

from oracle import dft, radial, structure

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


def to_qmajor(F):
    """[N, nky, nkx] -> [nky*nkx, N] in q order (ky-major, then kx)."""
    N = F.shape[0]
    return F.reshape(N, -1).T.copy()


# ---------------------------------------------------------------- DFT pins ---

def brute_dft(frames):
    """Four nested loops, math.cos/math.sin, full plane."""
    N, H, W = frames.shape
    out = np.zeros((N, H, W), dtype=np.complex128)
    for t in range(N):
        for ky in range(H):
            for kx in range(W):
                re = im = 0.0
                for y in range(H):
                    for x in range(W):
                        a = -2.0 * math.pi * (kx * x / W + ky * y / H)
                        v = float(frames[t, y, x])
                        re += v * math.cos(a)
                        im += v * math.sin(a)
                out[t, ky, kx] = complex(re, im)
    return out


@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 8, 7), (2, 6, 8)])
def test_dft_matches_brute_force(shape):
    frames = rng(1).integers(0, 4096, size=shape)
    full = brute_dft(frames)
    half = dft.dft_half_plane(frames)
    W = shape[2]
    np.testing.assert_allclose(half, full[:, :, : W // 2 + 1], rtol=0, atol=1e-12 * np.abs(full).max())


def test_dft_matches_library_rfft2():
    frames = rng(2).integers(0, 65536, size=(5, 12, 16))
    ref = np.fft.rfft2(frames.astype(np.float64), axes=(1, 2))
    got = dft.dft_half_plane(frames)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_dft_column_subset_equals_full():
    frames = rng(3).integers(0, 256, size=(4, 16, 24))
    full = dft.dft_half_plane(frames)
    kx = [0, 3, 12]
    ky = [0, 1, 8, 15]
    sub = dft.dft_columns(frames, kx, ky)
    np.testing.assert_allclose(sub, full[:, ky][:, :, kx], rtol=0, atol=1e-9)


def test_parseval_half_plane_weights():
    frames = rng(4).integers(0, 4096, size=(3, 10, 12))
    F = dft.dft_half_plane(frames)
    _, H, W = frames.shape
    kx = np.arange(W // 2 + 1)
    w = radial.weights(kx, W)
    lhs = (np.abs(F) ** 2 * w[None, None, :]).sum(axis=(1, 2))
    rhs = W * H * (frames.astype(np.float64) ** 2).sum(axis=(1, 2))
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_q_list_order_and_cut():
    kx, ky, kys = dft.q_list(8, 6)
    assert len(kx) == 6 * 5
    assert list(kx[:5]) == [0, 1, 2, 3, 4] and list(ky[:5]) == [0] * 5
    assert list(kys[::5]) == [0, 1, 2, 3, -2, -1]
    kx2, ky2, kys2 = dft.q_list(8, 6, k2_max=4)
    k2 = dft.k2_of(kx2, kys2, 8, 6)
    assert k2.max() <= 4
    # every kept q is in the full list, in the same relative order
    allk = list(zip(*dft.q_list(8, 6)[:2]))
    idx = [allk.index(p) for p in zip(kx2, ky2)]
    assert idx == sorted(idx)
    # non-square lattice measure: k2 proportional to (kx/W)^2 + (ky/H)^2
    assert dft.k2_of(1, 0, 8, 4) == 1 and dft.k2_of(0, 1, 8, 4) == 4


# ------------------------------------------------------- structure function ---

def test_golden_worked_example():
    rows = np.loadtxt(os.path.join(GOLDEN, "worked_example.txt"))
    frames = np.array([[[1, 2]], [[3, 5]], [[4, 4]]])
    F = to_qmajor(dft.dft_half_plane(frames))
    D = structure.structure_function_direct(F)
    np.testing.assert_allclose(D, rows[:, 2:], rtol=0, atol=1e-12)
    kx, _, kys = dft.q_list(2, 1)
    assert list(kx) == list(rows[:, 0].astype(int)) and list(kys) == list(rows[:, 1].astype(int))


def test_invariants_zero_lag_nonnegative_static():
    frames = rng(5).integers(0, 4096, size=(20, 8, 8))
    F = to_qmajor(dft.dft_half_plane(frames))
    D = structure.structure_function_direct(F)
    assert np.all(D[:, 0] == 0.0)
    assert np.all(D >= 0.0)
    static = np.repeat(frames[:1], 20, axis=0)
    Ds = structure.structure_function_direct(to_qmajor(dft.dft_half_plane(static)))
    assert np.all(Ds == 0.0)


def test_translating_pattern_closed_form():
    # I_t = I_0 shifted by t*v (periodic): D = 2|F0|^2 (1 - cos(phi m)),
    # phi = 2 pi (kx vx / W + ky vy / H)
    N, H, W, vx, vy = 16, 8, 12, 1, 2
    base = rng(6).integers(0, 4096, size=(H, W))
    frames = np.stack([np.roll(base, (t * vy, t * vx), axis=(0, 1)) for t in range(N)])
    F = dft.dft_half_plane(frames)
    D = structure.structure_function_direct(to_qmajor(F))
    kx, ky, _ = dft.q_list(W, H)
    phi = 2 * np.pi * (kx * vx / W + ky * vy / H)
    F0 = np.abs(to_qmajor(F)[:, 0]) ** 2
    m = np.arange(N)
    ref = 2 * F0[:, None] * (1 - np.cos(phi[:, None] * m[None, :]))
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-10 * ref.max())


def test_alternating_frames_closed_form():
    N, H, W = 11, 6, 8
    A = rng(7).integers(0, 4096, size=(H, W))
    B = rng(8).integers(0, 4096, size=(H, W))
    frames = np.stack([A if t % 2 == 0 else B for t in range(N)])
    D = structure.structure_function_direct(to_qmajor(dft.dft_half_plane(frames)))
    dAB = np.abs(to_qmajor(dft.dft_half_plane((A - B)[None]))[:, 0]) ** 2
    m = np.arange(N)
    ref = dAB[:, None] * (m % 2 == 1)[None, :]
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-10 * ref.max())


def test_linear_drift_closed_form():
    N, H, W = 9, 6, 6
    I0 = rng(9).integers(0, 1000, size=(H, W))
    J = rng(10).integers(-20, 20, size=(H, W))
    frames = np.stack([I0 + t * J for t in range(N)])
    D = structure.structure_function_direct(to_qmajor(dft.dft_half_plane(frames)))
    FJ = np.abs(to_qmajor(dft.dft_half_plane(J[None]))[:, 0]) ** 2
    m = np.arange(N)
    ref = FJ[:, None] * (m[None, :] ** 2)
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-10 * ref.max())


@pytest.mark.parametrize("t0", [0, 3, 6])
def test_single_impulse_closed_form(t0):
    N, H, W = 7, 4, 6
    J = rng(11).integers(1, 100, size=(H, W))
    frames = np.zeros((N, H, W), dtype=np.int64)
    frames[t0] = J
    D = structure.structure_function_direct(to_qmajor(dft.dft_half_plane(frames)))
    FJ = np.abs(to_qmajor(dft.dft_half_plane(J[None]))[:, 0]) ** 2
    m = np.arange(1, N)
    cnt = (t0 >= m).astype(float) + (t0 + m <= N - 1).astype(float)
    ref = FJ[:, None] * (cnt / (N - m))[None, :]
    np.testing.assert_allclose(D[:, 1:], ref, rtol=0, atol=1e-10 * ref.max())
    assert np.all(D[:, 0] == 0)


def test_weighted_sum_rule_exact_integer():
    frames = rng(12).integers(0, 4096, size=(13, 8, 10))
    N, H, W = frames.shape
    D = structure.structure_function_direct(to_qmajor(dft.dft_half_plane(frames)))
    kx, _, _ = dft.q_list(W, H)
    w = radial.weights(kx, W).astype(np.float64)
    for m in range(N):
        num, den = structure.structure_function_sum_rule_rhs(frames, m)
        lhs = (w * D[:, m]).sum()
        assert abs(lhs - num / den) <= 1e-12 * max(1.0, num / den)


# ------------------------------------ the Fourier route of Eq. (2) / App. B ---

def fourier_route(F):
    """D of one time sequence through the Fourier route, derived from the
    algebra rather than from the paper's procedure.  Expanding
    |F_n - F_{n-m}|^2 = |F_n|^2 + |F_{n-m}|^2 - 2 Re(conj(F_{n-m}) F_n)
    splits the sum of Eq. (1) into prefix sums S(k) = sum_{j<k} |F_j|^2 and the
    acyclic autocorrelation c(m) = sum_{n=m}^{N-1} conj(F_{n-m}) F_n.  A cyclic
    correlation of length P >= 2N - 1 has no wrap-around terms, so it equals
    the acyclic one, and by the correlation theorem it is the inverse DFT of
    |DFT(F zero-padded to P)|^2.  P = 2N - 1 here (not a power of two), with a
    library FFT, FP64."""
    N = len(F)
    X = np.fft.fft(F, n=2 * N - 1)
    c = np.fft.ifft(X * np.conj(X))[:N].real
    S = np.concatenate([[0.0], np.cumsum(np.abs(F) ** 2)])
    m = np.arange(N)
    return (S[N] - S[m] + S[N - m] - 2.0 * c) / (N - m)


@pytest.mark.parametrize("N", [2, 3, 5, 128, 1000])
def test_direct_difference_equals_fourier_route(N):
    """The method's exactness claim (Appendix B: the zero-padded transform gives
    Eq. (1) exactly): the oracle's direct differences equal the Fourier route."""
    r = rng(13 + N)
    F = r.standard_normal((6, N)) + 1j * r.standard_normal((6, N)) + 3.0
    D = structure.structure_function_direct(F, impl="numpy")
    for q in range(F.shape[0]):
        ref = fourier_route(F[q])
        np.testing.assert_allclose(D[q], ref, rtol=0, atol=1e-12 * np.abs(ref).max() + 1e-14)


def test_eq_b3_recursion_is_prefix_sum_form():
    r = rng(14)
    N = 257
    a = r.random(N)
    d_a = np.zeros(N + 1)
    for n in range(N):
        d_a[N - n - 1] = n / (n + 1) * d_a[N - n] + (a[n] + a[N - n - 1]) / (n + 1)
    S = np.concatenate([[0.0], np.cumsum(a)])
    m = np.arange(N)
    closed = (S[N - m] + S[N] - S[m]) / (N - m)
    np.testing.assert_allclose(d_a[:N], closed, rtol=1e-13)


def test_native_and_numpy_direct_difference_agree():
    r = rng(15)
    F = r.standard_normal((37, 90)) + 1j * r.standard_normal((37, 90))
    a = structure.structure_function_direct(F, impl="numpy")
    b = structure.structure_function_direct(F, impl="c", threads=4)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13)
    b2 = structure.structure_function_direct(F, max_lag=17, impl="c")
    np.testing.assert_allclose(b2, a[:, :17], rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ binning ---

@pytest.mark.parametrize("W,H", [(16, 16), (12, 8), (8, 24)])
def test_bin_counts_match_full_plane_lattice(W, H):
    kx, _, kys = dft.q_list(W, H)
    k2 = dft.k2_of(kx, kys, W, H)
    T = np.array([0, 1, 3, 7, 13, 21, 40, 100, 1000], dtype=np.int64)
    _, counts, b = radial.radial_average(np.zeros((len(kx), 2)), kx, kys, W, H, T)
    # brute force over the full plane kx in (-W/2, W/2], ky in (-H/2, H/2]
    brute = np.zeros(len(T) - 1, dtype=np.int64)
    for fx in range(-W // 2 + 1, W // 2 + 1):
        for fy in range(-H // 2 + 1, H // 2 + 1):
            kk = int(dft.k2_of(abs(fx), fy, W, H))
            for i in range(len(T) - 1):
                if T[i] <= kk < T[i + 1]:
                    brute[i] += 1
    np.testing.assert_array_equal(counts, brute)
    assert np.all((b == -1) == ((k2 < T[0]) | (k2 >= T[-1])))


def test_integer_bins_are_rounded_magnitude():
    b = np.arange(60)
    T = b * b - b + 1
    T[0] = 0
    k2 = np.arange(0, 3000)
    idx = radial.bin_index(k2, T)
    expect = np.array([int(math.floor(math.sqrt(k) + 0.5)) for k in k2])
    expect[expect >= 59] = -1
    np.testing.assert_array_equal(idx, expect)


def test_radial_average_weighted_mean():
    W, H = 8, 6
    kx, _, kys = dft.q_list(W, H)
    D = rng(16).random((len(kx), 4))
    T = np.array([0, 10, 40, 200], dtype=np.int64)  # k2 = 9 kx^2 + 16 ky^2 here
    Dbar, counts, b = radial.radial_average(D, kx, kys, W, H, T)
    for i in range(3):
        sel = np.flatnonzero(b == i)
        num = np.zeros(4)
        den = 0
        for q in sel:
            w = 2 if 0 < kx[q] < W // 2 else 1
            num += w * D[q]
            den += w
        np.testing.assert_allclose(Dbar[i], num / den, rtol=1e-14)
        assert counts[i] == den
