"""Image structure function by direct differences, FP64 (oracle; test only).

Definition (section "The algorithm", Eq. (1)).  The printed equation pairs
I_{n-m} with I_m, which does not depend on the summation index; the text that
follows Eq. (2) describes the two squared-modulus averages as running over the
first and the last N-m elements, which fixes the reading

    D(q, m) = 1/(N-m) * sum_{n=m}^{N-1} |F(q, n) - F(q, n-m)|^2 ,

with F(q, t) the 2-D transform of frame t at wave vector q and m = 0..N-1 the
lag in frames.  This is what the FFT-in-time method of Appendix B reaches
exactly (its zero padding removes the cyclic wrap), so the oracle is this
definition written out, O(N^2) per wave vector, with no FFT.

Two implementations of the same sum: a NumPy one over all q at once per lag,
and a plain-C one (``direct_diff.c``, a double loop per q) used for sizes where
NumPy would take minutes.  Both accumulate in FP64.
"""

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct_diff.c")
_LIB = os.path.join(_HERE, "liboracle_direct.so")
_lock = threading.Lock()
_lib = None


def build_native(force=False):
    """Compile the C direct-difference routine with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _native():
    global _lib
    with _lock:
        if _lib is None:
            build_native()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_direct_diff.restype = None
            lib.oracle_direct_diff.argtypes = [
                ctypes.c_void_p, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                ctypes.c_void_p, ctypes.c_int]
            _lib = lib
    return _lib


def _direct_numpy(F, M):
    Q, N = F.shape
    D = np.zeros((Q, M), dtype=np.float64)
    for m in range(1, M):
        diff = F[:, m:] - F[:, :N - m]          # pairs (n, n-m), n = m..N-1
        D[:, m] = (diff.real ** 2 + diff.imag ** 2).sum(axis=1) / (N - m)
    return D


def structure_function_direct(F, max_lag=None, impl="auto", threads=None):
    """D[q, m] for m in [0, max_lag) from time series F[q, t] (complex).

    F: complex array [Q, N] (q-major, time contiguous).  Returns float64 [Q, M].
    impl: "numpy", "c", or "auto" (C when Q*N*M is large).
    """
    F = np.ascontiguousarray(F, dtype=np.complex128)
    Q, N = F.shape
    M = N if max_lag in (None, 0) else int(max_lag)
    if not (1 <= M <= N):
        raise ValueError("max_lag must be in [1, N]")
    if impl == "auto":
        impl = "c" if Q * N * M > 2e7 else "numpy"
    if impl == "numpy":
        return _direct_numpy(F, M)
    D = np.empty((Q, M), dtype=np.float64)
    nt = int(threads or os.cpu_count() or 1)
    _native().oracle_direct_diff(F.ctypes.data, Q, N, M, D.ctypes.data, nt)
    return D


def structure_function_sum_rule_rhs(frames, m):
    """Exact integer right-hand side of the weighted sum rule at lag m.

    Parseval applied to the difference images gives
        sum over the full plane of D(q, m) = P/(N-m) * sum_{n=m}^{N-1} sum_x (I_n - I_{n-m})^2
    with P = W*H pixels.  Returned as the exact rational (numerator, denominator)
    in Python integers.
    """
    frames = np.asarray(frames).astype(np.int64)
    N, H, W = frames.shape
    tot = 0
    for n in range(m, N):
        d = frames[n] - frames[n - m]
        tot += int((d * d).sum())
    return tot * W * H, N - m
