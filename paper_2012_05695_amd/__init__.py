"""DDM image structure function via a Fourier transform in time, on MI355X.

Hot path (arXiv 2012.05695, section "The algorithm" and Appendix B): a 2-D FFT
of every frame, a transpose to per-wave-vector time series, and for each wave
vector a zero-padded time FFT -> |.|^2 -> inverse FFT autocorrelation combined
with |F|^2 prefix sums into D(q, m); then azimuthal |q| binning.  All of it runs
in hand-written HIP kernels behind the C ABI of ``include/ddm.h``.

``Plan`` and the other binding names load ``libddm.so`` on first access and
raise if it is missing; ``synth`` (seeded input stacks) needs no library.
"""

_API = {"Plan", "DdmError", "integer_bin_thresholds", "log_bin_thresholds", "abi_version",
        "last_error", "log_lags", "sample_curves", "fit", "Mlp", "Batch"}


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)


__all__ = sorted(_API) + ["synth"]
