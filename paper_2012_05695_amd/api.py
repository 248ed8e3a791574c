"""Python binding of libddm (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI of
``include/ddm.h``; this module checks tensor shapes and dtypes, passes device
pointers and the current HIP stream, and turns status codes into exceptions.
PyTorch provides device memory and streams.
"""

import ctypes

import numpy as np
import torch

from . import _lib as L

_lib = L.load()


class DdmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (L.STATUS_NAMES.get(status, str(status)), message))
        self.status = status


def _check(st):
    if st == L.DDM_OK:
        return st
    if st == L.DDM_WARN_FP16_SATURATED:
        return st
    raise DdmError(st, (_lib.ddm_last_error() or b"").decode())


def last_error():
    return (_lib.ddm_last_error() or b"").decode()


def abi_version():
    return int(_lib.ddm_abi_version())


NOALLOC_SCRATCH_BYTES = L.DDM_NOALLOC_SCRATCH_BYTES

_PIX = {"u8": L.DDM_PIX_U8, "u16": L.DDM_PIX_U16}
_PIX_DTYPES = {L.DDM_PIX_U8: (torch.uint8,), L.DDM_PIX_U16: (torch.uint16, torch.int16)}
_SPEC = {"f32": L.DDM_SPEC_F32, "f16": L.DDM_SPEC_F16_QSCALED}
_PAD = {"pow2": L.DDM_PAD_POW2, "minimal": L.DDM_PAD_MINIMAL}
_METHOD = {"fourier": L.DDM_METHOD_FOURIER, "direct": L.DDM_METHOD_DIRECT, "auto": L.DDM_METHOD_AUTO}
_METHOD_NAME = {v: k for k, v in _METHOD.items()}


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require(t, name, dtypes, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on a HIP device (got %s)" % (name, t.device))
    if device is not None and t.device.index != device:
        raise ValueError("%s is on device %s, plan on cuda:%d" % (name, t.device, device))
    if t.dtype not in dtypes:
        raise TypeError("%s dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Plan:
    """A structure-function plan for W x H frames, N per stack.

    Mirrors ``ddm_plan_create``; see include/ddm.h for the meaning of each field.
    """

    def __init__(self, width, height, n_frames, max_lag=0, pixel="u16", spectrum="f32",
                 precondition=True, k2_max=-1, padding="pow2", method="fourier", stream=None, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self.width, self.height, self.n_frames = int(width), int(height), int(n_frames)
        self.pixel = _PIX[pixel] if isinstance(pixel, str) else int(pixel)
        self._stream = stream
        d = L.PlanDesc()
        _lib.ddm_plan_desc_init(ctypes.byref(d))
        d.width, d.height, d.n_frames = self.width, self.height, self.n_frames
        d.max_lag = int(max_lag)
        d.pixel = self.pixel
        d.spectrum = _SPEC[spectrum] if isinstance(spectrum, str) else int(spectrum)
        d.precondition = 1 if precondition else 0
        d.k2_max = int(k2_max)
        d.padding = _PAD[padding] if isinstance(padding, str) else int(padding)
        d.method = _METHOD[method] if isinstance(method, str) else int(method)
        with torch.cuda.device(self.device):
            d.stream = _stream_handle(stream).value
        self._desc = d
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_plan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        nq, ml, n2 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.ddm_plan_query(h, ctypes.byref(nq), ctypes.byref(ml), ctypes.byref(n2)))
        self.n_q, self.max_lag, self.n2 = int(nq.value), int(ml.value), int(n2.value)
        self._ws = None
        self.last_status = L.DDM_OK

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                _check(_lib.ddm_plan_destroy(self._h))
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- queries --
    def q_index(self):
        kx = np.empty(self.n_q, dtype=np.int32)
        ky = np.empty(self.n_q, dtype=np.int32)
        _check(_lib.ddm_plan_q_index(self._h, kx.ctypes.data, ky.ctypes.data))
        return kx, ky

    @property
    def method(self):
        """Step two's method: "fourier" or "direct" (ddm_plan_method)."""
        m = ctypes.c_int32()
        _check(_lib.ddm_plan_method(self._h, ctypes.byref(m)))
        return _METHOD_NAME[int(m.value)]

    def workspace_size(self):
        mn, full = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.ddm_plan_workspace_size(self._h, ctypes.byref(mn), ctypes.byref(full)))
        return int(mn.value), int(full.value)

    def set_workspace(self, ws):
        _require(ws, "workspace", (torch.uint8,), (ws.numel(),), self.device)
        _check(_lib.ddm_plan_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        self._ws = ws

    def allocate_workspace(self, nbytes=None):
        mn, full = self.workspace_size()
        n = full if nbytes is None else max(int(nbytes), mn)
        ws = torch.empty(n, dtype=torch.uint8, device="cuda:%d" % self.device)
        self.set_workspace(ws)
        return ws

    def autotune(self):
        """Time the time-kernel launch shapes (and, for method "auto", the direct
        kernel, keeping the faster method) on this plan's workspace; returns
        (E, qpw, ms of step two per call)."""
        if self._ws is None:
            self.allocate_workspace()
        E, q, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_plan_autotune(self._h, ctypes.byref(E), ctypes.byref(q), ctypes.byref(ms)))
        return int(E.value), int(q.value), float(ms.value)

    # -- profiling (event pairs around launches on the plan's stream) --
    KERNELS = {"row": L.DDM_KERNEL_ROW, "col": L.DDM_KERNEL_COL, "time": L.DDM_KERNEL_TIME,
               "radial": L.DDM_KERNEL_RADIAL, "step1": L.DDM_KERNEL_STEP1}

    def set_profiling(self, kinds=()):
        mask = 0
        for k in kinds:
            mask |= self.KERNELS[k]
        _check(_lib.ddm_plan_set_profiling(self._h, mask))

    def profile(self, kind):
        """(total device ms, launches) of one kernel kind since set_profiling."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib.ddm_plan_get_profile(self._h, self.KERNELS[kind], ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    # -- computations --
    def _frames_ok(self, frames):
        _require(frames, "frames", _PIX_DTYPES[self.pixel],
                 (self.n_frames, self.height, self.width), self.device)

    def structure_function(self, frames, out=None):
        """D [n_q, max_lag] float32 of frames [N, H, W] (device tensors)."""
        self._frames_ok(frames)
        if self._ws is None:
            self.allocate_workspace()
        if out is None:
            out = torch.empty((self.n_q, self.max_lag), dtype=torch.float32, device=frames.device)
        _require(out, "D", (torch.float32,), (self.n_q, self.max_lag), self.device)
        with torch.cuda.device(self.device):
            self.last_status = _check(_lib.ddm_structure_function(self._h, ctypes.c_void_p(frames.data_ptr()),
                                                                  ctypes.c_void_p(out.data_ptr())))
        return out

    def structure_function_host(self, frames_host, staging, out=None):
        """D from frames in host memory (a CPU tensor, pinned for overlapped
        copies) through the device staging buffer `staging` (uint8 tensor;
        ddm_structure_function_host).  The frames must stay alive until the
        stream has passed the call."""
        if not isinstance(frames_host, torch.Tensor) or frames_host.device.type != "cpu":
            raise ValueError("frames_host must be a CPU tensor")
        if frames_host.dtype not in _PIX_DTYPES[self.pixel] or \
                tuple(frames_host.shape) != (self.n_frames, self.height, self.width) or \
                not frames_host.is_contiguous():
            raise ValueError("frames_host must be a contiguous [N, H, W] tensor of the plan's pixel type")
        _require(staging, "staging", (torch.uint8,), (staging.numel(),), self.device)
        if self._ws is None:
            self.allocate_workspace()
        if out is None:
            out = torch.empty((self.n_q, self.max_lag), dtype=torch.float32, device="cuda:%d" % self.device)
        _require(out, "D", (torch.float32,), (self.n_q, self.max_lag), self.device)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_structure_function_host(self._h, ctypes.c_void_p(frames_host.data_ptr()),
                                                    ctypes.c_void_p(staging.data_ptr()), staging.numel(),
                                                    ctypes.c_void_p(out.data_ptr())))
        return out

    def structure_function_noalloc(self, frames, out=None):
        """As structure_function, on the library's static device scratch instead
        of a workspace (ddm_structure_function_noalloc): no device allocation
        in the call when `out` is given."""
        self._frames_ok(frames)
        if out is None:
            out = torch.empty((self.n_q, self.max_lag), dtype=torch.float32, device=frames.device)
        _require(out, "D", (torch.float32,), (self.n_q, self.max_lag), self.device)
        with torch.cuda.device(self.device):
            self.last_status = _check(_lib.ddm_structure_function_noalloc(
                self._h, ctypes.c_void_p(frames.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def status(self):
        """Synchronise and report the outcomes of every call since the last
        report (ddm_plan_status): raises DdmError on a failed step one; returns
        DDM_OK or DDM_WARN_FP16_SATURATED."""
        with torch.cuda.device(self.device):
            return _check(_lib.ddm_plan_status(self._h))

    def fp16_saturations(self):
        """Spectrum components clipped by the FP16 store since plan creation (syncs)."""
        c = ctypes.c_int64()
        _check(_lib.ddm_plan_fp16_saturations(self._h, ctypes.byref(c)))
        return int(c.value)

    def image_spectra(self, frames, out=None):
        """F [n_q, N] complex64: step one only (frame 0 subtracted if the plan preconditions)."""
        self._frames_ok(frames)
        if self._ws is None:
            self.allocate_workspace()
        if out is None:
            out = torch.empty((self.n_q, self.n_frames), dtype=torch.complex64, device=frames.device)
        _require(out, "spectra", (torch.complex64,), (self.n_q, self.n_frames), self.device)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_image_spectra(self._h, ctypes.c_void_p(frames.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr())))
        return out

    def structure_from_spectra(self, spectra, out=None):
        """D [n_q, max_lag] float32 from time series [n_q, N] complex64: step two only."""
        _require(spectra, "spectra", (torch.complex64,), (self.n_q, self.n_frames), self.device)
        if out is None:
            out = torch.empty((self.n_q, self.max_lag), dtype=torch.float32, device=spectra.device)
        _require(out, "D", (torch.float32,), (self.n_q, self.max_lag), self.device)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_structure_from_spectra(self._h, ctypes.c_void_p(spectra.data_ptr()),
                                                   ctypes.c_void_p(out.data_ptr())))
        return out

    def radial_average(self, D, thresholds, bin_of_q=True):
        """(Dbar [n_bins, M] float64, counts [n_bins] int64, bin_of_q [n_q] int32 or None)."""
        _require(D, "D", (torch.float32,), (self.n_q, self.max_lag), self.device)
        thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.int64))
        nb = len(thr) - 1
        if nb < 0:
            raise ValueError("thresholds needs at least one entry")
        dev = D.device
        Dbar = torch.empty((max(nb, 0), self.max_lag), dtype=torch.float64, device=dev)
        counts = torch.empty((max(nb, 0),), dtype=torch.int64, device=dev)
        boq = torch.empty((self.n_q,), dtype=torch.int32, device=dev) if bin_of_q else None
        with torch.cuda.device(self.device):
            _check(_lib.ddm_radial_average(
                self._h, ctypes.c_void_p(D.data_ptr()), ctypes.c_void_p(thr.ctypes.data), nb,
                ctypes.c_void_p(Dbar.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                ctypes.c_void_p(boq.data_ptr() if boq is not None else 0)))
        return Dbar, counts, boq


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def log_lags(n_frames, K=64):
    """K log-spaced fractional lags from 1 to N-1 (float32)."""
    return np.geomspace(1.0, float(n_frames - 1), K).astype(np.float32)


def sample_curves(D, lags, stream=None):
    """Rows of D [n, M] sampled at fractional lags -> (curves [n, K] / row max, scale [n])."""
    lags = np.ascontiguousarray(np.asarray(lags, dtype=np.float32))
    n, M = D.shape
    _require(D, "D", (torch.float32,), (n, M), None)
    K = len(lags)
    curves = torch.empty((n, K), dtype=torch.float32, device=D.device)
    scale = torch.empty((n,), dtype=torch.float32, device=D.device)
    with torch.cuda.device(D.device):
        _check(_lib.ddm_sample_curves(_ptr(D), n, M, ctypes.c_void_p(lags.ctypes.data), K, _ptr(curves),
                                      _ptr(scale), _stream_handle(stream)))
    return curves, scale


def fit(curves, lags, init=None, fallback=True, max_iter=200, ftol=1e-7, xtol=1e-7, gtol=1e-3,
        lambda0=1e-3, stream=None):
    """LM fit of every row of curves [n, K] -> (params [n, 3] = A, B, tau; iters [n]; flags [n]).

    init: optional [n, 3] float32 (A, B, log tau) start; else the default start.
    fallback (with init): True refits from the default start the curves that do
    not converge; "best" starts each curve from whichever of init and the default
    start has the lower cost; "gate" starts from init where its tau lies within
    [m_1 / 4, 4 m_K] and its A is at least 5% of |A| + |B|, else from the default
    start; False fits from init only.
    """
    lags = np.ascontiguousarray(np.asarray(lags, dtype=np.float32))
    n, K = curves.shape
    _require(curves, "curves", (torch.float32,), (n, K), None)
    if init is not None:
        _require(init, "init", (torch.float32,), (n, 3), None)
    d = L.FitDesc()
    _lib.ddm_fit_desc_init(ctypes.byref(d))
    d.K, d.max_iter = K, int(max_iter)
    d.fallback = {"best": 2, "gate": 3}.get(fallback, 1 if fallback is True else 0) \
        if isinstance(fallback, (str, bool)) else int(fallback)
    d.ftol, d.xtol, d.gtol, d.lambda0 = float(ftol), float(xtol), float(gtol), float(lambda0)
    with torch.cuda.device(curves.device):
        d.stream = _stream_handle(stream).value
    params = torch.empty((n, 3), dtype=torch.float32, device=curves.device)
    iters = torch.empty((n,), dtype=torch.int32, device=curves.device)
    flags = torch.empty((n,), dtype=torch.int32, device=curves.device)
    with torch.cuda.device(curves.device):
        _check(_lib.ddm_fit(ctypes.byref(d), _ptr(curves), ctypes.c_void_p(lags.ctypes.data), n, _ptr(init),
                            _ptr(params), _ptr(iters), _ptr(flags)))
    return params, iters, flags


def integer_bin_thresholds(n_bins):
    """Thresholds of the bins b = round(|k|), b = 0..n_bins-1, on integer k2.

    round(sqrt(k2)) = b  <=>  b^2 - b + 1 <= k2 <= b^2 + b, so T_0 = 0 and
    T_b = b^2 - b + 1.
    """
    b = np.arange(n_bins + 1, dtype=np.int64)
    t = b * b - b + 1
    t[0] = 0
    return t


def log_bin_thresholds(n_bins, k_min, k_max):
    """n_bins logarithmic |k| bins with edges geomspace(k_min, k_max, n_bins+1).

    Each edge e becomes the integer threshold ceil(e^2) on k2 (so that
    k2 >= T <=> |k| >= e for integer k2, with e^2 evaluated in FP64); where low
    edges are closer than one lattice step, equal thresholds give empty bins.
    """
    e = np.geomspace(float(k_min), float(k_max), int(n_bins) + 1)
    t = np.ceil(e * e).astype(np.int64)
    t[-1] = max(t[-1], int(np.floor(k_max * k_max)) + 1)
    return t


class Mlp:
    """The fit-initialisation network (ddm_mlp_* of include/ddm.h)."""

    N_PARAMS = L.DDM_MLP_NPARAMS

    def __init__(self, seed=0, max_batch=4096, stream=None, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_mlp_create(int(seed), self.max_batch, _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.loss_dev = torch.zeros(1, dtype=torch.float32, device="cuda:%d" % self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                _check(_lib.ddm_mlp_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        p = np.empty(self.N_PARAMS, dtype=np.float32)
        _check(_lib.ddm_mlp_get_params(self._h, ctypes.c_void_p(p.ctypes.data)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        assert p.shape == (self.N_PARAMS,)
        _check(_lib.ddm_mlp_set_params(self._h, ctypes.c_void_p(p.ctypes.data)))

    def get_state(self):
        p, m, v = (np.empty(self.N_PARAMS, dtype=np.float32) for _ in range(3))
        st = ctypes.c_int64()
        _check(_lib.ddm_mlp_get_state(self._h, ctypes.c_void_p(p.ctypes.data), ctypes.c_void_p(m.ctypes.data),
                                      ctypes.c_void_p(v.ctypes.data), ctypes.byref(st)))
        return {"params": p, "adam_m": m, "adam_v": v, "step": int(st.value)}

    def set_state(self, s):
        p, m, v = (np.ascontiguousarray(np.asarray(s[k], dtype=np.float32)) for k in ("params", "adam_m", "adam_v"))
        _check(_lib.ddm_mlp_set_state(self._h, ctypes.c_void_p(p.ctypes.data), ctypes.c_void_p(m.ctypes.data),
                                      ctypes.c_void_p(v.ctypes.data), int(s["step"])))

    def forward(self, x, out=None):
        n = x.shape[0]
        _require(x, "x", (torch.float32,), (n, L.DDM_MLP_IN), self.device)
        if out is None:
            out = torch.empty((n, L.DDM_MLP_OUT), dtype=torch.float32, device=x.device)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_mlp_forward(self._h, _ptr(x), n, _ptr(out)))
        return out

    def gradient(self, x, t):
        """(grad [N_PARAMS] float32 numpy, loss) for one batch (host sync)."""
        B = x.shape[0]
        _require(x, "x", (torch.float32,), (B, L.DDM_MLP_IN), self.device)
        _require(t, "t", (torch.float32,), (B, L.DDM_MLP_OUT), self.device)
        g = np.empty(self.N_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_mlp_gradient(self._h, _ptr(x), _ptr(t), B, ctypes.c_void_p(g.ctypes.data),
                                         ctypes.byref(loss)))
        return g, float(loss.value)

    def adam_step(self, lr):
        _check(_lib.ddm_mlp_adam_step(self._h, float(lr)))

    def train_step(self, x, t, lr):
        """One asynchronous step; the batch loss lands in self.loss_dev."""
        B = x.shape[0]
        _require(x, "x", (torch.float32,), (B, L.DDM_MLP_IN), self.device)
        _require(t, "t", (torch.float32,), (B, L.DDM_MLP_OUT), self.device)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_mlp_train_step(self._h, _ptr(x), _ptr(t), B, float(lr), _ptr(self.loss_dev)))


class Batch:
    """Independent stacks of uneven sizes in one graph launch (ddm_batch_* of include/ddm.h).

    shapes: list of (W, H, N) or dicts with Plan keyword fields (width, height,
    n_frames, max_lag, pixel, precondition, k2_max, padding, method)."""

    def __init__(self, shapes, lanes=4, padding="pow2", stream=None, device=None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        descs = (L.PlanDesc * len(shapes))()
        self.shapes = []
        for i, sh in enumerate(shapes):
            if not isinstance(sh, dict):
                sh = {"width": sh[0], "height": sh[1], "n_frames": sh[2]}
            d = descs[i]
            _lib.ddm_plan_desc_init(ctypes.byref(d))
            d.width, d.height, d.n_frames = int(sh["width"]), int(sh["height"]), int(sh["n_frames"])
            d.max_lag = int(sh.get("max_lag", 0))
            pix = sh.get("pixel", "u16")
            d.pixel = _PIX[pix] if isinstance(pix, str) else int(pix)
            d.precondition = 1 if sh.get("precondition", True) else 0
            d.k2_max = int(sh.get("k2_max", -1))
            pad = sh.get("padding", padding)
            d.padding = _PAD[pad] if isinstance(pad, str) else int(pad)
            meth = sh.get("method", "fourier")
            d.method = _METHOD[meth] if isinstance(meth, str) else int(meth)
            self.shapes.append(sh)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_batch_create(descs, len(shapes), int(lanes), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._descs = descs
        self.n_q, self.max_lag, self.lane = [], [], []
        for i in range(len(shapes)):
            nq, ml, ln = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
            _check(_lib.ddm_batch_query(h, i, ctypes.byref(nq), ctypes.byref(ml), ctypes.byref(ln)))
            self.n_q.append(int(nq.value))
            self.max_lag.append(int(ml.value))
            self.lane.append(int(ln.value))
        self._ws = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                _check(_lib.ddm_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self):
        b = ctypes.c_size_t()
        _check(_lib.ddm_batch_workspace_size(self._h, ctypes.byref(b)))
        return int(b.value)

    def allocate_workspace(self):
        ws = torch.empty(self.workspace_size(), dtype=torch.uint8, device="cuda:%d" % self.device)
        _check(_lib.ddm_batch_set_workspace(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        self._ws = ws
        return ws

    def autotune(self):
        if self._ws is None:
            self.allocate_workspace()
        with torch.cuda.device(self.device):
            _check(_lib.ddm_batch_autotune(self._h))

    def set_bins(self, stack, thresholds):
        """|q| bins of one stack, computed inside the batch (ddm_batch_set_bins);
        an empty or one-entry threshold list removes them."""
        thr = np.ascontiguousarray(np.asarray(thresholds, dtype=np.int64))
        nb = max(len(thr) - 1, 0)
        if len(thr) == 0:
            thr = np.zeros(1, dtype=np.int64)
        with torch.cuda.device(self.device):
            _check(_lib.ddm_batch_set_bins(self._h, int(stack), ctypes.c_void_p(thr.ctypes.data), nb))
        self.n_bins = getattr(self, "n_bins", [0] * len(self._descs))
        self.n_bins[int(stack)] = nb

    def structure_function_binned(self, frames, outs=None, dbar=None, counts=None):
        """frames -> (D list, Dbar list, counts list); stacks without bins give None.
        Passing the lists of an earlier call reuses them (and the captured graph)."""
        n = len(self._descs)
        nbins = getattr(self, "n_bins", [0] * n)
        if dbar is None:
            dbar = [torch.empty((nbins[i], self.max_lag[i]), dtype=torch.float64, device=frames[i].device)
                    if nbins[i] else None for i in range(n)]
        if counts is None:
            counts = [torch.empty((nbins[i],), dtype=torch.int64, device=frames[i].device) if nbins[i] else None
                      for i in range(n)]
        cnt = counts
        for i in range(n):
            if nbins[i]:
                _require(dbar[i], "Dbar[%d]" % i, (torch.float64,), (nbins[i], self.max_lag[i]), self.device)
                _require(cnt[i], "counts[%d]" % i, (torch.int64,), (nbins[i],), self.device)
        outs = self.structure_function(frames, outs, _bins=(dbar, cnt))
        return outs, dbar, cnt

    def structure_function(self, frames, outs=None, _bins=None):
        """frames: list of [N, H, W] device tensors -> list of D [n_q, M] float32."""
        n = len(self._descs)
        assert len(frames) == n
        if self._ws is None:
            self.allocate_workspace()
        if outs is None:
            outs = [torch.empty((self.n_q[i], self.max_lag[i]), dtype=torch.float32, device=frames[i].device)
                    for i in range(n)]
        for i in range(n):
            d = self._descs[i]
            _require(frames[i], "frames[%d]" % i, _PIX_DTYPES[d.pixel], (d.n_frames, d.height, d.width), self.device)
            _require(outs[i], "D[%d]" % i, (torch.float32,), (self.n_q[i], self.max_lag[i]), self.device)
        fp = (ctypes.c_void_p * n)(*[f.data_ptr() for f in frames])
        dp = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        with torch.cuda.device(self.device):
            if _bins is None:
                _check(_lib.ddm_batch_structure_function(self._h, fp, dp))
            else:
                bp = (ctypes.c_void_p * n)(*[t.data_ptr() if t is not None else 0 for t in _bins[0]])
                cp = (ctypes.c_void_p * n)(*[t.data_ptr() if t is not None else 0 for t in _bins[1]])
                _check(_lib.ddm_batch_structure_function_binned(self._h, fp, dp, bp, cp))
        return outs

    def status(self):
        """Per-stack statuses of every call since the last report
        (ddm_batch_status, synchronises): a list of DDM_OK / DDM_ERR_HIP codes;
        does not raise."""
        n = len(self._descs)
        out = (ctypes.c_int32 * n)()
        with torch.cuda.device(self.device):
            st = _lib.ddm_batch_status(self._h, out)
        if st not in (L.DDM_OK, L.DDM_ERR_HIP):
            _check(st)
        return [int(x) for x in out]
