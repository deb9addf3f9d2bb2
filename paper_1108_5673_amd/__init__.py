"""MI355X partial-wave-analysis likelihood: Python binding of libpwa.

The extended unbinned negative log-likelihood of a partial-wave fit and its
analytic gradient (arXiv:1108.5673, Sec. 2, Eq. 3), evaluated by hand-written
HIP kernels for gfx950 behind the C ABI of include/pwa.h.  This module only
marshals arguments: every step of an evaluation runs in the library's kernels.
PyTorch, when used, supplies device memory and the current stream.

    from paper_1108_5673_amd import Model
    m = Model(data_amplitudes, mc_amplitudes, n_gen, form="table")
    nll, grad = m.nll_grad(V)          # grad = [dRe V_0, dIm V_0, ...]
"""
from __future__ import annotations

import ctypes
import warnings

import numpy as np

from . import _native
from ._native import PWAError

__all__ = ["Model", "PWAError", "nll_batched", "NLLFunction", "FORMS"]

FORMS = {
    "table": _native.PWA_FORM_TABLE,                    # complex64 table, fused kernel
    "amplitude": _native.PWA_FORM_AMPLITUDE,            # complex64 amplitudes
    "table_fp64_plain": _native.PWA_PRECISION_FP64_PLAIN,   # complex128 table, two passes
    "table_fp64": _native.PWA_PRECISION_FP64_FUSED,     # complex128 table, fused kernel
    "amplitude_bf16": _native.PWA_FORM_AMPLITUDE_BF16,  # bfloat16 amplitudes, matrix cores
    "amplitude_fp16": _native.PWA_FORM_AMPLITUDE_FP16,  # float16 amplitudes, matrix cores
}


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _current_stream():
    """torch's current HIP stream if torch has initialised the device, else NULL."""
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def _buffer(x, what: str):
    """(pointer, is_complex128, keepalive, shape) of a complex numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        if x.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("%s must be complex64 or complex128, got %s" % (what, x.dtype))
        x = x.contiguous()
        return ctypes.c_void_p(x.data_ptr()), x.dtype == torch.complex128, x, tuple(x.shape)
    a = np.asarray(x)
    if a.dtype not in (np.complex64, np.complex128):
        raise TypeError("%s must be complex64 or complex128, got %s" % (what, a.dtype))
    a = np.ascontiguousarray(a)
    return ctypes.c_void_p(a.ctypes.data), a.dtype == np.complex128, a, a.shape


def _v_array(v, n_waves: int) -> np.ndarray:
    """Production amplitudes as 2W doubles (re, im interleaved)."""
    if (type(v) is np.ndarray and v.dtype == np.float64 and v.ndim == 1
            and v.shape[0] == 2 * n_waves and v.flags.c_contiguous):
        return v
    if _is_torch(v):
        v = v.detach().cpu().numpy()
    a = np.asarray(v)
    if np.iscomplexobj(a):
        a = np.ascontiguousarray(a.astype(np.complex128)).view(np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    if a.shape[0] != 2 * n_waves:
        raise ValueError("expected %d waves (%d doubles), got %d doubles"
                         % (n_waves, 2 * n_waves, a.shape[0]))
    return a


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Model:
    """One data sample, its MC integral matrix and the device-resident table or
    amplitudes (built once; Sec. 2, the paragraph after Eq. 3).

    data:  (N, W) complex decay amplitudes, or with input_is_table=True an
           (N, W(W+1)/2) packed Hermitian table; numpy or torch, host or device.
    mc:    (N_acc, W) accepted MC amplitudes, or None for M = 0.
    n_gen: number of generated MC events.
    form:  "table" | "amplitude" | "table_fp64_plain" | "table_fp64".
    """

    def __init__(self, data, mc=None, n_gen: int = 1, form: str = "table",
                 input_is_table: bool = False, n_waves: int | None = None, stream=None):
        L = _native.lib()
        if form not in FORMS:
            raise ValueError("form must be one of %s" % sorted(FORMS))
        dptr, d128, self._data_keep, dshape = _buffer(data, "data")
        if len(dshape) != 2:
            raise ValueError("data must be 2-D")
        n = int(dshape[0])
        if input_is_table:
            p = int(dshape[1])
            w = int(round((np.sqrt(8 * p + 1) - 1) / 2))
            if w * (w + 1) // 2 != p:
                raise ValueError("table width %d is not W(W+1)/2" % p)
        else:
            w = int(dshape[1])
        if n_waves is not None and n_waves != w:
            raise ValueError("n_waves %d does not match data (%d)" % (n_waves, w))
        flags = FORMS[form]
        if input_is_table:
            flags |= _native.PWA_INPUT_IS_TABLE
        if d128:
            flags |= _native.PWA_DATA_COMPLEX128
        if mc is not None:
            mptr, m128, mkeep, mshape = _buffer(mc, "mc")
            if len(mshape) != 2 or mshape[1] != w:
                raise ValueError("mc must be (N_acc, %d)" % w)
            n_acc = int(mshape[0])
            if m128:
                flags |= _native.PWA_MC_COMPLEX128
        else:
            mptr, mkeep, n_acc = None, None, 0
        self._stream = stream if stream is not None else _current_stream()
        handle = ctypes.c_void_p()
        _native.check(L.pwa_build_table(dptr, n, w, mptr, n_acc, int(n_gen), flags,
                                        self._stream, ctypes.byref(handle)))
        self._h = handle
        self._data_keep = None          # the library holds its own copy
        del mkeep
        self.n_data, self.n_waves, self.form = n, w, form
        self.n_packed = w * (w + 1) // 2
        self._setup_call_buffers(L)

    def _setup_call_buffers(self, L):
        # V in and the gradient out go through buffers owned by the model, so a
        # call passes cached addresses (taking an array's address costs more
        # than copying 2W doubles)
        self._vbuf = np.empty(2 * self.n_waves, np.float64)
        self._gbuf = np.empty(2 * self.n_waves, np.float64)
        self._vaddr, self._gaddr = self._vbuf.ctypes.data, self._gbuf.ctypes.data
        self._nllv = ctypes.c_double(0.0)
        self._nllp = ctypes.byref(self._nllv)
        self._fn_nll, self._fn_grad = L.pwa_nll, L.pwa_nll_grad

    # -- evaluation ---------------------------------------------------------
    def _handle(self):
        if not self._h:
            raise RuntimeError("model has been freed")
        return self._h

    def nll(self, v) -> float:
        np.copyto(self._vbuf, _v_array(v, self.n_waves))
        st = self._fn_nll(self._handle(), self._vaddr, self._nllp, self._stream)
        if st:
            if _native.check(st) == _native.PWA_WARN_DEGENERATE:
                warnings.warn("degenerate event (I <= 0): NLL is +inf")
        return self._nllv.value

    def nll_grad(self, v):
        """(NLL, gradient as 2W doubles [dRe V_0, dIm V_0, ...])."""
        np.copyto(self._vbuf, _v_array(v, self.n_waves))
        st = self._fn_grad(self._handle(), self._vaddr, self._nllp, self._gaddr, self._stream)
        if st:
            if _native.check(st) == _native.PWA_WARN_DEGENERATE:
                warnings.warn("degenerate event (I <= 0): NLL is +inf, gradient NaN")
        return self._nllv.value, self._gbuf.copy()

    def nll_grad_async(self, v_dev, out_dev, grad: bool = True, stream=None) -> None:
        """Enqueue one evaluation: V read from the device tensor v_dev (2W
        float64) when it runs, [nll, n_bad, grad 2W] written to out_dev (float64,
        2 + 2W; the first two without grad).  Stream-ordered, capturable in a
        graph; no synchronisation."""
        import torch
        for t, what, n in ((v_dev, "v_dev", 2 * self.n_waves),
                           (out_dev, "out_dev", 2 + 2 * self.n_waves if grad else 2)):
            if not (_is_torch(t) and t.is_cuda and t.dtype == torch.float64
                    and t.is_contiguous() and t.numel() >= n):
                raise ValueError("%s must be a contiguous CUDA float64 tensor of >= %d values"
                                 % (what, n))
        s = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        fn = _native.lib().pwa_nll_grad_async if grad else _native.lib().pwa_nll_async
        _native.check(fn(self._handle(), ctypes.c_void_p(v_dev.data_ptr()),
                         ctypes.c_void_p(out_dev.data_ptr()), ctypes.c_void_p(s)))

    # -- inspection ---------------------------------------------------------
    def nll_grad_hess(self, v):
        """(NLL, gradient (2W,), FUMILI matrix (2W, 2W)); amplitude form."""
        va = _v_array(v, self.n_waves)
        out = ctypes.c_double(0.0)
        g = np.zeros(2 * self.n_waves, np.float64)
        h = np.zeros((2 * self.n_waves, 2 * self.n_waves), np.float64)
        st = _native.check(_native.lib().pwa_nll_grad_hess(self._handle(), va.ctypes.data,
                                                           ctypes.byref(out), g.ctypes.data,
                                                           h.ctypes.data, self._stream))
        if st == _native.PWA_WARN_DEGENERATE:
            warnings.warn("degenerate event (I <= 0): NLL is +inf, gradient and matrix NaN")
        return out.value, g, h

    def info(self) -> dict:
        inf = _native.Info()
        _native.check(_native.lib().pwa_model_info(self._handle(), ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _native.Info._fields_}

    def table(self) -> np.ndarray:
        """The stored table in canonical packed (N, P) layout; for the
        amplitude forms the stored amplitudes as complex64 (N, W)."""
        if self.form in ("amplitude", "amplitude_bf16", "amplitude_fp16"):
            out = np.zeros((self.n_data, self.n_waves), np.complex64)
        else:
            dt = np.complex64 if self.form == "table" else np.complex128
            out = np.zeros((self.n_data, self.n_packed), dt)
        _native.check(_native.lib().pwa_copy_table(self._handle(), out.ctypes.data, self._stream))
        return out

    def mc_matrix(self) -> np.ndarray:
        out = np.zeros((self.n_waves, self.n_waves), np.complex128)
        _native.check(_native.lib().pwa_copy_mc_matrix(self._handle(), out.ctypes.data,
                                                       self._stream))
        return out

    def set_mc_matrix(self, M) -> None:
        a = np.ascontiguousarray(np.asarray(M, np.complex128))
        if a.shape != (self.n_waves, self.n_waves):
            raise ValueError("M must be (W, W)")
        _native.check(_native.lib().pwa_set_mc_matrix(self._handle(), a.ctypes.data,
                                                      self._stream))

    def amplitude_shape(self):
        """(lanes per event, waves per lane) of a FP32 amplitude-form model."""
        q, wl = ctypes.c_int32(0), ctypes.c_int32(0)
        _native.check(_native.lib().pwa_get_amplitude_shape(self._handle(), ctypes.byref(q),
                                                            ctypes.byref(wl)))
        return q.value, wl.value

    def set_amplitude_shape(self, lanes_per_event: int, waves_per_lane: int) -> None:
        _native.check(_native.lib().pwa_set_amplitude_shape(self._handle(), int(lanes_per_event),
                                                            int(waves_per_lane), self._stream))

    def tune_amplitude_shape(self, evals: int = 5):
        """Time the candidate storage shapes, keep the fastest; returns it."""
        q, wl = ctypes.c_int32(0), ctypes.c_int32(0)
        _native.check(_native.lib().pwa_tune_amplitude_shape(self._handle(), int(evals),
                                                             self._stream, ctypes.byref(q),
                                                             ctypes.byref(wl)))
        return q.value, wl.value

    def set_timing(self, enable, every: int = 1) -> None:
        """Time every `every`-th evaluation's main kernel (off when enable is false)."""
        _native.check(_native.lib().pwa_set_timing(self._handle(),
                                                   int(every) if enable else 0))

    def timing(self):
        """(total device milliseconds of the main kernel, launches) since the last call."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _native.check(_native.lib().pwa_get_timing(self._handle(), ctypes.byref(ms),
                                                   ctypes.byref(n)))
        return ms.value, n.value

    def read_ceiling(self, reps: int = 5) -> dict:
        """Achievable read bandwidth on the stored data: the fastest of `reps`
        passes of the fused kernel's own loads with the arithmetic taken out
        (tiled table forms) or of a plain non-temporal reader (other forms)."""
        ms = ctypes.c_double(0.0)
        nb = ctypes.c_int64(0)
        _native.check(_native.lib().pwa_read_ceiling(self._handle(), int(reps), self._stream,
                                                     ctypes.byref(ms), ctypes.byref(nb)))
        return {"ms": ms.value, "bytes": nb.value, "gbs": nb.value / (ms.value * 1e-3) / 1e9}

    def build_timing(self) -> dict:
        """Device milliseconds of the table preparation and of the MC integral."""
        t = ctypes.c_double(0.0)
        mc = ctypes.c_double(0.0)
        _native.check(_native.lib().pwa_build_timing(self._handle(), ctypes.byref(t),
                                                     ctypes.byref(mc)))
        return {"table_ms": t.value, "mc_ms": mc.value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            _native.lib().pwa_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _addr(a: np.ndarray) -> int:
    return a.__array_interface__["data"][0]


def _batch_rows(v, n_waves: int) -> np.ndarray:
    """(K, 2W) float64 C-contiguous view or copy of K parameter vectors."""
    a = v.detach().cpu().numpy() if _is_torch(v) else v
    if not isinstance(a, np.ndarray) or a.dtype.kind == "c":
        a = np.asarray(a)
        if a.dtype.kind == "c":
            a = np.ascontiguousarray(a, np.complex128).view(np.float64)
    return np.ascontiguousarray(a, np.float64).reshape(-1, 2 * n_waves)


def nll_batched(models, vs, grad: bool = True, stream=None):
    """Evaluate K_m parameter sets on each of several models.

    vs[m] is a (K_m, W_m) complex or (K_m, 2 W_m) real array.  Returns a list of
    (nll (K_m,), grad (K_m, 2 W_m) or None) per model.
    """
    L = _native.lib()
    n = len(models)
    rows = [_batch_rows(v, m.n_waves) for m, v in zip(models, vs)]
    ks = [a.shape[0] for a in rows]
    if n == 1:
        vall = rows[0]
    else:
        vall = np.concatenate([a.ravel() for a in rows]) if rows else np.zeros(0)
    total = sum(ks)
    nll = np.empty(total, np.float64)
    g = np.empty(sum(k * 2 * m.n_waves for k, m in zip(ks, models)), np.float64) if grad else None
    handles = (ctypes.c_void_p * max(1, n))(*[m._handle() for m in models])
    karr = (ctypes.c_int32 * max(1, n))(*ks)
    st = stream if stream is not None else (models[0]._stream if models else None)
    status = _native.check(L.pwa_nll_batched(handles, n, karr, _addr(vall), _addr(nll),
                                             _addr(g) if grad else None, st))
    if status == _native.PWA_WARN_DEGENERATE:
        warnings.warn("degenerate evaluation(s): NLL +inf")
    out, pos, gpos = [], 0, 0
    for m, k in zip(models, ks):
        gi = None
        if grad:
            gi = g[gpos:gpos + k * 2 * m.n_waves].reshape(k, 2 * m.n_waves)
            gpos += k * 2 * m.n_waves
        out.append((nll[pos:pos + k], gi))
        pos += k
    return out


class Batch:
    """A fixed list of models evaluated together through one pwa_nll_batched
    call per step, with the handle list, counts, parameter layout and output
    buffers set up once (for callers that evaluate the same models every
    iteration, such as a fit of many models or many starting points).

    ks[m] parameter vectors of model m per call (default 1 each).  The
    parameters of a call are one flat float64 array of `size` values: model
    0's K_0 x 2W_0 (re, im interleaved), then model 1's, ...  `params[m]` is a
    (K_m, 2W_m) view of an internal array of that layout, which a call uses
    when it is given no array.  A call returns `results`: a list of
    (nll (K_m,), grad (K_m, 2W_m) or None) views of output buffers that the
    next call overwrites.
    """

    def __init__(self, models, ks=None, grad: bool = True, stream=None):
        self.models = list(models)
        n = len(self.models)
        self.ks = [1] * n if ks is None else [int(k) for k in ks]
        if len(self.ks) != n or any(k < 0 for k in self.ks):
            raise ValueError("ks must hold one non-negative count per model")
        widths = [2 * m.n_waves for m in self.models]
        off = np.cumsum([0] + [k * w for k, w in zip(self.ks, widths)])
        self.size = int(off[-1])
        self._handles = (ctypes.c_void_p * max(1, n))(*[m._handle() for m in self.models])
        self._karr = (ctypes.c_int32 * max(1, n))(*self.ks)
        self._v = np.zeros(max(1, self.size), np.float64)
        self._nll = np.empty(max(1, sum(self.ks)), np.float64)
        self._g = np.empty(max(1, self.size), np.float64) if grad else None
        self.params = [self._v[off[i]:off[i + 1]].reshape(k, w)
                       for i, (k, w) in enumerate(zip(self.ks, widths))]
        pos = np.cumsum([0] + self.ks)
        self.results = [(self._nll[pos[i]:pos[i + 1]],
                         self._g[off[i]:off[i + 1]].reshape(k, w) if grad else None)
                        for i, (k, w) in enumerate(zip(self.ks, widths))]
        self._stream = stream if stream is not None else (self.models[0]._stream if n else None)
        self._nll_addr, self._g_addr = _addr(self._nll), (_addr(self._g) if grad else None)

    def __call__(self, v=None):
        if v is None:
            a = self._v
        else:
            a = v.detach().cpu().numpy() if _is_torch(v) else v
            if (not isinstance(a, np.ndarray) or a.dtype != np.float64
                    or not a.flags.c_contiguous):
                a = np.ascontiguousarray(a, np.float64)
            if a.size != self.size:
                raise ValueError("expected %d parameter values, got %d" % (self.size, a.size))
        for m in self.models:
            m._handle()   # raises if a model was freed
        status = _native.check(_native.lib().pwa_nll_batched(
            self._handles, len(self.models), self._karr, _addr(a), self._nll_addr, self._g_addr,
            self._stream))
        if status == _native.PWA_WARN_DEGENERATE:
            warnings.warn("degenerate evaluation(s): NLL +inf")
        return self.results


def __getattr__(name):
    if name == "NLLFunction":
        from .autograd import NLLFunction
        return NLLFunction
    raise AttributeError(name)
