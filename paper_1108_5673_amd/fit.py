"""Fit drivers: limited-memory BFGS through the library's C ABI.

    from paper_1108_5673_amd import fit
    v, res = fit.fit_lbfgs(model, v0)              # NLL(V) on the GPU, gauge Im V_0 = 0
    v, res = fit.fit_fumili(model, v0)             # damped Newton on the FUMILI matrix
    x, res = fit.minimize_lbfgs(fun, x0)           # fun(x) -> (f, g), any objective
    x, res = fit.minimize_newton(fun, x0)          # fun(x) -> (f, g, H)

The minimiser runs in the library (include/pwa.h, pwa_lbfgs_minimize); this
module only marshals arguments and wraps a Python objective as a C callback.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native

STATUS = {
    _native.PWA_LBFGS_CONVERGED_GRADIENT: "converged (gradient)",
    _native.PWA_LBFGS_CONVERGED_VALUE: "converged (value)",
    _native.PWA_LBFGS_MAX_ITERATIONS: "iteration limit",
    _native.PWA_LBFGS_LINE_SEARCH_FAILED: "line search failed",
}


def _options(**kw) -> _native.LbfgsOptions:
    opt = _native.LbfgsOptions()
    _native.lib().pwa_lbfgs_default_options(ctypes.byref(opt))
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(opt, k):
            raise TypeError("unknown L-BFGS option %r" % k)
        setattr(opt, k, v)
    return opt


def _result(r: _native.LbfgsResult) -> dict:
    return {"status": r.status, "message": STATUS.get(r.status, "?"), "iterations": r.iterations,
            "evaluations": r.evaluations, "f": r.f, "grad_norm": r.grad_norm}


def minimize_lbfgs(fun, x0, **options):
    """Minimise fun (x -> (f, g)) from x0; returns (x, result dict)."""
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).ravel().copy())
    n = x.size
    err = []

    def cb(_ctx, xp, fp, gp):
        try:
            xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            f, g = fun(xv)
            fp[0] = float(f)
            np.ctypeslib.as_array(gp, shape=(n,))[:] = np.asarray(g, dtype=np.float64).ravel()
            return 0
        except Exception as e:          # reported after the call returns
            err.append(e)
            return _native.PWA_ERR_INVALID

    c_cb = _native.OBJECTIVE(cb)
    res = _native.LbfgsResult()
    opt = _options(**options)
    status = _native.lib().pwa_lbfgs_minimize(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              c_cb, None, ctypes.byref(opt), ctypes.byref(res))
    if err:
        raise err[0]
    _native.check(status)
    return x, _result(res)


def fit_lbfgs(model, v0, stream=None, **options):
    """Fit V on a model from v0 ((W,) complex or (2W,) real); returns
    (V as (W,) complex128, result dict)."""
    a = np.asarray(v0)
    if np.iscomplexobj(a):
        a = a.astype(np.complex128).view(np.float64)
    x = np.ascontiguousarray(a, dtype=np.float64).ravel().copy()
    if x.size != 2 * model.n_waves:
        raise ValueError("expected %d waves" % model.n_waves)
    res = _native.LbfgsResult()
    opt = _options(**options)
    st = stream if stream is not None else model._stream
    status = _native.lib().pwa_fit_lbfgs(model._handle(),
                                         x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         ctypes.byref(opt), ctypes.byref(res), st)
    _native.check(status)
    return x.view(np.complex128).copy(), _result(res)


def minimize_newton(fun, x0, **options):
    """Minimise fun (x -> (f, g, H)) from x0 with damped Newton steps; returns
    (x, result dict).  At trial points the library asks for f and g only and
    the H fun returns is not used."""
    x = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).ravel().copy())
    n = x.size
    err = []

    def cb(_ctx, xp, fp, gp, hp):
        try:
            f, g, H = fun(np.ctypeslib.as_array(xp, shape=(n,)).copy())
            fp[0] = float(f)
            np.ctypeslib.as_array(gp, shape=(n,))[:] = np.asarray(g, dtype=np.float64).ravel()
            if hp:   # NULL at trial points: f and g only
                np.ctypeslib.as_array(hp, shape=(n * n,))[:] = np.asarray(H, dtype=np.float64).ravel()
            return 0
        except Exception as e:          # reported after the call returns
            err.append(e)
            return _native.PWA_ERR_INVALID

    c_cb = _native.OBJECTIVE_HESS(cb)
    res = _native.LbfgsResult()
    opt = _options(**options)
    status = _native.lib().pwa_newton_minimize(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               c_cb, None, ctypes.byref(opt), ctypes.byref(res))
    if err:
        raise err[0]
    _native.check(status)
    return x, _result(res)


def fit_fumili(model, v0, stream=None, **options):
    """Fit V on an amplitude-form model with damped Newton steps on the FUMILI
    matrix; returns (V as (W,) complex128, result dict)."""
    a = np.asarray(v0)
    if np.iscomplexobj(a):
        a = a.astype(np.complex128).view(np.float64)
    x = np.ascontiguousarray(a, dtype=np.float64).ravel().copy()
    if x.size != 2 * model.n_waves:
        raise ValueError("expected %d waves" % model.n_waves)
    res = _native.LbfgsResult()
    opt = _options(**options)
    st = stream if stream is not None else model._stream
    status = _native.lib().pwa_fit_fumili(model._handle(),
                                          x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          ctypes.byref(opt), ctypes.byref(res), st)
    _native.check(status)
    return x.view(np.complex128).copy(), _result(res)
