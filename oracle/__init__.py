"""Python access to the plain FP64 CPU oracle (``pwa_oracle.c``).

Test infrastructure only: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this module; the product library never does.  It
shares no code with the HIP path.

Every function takes numpy arrays (complex128 unless stated) and returns numpy
arrays or floats.  ``build()`` compiles ``liboracle.so`` next to this file with
gcc (plain IEEE FP64: no fast-math, no FMA contraction); ``load()`` builds it on
first use if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "pwa_oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fcx-limited-range"]

_lib = None


def build(source: str = SOURCE, output: str = LIBRARY) -> str:
    """Compile the oracle with gcc into ``output`` and return its path."""
    tmp = output + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, source, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, output)
    return output


def _bind(lib):
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    p = ctypes.c_void_p
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_mc_matrix.argtypes = [p, i64, i32, i64, p]
    lib.oracle_table_from_amplitudes.argtypes = [p, i64, i32, p]
    lib.oracle_intensity_amp.argtypes = [p, i64, i32, p, p]
    lib.oracle_intensity_table.argtypes = [p, i64, i32, p, p]
    lib.oracle_mc_term.argtypes = [p, i32, p, p]
    lib.oracle_mc_term.restype = d
    lib.oracle_nll_table.argtypes = [p, i64, i32, p, p, p, p]
    lib.oracle_nll_table.restype = i64
    lib.oracle_nll_amp.argtypes = [p, i64, i32, p, p, p, p]
    lib.oracle_nll_amp.restype = i64
    if hasattr(lib, "oracle_fumili_amp"):
        lib.oracle_fumili_amp.argtypes = [p, i64, i32, p, p]
        lib.oracle_fumili_amp.restype = i64
    return lib


def load(path: str | None = None):
    """Load (building first if needed) the oracle library.

    With ``path`` given, load that file instead of the default one; the
    result is not cached (used by the tests that plant mistakes in a copy).
    """
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build()
        _lib = _bind(ctypes.CDLL(LIBRARY))
    return _lib


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class Oracle:
    """Thin wrapper over one loaded copy of the oracle library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_num_threads(self, n: int) -> None:
        self.lib.oracle_set_num_threads(int(n))

    def mc_matrix(self, B, n_gen: int) -> np.ndarray:
        """M_aa' = (1/N_gen) sum_j B_ja conj(B_ja')   (Eq. 3, inner bracket)."""
        B = _c128(B)
        n, w = B.shape
        M = np.zeros((w, w), np.complex128)
        self.lib.oracle_mc_matrix(_ptr(B), n, w, int(n_gen), _ptr(M))
        return M

    def table(self, A) -> np.ndarray:
        """Packed per-event table T_i,aa' = A_ia conj(A_ia'), a <= a' (Sec. 2)."""
        A = _c128(A)
        n, w = A.shape
        T = np.zeros((n, w * (w + 1) // 2), np.complex128)
        self.lib.oracle_table_from_amplitudes(_ptr(A), n, w, _ptr(T))
        return T

    def table_fp32(self, A) -> np.ndarray:
        """The single-precision stored table: each FP64 entry rounded to the
        nearest complex64 component-wise (the paper keeps the table in single
        precision, Sec. 4; for complex64 amplitudes every product is exact in
        FP64, so this is one rounding of an exactly formed sum)."""
        return self.table(A).astype(np.complex64)

    def intensity_amp(self, A, V) -> np.ndarray:
        A = _c128(A)
        V = _c128(V)
        n, w = A.shape
        out = np.zeros(n, np.float64)
        self.lib.oracle_intensity_amp(_ptr(A), n, w, _ptr(V), _ptr(out))
        return out

    def intensity_table(self, T, V) -> np.ndarray:
        T = _c128(T)
        V = _c128(V)
        w = V.shape[0]
        n = T.shape[0]
        assert T.shape[1] == w * (w + 1) // 2
        out = np.zeros(n, np.float64)
        self.lib.oracle_intensity_table(_ptr(T), n, w, _ptr(V), _ptr(out))
        return out

    def mc_term(self, M, V):
        M = _c128(M)
        V = _c128(V)
        im = ctypes.c_double(0.0)
        re = self.lib.oracle_mc_term(_ptr(M), V.shape[0], _ptr(V), ctypes.byref(im))
        return re, im.value

    def _nll(self, fn, X, n, w, M, V, grad: bool):
        M = _c128(M)
        V = _c128(V)
        assert V.shape == (w,) and M.shape == (w, w)
        nll = ctypes.c_double(0.0)
        g = np.zeros(2 * w, np.float64) if grad else None
        nbad = fn(_ptr(X), n, w, _ptr(M), _ptr(V), ctypes.byref(nll),
                  _ptr(g) if grad else None)
        return nll.value, g, int(nbad)

    def nll_table(self, T, M, V, grad: bool = True):
        """(NLL, gradient [dRe V_0, dIm V_0, ...] or None, n_degenerate)."""
        T = _c128(T)
        w = _c128(V).shape[0]
        return self._nll(self.lib.oracle_nll_table, T, T.shape[0], w, M, V, grad)

    def nll_amp(self, A, M, V, grad: bool = True):
        """(NLL, gradient [dRe V_0, dIm V_0, ...] or None, n_degenerate)."""
        A = _c128(A)
        return self._nll(self.lib.oracle_nll_amp, A, A.shape[0], A.shape[1], M, V, grad)


    def fumili_amp(self, A, V):
        """(H, n_degenerate): the FUMILI matrix (2W x 2W over theta = (Re V_0,
        Im V_0, ...)): the sum over events of J_i J_i^T, J_i = grad ln I_i."""
        A = _c128(A)
        V = _c128(V)
        W = A.shape[1]
        H = np.zeros((2 * W, 2 * W), np.float64)
        nbad = self.lib.oracle_fumili_amp(_ptr(A), A.shape[0], W, _ptr(V), _ptr(H))
        return H, int(nbad)


_default = None


def get() -> Oracle:
    """The process-wide oracle instance over the default library."""
    global _default
    if _default is None:
        _default = Oracle()
    return _default
