"""pwa_nll_batched_noalloc: the matrix-core K-vector evaluation with all of
its buffers in the library's static device array (needs an MI355X).

Checked through the C ABI against the existing entry point pwa_nll_batched on
the same model and vectors, on two calls in a row, the second with a smaller
input (fewer vectors on a smaller model), so that the second call runs over
the array the first one left behind:
  * when the records of pwa_nll_batched's event chunks fit in the array, both
    run the same kernels over the same chunks: bit for bit equal;
  * when they do not (many vectors at a wide W), the events are cut into fewer,
    longer chunks, whose FP32 records each add more tiles: both results are
    held to the derived bounds against the oracle on the identical 16-bit
    amplitudes (tests/test_gpu_matrix.py), and to each other within the sum of
    those bounds.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import _native, synth
from test_gpu_matrix import _bounds, _round16

pytestmark = pytest.mark.gpu


def _noalloc(model, V):
    """One pwa_nll_batched_noalloc call: V (k, W) complex -> (nll (k,), grad (k, 2W))."""
    import torch
    k, w = V.shape
    v = torch.from_numpy(np.ascontiguousarray(V.astype(np.complex128)).view(np.float64)
                         .reshape(k, 2 * w)).cuda()
    out = torch.full((k, 2 + 2 * w), np.nan, dtype=torch.float64, device="cuda")
    st = _native.lib().pwa_nll_batched_noalloc(model._handle(), k, ctypes.c_void_p(v.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _native.PWA_OK, _native.last_error()
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.all(o[:, 1] == 0.0)
    return o[:, 0], o[:, 2:]


def _sample(w, n, k, seed):
    s = synth.small_sample(w, n, 2 * n, seed, n_points=k)
    return s, s.data.astype(np.complex64), s.mc.astype(np.complex64)


@pytest.mark.parametrize("form", ["amplitude_bf16", "amplitude_fp16"])
def test_noalloc_equals_batched_bitwise(form):
    # first call: 96 vectors on 20 waves; second: 17 vectors on 7 waves
    for w, n, k, seed in ((20, 30_011, 96, 1), (7, 5_003, 17, 2)):
        s, d, mc = _sample(w, n, k, seed)
        model = pwa.Model(d, mc, 4 * n, form=form)
        V = np.asarray(s.points)
        nll_a, g_a = _noalloc(model, V)
        [(nll_b, g_b)] = pwa.nll_batched([model], [s.points])
        assert np.array_equal(nll_a, nll_b) and np.array_equal(g_a, g_b), (form, w, k)
        model.close()


@pytest.mark.parametrize("form", ["amplitude_bf16", "amplitude_fp16"])
def test_noalloc_fewer_chunks_within_bounds(form):
    # 1024 vectors at 64 waves: the records of pwa_nll_batched's chunks do not
    # fit, the variant runs fewer chunks; then a smaller call on the same array
    o = oracle.get()
    for w, n, k, seed in ((64, 20_000, 1024, 3), (33, 4_000, 40, 4)):
        s, d, mc = _sample(w, n, k, seed)
        model = pwa.Model(d, mc, 4 * n, form=form)
        V = np.asarray(s.points)
        nll_a, g_a = _noalloc(model, V)
        [(nll_b, g_b)] = pwa.nll_batched([model], [s.points])
        A = _round16(d, form)
        M = o.mc_matrix(mc.astype(np.complex128), 4 * n)
        for j in (0, k // 3, k - 1):
            rn, rg, nbad = o.nll_amp(A, M, s.points[j])
            assert nbad == 0
            bn, bg = _bounds(A, s.points[j], form, rn, rg)
            assert abs(nll_a[j] - rn) <= bn and np.linalg.norm(g_a[j] - rg) <= bg, (form, w, j)
            assert abs(nll_b[j] - rn) <= bn and np.linalg.norm(g_b[j] - rg) <= bg, (form, w, j)
            assert abs(nll_a[j] - nll_b[j]) <= 2 * bn
            assert np.linalg.norm(g_a[j] - g_b[j]) <= 2 * bg
        model.close()


def test_noalloc_rejects_what_does_not_fit():
    import torch
    s, d, mc = _sample(8, 100, 2, 5)
    L = _native.lib()
    v = torch.zeros(2048 * 16, dtype=torch.float64, device="cuda")
    out = torch.zeros(2048 * 18, dtype=torch.float64, device="cuda")
    table = pwa.Model(d, mc, 200, form="table")
    # another form, k out of range: refused before anything is enqueued
    assert L.pwa_nll_batched_noalloc(table._handle(), 2, ctypes.c_void_p(v.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), None) == _native.PWA_ERR_INVALID
    model = pwa.Model(d, mc, 200, form="amplitude_bf16")
    for k in (0, 1025):
        assert L.pwa_nll_batched_noalloc(model._handle(), k, ctypes.c_void_p(v.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), None) == \
            _native.PWA_ERR_INVALID
    assert "k must be" in _native.last_error()
    table.close()
    model.close()
