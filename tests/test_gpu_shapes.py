"""Storage shapes of the FP32 amplitude form (needs an MI355X).

The amplitudes of an event are spread over 1-16 lanes with 2-16 waves each
(include/pwa.h, pwa_set_amplitude_shape).  Every shape must hold the same
amplitudes (read back bit for bit), give the NLL, gradient and FUMILI matrix of
the FP64 oracle on those amplitudes (NLL 1e-10 relative, gradient 1e-9,
matrix 1e-10: FP64 sums in different orders), repeat bit for bit when a shape
is set again, and keep a cached multi-model plan consistent.
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth
from paper_1108_5673_amd._native import PWAError

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def _shapes(W):
    out = []
    for q in (1, 2, 4, 8, 16):
        for wl in range(2, 17, 2):
            if q * wl >= W and q * wl <= 2 * W + 32:
                out.append((q, wl))
    return out


@pytest.mark.parametrize("w,n", [(3, 1000), (13, 3001), (20, 4099), (32, 2500), (48, 1500),
                                 (100, 700)])
def test_every_shape_matches_oracle(w, n):
    o = oracle.get()
    s = synth.small_sample(w, n, 2 * n + 3, seed=7000 + w, n_points=1)
    d, mc = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d, mc, 2 * n + 3, form="amplitude")
    V = s.points[0]
    M = o.mc_matrix(mc.astype(np.complex128), 2 * n + 3)
    rn, rg, nbad = o.nll_amp(d.astype(np.complex128), M, V)
    assert nbad == 0
    Href, _ = o.fumili_amp(d.astype(np.complex128), V)
    first = model.amplitude_shape()
    n0, g0 = model.nll_grad(V)
    for q, wl in _shapes(w):
        print("shape", w, n, q, wl, flush=True)
        model.set_amplitude_shape(q, wl)
        assert model.amplitude_shape() == (q, wl)
        assert np.array_equal(model.table(), d)
        nll, g = model.nll_grad(V)
        assert abs(nll - rn) <= 1e-10 * max(1.0, abs(rn)), (q, wl, nll, rn)
        assert _rel(g, rg) <= 1e-9, (q, wl, _rel(g, rg))
        _, _, H = model.nll_grad_hess(V)
        assert _rel(H, Href) <= 1e-10, (q, wl)
    model.set_amplitude_shape(*first)
    n1, g1 = model.nll_grad(V)
    assert n1 == n0 and np.array_equal(g1, g0)
    model.close()


def test_invalid_shapes_rejected():
    s = synth.small_sample(20, 500, 1000, seed=71, n_points=1)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 1000,
                      form="amplitude")
    before = model.amplitude_shape()
    for q, wl in [(3, 8), (2, 5), (1, 18), (2, 8), (32, 2), (0, 20)]:
        with pytest.raises(PWAError):
            model.set_amplitude_shape(q, wl)
    assert model.amplitude_shape() == before
    model.close()
    t = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 1000, form="table")
    with pytest.raises(PWAError):
        t.amplitude_shape()
    t.close()


def test_tune_keeps_results():
    o = oracle.get()
    s = synth.small_sample(32, 20000, 30000, seed=72, n_points=1)
    d, mc = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d, mc, 30000, form="amplitude")
    q, wl = model.tune_amplitude_shape(evals=3)
    assert (q, wl) == model.amplitude_shape() and q * wl >= 32
    assert np.array_equal(model.table(), d)
    M = o.mc_matrix(mc.astype(np.complex128), 30000)
    rn, rg, _ = o.nll_amp(d.astype(np.complex128), M, s.points[0])
    nll, g = model.nll_grad(s.points[0])
    assert abs(nll - rn) <= 1e-10 * abs(rn) and _rel(g, rg) <= 1e-9
    model.close()


def test_multi_plan_follows_shape_change():
    ms = []
    for i, (w, n) in enumerate([(20, 3000), (13, 2000), (40, 1000)]):
        s = synth.small_sample(w, n, 2 * n, seed=80 + i, n_points=2)
        ms.append((pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 2 * n,
                             form="amplitude"), s))
    models = [m for m, _ in ms]
    vs = [s.points for _, s in ms]
    r1 = pwa.nll_batched(models, vs)
    models[0].set_amplitude_shape(4, 6)          # 24 waves per row instead of 20
    r2 = pwa.nll_batched(models, vs)
    for (m, s), (a, ga), (b, gb) in zip(ms, r1, r2):
        for j in range(2):
            n1, g1 = m.nll_grad(s.points[j])
            assert abs(b[j] - n1) <= 1e-10 * abs(n1) and _rel(gb[j], g1) <= 1e-9
            assert abs(a[j] - b[j]) <= 1e-10 * abs(a[j]) and _rel(ga[j], gb[j]) <= 1e-9
    for m in models:
        m.close()
