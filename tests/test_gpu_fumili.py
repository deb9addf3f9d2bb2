"""The FUMILI second-derivative matrix of the amplitude form (needs an MI355X).

Against the oracle's plain definition (FP64 both sides, different summation
orders: ||dH||_F / ||H||_F <= 1e-10) at sizes spanning several tiles and a
ragged last tile, both kernels (up to 4 blocks of 16 parameters, W <= 32: all
block pairs in each wavefront; wider: J staged in LDS once per event and the
block pairs split over 16 wavefronts, from 5 to 16 blocks, one and several
tiles per block), degenerate events, and at 2x10^6 events x 32 waves through
the identities that hold at any size: theta^T H theta = 4 N and H (i V) = 0.
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth

pytestmark = pytest.mark.gpu


def _frob(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("w,n", [(1, 1), (2, 70), (4, 1000), (7, 4099), (20, 5000), (33, 700),
                                 (48, 2000), (64, 300), (72, 70_001), (77, 500), (100, 700),
                                 (113, 9_999), (128, 300), (128, 20_033)])
def test_fumili_matches_oracle(w, n):
    o = oracle.get()
    s = synth.small_sample(w, n, 3 * n + 7, seed=4000 + 10 * w + n, n_points=2)
    d, mc = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d, mc, 3 * n + 7, form="amplitude")
    for V in s.points:
        nll, g, H = model.nll_grad_hess(V)
        Href, nbad = o.fumili_amp(d.astype(np.complex128), V)
        assert nbad == 0
        assert H.shape == (2 * w, 2 * w)
        assert _frob(H, Href) <= 1e-10, (w, n, _frob(H, Href))
        nll2, g2 = model.nll_grad(V)
        assert nll == nll2 and np.array_equal(g, g2)
    model.close()


def test_fumili_degenerate():
    s = synth.small_sample(5, 400, 500, seed=31, n_points=1)
    d = s.data.astype(np.complex64)
    d[17] = 0.0
    model = pwa.Model(d, s.mc.astype(np.complex64), 500, form="amplitude")
    with pytest.warns(UserWarning):
        nll, g, H = model.nll_grad_hess(s.points[0])
    assert np.isinf(nll) and np.all(np.isnan(g)) and np.all(np.isnan(H))
    model.close()


def test_fumili_wrong_form_rejected():
    s = synth.small_sample(3, 100, 100, seed=32, n_points=1)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 100, form="table")
    with pytest.raises(pwa.PWAError):
        model.nll_grad_hess(s.points[0])
    model.close()


def test_fumili_full_size_identities():
    s = synth.make_sample("w32_n2m", n_points=3)
    d, mc = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    model = pwa.Model(d, mc, s.n_gen, form="amplitude")
    n = d.shape[0]
    for V in s.points:
        nll, g, H = model.nll_grad_hess(V)
        th = np.ascontiguousarray(V.astype(np.complex128)).view(np.float64)
        assert abs(th @ H @ th - 4 * n) <= 1e-9 * 4 * n
        phi = np.ascontiguousarray((1j * V).astype(np.complex128)).view(np.float64)
        assert np.linalg.norm(H @ phi) <= 1e-9 * np.linalg.norm(H) * np.linalg.norm(phi)
    model.close()
