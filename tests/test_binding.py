"""Host-side layout of the Python binding's Batch object (no GPU needed: the
models are stand-ins that only carry a wave count and a handle)."""
import numpy as np
import pytest

import paper_1108_5673_amd as pwa


class _Stub:
    def __init__(self, w):
        self.n_waves = w
        self._stream = None

    def _handle(self):
        return 1


def test_batch_layout():
    models = [_Stub(3), _Stub(1), _Stub(5)]
    b = pwa.Batch(models, ks=[2, 0, 3])
    assert b.size == 2 * 6 + 0 + 3 * 10
    assert [p.shape for p in b.params] == [(2, 6), (0, 2), (3, 10)]
    assert [r[0].shape for r in b.results] == [(2,), (0,), (3,)]
    assert [r[1].shape for r in b.results] == [(2, 6), (0, 2), (3, 10)]
    # the views tile one flat array in model order
    for i, p in enumerate(b.params):
        p[...] = i + 1
    assert np.array_equal(b._v[:b.size], np.repeat([1.0, 3.0], [12, 30]))


def test_batch_default_counts_and_no_grad():
    b = pwa.Batch([_Stub(2), _Stub(4)], grad=False)
    assert b.ks == [1, 1] and b.size == 4 + 8
    assert all(g is None for _, g in b.results)


def test_batch_rejects_bad_counts():
    with pytest.raises(ValueError):
        pwa.Batch([_Stub(2), _Stub(4)], ks=[1])
    with pytest.raises(ValueError):
        pwa.Batch([_Stub(2)], ks=[-1])
