"""The largest models: offsets beyond 32 bits (needs an MI355X).

A sample of 10^6 events replicated K times has K copies of every event, so by
Eq. 3 its data term is K times the sample's and the MC term is unchanged:
    NLL_K(V) = K (NLL_1(V) - mu(V)) + mu(V),
    G_K(V)   = K G_1(V) - (K - 1) g_mu(V),
with g_mu the gradient of mu alone.  NLL_1, G_1 and mu come from the oracle on
the sample (on the identical stored inputs of each form); g_mu from the
oracle too, as 2 G_1 - G_2 on a doubled subset (the same identity at K = 2).
The replicated models are the largest of the test suite:
  * complex64 table, 24 x 10^6 events x 20 waves: 38.4 GB stored, 4.8 x 10^9
    stored entries (beyond 2^32);
  * FP32 amplitudes, 1.1 x 10^8 events x 20 waves: 2.2 x 10^9 amplitudes
    (beyond 2^31), 17.6 GB;
  * bf16 amplitudes on the matrix cores, 1.1 x 10^8 events x 20 waves, 64
    vectors: 49 GB of operand tiles (1.05 x 10^10 16-bit forward-operand
    elements).
Tolerances: FP64 sums of N terms in different orders for the table and FP32
amplitude forms (as at full size: 1e-12 max(|NLL|, N), 1e-10 on the
gradient); for the matrix form the derived per-event bounds of
test_gpu_matrix.py on the sample, times K.
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth
from test_gpu_matrix import _bounds, _round16

pytestmark = pytest.mark.gpu

N1 = 1_000_000
W = 20


@pytest.fixture(scope="module")
def base():
    s = synth.small_sample(W, N1, 200_000, seed=24_680, n_points=2)
    d32, mc32 = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    o = oracle.get()
    M = o.mc_matrix(mc32.astype(np.complex128), 400_000)
    return s, d32, mc32, M, o


def _g_mu(o, X, M, V, nll_fn):
    """Gradient of mu alone: 2 G_1 - G_2 on the first 1000 rows of X and on
    those rows twice."""
    x = X[:1000]
    _, g1, _ = nll_fn(x, M, V)
    _, g2, _ = nll_fn(np.concatenate([x, x]), M, V)
    return 2 * g1 - g2


def _replicated(d32, k):
    import torch
    return torch.from_numpy(d32).cuda().repeat(k, 1)


def _check(model, k, V, rn, rg, mu, gmu, tol_nll, tol_g):
    nll, g = model.nll_grad(V)
    want_nll = k * (rn - mu) + mu
    want_g = k * rg - (k - 1) * gmu
    assert abs(nll - want_nll) <= tol_nll, (nll, want_nll, tol_nll)
    assert np.linalg.norm(g - want_g) <= tol_g, (np.linalg.norm(g - want_g), tol_g)


def test_table_24m_events(base):
    import torch
    s, d32, mc32, M, o = base
    k = 24
    T = o.table_fp32(d32).astype(np.complex128)      # the identical stored table
    big = _replicated(d32, k)
    model = pwa.Model(big, mc32, 400_000, form="table")
    del big
    torch.cuda.empty_cache()
    assert model.info()["n_data"] == k * N1
    for V in s.points:
        rn, rg, nbad = o.nll_table(T, M, V)
        assert nbad == 0
        mu, _ = o.mc_term(M, V)
        gmu = _g_mu(o, T, M, V, o.nll_table)
        n = k * N1
        want = k * (rn - mu) + mu
        _check(model, k, V, rn, rg, mu, gmu, 1e-12 * max(abs(want), n),
               1e-10 * np.linalg.norm(k * rg - (k - 1) * gmu))
    model.close()


def test_amplitude_110m_events(base):
    import torch
    s, d32, mc32, M, o = base
    k = 110
    A = d32.astype(np.complex128)
    big = _replicated(d32, k)
    model = pwa.Model(big, mc32, 400_000, form="amplitude")
    del big
    torch.cuda.empty_cache()
    assert model.info()["n_data"] == k * N1
    for V in s.points:
        rn, rg, nbad = o.nll_amp(A, M, V)
        assert nbad == 0
        mu, _ = o.mc_term(M, V)
        gmu = _g_mu(o, A, M, V, o.nll_amp)
        n = k * N1
        want = k * (rn - mu) + mu
        _check(model, k, V, rn, rg, mu, gmu, 1e-12 * max(abs(want), n),
               1e-10 * np.linalg.norm(k * rg - (k - 1) * gmu))
    model.close()


def test_matrix_bf16_110m_events(base):
    import torch
    s, d32, mc32, M, o = base
    k, form = 110, "amplitude_bf16"
    A = _round16(d32, form)                          # the identical stored amplitudes
    big = _replicated(d32, k)
    model = pwa.Model(big, mc32, 400_000, form=form)
    del big
    torch.cuda.empty_cache()
    assert model.info()["n_data"] == k * N1
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 110, 64])))
    Vs = synth.random_v(rng, W, 64)
    [(nll_b, g_b)] = pwa.nll_batched([model], [Vs])
    for j in (0, 31, 63):
        V = Vs[j]
        rn, rg, nbad = o.nll_amp(A, M, V)
        assert nbad == 0
        mu, _ = o.mc_term(M, V)
        gmu = _g_mu(o, A, M, V, o.nll_amp)
        b_nll, b_g = _bounds(A, V, form, rn, rg)
        want_nll = k * (rn - mu) + mu
        want_g = k * rg - (k - 1) * gmu
        assert abs(nll_b[j] - want_nll) <= k * b_nll, (j, nll_b[j], want_nll, k * b_nll)
        assert np.linalg.norm(g_b[j] - want_g) <= k * b_g, (j, np.linalg.norm(g_b[j] - want_g), k * b_g)
    model.close()
