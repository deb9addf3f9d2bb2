"""Many evaluations of several FP32 amplitude models in one call (needs an
MI355X).

pwa_nll_batched over amplitude-form models runs every (model, vector)
evaluation as one work list: one launch of the amplitude kernel per class of
storage shape and one of the assembly, replayed from a graph captured once per
set of models.  Checked against the FP64 oracle per evaluation (tolerances as
for single calls: NLL 1e-10 relative, gradient 1e-9), against single calls,
across replays with other GPU work in between, after a model of the cached plan
is freed, and through the pwa.Batch object (bitwise the same as the list form).
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth

pytestmark = pytest.mark.gpu


def _rel(g, ref):
    return float(np.linalg.norm(np.asarray(g) - ref) / np.linalg.norm(ref))


def _models(spec, seed0=0):
    out = []
    for i, (w, n) in enumerate(spec):
        s = synth.small_sample(w, n, 2 * n + 5, seed=9000 + seed0 + i, n_points=3)
        d, mc = s.data.astype(np.complex64), s.mc.astype(np.complex64)
        m = pwa.Model(d, mc, 2 * n + 5, form="amplitude")
        out.append((m, s, d, mc))
    return out


def _ref(o, d, mc, n_gen, V):
    M = o.mc_matrix(mc.astype(np.complex128), n_gen)
    return o.nll_amp(d.astype(np.complex128), M, V)


SPEC = [(8, 1000), (20, 33), (48, 4099), (13, 777), (1, 64), (33, 2500), (64, 130), (80, 300)]


def test_multi_against_oracle():
    o = oracle.get()
    ms = _models(SPEC)
    ks = [1, 2, 3, 1, 2, 1, 3, 2]
    vs = [s.points[:k] for (m, s, d, mc), k in zip(ms, ks)]
    res = pwa.nll_batched([m for m, *_ in ms], vs)
    for (m, s, d, mc), (nll, g), k in zip(ms, res, ks):
        assert nll.shape == (k,) and g.shape == (k, 2 * m.n_waves)
        for j in range(k):
            rn, rg, nbad = _ref(o, d, mc, 2 * m.n_data + 5, s.points[j])
            assert nbad == 0
            assert abs(nll[j] - rn) <= 1e-10 * max(1.0, abs(rn)), (m.n_waves, j, nll[j], rn)
            assert _rel(g[j], rg) <= 1e-9, (m.n_waves, j, _rel(g[j], rg))
    for m, *_ in ms:
        m.close()


def test_multi_replays_with_work_in_between():
    ms = _models(SPEC[:5], seed0=50)
    models = [m for m, *_ in ms]
    rng = np.random.default_rng(3)
    first = None
    for rep in range(6):
        vs = [synth.random_v(rng, m.n_waves, 2) for m in models]
        res = pwa.nll_batched(models, vs)
        # eager work on the same GPU between replays, and its own check
        for m, v in zip(models, vs):
            for j in range(2):
                nll1, g1 = m.nll_grad(v[j])
                nllb, gb = res[models.index(m)][0][j], res[models.index(m)][1][j]
                assert abs(nllb - nll1) <= 1e-10 * max(1.0, abs(nll1))
                assert _rel(gb, g1) <= 1e-9
        if rep == 0:
            first = (vs, res)
    # the same vectors again: bitwise the same results
    vs, res = first
    again = pwa.nll_batched(models, vs)
    for (a, ga), (b, gb) in zip(res, again):
        assert np.array_equal(a, b) and np.array_equal(ga, gb)
    for m in models:
        m.close()


def test_multi_plan_dropped_when_model_freed():
    ms = _models(SPEC[:3], seed0=70)
    models = [m for m, *_ in ms]
    vs = [s.points[:2] for (m, s, d, mc) in ms]
    r1 = pwa.nll_batched(models, vs)
    models[1].close()
    keep = [models[0], models[2]]
    r2 = pwa.nll_batched(keep, [vs[0], vs[2]])
    assert np.array_equal(r1[0][0], r2[0][0]) and np.array_equal(r1[2][1], r2[1][1])
    for m in keep:
        m.close()


def test_batch_object_matches_list_form():
    ms = _models(SPEC[:4], seed0=90)
    models = [m for m, *_ in ms]
    ks = [2, 1, 3, 2]
    vs = [s.points[:k] for (m, s, d, mc), k in zip(ms, ks)]
    ref = pwa.nll_batched(models, vs)
    b = pwa.Batch(models, ks)
    flat = np.concatenate([np.ascontiguousarray(v, np.complex128).view(np.float64).ravel()
                           for v in vs])
    assert flat.size == b.size
    res = b(flat)
    for (n1, g1), (n2, g2), k, m in zip(ref, res, ks, models):
        assert n2.shape == (k,) and g2.shape == (k, 2 * m.n_waves)
        assert np.array_equal(n1, n2) and np.array_equal(g1, g2)
    # the same through the parameter views, after a call with other vectors
    b(flat[::-1].copy())
    for p, v in zip(b.params, vs):
        p[...] = np.ascontiguousarray(v, np.complex128).view(np.float64).reshape(p.shape)
    res = b()
    for (n1, g1), (n2, g2) in zip(ref, res):
        assert np.array_equal(n1, n2) and np.array_equal(g1, g2)
    with pytest.raises(ValueError):
        b(flat[:-1])
    models[2].close()
    with pytest.raises(RuntimeError):
        b(flat)
    for i in (0, 1, 3):
        models[i].close()


def test_two_batches_alternating_keep_their_plans():
    """Two Batch objects on different model sets, called in turn: each call
    replays its own cached plan (no recapture: a call takes well under the
    milliseconds a plan build with its allocations and graph capture costs),
    and every call gives its first call's results bit for bit."""
    import time
    ms1 = _models(SPEC[:3], seed0=110)
    ms2 = _models(SPEC[3:6], seed0=120)
    b1 = pwa.Batch([m for m, *_ in ms1], [2, 1, 2])
    b2 = pwa.Batch([m for m, *_ in ms2], [1, 3, 1])
    rng = np.random.default_rng(7)
    v1, v2 = rng.standard_normal(b1.size), rng.standard_normal(b2.size)
    first1 = [(n.copy(), g.copy()) for n, g in b1(v1)]
    first2 = [(n.copy(), g.copy()) for n, g in b2(v2)]
    times = []
    for _ in range(10):
        for b, v, first in ((b1, v1, first1), (b2, v2, first2)):
            t = time.perf_counter()
            res = b(v)
            times.append(time.perf_counter() - t)
            for (n, g), (n0, g0) in zip(res, first):
                assert np.array_equal(n, n0) and np.array_equal(g, g0)
    assert np.median(times) < 1.5e-3, np.median(times)
    for m, *_ in ms1 + ms2:
        m.close()
