"""HIP path against the FP64 oracle on identical inputs (needs an MI355X).

Inputs are the stored arrays both sides see: complex64 amplitudes for the
single-precision forms (the oracle widens them exactly and forms the same
single-precision table), complex128 for the double-precision forms.  The
oracle and the kernels share no code; only the seeded generator feeds both.

Tolerances (FP64 arithmetic on both sides, different summation orders):
NLL relative 1e-10 at small sizes; gradient ||dG|| / ||G|| <= 1e-9.  Tables are
compared bit for bit: each entry is the same IEEE operations on the same inputs.
"""
import math
import warnings

import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth

pytestmark = pytest.mark.gpu

FORMS = ["table", "amplitude", "table_fp64_plain", "table_fp64"]
SP_FORMS = ("table", "amplitude")


def _o():
    return oracle.get()


def _inputs(form, s):
    """(data, mc) as stored for the form, and their exact complex128 widening."""
    if form in SP_FORMS:
        d, m = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    else:
        d, m = s.data, s.mc
    return d, m, d.astype(np.complex128), m.astype(np.complex128)


def _reference(form, d128, m128, n_gen, V, grad=True):
    o = _o()
    M = o.mc_matrix(m128, n_gen)
    if form == "amplitude":
        return o.nll_amp(d128, M, V, grad)
    T = o.table(d128)
    if form == "table":
        T = T.astype(np.complex64).astype(np.complex128)
    return o.nll_table(T, M, V, grad)


def _rel(g, ref):
    return float(np.linalg.norm(np.asarray(g) - ref) / np.linalg.norm(ref))


def _check(form, w, n, n_mc, seed, points=2, nll_rtol=1e-10, g_rtol=1e-9):
    s = synth.small_sample(w, n, n_mc, seed, points)
    d, m, d128, m128 = _inputs(form, s)
    model = pwa.Model(d, m, 2 * n_mc, form=form)
    for V in s.points:
        nll, g = model.nll_grad(V)
        rn, rg, nbad = _reference(form, d128, m128, 2 * n_mc, V)
        assert nbad == 0
        assert abs(nll - rn) <= nll_rtol * max(1.0, abs(rn)), (form, w, n, nll, rn)
        assert _rel(g, rg) <= g_rtol, (form, w, n, _rel(g, rg))
        assert abs(model.nll(V) - nll) <= 1e-14 * max(1.0, abs(nll))
    model.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("w,n", [(1, 1), (1, 33), (2, 17), (3, 100), (4, 1000), (7, 4099),
                                 (11, 777), (20, 2049), (23, 300), (32, 1500), (36, 400),
                                 (44, 300), (48, 513), (56, 200), (64, 130)])
def test_parity_small(form, w, n):
    _check(form, w, n, 3 * n + 7, seed=100 * w + n)


@pytest.mark.parametrize("w", [33, 80, 128])
def test_parity_amplitude_wide(w):
    _check("amplitude", w, 700, 900, seed=w)


@pytest.mark.parametrize("form", ["table", "table_fp64_plain", "table_fp64"])
@pytest.mark.parametrize("w,n", [(1, 5), (4, 31), (20, 1001), (33, 65), (64, 17)])
def test_table_bit_exact(form, w, n):
    s = synth.small_sample(w, n, 4, seed=7 * w + n)
    d, _, d128, _ = _inputs(form, s)
    model = pwa.Model(d, None, 1, form=form)
    ref = _o().table(d128)
    if form == "table":
        ref = ref.astype(np.complex64)
    got = model.table()
    assert got.dtype == ref.dtype and np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("form", ["table", "table_fp64_plain", "table_fp64"])
@pytest.mark.parametrize("w,n", [(1, 3), (2, 17), (5, 40), (20, 33)])
def test_table_input_round_trip(form, w, n):
    """A canonical packed table given as input (PWA_INPUT_IS_TABLE) comes back
    bit for bit: the tiled forms keep its diagonal as real pairs (odd and even
    W), the plain form as it is."""
    o = _o()
    parts = [synth.small_sample(w, n, 4, seed=40 + k).data for k in (1, 2)]
    T = o.table(parts[0]) + o.table(parts[1])
    stored = T.astype(np.complex64) if form == "table" else T
    model = pwa.Model(stored, None, 1, form=form, input_is_table=True)
    got = model.table()
    assert got.dtype == stored.dtype
    assert np.array_equal(got.view(np.uint8), stored.view(np.uint8))
    model.close()


@pytest.mark.parametrize("form", ["table", "table_fp64_plain", "table_fp64"])
def test_non_hermitian_table_rejected(form):
    """A table whose diagonal has a non-zero imaginary part is not Hermitian
    and is refused (PWA_ERR_INVALID) before anything is stored."""
    o = _o()
    T = o.table(synth.small_sample(4, 50, 4, seed=44).data)
    T[17, 4] += 1e-3j                    # entry (1, 1): packed index 4 at W = 4
    stored = T.astype(np.complex64) if form == "table" else T
    with pytest.raises(pwa.PWAError) as e:
        pwa.Model(stored, None, 1, form=form, input_is_table=True)
    assert e.value.status == -1 and "Hermitian" in str(e.value)


@pytest.mark.parametrize("form", ["table", "amplitude", "amplitude_bf16"])
def test_oversized_model_refused_before_allocation(form):
    """A model whose build cannot fit in device memory (2^36 events: about
    110 TB as a 20-wave complex64 table) is refused with PWA_ERR_OOM by the
    pre-flight, before anything is allocated or the input is read (the buffer
    passed is far smaller than N x W; the check never touches it), and the
    library stays usable."""
    import ctypes
    from paper_1108_5673_amd import _native
    L = _native.lib()
    small = np.ones((4, 20), np.complex64)
    h = ctypes.c_void_p()
    st = L.pwa_build_table(small.ctypes.data, 1 << 36, 20, None, 0, 1, pwa.FORMS[form], None,
                           ctypes.byref(h))
    assert st == _native.PWA_ERR_OOM and h.value is None
    assert "device memory" in _native.last_error()
    _check(form if form != "amplitude_bf16" else "amplitude", 20, 1000, 500, seed=45)


@pytest.mark.parametrize("form", FORMS)
def test_mc_matrix(form):
    s = synth.small_sample(9, 10, 20_000, seed=3)
    _, m, _, m128 = _inputs(form, s)
    model = pwa.Model(s.data.astype(np.complex64 if form in SP_FORMS else np.complex128), m,
                      50_000, form=form)
    ref = _o().mc_matrix(m128, 50_000)
    got = model.mc_matrix()
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    assert np.array_equal(got, got.conj().T)


@pytest.mark.parametrize("c128", [False, True])
@pytest.mark.parametrize("w,n_acc", [(1, 1), (5, 63), (8, 1_001), (16, 4_097), (20, 64),
                                     (20, 65), (20, 40_017), (32, 20_011), (33, 777),
                                     (40, 3_001), (48, 10_007), (56, 999), (64, 9_999),
                                     (65, 33), (65, 5_000), (72, 70_001), (80, 31),
                                     (88, 4_095), (96, 300_007), (100, 1_025), (112, 12_345),
                                     (120, 777), (121, 20_000), (128, 2_049), (128, 65_537)])
def test_mc_matrix_sizes(c128, w, n_acc):
    """M over ragged tails, on the FP64 matrix cores in tiles of 16 of the 2W
    real components: 1 to 4 tiles with every tile pair in one wavefront
    (several blocks and steps per wavefront); 5 to 8 with the pairs split over
    the block's 4 wavefronts at compile time and the events staged through LDS
    (ragged chunks); 9 to 16 tiles (W 65..128) over 16 wavefronts with the
    pairs indexed at run time (every tile count, a single event chunk, many
    chunks per block, partly filled last tiles)."""
    s = synth.small_sample(w, 10, n_acc, seed=500 + w + n_acc)
    m = s.mc if c128 else s.mc.astype(np.complex64)
    model = pwa.Model(s.data.astype(np.complex64), m, 2 * n_acc + 1, form="amplitude")
    ref = _o().mc_matrix(m.astype(np.complex128), 2 * n_acc + 1)
    got = model.mc_matrix()
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref), (w, n_acc)
    assert np.array_equal(got, got.conj().T)
    model.close()


def test_no_mc_gives_zero_matrix():
    s = synth.small_sample(3, 50, 4, seed=4)
    model = pwa.Model(s.data.astype(np.complex64), None, 1, form="table")
    assert np.all(model.mc_matrix() == 0)
    V = s.points[0]
    rn, _, _ = _o().nll_table(_o().table_fp32(s.data.astype(np.complex64)).astype(np.complex128),
                              np.zeros((3, 3)), V)
    assert abs(model.nll(V) - rn) <= 1e-12 * abs(rn)


@pytest.mark.parametrize("form", FORMS)
def test_degenerate_event(form):
    s = synth.small_sample(3, 40, 60, seed=5)
    V = np.array([1.0 + 0.5j, -0.25 + 1j, 0.5 - 0.5j])
    A = s.data.copy()
    A[13] = [V[1], -V[0], 0.0]           # sum_a V_a A_a = 0 exactly (dyadic values)
    d = A.astype(np.complex64) if form in SP_FORMS else A
    model = pwa.Model(d, s.mc.astype(d.dtype), 100, form=form)
    with warnings.catch_warnings(record=True):
        warnings.simplefilter("always")
        nll, g = model.nll_grad(V)
    assert nll == math.inf and np.all(np.isnan(g))
    # the next call at a regular point is unaffected
    nll2, g2 = model.nll_grad(s.points[0])
    assert math.isfinite(nll2) and np.all(np.isfinite(g2))


@pytest.mark.parametrize("form", FORMS)
def test_bitwise_repeatable(form):
    s = synth.small_sample(20, 20_000, 1000, seed=6)
    d, m, _, _ = _inputs(form, s)
    model = pwa.Model(d, m, 2000, form=form)
    first = model.nll_grad(s.points[1])
    for _ in range(5):
        again = model.nll_grad(s.points[1])
        assert again[0] == first[0] and np.array_equal(again[1], first[1])


def test_general_psd_table_input():
    """PWA_INPUT_IS_TABLE: a rank-3 Hermitian PSD table, not A A^H."""
    o = _o()
    parts = [synth.small_sample(6, 700, 10, seed=k).data.astype(np.complex64) for k in (1, 2, 3)]
    T = sum(o.table(p.astype(np.complex128)) for p in parts)
    mc = synth.small_sample(6, 10, 900, seed=9).mc.astype(np.complex64)
    M = o.mc_matrix(mc.astype(np.complex128), 1800)
    for form, stored in (("table", T.astype(np.complex64)), ("table_fp64", T),
                         ("table_fp64_plain", T)):
        model = pwa.Model(stored, mc, 1800, form=form, input_is_table=True)
        assert model.n_waves == 6
        ref_T = stored.astype(np.complex128)
        for V in synth.small_sample(6, 1, 1, seed=11, n_points=3).points:
            nll, g = model.nll_grad(V)
            rn, rg, _ = o.nll_table(ref_T, M, V)
            assert abs(nll - rn) <= 1e-10 * abs(rn)
            assert _rel(g, rg) <= 1e-9


def test_set_mc_matrix():
    s = synth.small_sample(5, 300, 10, seed=12)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    M = X @ X.conj().T
    model = pwa.Model(s.data.astype(np.complex64), None, 1, form="amplitude")
    model.set_mc_matrix(M)
    assert np.array_equal(model.mc_matrix(), M)
    V = s.points[0]
    rn, rg, _ = _o().nll_amp(s.data.astype(np.complex64).astype(np.complex128), M, V)
    nll, g = model.nll_grad(V)
    assert abs(nll - rn) <= 1e-11 * abs(rn) and _rel(g, rg) <= 1e-10


def test_device_tensor_inputs_match_host_inputs():
    import torch
    s = synth.small_sample(8, 5000, 3000, seed=13)
    d, m = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    host = pwa.Model(d, m, 6000, form="table")
    dev = pwa.Model(torch.from_numpy(d).cuda(), torch.from_numpy(m).cuda(), 6000, form="table")
    for V in s.points:
        a, b = host.nll_grad(V), dev.nll_grad(V)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_batched_matches_single_calls():
    s1 = synth.small_sample(6, 3000, 2000, seed=14, n_points=3)
    s2 = synth.small_sample(11, 2000, 1000, seed=15, n_points=2)
    m1 = pwa.Model(s1.data.astype(np.complex64), s1.mc.astype(np.complex64), 4000, form="table")
    m2 = pwa.Model(s2.data.astype(np.complex64), s2.mc.astype(np.complex64), 2000,
                   form="amplitude")
    out = pwa.nll_batched([m1, m2], [s1.points, s2.points])
    for (nll, g), m, s in zip(out, (m1, m2), (s1, s2)):
        for k, V in enumerate(s.points):
            rn, rg = m.nll_grad(V)
            assert nll[k] == rn and np.array_equal(g[k], rg)
    out = pwa.nll_batched([m1], [s1.points], grad=False)
    assert np.array_equal(out[0][0], np.array([m1.nll(V) for V in s1.points]))


def test_autograd_function():
    import torch
    from paper_1108_5673_amd.autograd import NLLFunction
    s = synth.small_sample(4, 2000, 1000, seed=16)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 2000)
    V = s.points[0]
    v = torch.tensor(np.stack([V.real, V.imag], -1).ravel(), dtype=torch.float64,
                     requires_grad=True)
    loss = 3.0 * NLLFunction.apply(v, model)
    loss.backward()
    nll, g = model.nll_grad(V)
    assert abs(loss.item() - 3.0 * nll) <= 1e-12 * abs(nll)
    assert np.allclose(v.grad.numpy(), 3.0 * g, rtol=1e-14, atol=0)
    # real parametrisation: d|z|^2 / d(Re z, Im z) at z = 1 + 1j is (2, 2)
    z = torch.tensor([1.0, 1.0], dtype=torch.float64, requires_grad=True)
    (z[0] ** 2 + z[1] ** 2).backward()
    assert z.grad.tolist() == [2.0, 2.0]


def test_timing_counters():
    s = synth.small_sample(20, 50_000, 100, seed=17)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 200)
    model.set_timing(True)
    for V in s.points:
        model.nll_grad(V)
    ms, n = model.timing()
    assert n == len(s.points) and ms > 0
    model.set_timing(False)
    model.nll_grad(s.points[0])
    assert model.timing() == (0.0, 0)
    # every 4th evaluation: the 1st, 5th, 9th of 10; more launches than the
    # event ring holds are read back as the ring is reused
    model.set_timing(True, every=4)
    for k in range(10):
        model.nll_grad(s.points[k % len(s.points)])
    ms, n = model.timing()
    assert n == 3 and ms > 0
    model.set_timing(True)
    for k in range(150):
        model.nll_grad(s.points[k % len(s.points)])
    ms, n = model.timing()
    assert n == 150 and ms > 0
    model.set_timing(False)


def test_nonfinite_v_rejected():
    s = synth.small_sample(3, 10, 10, seed=18)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 20)
    with pytest.raises(pwa.PWAError) as e:
        model.nll(np.array([1.0, np.nan, 0, 0, 0, 0]))
    assert e.value.status == -5


def test_build_timing():
    s = synth.small_sample(8, 5000, 20000, seed=3)
    m = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 20000, form="table")
    t = m.build_timing()
    assert t["table_ms"] > 0.0 and t["mc_ms"] > 0.0
    m.close()
    m = pwa.Model(s.data.astype(np.complex64), None, 1, form="amplitude")
    t = m.build_timing()
    assert t["table_ms"] > 0.0 and t["mc_ms"] == 0.0
    m.close()


def test_read_ceiling():
    """The reference read of the stored data reports the stored bytes and a
    positive, physically possible bandwidth (below 8 TB/s of HBM3E plus the
    caches' help on a small table)."""
    s = synth.small_sample(20, 200_000, 100, seed=19)
    model = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), 200)
    r = model.read_ceiling(reps=3)
    # 200 stored entries per event at W = 20: 10 diagonal pairs + 190 off-diagonal
    assert r["bytes"] == 200_000 * 200 * 8 and r["ms"] > 0 and 0 < r["gbs"] < 50_000
    model.close()


@pytest.mark.parametrize("form,e", [("table", 8), ("table_fp64", 4)])
def test_table_subtile_override(form, e, monkeypatch):
    """The sub-tile widths kept for tuning (PWA_TABLE_SUBTILE, read when a
    model is built): 8 events per sub-tile for the complex64 table at W = 20,
    4 for the complex128 one, against the oracle with a ragged last tile."""
    monkeypatch.setenv("PWA_TABLE_SUBTILE", str(e))
    _check(form, 20, 2049, 3 * 2049 + 7, seed=2017)


def test_table_subtile_override_falls_back(monkeypatch):
    """A width with no kernel instance is ignored: the model keeps its default
    shape and gives the default model's results bit for bit."""
    s = synth.small_sample(20, 1500, 2000, seed=2018, n_points=1)
    d, m = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    ref = pwa.Model(d, m, 4000, form="table")
    monkeypatch.setenv("PWA_TABLE_SUBTILE", "3")
    odd = pwa.Model(d, m, 4000, form="table")
    (n0, g0), (n1, g1) = ref.nll_grad(s.points[0]), odd.nll_grad(s.points[0])
    assert n0 == n1 and np.array_equal(g0, g1)
    assert odd.info()["grid_blocks"] == ref.info()["grid_blocks"]
    ref.close()
    odd.close()
