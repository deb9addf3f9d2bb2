"""Parity on the named workloads at their full sizes (needs an MI355X).

Workloads (seeded, synthetic J/psi -> gamma K+K- shaped samples):
  w4_n10k   10k events, 4 waves, 10 random points: every form against the
            oracle, 1e-9 relative.
  w20_n1m   10^6 events, 20 waves, the complex64 table form in the launch
            configuration the benchmark times, at 8 of the 200 walk points:
            (a) against the oracle on the identical stored table, which isolates
            the kernels' arithmetic, and (b) against the oracle on the complex128
            amplitudes, which adds the single-precision storage: |dNLL| <= 1e-3
            and ||dG|| / ||G|| <= 1e-5.  The complex128 forms against the oracle
            on the complex128 table.
  w32_n2m   2x10^6 events, 32 waves, amplitude form, 20 random points: NLL and
            gradient against the oracle, and the gradient against Richardson-
            extrapolated central differences of the kernels' own NLL.
  w20_n1m_k256  256 random points on the 10^6-event table, one batched call:
            every entry equal to the single call at the same point, a sample
            against the oracle.
"""
import numpy as np
import pytest

import oracle
import paper_1108_5673_amd as pwa
from paper_1108_5673_amd import synth

pytestmark = pytest.mark.gpu

WALK_SAMPLE = [0, 1, 37, 99, 100, 150, 198, 199]


def _rel(g, ref):
    return float(np.linalg.norm(np.asarray(g) - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def o():
    return oracle.get()


@pytest.fixture(scope="module")
def w20():
    s = synth.make_sample("w20_n1m")
    d32 = s.data.astype(np.complex64)
    mc32 = s.mc.astype(np.complex64)
    return s, d32, mc32


def test_w4_n10k_all_forms(o):
    s = synth.make_sample("w4_n10k")
    assert s.data.shape == (10_000, 4) and s.mc.shape == (50_000, 4) and s.n_gen == 100_000
    for form in ["table_fp64_plain", "table_fp64", "table", "amplitude"]:
        sp = form in ("table", "amplitude")
        d = s.data.astype(np.complex64) if sp else s.data
        m = s.mc.astype(np.complex64) if sp else s.mc
        d128, m128 = d.astype(np.complex128), m.astype(np.complex128)
        M = o.mc_matrix(m128, s.n_gen)
        if form == "amplitude":
            ref = [o.nll_amp(d128, M, V) for V in s.points]
        else:
            T = o.table(d128)
            if form == "table":
                T = T.astype(np.complex64).astype(np.complex128)
            ref = [o.nll_table(T, M, V) for V in s.points]
        model = pwa.Model(d, m, s.n_gen, form=form)
        for V, (rn, rg, nbad) in zip(s.points, ref):
            nll, g = model.nll_grad(V)
            assert nbad == 0
            assert abs(nll - rn) <= 1e-9 * abs(rn), (form, nll, rn)
            assert _rel(g, rg) <= 1e-9, (form, _rel(g, rg))
        model.close()


def test_w20_n1m_table_complex64(o, w20):
    s, d32, mc32 = w20
    model = pwa.Model(d32, mc32, s.n_gen, form="table")
    info = model.info()
    assert info["n_data"] == 1_000_000 and info["n_waves"] == 20 and info["n_packed"] == 210
    # 200 stored entries: 10 pairs of the real diagonal + 190 off-diagonal
    assert info["stream_bytes"] == 1_000_000 * 200 * 8
    got = {k: model.nll_grad(s.points[k]) for k in WALK_SAMPLE}
    model.close()
    # (a) the identical stored table
    T = o.table(d32.astype(np.complex128)).astype(np.complex64).astype(np.complex128)
    M32 = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
    for k in WALK_SAMPLE:
        rn, rg, nbad = o.nll_table(T, M32, s.points[k])
        nll, g = got[k]
        assert nbad == 0
        assert abs(nll - rn) <= 1e-12 * max(abs(rn), 1e6), (k, nll, rn)
        assert _rel(g, rg) <= 1e-10, (k, _rel(g, rg))
    del T
    # (b) the FP64 oracle on the complex128 amplitudes
    M = o.mc_matrix(s.mc, s.n_gen)
    for k in WALK_SAMPLE:
        rn, rg, nbad = o.nll_amp(s.data, M, s.points[k])
        nll, g = got[k]
        assert abs(nll - rn) <= 1e-3, (k, nll, rn)
        assert _rel(g, rg) <= 1e-5, (k, _rel(g, rg))


@pytest.mark.parametrize("form", ["table_fp64_plain", "table_fp64"])
def test_w20_n1m_table_complex128(o, w20, form):
    s, _, _ = w20
    model = pwa.Model(s.data, s.mc, s.n_gen, form=form)
    pts = [0, 199]
    got = {k: model.nll_grad(s.points[k]) for k in pts}
    model.close()
    T = o.table(s.data)
    M = o.mc_matrix(s.mc, s.n_gen)
    for k in pts:
        rn, rg, _ = o.nll_table(T, M, s.points[k])
        nll, g = got[k]
        assert abs(nll - rn) <= 1e-12 * max(abs(rn), 1e6), (form, k, nll, rn)
        assert _rel(g, rg) <= 1e-10, (form, k, _rel(g, rg))


def test_w20_n1m_256_points_table_batched_call(o):
    """The 256 starting points of w20_n1m_k256 on the complex64 table through
    one pwa_nll_batched call (one table pass per point): equal to single calls
    bit for bit, and a sample against the oracle on the identical table."""
    k = synth.make_sample("w20_n1m_k256")
    assert k.points.shape == (256, 20) and k.data.shape == (1_000_000, 20)
    d, mc = k.data.astype(np.complex64), k.mc.astype(np.complex64)
    model = pwa.Model(d, mc, k.n_gen, form="table")
    [(nll_b, g_b)] = pwa.nll_batched([model], [k.points])
    assert nll_b.shape == (256,) and g_b.shape == (256, 40)
    for j in range(0, 256, 17):
        nll, g = model.nll_grad(k.points[j])
        assert nll == nll_b[j] and np.array_equal(g, g_b[j], equal_nan=True), j
    model.close()
    T = o.table(d.astype(np.complex128)).astype(np.complex64).astype(np.complex128)
    M = o.mc_matrix(mc.astype(np.complex128), k.n_gen)
    for j in [0, 85, 170, 255]:
        rn, rg, nbad = o.nll_table(T, M, k.points[j])
        if nbad:
            assert np.isinf(nll_b[j])
            continue
        assert abs(nll_b[j] - rn) <= 1e-12 * max(abs(rn), 1e6), (j, nll_b[j], rn)
        assert _rel(g_b[j], rg) <= 1e-10, (j, _rel(g_b[j], rg))


@pytest.mark.parametrize("form", ["amplitude_bf16", "amplitude_fp16"])
def test_w20_n1m_k256_matrix_cores(o, form):
    """The batched-starting-points workload at full size on the matrix cores:
    1M events, 20 waves, 256 vectors in one pass (8 column blocks, 256 event
    chunks of about 245 tiles each), vectors 0, 85, 170 and 255 against the
    oracle on the identical 16-bit amplitudes within the derived bounds of
    tests/test_gpu_matrix.py."""
    from test_gpu_matrix import _bounds, _round16
    k = synth.make_sample("w20_n1m_k256")
    d, mc = k.data.astype(np.complex64), k.mc.astype(np.complex64)
    model = pwa.Model(d, mc, k.n_gen, form=form)
    [(nll_b, g_b)] = pwa.nll_batched([model], [k.points])
    model.close()
    A = _round16(d, form)
    M = o.mc_matrix(mc.astype(np.complex128), k.n_gen)
    for j in (0, 85, 170, 255):
        rn, rg, nbad = o.nll_amp(A, M, k.points[j])
        assert nbad == 0
        b_nll, b_g = _bounds(A, k.points[j], form, rn, rg)
        assert abs(nll_b[j] - rn) <= b_nll, (form, j, nll_b[j], rn, b_nll)
        assert np.linalg.norm(g_b[j] - rg) <= b_g, (form, j, _rel(g_b[j], rg))


@pytest.fixture(scope="module")
def w32():
    s = synth.make_sample("w32_n2m")
    return s, s.data.astype(np.complex64), s.mc.astype(np.complex64)


def test_w32_n2m_amplitude_parity(o, w32):
    s, d32, mc32 = w32
    model = pwa.Model(d32, mc32, s.n_gen, form="amplitude")
    M = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
    d128 = d32.astype(np.complex128)
    for V in s.points:
        nll, g = model.nll_grad(V)
        rn, rg, nbad = o.nll_amp(d128, M, V)
        assert nbad == 0
        assert abs(nll - rn) <= 1e-12 * max(abs(rn), 2e6), (nll, rn)
        assert _rel(g, rg) <= 1e-10, _rel(g, rg)
    model.close()


def test_w32_n2m_gradient_vs_differences(w32):
    """The kernels' gradient against central differences of their own NLL at
    all 20 random points, h = 1e-4 as the workload states.  The truncation
    error of a central difference is c h^2 + O(h^4), so the difference of the
    h and h/2 estimates is 3/4 of it; the h = 1e-4 difference must agree with
    the gradient within twice that estimate (plus FP64 rounding of the NLL
    differences), and their Richardson combination (4 D(h/2) - D(h)) / 3,
    error O(h^4), to 1e-6 relative."""
    s, d32, mc32 = w32
    model = pwa.Model(d32, mc32, s.n_gen, form="amplitude")
    h = 1e-4
    assert len(s.points) == 20
    for j, V in enumerate(s.points):
        x = np.ascontiguousarray(V.astype(np.complex128)).view(np.float64).copy()
        nll0, g = model.nll_grad(x)

        def cd(step, i):
            xp, xm = x.copy(), x.copy()
            xp[i] += step
            xm[i] -= step
            return (model.nll(xp) - model.nll(xm)) / (2 * step)

        d1 = np.array([cd(h, i) for i in range(x.size)])
        d2 = np.array([cd(h / 2, i) for i in range(x.size)])
        trunc = 4.0 / 3.0 * np.abs(d1 - d2)
        rounding = 1e-15 * abs(nll0) / h * 8
        assert np.all(np.abs(d1 - g) <= 2 * trunc + rounding), (j, _rel(g, d1))
        rich = (4 * d2 - d1) / 3
        assert _rel(g, rich) <= 1e-6, (j, _rel(g, rich))
    model.close()


def test_w32_n2m_lbfgs_fit_from_random_start(o, w32):
    """A full fit (L-BFGS, gauge Im V_0 = 0) from a random start, which the
    driver first scales to mu = N: it reaches its gradient test, or its line
    search stops where the decrease of f is below the rounding of f (a 2M-term
    FP64 sum) with ||G|| <= 1e-11 |NLL|; the extended likelihood's stationarity
    then fixes mu = N (|mu - N| <= ||G|| ||V|| / 2 by the scale identity), and
    the fitted NLL agrees with the oracle at the fitted V."""
    from paper_1108_5673_amd import fit
    s, d32, mc32 = w32
    model = pwa.Model(d32, mc32, s.n_gen, form="amplitude")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 32, 1])))
    v0 = synth.random_v(rng, 32)
    nll0 = model.nll(v0)
    # the value test off: the fit must reach a gradient of 1e-12 |NLL|
    V, res = fit.fit_lbfgs(model, v0, grad_tol=1e-12, rel_f_tol=0.0)
    line_search_at_rounding = res["status"] == 3 and res["grad_norm"] <= 1e-11 * abs(res["f"])
    assert res["status"] == 0 or line_search_at_rounding, res
    assert V[0].imag == 0.0
    nll, g = model.nll_grad(V)
    assert nll == res["f"] and nll < nll0
    M = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
    rn, rg, _ = o.nll_amp(d32.astype(np.complex128), M, V)
    assert abs(nll - rn) <= 1e-12 * max(abs(rn), 2e6)
    mu, _ = o.mc_term(M, V)
    n = d32.shape[0]
    assert abs(mu - n) <= 0.5 * np.linalg.norm(g) * np.linalg.norm(V) + 1e-9 * n, (mu, n)
    assert abs(mu - n) <= 1e-6 * n, (mu, n)
    model.close()


def test_w32_n2m_fumili_fit(o, w32):
    """The FUMILI fit (gain-ratio damped Newton steps on pwa_nll_grad_hess)
    from a random start, which the driver first scales to mu = N: converged,
    mu = N at the end, NLL matching the oracle.  From a random start the steps
    cross several basins of the likelihood (148 iterations measured on this
    sample; L-BFGS takes about 1700 from the same start): the bound is loose."""
    from paper_1108_5673_amd import fit
    s, d32, mc32 = w32
    model = pwa.Model(d32, mc32, s.n_gen, form="amplitude")
    M = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 32, 2])))
    v0 = synth.random_v(rng, 32)
    n = d32.shape[0]
    V, res = fit.fit_fumili(model, v0, max_iterations=1000)
    assert res["status"] == 0 and res["iterations"] <= 400, res
    nll, g = model.nll_grad(V)
    rn, rg, _ = o.nll_amp(d32.astype(np.complex128), M, V)
    assert abs(nll - rn) <= 1e-12 * max(abs(rn), 2e6)
    # the scale identity sum_b Re(conj(G_b) V_b) = 2 (mu - N) bounds mu - N by
    # the gradient the fit stopped at
    mu, _ = o.mc_term(M, V)
    assert abs(mu - n) <= 0.5 * np.linalg.norm(g) * np.linalg.norm(V) + 1e-9 * n, (mu, n)
    model.close()


def test_w32_n2m_fumili_fit_near_solution(o, w32):
    """FUMILI in the regime the paper reports (Sec. 5: 5 to 10 iterations): a
    start near the generating point (5 % complex noise per wave), default
    tolerances: the gradient test is met within 10 iterations (3 measured;
    L-BFGS from such starts takes 150 to 350), the NLL there matches the
    oracle, and mu = N within the scale identity's bound."""
    from paper_1108_5673_amd import fit
    s, d32, mc32 = w32
    model = pwa.Model(d32, mc32, s.n_gen, form="amplitude")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([11085673, 32, 3])))
    v0 = s.v_true * (1 + 0.05 * (rng.standard_normal(32) + 1j * rng.standard_normal(32)))
    V, res = fit.fit_fumili(model, v0)
    assert res["status"] == 0 and res["iterations"] <= 10, res
    rn, _, _ = o.nll_amp(d32.astype(np.complex128),
                         o.mc_matrix(mc32.astype(np.complex128), s.n_gen), V)
    assert abs(res["f"] - rn) <= 1e-12 * max(abs(rn), 2e6), (res["f"], rn)
    n = d32.shape[0]
    M = o.mc_matrix(mc32.astype(np.complex128), s.n_gen)
    mu, _ = o.mc_term(M, V)
    _, g = model.nll_grad(V)
    assert abs(mu - n) <= 0.5 * np.linalg.norm(g) * np.linalg.norm(V) + 1e-9 * n, (mu, n)
    model.close()
