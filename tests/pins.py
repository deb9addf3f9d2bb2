"""Pins that tie the oracle to the paper and to mathematics, not to itself.

Each pin takes an ``oracle.Oracle`` and raises AssertionError when the oracle
disagrees with something the paper or the mathematics fixes:

  * hand-derived closed forms (W = 1; a 2-wave, 2-event example worked on paper);
  * exact rational brute force of Eq. 1 and Eq. 3 for one event, and a
    50-digit evaluation of the likelihood;
  * invariants: global phase, the Euler (scale) identity, non-negativity,
    additivity over samples, event-order independence;
  * the MC term against the event-by-event sum it abbreviates (fixes the
    conjugation convention of M);
  * the packed table against numpy's own products in triu order;
  * central finite differences (Richardson-extrapolated) of the oracle's NLL;
  * for the FUMILI matrix: the scale identity theta^T H theta = 4N, the phase
    null vector, one-event brute force by differences, additivity.

``ALL_PINS`` lists them; ``tests/test_oracle_mutations.py`` checks that a
plausible mistake planted anywhere in the oracle fails at least one.
"""
from __future__ import annotations

import math
from fractions import Fraction

import mpmath
import numpy as np

from paper_1108_5673_amd import synth


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))


def _sample(w, n, n_mc, seed, n_points=3):
    return synth.small_sample(w, n, n_mc, seed, n_points)


# ---------------------------------------------------------------- closed forms
def pin_hand_example(o):
    """W = 2, N = 2 worked by hand from Eq. 1 and Eq. 3.

    A_1 = (1, i), A_2 = (1, 1), V = (1, 1); MC B_1 = (1, 0), B_2 = (0, 1), N_gen = 4.
    I_1 = |1 + i|^2 = 2, I_2 = |1 + 1|^2 = 4, M = diag(1/4, 1/4), mu = 1/2,
    NLL = -ln 2 - ln 4 + 1/2.  Differentiating each term directly:
    dNLL/dRe V_1 = -2/2 - 4/4 + 1/2 = -3/2, dNLL/dIm V_1 = -2/2 - 0 + 0 = -1,
    dNLL/dRe V_2 = -2/2 - 4/4 + 1/2 = -3/2, dNLL/dIm V_2 = +2/2 - 0 + 0 = +1.
    """
    A = np.array([[1, 1j], [1, 1]], np.complex128)
    B = np.array([[1, 0], [0, 1]], np.complex128)
    V = np.array([1, 1], np.complex128)
    M = o.mc_matrix(B, 4)
    assert np.allclose(M, np.diag([0.25, 0.25]), rtol=0, atol=1e-15), M
    expect_nll = -math.log(2.0) - math.log(4.0) + 0.5
    expect_g = np.array([-1.5, -1.0, -1.5, 1.0])
    assert np.allclose(o.intensity_amp(A, V), [2.0, 4.0], rtol=1e-15)
    assert np.allclose(o.intensity_table(o.table(A), V), [2.0, 4.0], rtol=1e-15)
    for nll, g, nbad in (o.nll_amp(A, M, V), o.nll_table(o.table(A), M, V)):
        assert nbad == 0
        assert abs(nll - expect_nll) < 1e-14, (nll, expect_nll)
        assert np.allclose(g, expect_g, rtol=0, atol=1e-14), g


def pin_w1_closed_form(o):
    """W = 1: I_i = |V|^2 |A_i|^2, so NLL = -N ln|V|^2 - sum ln|A_i|^2 + |V|^2 M_11
    and G = 2 V (M_11 - N / |V|^2)."""
    s = _sample(1, 700, 900, 11)
    A, B = s.data, s.mc
    n_gen = 1800
    M = o.mc_matrix(B, n_gen)
    m11 = float(np.sum(np.abs(B[:, 0]) ** 2) / n_gen)
    assert abs(M[0, 0].real - m11) <= 1e-13 * m11 and abs(M[0, 0].imag) <= 1e-15 * m11
    for V in s.points:
        v2 = abs(V[0]) ** 2
        n = A.shape[0]
        expect = -n * math.log(v2) - float(np.sum(np.log(np.abs(A[:, 0]) ** 2))) + v2 * m11
        g = 2.0 * V[0] * (m11 - n / v2)
        for nll, grad, nbad in (o.nll_amp(A, M, V), o.nll_table(o.table(A), M, V)):
            assert nbad == 0
            assert abs(nll - expect) <= 1e-11 * abs(expect), (nll, expect)
            assert _rel(grad, [g.real, g.imag]) < 1e-11


# ------------------------------------------------------- exact brute force
def _q(x):
    return Fraction(float(x))       # exact: the inputs are dyadic rationals


def _cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def _conj(a):
    return (a[0], -a[1])


def pin_exact_one_event(o):
    """N = 1: Eq. 3's double sum and Eq. 1's modulus squared, in exact rational
    arithmetic, against the oracle; the likelihood against a 50-digit value."""
    rng = np.random.default_rng(5)
    W = 4
    # dyadic rationals are exact in binary floating point and in Fraction
    A = (rng.integers(-16, 17, W) + 1j * rng.integers(-16, 17, W)) / 8.0
    V = (rng.integers(-16, 17, W) + 1j * rng.integers(-16, 17, W)) / 4.0
    Bm = (rng.integers(-16, 17, (3, W)) + 1j * rng.integers(-16, 17, (3, W))) / 8.0
    n_gen = 5
    Aq = [(_q(z.real), _q(z.imag)) for z in A]
    Vq = [(_q(z.real), _q(z.imag)) for z in V]
    # Eq. 3, first bracket: sum_a sum_a' V_a V*_a' A_a A*_a'
    dbl = (Fraction(0), Fraction(0))
    for a in range(W):
        for ap in range(W):
            t = _cmul(_cmul(Vq[a], _conj(Vq[ap])), _cmul(Aq[a], _conj(Aq[ap])))
            dbl = (dbl[0] + t[0], dbl[1] + t[1])
    assert dbl[1] == 0
    # Eq. 1: |sum_a V_a A_a|^2
    s = (Fraction(0), Fraction(0))
    for a in range(W):
        t = _cmul(Vq[a], Aq[a])
        s = (s[0] + t[0], s[1] + t[1])
    assert s[0] ** 2 + s[1] ** 2 == dbl[0]
    exact_I = dbl[0]
    A1 = A[None, :]
    assert abs(o.intensity_amp(A1, V)[0] - float(exact_I)) <= 1e-15 * float(exact_I)
    assert abs(o.intensity_table(o.table(A1), V)[0] - float(exact_I)) <= 1e-14 * float(exact_I)
    # MC term: (1/N_gen) sum_j |sum_a V_a B_ja|^2, exact
    mu = Fraction(0)
    for j in range(Bm.shape[0]):
        s = (Fraction(0), Fraction(0))
        for a in range(W):
            t = _cmul(Vq[a], (_q(Bm[j, a].real), _q(Bm[j, a].imag)))
            s = (s[0] + t[0], s[1] + t[1])
        mu += s[0] ** 2 + s[1] ** 2
    mu /= n_gen
    M = o.mc_matrix(Bm, n_gen)
    mpmath.mp.dps = 50
    expect = -mpmath.log(mpmath.mpf(exact_I.numerator) / exact_I.denominator) + \
        mpmath.mpf(mu.numerator) / mu.denominator
    for nll, _, nbad in (o.nll_amp(A1, M, V), o.nll_table(o.table(A1), M, V)):
        assert nbad == 0
        assert abs(mpmath.mpf(nll) - expect) <= 1e-13 * max(1, abs(expect)), (nll, expect)


# ------------------------------------------------------------ conventions
def pin_mc_term_is_event_sum(o):
    """mu(V) from M equals (1/N_gen) sum_j |sum_a V_a B_ja|^2 evaluated event by
    event; only M_aa' = (1/N_gen) sum_j B_ja B*_ja' with mu = sum V_a V*_a' M_aa'
    passes this for complex B and W >= 2."""
    s = _sample(5, 10, 3000, 12)
    n_gen = 7000
    M = o.mc_matrix(s.mc, n_gen)
    assert np.allclose(M, M.conj().T, rtol=0, atol=1e-15 * np.abs(M).max())
    for V in s.points:
        direct = float(np.sum(np.abs(s.mc @ V) ** 2) / n_gen)
        mu, mu_im = o.mc_term(M, V)
        assert abs(mu - direct) <= 1e-12 * direct, (mu, direct)
        assert abs(mu_im) <= 1e-12 * direct
        # the likelihood uses the same term: NLL(data = empty) == mu
        nll, _, _ = o.nll_amp(np.zeros((0, 5), np.complex128), M, V)
        assert abs(nll - direct) <= 1e-12 * direct


def pin_table_layout(o):
    """Packed table: column k holds A_a conj(A_a') for the k-th (a, a') of numpy's
    triu_indices(W) (row-major upper triangle)."""
    s = _sample(6, 50, 10, 13)
    ia, ib = np.triu_indices(6)
    # complex64 amplitudes: every product is exact in FP64, so each entry is one
    # rounding of an exact value and must match bit for bit
    A = s.data.astype(np.complex64).astype(np.complex128)
    T = o.table(A)
    assert T.shape == (50, len(ia))
    assert np.array_equal(T, A[:, ia] * np.conj(A[:, ib]))
    T = o.table(s.data)
    scale = np.abs(s.data[:, ia]) * np.abs(s.data[:, ib])
    assert np.all(np.abs(T - s.data[:, ia] * np.conj(s.data[:, ib])) <= 4e-16 * scale)


def pin_forms_agree(o):
    """Table form (Eq. 3 literal) and amplitude form (Eq. 1) give the same NLL and
    gradient; the intensity from a general PSD table of rank 2 equals the sum of
    the two rank-1 intensities."""
    s = _sample(7, 400, 500, 14)
    M = o.mc_matrix(s.mc, 900)
    T = o.table(s.data)
    for V in s.points:
        a = o.nll_amp(s.data, M, V)
        t = o.nll_table(T, M, V)
        assert abs(a[0] - t[0]) <= 1e-12 * abs(a[0])
        assert _rel(t[1], a[1]) < 1e-11
        i_amp = o.intensity_amp(s.data, V)
        assert _rel(o.intensity_table(T, V), i_amp) < 1e-13
    A2 = _sample(7, 400, 10, 15).data
    T2 = o.table(A2)
    V = s.points[0]
    assert _rel(o.intensity_table(T + T2, V), o.intensity_amp(s.data, V) + o.intensity_amp(A2, V)) < 1e-13


# ------------------------------------------------------------- invariants
def pin_phase_invariance(o):
    """NLL(e^{i phi} V) = NLL(V); the gradient is orthogonal to i V:
    sum_b (-Re G_b Im V_b + Im G_b Re V_b) = 0."""
    s = _sample(6, 600, 800, 16)
    M = o.mc_matrix(s.mc, 1600)
    for V in s.points:
        nll, g, _ = o.nll_amp(s.data, M, V)
        for phi in (0.3, 2.1, -1.2):
            nll2, _, _ = o.nll_amp(s.data, M, V * np.exp(1j * phi))
            assert abs(nll2 - nll) <= 1e-12 * abs(nll)
        gc = g[0::2] + 1j * g[1::2]
        rot = float(np.sum(-gc.real * V.imag + gc.imag * V.real))
        assert abs(rot) <= 1e-12 * float(np.linalg.norm(gc) * np.linalg.norm(V))


def pin_scale_identity(o):
    """Euler's identity for the homogeneous parts of Eq. 3:
    sum_b (Re G_b Re V_b + Im G_b Im V_b) = 2 (mu - N)."""
    s = _sample(5, 500, 700, 17)
    M = o.mc_matrix(s.mc, 1000)
    T = o.table(s.data)
    for V in s.points:
        mu, _ = o.mc_term(M, V)
        for nll, g, _ in (o.nll_amp(s.data, M, V), o.nll_table(T, M, V)):
            gc = g[0::2] + 1j * g[1::2]
            lhs = float(np.sum(gc.real * V.real + gc.imag * V.imag))
            rhs = 2.0 * (mu - s.data.shape[0])
            assert abs(lhs - rhs) <= 1e-11 * max(abs(rhs), 1.0), (lhs, rhs)


def pin_nonnegative(o):
    """I_i >= 0 for a positive semi-definite table (rank 1 and rank 3)."""
    s = _sample(8, 300, 10, 18)
    T = o.table(s.data) + o.table(_sample(8, 300, 10, 19).data) + o.table(_sample(8, 300, 10, 20).data)
    for V in s.points:
        assert np.all(o.intensity_table(T, V) >= 0)
        assert np.all(o.intensity_amp(s.data, V) >= 0)


def pin_additivity_permutation(o):
    """The data term is a sum over independent events: D(s1 + s2) = D(s1) + D(s2),
    the data gradient adds the same way, and event order does not matter."""
    s = _sample(5, 900, 400, 21)
    M = o.mc_matrix(s.mc, 800)
    V = s.points[1]
    mu, _ = o.mc_term(M, V)
    n_all, g_all, _ = o.nll_amp(s.data, M, V)
    n_1, g_1, _ = o.nll_amp(s.data[:350], M, V)
    n_2, g_2, _ = o.nll_amp(s.data[350:], M, V)
    assert abs((n_all - mu) - ((n_1 - mu) + (n_2 - mu))) <= 1e-12 * abs(n_all)
    gmu = 2.0 * (V @ M)
    gmu = np.stack([gmu.real, gmu.imag], -1).ravel()
    assert _rel(g_all - gmu, (g_1 - gmu) + (g_2 - gmu)) < 1e-12
    perm = np.random.default_rng(3).permutation(900)
    n_p, g_p, _ = o.nll_table(o.table(s.data[perm]), M, V)
    assert abs(n_p - n_all) <= 1e-12 * abs(n_all)
    assert _rel(g_p, g_all) < 1e-12


def pin_degenerate(o):
    """An event with sum_a V_a A_ia = 0 has I_i = 0: the likelihood is undefined
    (NLL = +inf, gradient NaN) and the event is counted."""
    s = _sample(3, 20, 50, 22)
    A = s.data.copy()
    V = np.array([1.0 + 0.5j, -0.25 + 1j, 0.5 - 0.5j])
    A[7] = [V[1], -V[0], 0.0]          # V_0 V_1 - V_1 V_0 = 0
    M = o.mc_matrix(s.mc, 100)
    for nll, g, nbad in (o.nll_amp(A, M, V), o.nll_table(o.table(A), M, V)):
        assert nbad == 1 and nll == math.inf and np.all(np.isnan(g))


# ------------------------------------------------------------ derivatives
def pin_finite_differences(o):
    """Central differences of the oracle's own NLL, Richardson-extrapolated,
    against its analytic gradient (both forms)."""
    s = _sample(4, 300, 500, 23)
    M = o.mc_matrix(s.mc, 1000)
    T = o.table(s.data)
    for V in s.points[:2]:
        for f in (lambda v: o.nll_amp(s.data, M, v, grad=False)[0],
                  lambda v: o.nll_table(T, M, v, grad=False)[0]):
            fd = np.zeros(8)
            for k in range(8):
                e = np.zeros(4, np.complex128)
                e[k // 2] = 1.0 if k % 2 == 0 else 1.0j

                def cd(h):
                    return (f(V + h * e) - f(V - h * e)) / (2 * h)
                fd[k] = (4.0 * cd(5e-4) - cd(1e-3)) / 3.0
            _, g, _ = o.nll_amp(s.data, M, V)
            assert _rel(fd, g) < 1e-7, (fd, g)


def pin_thread_independence(o):
    """The fixed-chunk summation gives bit-identical results for 1 and many threads."""
    s = _sample(6, 30_000, 20_000, 24)
    before = o.num_threads()
    res, mats = [], []
    try:
        for nt in (1, max(4, before)):
            o.set_num_threads(nt)
            mats.append(o.mc_matrix(s.mc, 40_000))
            res.append(o.nll_amp(s.data, mats[-1], s.points[0]))
    finally:
        o.set_num_threads(before)
    assert np.array_equal(mats[0], mats[1])
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])


# ---------------------------------------------- FUMILI second derivatives
def _theta(V):
    return np.ascontiguousarray(np.asarray(V, np.complex128)).view(np.float64)


def pin_fumili_scale_identity(o):
    """I_i is homogeneous of degree 2 in theta, so theta . grad ln I_i = 2 for
    every event and theta^T (sum_i J_i J_i^T) theta = 4 N exactly."""
    s = _sample(5, 3000, 10, 41)
    for V in s.points:
        H, nbad = o.fumili_amp(s.data, V)
        assert nbad == 0
        th = _theta(V)
        assert abs(th @ H @ th - 4 * 3000) <= 1e-10 * 4 * 3000
        assert _rel(H, H.T) < 1e-14


def pin_fumili_phase_null_vector(o):
    """A global phase does not change I_i: theta' = i V (as reals) is a null
    vector, and the matrix is positive semidefinite."""
    s = _sample(4, 2000, 10, 42)
    V = s.points[0]
    H, _ = o.fumili_amp(s.data, V)
    phi = _theta(1j * V)
    assert np.linalg.norm(H @ phi) <= 1e-11 * np.linalg.norm(H) * np.linalg.norm(phi)
    assert np.linalg.eigvalsh(H).min() >= -1e-10 * np.abs(H).max()


def pin_fumili_one_event_brute_force(o):
    """One event: the matrix is J J^T with J the gradient of ln I, here taken
    by Richardson-extrapolated central differences of |sum_a V_a A_a|^2."""
    rng = np.random.default_rng(43)
    W = 3
    A = rng.standard_normal((1, W)) + 1j * rng.standard_normal((1, W))
    V = rng.standard_normal(W) + 1j * rng.standard_normal(W)
    th = _theta(V).copy()

    def lnI(t):
        v = t.view(np.complex128)
        s_ = np.sum(v * A[0])
        return math.log(s_.real ** 2 + s_.imag ** 2)

    J = np.zeros(2 * W)
    for k in range(2 * W):
        e = np.zeros(2 * W)
        e[k] = 1.0

        def cd(h):
            return (lnI(th + h * e) - lnI(th - h * e)) / (2 * h)
        J[k] = (4.0 * cd(1e-4) - cd(2e-4)) / 3.0
    H, _ = o.fumili_amp(A, V)
    assert _rel(H, np.outer(J, J)) < 1e-8, (H, np.outer(J, J))


def pin_fumili_additivity(o):
    """The matrix is a sum over events: two halves add to the whole."""
    s = _sample(6, 2000, 10, 45)
    V = s.points[0]
    H, _ = o.fumili_amp(s.data, V)
    H1, _ = o.fumili_amp(s.data[:700], V)
    H2, _ = o.fumili_amp(s.data[700:], V)
    assert _rel(H1 + H2, H) < 1e-12


ALL_PINS = [
    pin_hand_example, pin_w1_closed_form, pin_exact_one_event, pin_mc_term_is_event_sum,
    pin_table_layout, pin_forms_agree, pin_phase_invariance, pin_scale_identity,
    pin_nonnegative, pin_additivity_permutation, pin_degenerate, pin_finite_differences,
    pin_thread_independence, pin_fumili_scale_identity, pin_fumili_phase_null_vector,
    pin_fumili_one_event_brute_force, pin_fumili_additivity,
]
