"""The L-BFGS fit driver of the library, on the CPU.

The minimiser is host code (include/pwa.h, pwa_lbfgs_minimize) that takes its
objective as a callback, so it is checked here without a GPU: against closed-
form minima, on the Rosenbrock valley, against scipy's L-BFGS-B on the oracle's
NLL of a small sample, and for its error paths.  At a stationary point of
Eq. 3 the extended likelihood fixes mu = N exactly (the scale identity
sum_b Re(conj(G_b) V_b) = 2 (mu - N)), which the fitted point must meet.
"""
import numpy as np
import pytest
import scipy.optimize

import oracle
from paper_1108_5673_amd import fit, synth


def test_quadratic_closed_form():
    rng = np.random.default_rng(5)
    n = 24
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    # the value test off: the gradient test alone must stop it
    x, res = fit.minimize_lbfgs(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b), np.zeros(n),
                                grad_tol=1e-11, rel_f_tol=0.0)
    assert res["status"] == 0 and res["grad_norm"] <= 1e-11, res
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("n", [2, 10])
def test_rosenbrock(n):
    def f(x):
        v = np.sum(100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2)
        g = np.zeros_like(x)
        g[:-1] = -400.0 * x[:-1] * (x[1:] - x[:-1] ** 2) - 2.0 * (1 - x[:-1])
        g[1:] += 200.0 * (x[1:] - x[:-1] ** 2)
        return v, g

    x0 = np.full(n, -1.2)
    x0[1::2] = 1.0
    x, res = fit.minimize_lbfgs(f, x0, grad_tol=1e-12, max_iterations=5000)
    assert res["status"] in (0, 1), res
    np.testing.assert_allclose(x, np.ones(n), atol=1e-6)


def test_fixed_coordinate_stays():
    x, res = fit.minimize_lbfgs(lambda x: (np.sum((x - 3.0) ** 2), 2 * (x - 3.0)),
                                np.array([0.0, 0.5, 0.0]), fixed_index=1)
    assert x[1] == 0.5
    np.testing.assert_allclose(x[[0, 2]], [3.0, 3.0], atol=1e-8)


def test_objective_error_is_returned():
    calls = []

    def bad(x):
        calls.append(1)
        raise ValueError("objective failed")

    with pytest.raises(ValueError):
        fit.minimize_lbfgs(bad, np.zeros(3))
    assert len(calls) == 1


def test_outside_domain_shortens_the_step():
    # f = -log(1 - x^2) summed: finite only inside (-1, 1); minimum at 0
    def f(x):
        if np.any(np.abs(x) >= 1.0):
            return np.inf, np.zeros_like(x)
        return -np.sum(np.log1p(-x * x)), 2 * x / (1 - x * x)

    x, res = fit.minimize_lbfgs(f, np.array([0.9, -0.5]))
    assert res["status"] in (0, 1), res
    np.testing.assert_allclose(x, 0.0, atol=1e-8)


def test_pwa_fit_matches_scipy_and_scale_identity():
    o = oracle.get()
    s = synth.make_sample("w4_n10k", n_data=3000, n_gen=20000, n_acc=10000, n_points=1)
    A, M = s.data, o.mc_matrix(s.mc, s.n_gen)
    W = A.shape[1]

    def nll(x):
        f, g, nbad = o.nll_amp(A, M, x.view(np.complex128))
        return (np.inf if nbad else f), g

    rng = np.random.default_rng(11)
    v0 = s.v_true * np.exp(0.7j) + 0.2 * (rng.standard_normal(W) + 1j * rng.standard_normal(W))
    v0 = v0 * np.exp(-1j * np.angle(v0[0]))                 # gauge: V_0 real
    x0 = np.ascontiguousarray(v0).view(np.float64).copy()
    x0[1] = 0.0
    x, res = fit.minimize_lbfgs(nll, x0, fixed_index=1, grad_tol=1e-12)
    assert res["status"] in (0, 1), res
    assert x[1] == 0.0
    f_fit, g_fit = nll(x)
    assert np.linalg.norm(g_fit) <= 1e-6 * abs(f_fit)

    free = [k for k in range(2 * W) if k != 1]

    def nll_free(z):
        xx = x0.copy()
        xx[free] = z
        f, g = nll(xx)
        return f, g[free]

    ref = scipy.optimize.minimize(nll_free, x0[free], jac=True, method="L-BFGS-B",
                                  options={"ftol": 1e-15, "gtol": 1e-10, "maxiter": 10000})
    assert abs(f_fit - ref.fun) <= 1e-9 * abs(ref.fun), (f_fit, ref.fun)

    # stationary point of the extended likelihood: mu = N
    V = x.view(np.complex128)
    mu = o.mc_term(M, V)
    mu = mu[0] if isinstance(mu, tuple) else mu
    assert abs(mu - A.shape[0]) <= 1e-6 * A.shape[0], (mu, A.shape[0])


def test_newton_quadratic_one_step():
    rng = np.random.default_rng(9)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    x, res = fit.minimize_newton(lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b, A), np.zeros(n),
                                 grad_tol=1e-12, rel_f_tol=0.0)
    assert res["status"] == 0 and res["iterations"] <= 3, res
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def test_newton_rosenbrock():
    def f(x):
        v = 100.0 * (x[1] - x[0] ** 2) ** 2 + (1 - x[0]) ** 2
        g = np.array([-400.0 * x[0] * (x[1] - x[0] ** 2) - 2.0 * (1 - x[0]), 200.0 * (x[1] - x[0] ** 2)])
        H = np.array([[1200.0 * x[0] ** 2 - 400.0 * x[1] + 2.0, -400.0 * x[0]], [-400.0 * x[0], 200.0]])
        return v, g, H

    x, res = fit.minimize_newton(f, np.array([-1.2, 1.0]), grad_tol=1e-12, max_iterations=500)
    assert res["status"] in (0, 1), res
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-8)


def test_fumili_fit_matches_lbfgs_minimum():
    """FUMILI steps on the oracle's NLL, gradient and FUMILI matrix reach the
    same minimum as L-BFGS, in few iterations (the paper's fits take 5-10)."""
    o = oracle.get()
    s = synth.make_sample("w4_n10k", n_data=3000, n_gen=20000, n_acc=10000, n_points=1)
    A, M = s.data, o.mc_matrix(s.mc, s.n_gen)

    def fgh(x):
        V = x.view(np.complex128)
        f, g, nbad = o.nll_amp(A, M, V)
        H, _ = o.fumili_amp(A, V)
        return (np.inf if nbad else f), g, H

    rng = np.random.default_rng(11)
    W = A.shape[1]
    # start in the basin of the generating point: its direction, slightly
    # perturbed, scaled so that mu = N (the extended likelihood's scale);
    # both methods then find the same minimum
    v0 = s.v_true * np.exp(0.7j) + 0.05 * (rng.standard_normal(W) + 1j * rng.standard_normal(W))
    v0 = v0 * np.exp(-1j * np.angle(v0[0]))
    v0 = v0 * np.sqrt(A.shape[0] / o.mc_term(M, v0)[0])
    x0 = np.ascontiguousarray(v0).view(np.float64).copy()
    x0[1] = 0.0
    xn, rn = fit.minimize_newton(fgh, x0, fixed_index=1, grad_tol=1e-10)
    xl, rl = fit.minimize_lbfgs(lambda x: fgh(x)[:2], x0, fixed_index=1, grad_tol=1e-10)
    assert rn["status"] in (0, 1) and rl["status"] in (0, 1), (rn, rl)
    assert rn["iterations"] < rl["iterations"], (rn, rl)
    assert abs(rn["f"] - rl["f"]) <= 1e-9 * abs(rl["f"])
