// fit.cpp -- fit drivers on the host: limited-memory BFGS over the NLL and its
// analytic gradient.
//
// The paper's fits repeat a minimisation of Eq. 3 with analytic derivatives
// (Sec. 2, Sec. 4).  This file provides the minimiser: the two-loop recursion
// of limited-memory BFGS for the search direction and a line search that
// enforces the strong Wolfe conditions (bracketing, then zoom with safeguarded
// cubic interpolation), as published in Nocedal and Wright, Numerical
// Optimization, 2nd ed., Algorithms 7.4, 3.5 and 3.6, with the approximate
// Wolfe test of Hager and Zhang (SIAM J. Optim. 16, 2005) once the decrease of
// f is below its rounding.  Each objective call on a
// model is one pwa_nll_grad evaluation on the GPU; the minimiser itself is a
// few vector operations over 2W numbers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pwa.h"

namespace {

double dot(const std::vector<double>& a, const std::vector<double>& b)
{
    double s = 0.0;
    for (size_t k = 0; k < a.size(); ++k) s += a[k] * b[k];
    return s;
}

double norm2(const std::vector<double>& a) { return std::sqrt(dot(a, a)); }

// Minimiser of the cubic through (a, fa, ga) and (b, fb, gb), kept inside the
// interval shrunk by 10 % at both ends; bisection when the cubic has no usable
// minimiser.
double cubic_step(double a, double fa, double ga, double b, double fb, double gb)
{
    const double lo = std::min(a, b), hi = std::max(a, b);
    const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - ga * gb;
    double t = 0.5 * (a + b);
    if (disc >= 0.0 && std::isfinite(disc)) {
        const double d2 = std::copysign(std::sqrt(disc), b - a);
        const double den = gb - ga + 2.0 * d2;
        if (den != 0.0) {
            const double c = b - (b - a) * (gb + d2 - d1) / den;
            if (std::isfinite(c)) t = c;
        }
    }
    const double margin = 0.1 * (hi - lo);
    if (!(t > lo + margin && t < hi - margin)) t = 0.5 * (a + b);
    return t;
}

struct Objective {
    pwa_objective fn;
    void* ctx;
    int fixed;
    int evaluations = 0;

    // f and g at x; the gauge coordinate's derivative is dropped so that the
    // minimiser never moves it
    int operator()(const std::vector<double>& x, double& f, std::vector<double>& g)
    {
        ++evaluations;
        const int rc = fn(ctx, x.data(), &f, g.data());
        if (fixed >= 0) g[fixed] = 0.0;
        if (rc < 0) return rc;
        if (!std::isfinite(f)) f = INFINITY;
        return 0;
    }
};

// Strong Wolfe line search along d from x (value f0, slope d0 < 0).  On success
// x, f, g hold the accepted point.  Returns 0 on success, 1 if no acceptable
// step was found, < 0 on an objective error.
int wolfe_search(Objective& obj, std::vector<double>& x, double& f, std::vector<double>& g,
                 const std::vector<double>& d, double step0)
{
    const double c1 = 1e-4, c2 = 0.9;
    const double f0 = f, d0 = dot(g, d);
    const std::vector<double> x0 = x;
    std::vector<double> xt(x.size()), gt(x.size());
    auto eval = [&](double a, double& fa, double& da) {
        for (size_t k = 0; k < x.size(); ++k) xt[k] = x0[k] + a * d[k];
        const int rc = obj(xt, fa, gt);
        da = std::isfinite(fa) ? dot(gt, d) : NAN;
        return rc;
    };
    auto accept = [&](double fa) {
        x = xt;
        f = fa;
        g = gt;
        return 0;
    };
    // Near a minimiser the decrease of f along d falls below the rounding of
    // f itself while the slope is still accurate; a step is then also taken
    // when f has not grown beyond that rounding and the slope has the
    // approximate Wolfe bracket of Hager and Zhang (c2 d0 <= da <= (1 - 2 c1) |d0|).
    const double f_noise = 1e-14 * std::fabs(f0);
    auto approx_ok = [&](double fa, double da) {
        return std::isfinite(fa) && fa <= f0 + f_noise && da >= c2 * d0 &&
               da <= (1.0 - 2.0 * c1) * (-d0);
    };
    auto zoom = [&](double lo, double flo, double dlo, double hi, double fhi, double dhi) {
        for (int it = 0; it < 30; ++it) {
            double a;
            if (std::isfinite(fhi) && std::isfinite(dhi)) a = cubic_step(lo, flo, dlo, hi, fhi, dhi);
            else a = 0.5 * (lo + hi);
            double fa, da;
            const int rc = eval(a, fa, da);
            if (rc < 0) return rc;
            if (approx_ok(fa, da) && !(fa <= f0 + c1 * a * d0)) return accept(fa);
            if (!std::isfinite(fa) || fa > f0 + c1 * a * d0 || fa >= flo) {
                hi = a;
                fhi = fa;
                dhi = da;
            } else {
                if (std::fabs(da) <= -c2 * d0) return accept(fa);
                if (da * (hi - lo) >= 0.0) {
                    hi = lo;
                    fhi = flo;
                    dhi = dlo;
                }
                lo = a;
                flo = fa;
                dlo = da;
            }
            if (std::fabs(hi - lo) <= 1e-16 * std::max(1.0, std::fabs(lo))) break;
        }
        // no step met the curvature condition: keep the best sufficient decrease
        if (lo > 0.0 && flo < f0) {
            double fa, da;
            const int rc = eval(lo, fa, da);
            if (rc < 0) return rc;
            return accept(fa);
        }
        return 1;
    };

    double a_prev = 0.0, f_prev = f0, d_prev = d0;
    double a = step0;
    for (int it = 0; it < 40; ++it) {
        double fa, da;
        const int rc = eval(a, fa, da);
        if (rc < 0) return rc;
        if (approx_ok(fa, da) && !(fa <= f0 + c1 * a * d0)) return accept(fa);
        if (!std::isfinite(fa) || fa > f0 + c1 * a * d0 || (it > 0 && fa >= f_prev))
            return zoom(a_prev, f_prev, d_prev, a, fa, da);
        if (std::fabs(da) <= -c2 * d0) return accept(fa);
        if (da >= 0.0) return zoom(a, fa, da, a_prev, f_prev, d_prev);
        a_prev = a;
        f_prev = fa;
        d_prev = da;
        a *= 2.0;
    }
    return 1;
}

}  // namespace

extern "C" {

void pwa_lbfgs_default_options(pwa_lbfgs_options* opt)
{
    if (!opt) return;
    opt->max_iterations = 2000;
    opt->history = 10;
    opt->grad_tol = 1e-9;
    opt->rel_f_tol = 1e-15;
    opt->fixed_index = -1;
}

int pwa_lbfgs_minimize(int32_t n, double* x_io, pwa_objective fn, void* ctx,
                       const pwa_lbfgs_options* options, pwa_lbfgs_result* res)
{
    if (n < 1 || !x_io || !fn || !res) return PWA_ERR_INVALID;
    pwa_lbfgs_options opt;
    pwa_lbfgs_default_options(&opt);
    if (options) opt = *options;
    if (opt.history < 1 || opt.max_iterations < 0 || opt.fixed_index >= n) return PWA_ERR_INVALID;
    std::memset(res, 0, sizeof *res);

    Objective obj{fn, ctx, opt.fixed_index};
    std::vector<double> x(x_io, x_io + n), g(n), d(n), q(n);
    double f = 0.0;
    int rc = obj(x, f, g);
    if (rc < 0) return rc;
    if (!std::isfinite(f)) return PWA_WARN_DEGENERATE;

    const int m = opt.history;
    std::vector<std::vector<double>> S(m, std::vector<double>(n)), Y(m, std::vector<double>(n));
    std::vector<double> rho(m), alpha(m);
    int stored = 0, head = 0;   // ring buffer of the last `stored` pairs, newest at head - 1
    int status = PWA_LBFGS_MAX_ITERATIONS;
    int iter = 0;
    int small_steps = 0;
    for (; iter < opt.max_iterations; ++iter) {
        const double gn = norm2(g);
        if (gn <= opt.grad_tol * std::max(1.0, std::fabs(f))) {
            status = PWA_LBFGS_CONVERGED_GRADIENT;
            break;
        }
        // two-loop recursion: d = -H g with H0 = (s'y / y'y) I
        q = g;
        for (int j = 0; j < stored; ++j) {
            const int k = (head - 1 - j + m) % m;
            alpha[k] = rho[k] * dot(S[k], q);
            for (int i = 0; i < n; ++i) q[i] -= alpha[k] * Y[k][i];
        }
        double gamma = 1.0;
        if (stored > 0) {
            const int k = (head - 1 + m) % m;
            gamma = dot(S[k], Y[k]) / dot(Y[k], Y[k]);
        }
        for (int i = 0; i < n; ++i) q[i] *= gamma;
        for (int j = stored - 1; j >= 0; --j) {
            const int k = (head - 1 - j + m) % m;
            const double beta = rho[k] * dot(Y[k], q);
            for (int i = 0; i < n; ++i) q[i] += (alpha[k] - beta) * S[k][i];
        }
        for (int i = 0; i < n; ++i) d[i] = -q[i];
        if (opt.fixed_index >= 0) d[opt.fixed_index] = 0.0;
        double slope = dot(g, d);
        if (!(slope < 0.0)) {   // not a descent direction: restart from steepest descent
            stored = 0;
            for (int i = 0; i < n; ++i) d[i] = -g[i];
            slope = -gn * gn;
        }
        const double step0 = stored == 0 ? std::min(1.0, 1.0 / gn) : 1.0;

        const std::vector<double> x_old = x, g_old = g;
        const double f_old = f;
        rc = wolfe_search(obj, x, f, g, d, step0);
        if (rc < 0) return rc;
        if (rc == 1) {
            if (stored > 0) {   // drop the curvature memory once and retry
                stored = 0;
                continue;
            }
            status = PWA_LBFGS_LINE_SEARCH_FAILED;
            break;
        }
        // curvature pair
        std::vector<double>& s = S[head];
        std::vector<double>& y = Y[head];
        for (int i = 0; i < n; ++i) {
            s[i] = x[i] - x_old[i];
            y[i] = g[i] - g_old[i];
        }
        const double sy = dot(s, y);
        if (sy > 1e-300) {
            rho[head] = 1.0 / sy;
            head = (head + 1) % m;
            stored = std::min(stored + 1, m);
        }
        if (opt.rel_f_tol > 0.0 && f_old - f <= opt.rel_f_tol * std::max(1.0, std::fabs(f))) {
            if (++small_steps >= 3) {
                status = PWA_LBFGS_CONVERGED_VALUE;
                ++iter;
                break;
            }
        } else {
            small_steps = 0;
        }
    }
    std::memcpy(x_io, x.data(), sizeof(double) * n);
    res->status = status;
    res->iterations = iter;
    res->evaluations = obj.evaluations;
    res->f = f;
    res->grad_norm = norm2(g);
    return PWA_OK;
}

}  // extern "C"

namespace {

struct ModelCtx {
    const pwa_model* model;
    void* stream;
};

// Gauge: the NLL does not depend on a global phase of V, so V_0 is rotated
// onto the positive real axis (the fits then hold Im V_0 at zero).
void gauge_rotate(double* v, int W)
{
    const double r = std::hypot(v[0], v[1]);
    if (r > 0.0) {
        const double c = v[0] / r, s = -v[1] / r;   // multiply by exp(-i arg V_0)
        for (int a = 0; a < W; ++a) {
            const double re = v[2 * a], im = v[2 * a + 1];
            v[2 * a] = re * c - im * s;
            v[2 * a + 1] = re * s + im * c;
        }
        v[1] = 0.0;
    }
}

// Scale: along V -> s V the extended likelihood of Eq. 3 changes as
// -N ln s^2 + s^2 mu(V) (the data term gains -ln s^2 per event), whose minimum
// is at s^2 = N / mu(V).  The fits start from that point of the start's ray
// (mu(V) = sum_ab V_a V*_b M_ab from the model's M); nothing is done when
// mu(V) is not positive (no MC events).  Both fit drivers scale their start:
// it is the best point of the start's ray, and there FUMILI's matrix has the
// true curvature along V (4N against 2N + 2 mu(V), equal at mu = N).
int scale_start(const pwa_model* model, double* v, int W, int64_t n, void* stream)
{
    std::vector<double> M((size_t)2 * W * W);
    const int rc = pwa_copy_mc_matrix(model, M.data(), stream);
    if (rc != PWA_OK) return rc;
    double mu = 0.0;
    for (int a = 0; a < W; ++a)
        for (int b = 0; b < W; ++b) {
            // Re(V_a M_ab conj(V_b))
            const double mr = M[2 * ((size_t)a * W + b)], mi = M[2 * ((size_t)a * W + b) + 1];
            const double tr = v[2 * a] * mr - v[2 * a + 1] * mi, ti = v[2 * a] * mi + v[2 * a + 1] * mr;
            mu += tr * v[2 * b] + ti * v[2 * b + 1];
        }
    if (mu > 0.0 && std::isfinite(mu)) {
        const double sc = std::sqrt((double)n / mu);
        for (int k = 0; k < 2 * W; ++k) v[k] *= sc;
    }
    return PWA_OK;
}

int model_objective(void* ctx, const double* x, double* f, double* g)
{
    const ModelCtx* c = static_cast<const ModelCtx*>(ctx);
    const int rc = pwa_nll_grad(c->model, x, f, g, c->stream);
    if (rc == PWA_WARN_DEGENERATE) {
        *f = INFINITY;
        return 0;
    }
    return rc;
}

}  // namespace

extern "C" int pwa_fit_lbfgs(const pwa_model* model, double* v, const pwa_lbfgs_options* options,
                             pwa_lbfgs_result* res, void* hip_stream)
{
    if (!model || !v || !res) return PWA_ERR_INVALID;
    pwa_info info;
    int rc = pwa_model_info(model, &info);
    if (rc != PWA_OK) return rc;
    const int W = info.n_waves;
    pwa_lbfgs_options opt;
    pwa_lbfgs_default_options(&opt);
    if (options) opt = *options;
    gauge_rotate(v, W);
    rc = scale_start(model, v, W, info.n_data, hip_stream);
    if (rc != PWA_OK) return rc;
    opt.fixed_index = 1;
    ModelCtx ctx{model, hip_stream};
    return pwa_lbfgs_minimize(2 * W, v, model_objective, &ctx, &opt, res);
}

// ---- FUMILI-style fit: damped Newton steps on the FUMILI matrix ------------
// With f, g and the FUMILI matrix H at x: solve (H + lambda D) d = -g by
// Cholesky (D the diagonal of H, lambda raised until the factorisation
// succeeds) and compare the actual decrease f(x) - f(x + d) with the one the
// quadratic model predicts, -(g.d + d.H.d / 2) (Levenberg-Marquardt with the
// gain ratio rho of the two; FUMILI is the Gauss-Newton method of likelihood
// fits).  rho > 1e-4: the step is taken, and lambda is divided by 5 when
// rho > 0.75 or multiplied by 4 when rho < 0.25; otherwise x stays and lambda
// is multiplied by 4.  A trial point costs f and g only; H is computed at the
// points taken.
namespace {

// In-place Cholesky of the n x n row-major A (lower factor); false if A is not
// positive definite.
bool cholesky(std::vector<double>& A, int n)
{
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        d = std::sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double x = A[i * n + j];
            for (int k = 0; k < j; ++k) x -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = x / d;
        }
    }
    return true;
}

void cholesky_solve(const std::vector<double>& L, int n, std::vector<double>& b)
{
    for (int i = 0; i < n; ++i) {
        double x = b[i];
        for (int k = 0; k < i; ++k) x -= L[i * n + k] * b[k];
        b[i] = x / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double x = b[i];
        for (int k = i + 1; k < n; ++k) x -= L[k * n + i] * b[k];
        b[i] = x / L[i * n + i];
    }
}

}  // namespace

extern "C" int pwa_newton_minimize(int32_t n, double* x_io, pwa_objective_hess fn, void* ctx,
                                   const pwa_lbfgs_options* options, pwa_lbfgs_result* res)
{
    if (n < 1 || !x_io || !fn || !res) return PWA_ERR_INVALID;
    pwa_lbfgs_options opt;
    pwa_lbfgs_default_options(&opt);
    if (options) opt = *options;
    if (opt.max_iterations < 0 || opt.fixed_index >= n) return PWA_ERR_INVALID;
    std::memset(res, 0, sizeof *res);
    std::vector<double> x(x_io, x_io + n), g(n), H((size_t)n * n), L((size_t)n * n), d(n),
        xt(n), gt(n), Hd(n);
    int evals = 0;
    const int k = opt.fixed_index;
    // f and g at xx, and H when HH is given; the fixed coordinate gets a zero
    // gradient, a unit diagonal and no coupling
    auto eval = [&](const std::vector<double>& xx, double& f, std::vector<double>& gg,
                    std::vector<double>* HH) {
        ++evals;
        const int rc = fn(ctx, xx.data(), &f, gg.data(), HH ? HH->data() : nullptr);
        if (rc < 0) return rc;
        if (!std::isfinite(f)) f = INFINITY;
        if (k >= 0) {
            gg[k] = 0.0;
            if (HH) {
                for (int i = 0; i < n; ++i) (*HH)[(size_t)i * n + k] = (*HH)[(size_t)k * n + i] = 0.0;
                (*HH)[(size_t)k * n + k] = 1.0;
            }
        }
        return 0;
    };
    double f = 0.0;
    int rc = eval(x, f, g, &H);
    if (rc < 0) return rc;
    if (!std::isfinite(f)) return PWA_WARN_DEGENERATE;
    double lambda = 1e-6;   // nearly a Newton step at first; raised 4x per step not taken
    int status = PWA_LBFGS_MAX_ITERATIONS;
    int iter = 0, small_steps = 0, rejected = 0;
    while (iter < opt.max_iterations) {
        const double gn = norm2(g);
        if (gn <= opt.grad_tol * std::max(1.0, std::fabs(f))) {
            status = PWA_LBFGS_CONVERGED_GRADIENT;
            break;
        }
        // damped system, damping raised until positive definite
        bool ok = false;
        for (int tries = 0; tries < 60 && !ok; ++tries) {
            L = H;
            for (int i = 0; i < n; ++i) L[(size_t)i * n + i] += lambda * std::max(H[(size_t)i * n + i], 1e-300);
            ok = cholesky(L, n);
            if (!ok) lambda = std::max(lambda * 10.0, 1e-8);
        }
        if (!ok) {
            status = PWA_LBFGS_LINE_SEARCH_FAILED;
            break;
        }
        for (int i = 0; i < n; ++i) d[i] = -g[i];
        cholesky_solve(L, n, d);
        // predicted decrease of the quadratic model
        for (int i = 0; i < n; ++i) {
            double t = 0.0;
            for (int j = 0; j < n; ++j) t += H[(size_t)i * n + j] * d[j];
            Hd[i] = t;
        }
        const double pred = -(dot(g, d) + 0.5 * dot(d, Hd));
        for (int i = 0; i < n; ++i) xt[i] = x[i] + d[i];
        double ft = 0.0;
        rc = eval(xt, ft, gt, nullptr);
        if (rc < 0) return rc;
        const double noise = 1e-14 * std::fabs(f);
        const double actual = f - ft;
        const double rho = pred > 0.0 ? actual / pred : -1.0;
        // taken: a real decrease in line with the model, or, once the model's
        // predicted decrease is below rounding, a step that raises f by no
        // more than rounding
        const bool take = std::isfinite(ft) && (rho > 1e-4 || (pred <= noise && ft <= f + noise));
        if (!take) {
            lambda = std::max(lambda * 4.0, 1e-6);
            if (++rejected > 40) {
                status = PWA_LBFGS_LINE_SEARCH_FAILED;
                break;
            }
            continue;
        }
        rejected = 0;
        ++iter;
        if (rho > 0.75) lambda = std::max(lambda * 0.2, 1e-12);
        else if (rho < 0.25) lambda *= 4.0;
        x = xt;
        g = gt;
        const double f_old = f;
        rc = eval(x, f, g, &H);   // H at the new point (f, g again with it)
        if (rc < 0) return rc;
        if (opt.rel_f_tol > 0.0 && f_old - f <= opt.rel_f_tol * std::max(1.0, std::fabs(f))) {
            if (++small_steps >= 3) {
                status = PWA_LBFGS_CONVERGED_VALUE;
                break;
            }
        } else {
            small_steps = 0;
        }
    }
    std::memcpy(x_io, x.data(), sizeof(double) * n);
    res->status = status;
    res->iterations = iter;
    res->evaluations = evals;
    res->f = f;
    res->grad_norm = norm2(g);
    return PWA_OK;
}

namespace {

int model_objective_hess(void* ctx, const double* x, double* f, double* g, double* H)
{
    const ModelCtx* c = static_cast<const ModelCtx*>(ctx);
    const int rc = H ? pwa_nll_grad_hess(c->model, x, f, g, H, c->stream)
                     : pwa_nll_grad(c->model, x, f, g, c->stream);
    if (rc == PWA_WARN_DEGENERATE) {
        *f = INFINITY;
        return 0;
    }
    return rc;
}

}  // namespace

extern "C" int pwa_fit_fumili(const pwa_model* model, double* v, const pwa_lbfgs_options* options,
                              pwa_lbfgs_result* res, void* hip_stream)
{
    if (!model || !v || !res) return PWA_ERR_INVALID;
    pwa_info info;
    int rc = pwa_model_info(model, &info);
    if (rc != PWA_OK) return rc;
    const int W = info.n_waves;
    pwa_lbfgs_options opt;
    pwa_lbfgs_default_options(&opt);
    if (options) opt = *options;
    gauge_rotate(v, W);
    rc = scale_start(model, v, W, info.n_data, hip_stream);
    if (rc != PWA_OK) return rc;
    opt.fixed_index = 1;
    ModelCtx ctx{model, hip_stream};
    return pwa_newton_minimize(2 * W, v, model_objective_hess, &ctx, &opt, res);
}
