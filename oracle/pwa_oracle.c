/*
 * pwa_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the
 * extended unbinned negative log-likelihood of a partial-wave fit
 * (arXiv:1108.5673, Sec. 2, Eqs. 1-3) and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  The HIP library never links, loads or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP path: both sides receive the same arrays and nothing else.
 *
 * Notation (Sec. 2):
 *   V_a             complex production amplitude of wave a (the fit parameters)
 *   A_a(Omega_i)    complex decay amplitude of wave a for data event i
 *   B_ja            decay amplitude of wave a for accepted MC event j
 *   I(Omega)        = |sum_a V_a A_a(Omega)|^2                          (Eq. 1)
 *   -ln L           = - sum_i ln( sum_a sum_a' V_a V*_a' A_a A*_a' )
 *                     + sum_a sum_a' V_a V*_a' M_aa'                    (Eq. 3)
 *   M_aa'           = (1/N_gen) sum_{j in accepted MC} B_ja B*_ja'       (Eq. 3, inner bracket)
 *   T_i,aa'         = A_a(Omega_i) A*_a'(Omega_i), the per-event lookup table
 *                     that can be precomputed when masses and widths are
 *                     fixed (Sec. 2, the paragraph after Eq. 3).
 *
 * Readings of the paper taken here (the paper writes Eq. 3 with a
 * proportionality sign and gives no gradient):
 *   - NLL = D + mu exactly, with D = -sum_i ln I_i and mu the MC term; no
 *     additive constants are kept.
 *   - The table is stored packed: only entries a <= a' in row-major order of
 *     the upper triangle; T_i,a'a = conj(T_i,aa') restores the rest, since
 *     T_i is Hermitian by construction.
 *   - Gradient with respect to the real and imaginary part of V_b, returned
 *     as G_b = dNLL/dRe V_b + i dNLL/dIm V_b.  Differentiating Eq. 3:
 *         dI_i/dRe V_b + i dI_i/dIm V_b = 2 sum_a V_a T_i,ab
 *     so  G_b = 2 sum_a V_a (M_ab - U_ab),  U_ab = sum_i T_i,ab / I_i,
 *     and in amplitude form  G_b = 2 sum_a V_a M_ab - 2 sum_i S_i A*_ib / I_i
 *     with S_i = sum_a V_a A_ia.
 *   - An event with I_i <= 0 or a non-finite I_i makes the likelihood
 *     undefined: the NLL is +inf, the gradient NaN, and the number of such
 *     events is returned; nothing is clamped.
 *
 * Summation: events are split into fixed chunks of ORACLE_CHUNK events; each
 * chunk is summed in event order with Neumaier compensation and the chunk
 * sums are combined in chunk order, again compensated.  The result therefore
 * does not depend on the number of OpenMP threads.
 *
 * Complex arrays are interleaved (re, im) doubles, row-major.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CHUNK 8192

typedef double complex cplx;

/* ---- compensated (Neumaier) summation -------------------------------- */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_value(const nsum* a) { return a->s + a->c; }

static int64_t n_chunks(int64_t n) { return (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK; }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* packed index of (a, a') with a <= a' in the row-major upper triangle */
static int64_t packed_index(int32_t W, int32_t a, int32_t ap)
{
    /* rows 0..a-1 hold W, W-1, ..., W-a+1 entries */
    return (int64_t)a * W - (int64_t)a * (a - 1) / 2 + (ap - a);
}

/* T_i,aa' of a packed Hermitian table, any a, a' (Hermitian completion) */
static cplx table_entry(const cplx* Ti, int32_t W, int32_t a, int32_t ap)
{
    if (a <= ap) return Ti[packed_index(W, a, ap)];
    return conj(Ti[packed_index(W, ap, a)]);
}

/* ---- Eq. 3 inner bracket: M_aa' = (1/N_gen) sum_j B_ja B*_ja' ------------ */
void oracle_mc_matrix(const double* Bri, int64_t n_acc, int32_t W, int64_t n_gen, double* Mri)
{
    const cplx* B = (const cplx*)Bri;
    cplx* M = (cplx*)Mri;
    const int64_t nc = n_chunks(n_acc);
    const int64_t WW = (int64_t)W * W;
    nsum* part = calloc((size_t)(nc > 0 ? nc : 1) * WW * 2, sizeof(nsum));

    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        nsum* p = part + c * WW * 2;
        int64_t j1 = (c + 1) * ORACLE_CHUNK < n_acc ? (c + 1) * ORACLE_CHUNK : n_acc;
        for (int64_t j = c * ORACLE_CHUNK; j < j1; ++j)
            for (int32_t a = 0; a < W; ++a)
                for (int32_t ap = 0; ap < W; ++ap) {
                    cplx x = B[j * W + a] * conj(B[j * W + ap]);
                    nsum_add(&p[2 * (a * W + ap)], creal(x));
                    nsum_add(&p[2 * (a * W + ap) + 1], cimag(x));
                }
    }
    for (int64_t k = 0; k < WW; ++k) {
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t c = 0; c < nc; ++c) {
            nsum_add(&re, nsum_value(&part[c * WW * 2 + 2 * k]));
            nsum_add(&im, nsum_value(&part[c * WW * 2 + 2 * k + 1]));
        }
        M[k] = (nsum_value(&re) + I * nsum_value(&im)) / (double)n_gen;
    }
    free(part);
}

/* ---- Sec. 2: the per-event lookup table T_i,aa' = A_ia A*_ia', a <= a' ---- */
void oracle_table_from_amplitudes(const double* Ari, int64_t N, int32_t W, double* Tri)
{
    const cplx* A = (const cplx*)Ari;
    cplx* T = (cplx*)Tri;
    const int64_t P = (int64_t)W * (W + 1) / 2;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int32_t a = 0; a < W; ++a)
            for (int32_t ap = a; ap < W; ++ap)
                T[i * P + packed_index(W, a, ap)] = A[i * W + a] * conj(A[i * W + ap]);
}

/* ---- Eq. 1: I_i = |sum_a V_a A_ia|^2 ------------------------------------ */
void oracle_intensity_amp(const double* Ari, int64_t N, int32_t W, const double* Vri, double* Iout)
{
    const cplx* A = (const cplx*)Ari;
    const cplx* V = (const cplx*)Vri;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        cplx s = 0;
        for (int32_t a = 0; a < W; ++a) s += V[a] * A[i * W + a];
        Iout[i] = creal(s) * creal(s) + cimag(s) * cimag(s);
    }
}

/* ---- Eq. 3 first bracket: I_i = sum_a sum_a' V_a V*_a' T_i,aa' ---------- */
static double intensity_table_one(const cplx* Ti, int32_t W, const cplx* V)
{
    cplx s = 0;
    for (int32_t a = 0; a < W; ++a)
        for (int32_t ap = 0; ap < W; ++ap)
            s += V[a] * conj(V[ap]) * table_entry(Ti, W, a, ap);
    return creal(s);   /* the imaginary part vanishes for Hermitian T */
}

void oracle_intensity_table(const double* Tri, int64_t N, int32_t W, const double* Vri, double* Iout)
{
    const cplx* T = (const cplx*)Tri;
    const cplx* V = (const cplx*)Vri;
    const int64_t P = (int64_t)W * (W + 1) / 2;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) Iout[i] = intensity_table_one(T + i * P, W, V);
}

/* ---- Eq. 3 second term: mu = sum_a sum_a' V_a V*_a' M_aa' ------------------ */
double oracle_mc_term(const double* Mri, int32_t W, const double* Vri, double* imag_part)
{
    const cplx* M = (const cplx*)Mri;
    const cplx* V = (const cplx*)Vri;
    nsum re = {0, 0}, im = {0, 0};
    for (int32_t a = 0; a < W; ++a)
        for (int32_t ap = 0; ap < W; ++ap) {
            cplx x = V[a] * conj(V[ap]) * M[a * W + ap];
            nsum_add(&re, creal(x));
            nsum_add(&im, cimag(x));
        }
    if (imag_part) *imag_part = nsum_value(&im);
    return nsum_value(&re);
}

/* Common tail: NLL = D + mu, G_b = 2 sum_a V_a (M_ab - U_ab). */
static void assemble(int32_t W, const cplx* M, const cplx* V, double sum_ln,
                     const cplx* U /* W*W, may be NULL */, int64_t nbad,
                     double* nll, double* grad)
{
    if (nbad > 0) {
        *nll = INFINITY;
        if (grad) for (int32_t k = 0; k < 2 * W; ++k) grad[k] = NAN;
        return;
    }
    *nll = -sum_ln + oracle_mc_term((const double*)M, W, (const double*)V, NULL);
    if (!grad) return;
    for (int32_t b = 0; b < W; ++b) {
        cplx g = 0;
        for (int32_t a = 0; a < W; ++a) g += V[a] * (M[a * W + b] - U[a * W + b]);
        g *= 2.0;
        grad[2 * b] = creal(g);
        grad[2 * b + 1] = cimag(g);
    }
}

/* ---- NLL (+ gradient) from a packed table ------------------------------ */
int64_t oracle_nll_table(const double* Tri, int64_t N, int32_t W, const double* Mri,
                         const double* Vri, double* nll, double* grad)
{
    const cplx* T = (const cplx*)Tri;
    const cplx* V = (const cplx*)Vri;
    const int64_t P = (int64_t)W * (W + 1) / 2;
    const int64_t WW = (int64_t)W * W;
    const int64_t nc = n_chunks(N);
    nsum* dpart = calloc((size_t)(nc > 0 ? nc : 1), sizeof(nsum));
    nsum* upart = grad ? calloc((size_t)(nc > 0 ? nc : 1) * WW * 2, sizeof(nsum)) : NULL;
    int64_t* bad = calloc((size_t)(nc > 0 ? nc : 1), sizeof(int64_t));

    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i1 = (c + 1) * ORACLE_CHUNK < N ? (c + 1) * ORACLE_CHUNK : N;
        for (int64_t i = c * ORACLE_CHUNK; i < i1; ++i) {
            const cplx* Ti = T + i * P;
            double Ii = intensity_table_one(Ti, W, V);
            if (!(Ii > 0.0) || !isfinite(Ii)) { bad[c]++; continue; }
            nsum_add(&dpart[c], log(Ii));
            if (!upart) continue;
            nsum* u = upart + c * WW * 2;
            for (int32_t a = 0; a < W; ++a)
                for (int32_t b = 0; b < W; ++b) {
                    cplx x = table_entry(Ti, W, a, b) / Ii;
                    nsum_add(&u[2 * (a * W + b)], creal(x));
                    nsum_add(&u[2 * (a * W + b) + 1], cimag(x));
                }
        }
    }

    nsum d = {0, 0};
    int64_t nbad = 0;
    for (int64_t c = 0; c < nc; ++c) { nsum_add(&d, nsum_value(&dpart[c])); nbad += bad[c]; }
    cplx* U = NULL;
    if (grad) {
        U = calloc((size_t)(WW > 0 ? WW : 1), sizeof(cplx));
        for (int64_t k = 0; k < WW; ++k) {
            nsum re = {0, 0}, im = {0, 0};
            for (int64_t c = 0; c < nc; ++c) {
                nsum_add(&re, nsum_value(&upart[c * WW * 2 + 2 * k]));
                nsum_add(&im, nsum_value(&upart[c * WW * 2 + 2 * k + 1]));
            }
            U[k] = nsum_value(&re) + I * nsum_value(&im);
        }
    }
    assemble(W, (const cplx*)Mri, V, nsum_value(&d), U, nbad, nll, grad);
    free(U); free(dpart); free(upart); free(bad);
    return nbad;
}

/* ---- NLL (+ gradient) from amplitudes, Eq. 1 inside Eq. 3 ---------------- */
int64_t oracle_nll_amp(const double* Ari, int64_t N, int32_t W, const double* Mri,
                       const double* Vri, double* nll, double* grad)
{
    const cplx* A = (const cplx*)Ari;
    const cplx* V = (const cplx*)Vri;
    const cplx* M = (const cplx*)Mri;
    const int64_t nc = n_chunks(N);
    nsum* dpart = calloc((size_t)(nc > 0 ? nc : 1), sizeof(nsum));
    nsum* gpart = grad ? calloc((size_t)(nc > 0 ? nc : 1) * W * 2, sizeof(nsum)) : NULL;
    int64_t* bad = calloc((size_t)(nc > 0 ? nc : 1), sizeof(int64_t));

    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i1 = (c + 1) * ORACLE_CHUNK < N ? (c + 1) * ORACLE_CHUNK : N;
        for (int64_t i = c * ORACLE_CHUNK; i < i1; ++i) {
            cplx s = 0;
            for (int32_t a = 0; a < W; ++a) s += V[a] * A[i * W + a];
            double Ii = creal(s) * creal(s) + cimag(s) * cimag(s);
            if (!(Ii > 0.0) || !isfinite(Ii)) { bad[c]++; continue; }
            nsum_add(&dpart[c], log(Ii));
            if (!gpart) continue;
            nsum* g = gpart + c * W * 2;
            for (int32_t b = 0; b < W; ++b) {
                cplx x = s * conj(A[i * W + b]) / Ii;
                nsum_add(&g[2 * b], creal(x));
                nsum_add(&g[2 * b + 1], cimag(x));
            }
        }
    }

    nsum d = {0, 0};
    int64_t nbad = 0;
    for (int64_t c = 0; c < nc; ++c) { nsum_add(&d, nsum_value(&dpart[c])); nbad += bad[c]; }
    if (nbad > 0 || !grad) {
        assemble(W, M, V, nsum_value(&d), NULL, nbad, nll, grad);
    } else {
        *nll = -nsum_value(&d) + oracle_mc_term(Mri, W, Vri, NULL);
        for (int32_t b = 0; b < W; ++b) {
            nsum re = {0, 0}, im = {0, 0};
            for (int64_t c = 0; c < nc; ++c) {
                nsum_add(&re, nsum_value(&gpart[c * W * 2 + 2 * b]));
                nsum_add(&im, nsum_value(&gpart[c * W * 2 + 2 * b + 1]));
            }
            cplx mv = 0;
            for (int32_t a = 0; a < W; ++a) mv += V[a] * M[a * W + b];
            cplx g = 2.0 * mv - 2.0 * (nsum_value(&re) + I * nsum_value(&im));
            grad[2 * b] = creal(g);
            grad[2 * b + 1] = cimag(g);
        }
    }
    free(dpart); free(gpart); free(bad);
    return nbad;
}

/* ---- FUMILI second derivatives --------------------------------------
 * The paper's fits use FUMILI with analytic gradients and Hessian (Sec. 5).
 * FUMILI replaces the Hessian of -ln L by the sum over events of the outer
 * products of the gradients of ln f, dropping the second derivatives of f.
 * For the extended likelihood of Eq. 3 the dropped part of the data term,
 * -sum_i (d2 I_i / dtheta2) / I_i, has the expectation -d2 mu / dtheta2 over
 * samples drawn from the model, so it cancels the Hessian of the MC term on
 * average and the matrix is the data sum alone (the observed information):
 *   theta = (Re V_0, Im V_0, Re V_1, ...),
 *   dI_i/dRe V_b = 2 Re(conj(S_i) A_ib),  dI_i/dIm V_b = -2 Im(conj(S_i) A_ib),
 *   J_i = grad_theta ln I_i = grad_theta I_i / I_i,   H = sum_i J_i J_i^T.
 * oracle_fumili_amp fills H (2W x 2W, row-major) and returns the number of
 * degenerate events (then H is NaN).  Per chunk and entry the event sums are
 * compensated, chunks added in order.
 */
int64_t oracle_fumili_amp(const double* Ari, int64_t N, int32_t W, const double* Vri, double* H)
{
    const cplx* A = (const cplx*)Ari;
    const cplx* V = (const cplx*)Vri;
    const int32_t P = 2 * W;
    const int64_t nc = n_chunks(N);
    nsum* hpart = calloc((size_t)(nc > 0 ? nc : 1) * P * P, sizeof(nsum));
    int64_t* bad = calloc((size_t)(nc > 0 ? nc : 1), sizeof(int64_t));

    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i1 = (c + 1) * ORACLE_CHUNK < N ? (c + 1) * ORACLE_CHUNK : N;
        double* J = malloc(sizeof(double) * P);
        nsum* h = hpart + c * P * P;
        for (int64_t i = c * ORACLE_CHUNK; i < i1; ++i) {
            cplx s = 0;
            for (int32_t a = 0; a < W; ++a) s += V[a] * A[i * W + a];
            double Ii = creal(s) * creal(s) + cimag(s) * cimag(s);
            if (!(Ii > 0.0) || !isfinite(Ii)) { bad[c]++; continue; }
            for (int32_t b = 0; b < W; ++b) {
                cplx z = conj(s) * A[i * W + b];
                J[2 * b] = 2.0 * creal(z) / Ii;
                J[2 * b + 1] = -2.0 * cimag(z) / Ii;
            }
            for (int32_t p = 0; p < P; ++p)
                for (int32_t q = 0; q < P; ++q) nsum_add(&h[p * P + q], J[p] * J[q]);
        }
        free(J);
    }
    int64_t nbad = 0;
    for (int64_t c = 0; c < nc; ++c) nbad += bad[c];
    for (int32_t p = 0; p < P; ++p)
        for (int32_t q = 0; q < P; ++q) {
            nsum t = {0, 0};
            for (int64_t c = 0; c < nc; ++c) nsum_add(&t, nsum_value(&hpart[c * P * P + p * P + q]));
            H[p * P + q] = nbad > 0 ? NAN : nsum_value(&t);
        }
    free(hpart);
    free(bad);
    return nbad;
}
