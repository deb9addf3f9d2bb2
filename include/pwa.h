/*
 * pwa.h -- C ABI of the MI355X partial-wave-analysis likelihood library.
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the extended
 * unbinned negative log-likelihood of a partial-wave fit and its analytic
 * gradient (arXiv:1108.5673, Sec. 2, Eq. 3):
 *
 *   NLL(V) = - sum_i ln I_i(V) + mu(V)
 *   I_i(V) = sum_a sum_a' V_a V*_a' T_i,aa',   T_i,aa' = A_a(Omega_i) A*_a'(Omega_i)
 *   mu(V)  = sum_a sum_a' V_a V*_a' M_aa',     M_aa' = (1/N_gen) sum_{j acc} B_ja B*_ja'
 *
 * where V (W complex numbers) are the production amplitudes being fitted,
 * A the decay amplitudes of the N data events and B those of the accepted
 * Monte Carlo events.  No constant is added to Eq. 3.  The gradient is
 * returned with respect to the real and imaginary parts of V:
 *   grad[2b] = dNLL/dRe V_b,  grad[2b+1] = dNLL/dIm V_b.
 *
 * Because masses and widths are fixed during the fit, the per-event products
 * T_i and the MC matrix M are computed once, when the model is built
 * (Sec. 2, the paragraph after Eq. 3); each evaluation then streams the
 * device-resident table and moves only V to the device and the NLL and
 * gradient back (Sec. 5: only fit parameters, likelihood and derivatives
 * cross the bus).
 *
 * Conventions for every function:
 *   - Complex numbers are interleaved (re, im) pairs; arrays are row-major.
 *   - V, nll and grad are host pointers.  V has 2W doubles (re, im per wave).
 *   - Each evaluation call is synchronous: it enqueues its work on hip_stream
 *     (a hipStream_t; NULL means the default stream) and returns once the
 *     results are in host memory (the last kernel writes them to pinned host
 *     memory; the call polls a completion word and reports stream errors).
 *   - No exception or abort crosses the ABI.  Every function returns a status
 *     (pwa_status); pwa_last_error() gives a message for the last non-OK
 *     status of the calling thread.
 *   - A model is not safe for concurrent calls from several threads: it owns
 *     one set of scratch buffers.  Distinct models may be used concurrently.
 *   - Degenerate events: if any event has I_i <= 0 or a non-finite I_i the
 *     likelihood is undefined; the call returns PWA_WARN_DEGENERATE, sets
 *     *nll = +INFINITY and fills grad with NaN.  Nothing is clamped.
 */
#ifndef PWA_H
#define PWA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwa_model pwa_model;

typedef enum pwa_status {
    PWA_OK = 0,
    PWA_WARN_DEGENERATE = 1,      /* some I_i <= 0 or non-finite: *nll = +INFINITY, grad NaN   */
    PWA_ERR_INVALID = -1,         /* bad argument (NULL pointer, size out of range, bad flags) */
    PWA_ERR_OOM = -2,             /* device or pinned host allocation failed                   */
    PWA_ERR_DEVICE = -3,          /* a HIP runtime call or kernel launch failed                */
    PWA_ERR_NO_DEVICE = -4,       /* no HIP device is visible to this process                  */
    PWA_ERR_NONFINITE_INPUT = -5  /* V holds a NaN or infinity                                 */
} pwa_status;

typedef enum pwa_flags {
    /* Evaluation form (exactly one of the six must be given). */
    PWA_FORM_TABLE = 1,              /* complex64 packed table, fused one-pass NLL+gradient kernel */
    PWA_FORM_AMPLITUDE = 2,          /* complex64 amplitudes, S_i = sum_a V_a A_ia per event (Eq. 1) */
    PWA_PRECISION_FP64_PLAIN = 8,    /* complex128 packed table, plain two-pass FP64 kernels       */
    PWA_PRECISION_FP64_FUSED = 64,   /* complex128 packed table, fused one-pass kernel            */
    PWA_FORM_AMPLITUDE_BF16 = 128,   /* amplitudes stored in bfloat16, matrix-core kernel that
                                        evaluates any number of V together (S = A V as a GEMM)  */
    PWA_FORM_AMPLITUDE_FP16 = 256,   /* the same with amplitudes stored in float16               */
    /* Input description. */
    PWA_INPUT_IS_TABLE = 4,          /* `data` is an N x P packed Hermitian table, P = W(W+1)/2,
                                        entries (a, a') with a <= a' in row-major order of the
                                        upper triangle; any Hermitian positive semi-definite
                                        per-event table is accepted, not only rank one.  A
                                        diagonal entry with a non-zero imaginary part makes
                                        the build fail with PWA_ERR_INVALID (the stored
                                        table keeps the diagonal real).  Table forms only.     */
    PWA_DATA_COMPLEX128 = 16,        /* `data` elements are complex128 (default complex64)        */
    PWA_MC_COMPLEX128 = 32           /* `mc_amp` elements are complex128 (default complex64)      */
} pwa_flags;

/* Largest wave count per form. */
#define PWA_MAX_WAVES_TABLE 64
#define PWA_MAX_WAVES_AMPLITUDE 128
#define PWA_MAX_WAVES_MATRIX 64      /* PWA_FORM_AMPLITUDE_BF16 / _FP16 */

/*
 * pwa_build_table -- build a model: the per-event table (or the device copy
 * of the amplitudes) and the MC matrix M (Sec. 2, Eq. 3 and the paragraph
 * after it).
 *
 *   data      N x W amplitudes A_ia, or with PWA_INPUT_IS_TABLE an N x P packed
 *             table; complex64 unless PWA_DATA_COMPLEX128.  Host or device
 *             memory (detected).  Copied: the caller keeps ownership and may
 *             free it when the call returns.
 *   n_data    N >= 1.
 *   n_waves   W, 1 <= W <= PWA_MAX_WAVES_TABLE (table forms),
 *             PWA_MAX_WAVES_AMPLITUDE (amplitude form) or PWA_MAX_WAVES_MATRIX
 *             (16-bit amplitude forms).
 *   mc_amp    N_acc x W accepted MC amplitudes B_ja (complex64 unless
 *             PWA_MC_COMPLEX128), host or device; copied.  May be NULL only
 *             when n_mc_acc == 0, which gives M = 0.
 *   n_mc_acc  N_acc >= 0.
 *   n_mc_gen  N_gen >= 1, the number of generated MC events (Eq. 3 divides by
 *             it, not by N_acc).
 *   flags     pwa_flags.
 *   out       receives the new model; *out is NULL on error.
 *
 * Before anything is allocated or copied, the build estimates its peak device
 * memory (staged input, stored table or amplitudes, MC staging and records)
 * and returns PWA_ERR_OOM, with the estimate and the free memory in
 * pwa_last_error(), when hipMemGetInfo reports less free.
 *
 * Table forms compute T_i,aa' in FP64 from the given amplitudes (each product
 * formed with a separately rounded multiply and add) and store it at the
 * form's precision, rounded to nearest.  M is accumulated in FP64.  The
 * amplitude form keeps the amplitudes in complex64 (complex128 input is
 * rounded to nearest).  The 16-bit amplitude forms store the real and
 * imaginary parts in bfloat16 or float16, rounded to nearest from complex64
 * (complex128 input is rounded to float first; float16 results below 2^-14 in
 * magnitude are stored as zero); they evaluate through the
 * matrix cores: each call, single or batched, runs one pass over the events
 * for all its vectors, with V split into two 16-bit parts (16 significant bits
 * for bfloat16, 22 for float16; the first-order share of the NLL of what the
 * parts leave out is added back), FP32 products and FP64 sums across events.
 */
int pwa_build_table(const void* data, int64_t n_data, int32_t n_waves,
                    const void* mc_amp, int64_t n_mc_acc, int64_t n_mc_gen,
                    uint32_t flags, void* hip_stream, pwa_model** out);

/*
 * pwa_nll -- NLL(V) of Eq. 3.  v: 2W doubles (host).  *nll receives the value.
 */
int pwa_nll(const pwa_model* model, const double* v, double* nll, void* hip_stream);

/*
 * pwa_nll_grad -- NLL(V) and its gradient in one pass over the events.
 * grad receives 2W doubles: dNLL/dRe V_b, dNLL/dIm V_b.  The gradient is
 *   G_b = 2 sum_a V_a (M_ab - U_ab),  U_ab = sum_i T_i,ab / I_i
 * (the derivative of Eq. 3; the paper's fitter uses analytic gradients,
 * Sec. 4 and Sec. 5).
 */
int pwa_nll_grad(const pwa_model* model, const double* v, double* nll, double* grad,
                 void* hip_stream);

/*
 * Asynchronous twins of pwa_nll and pwa_nll_grad for stream-ordered use and
 * HIP graph capture: V is read from device memory (v_dev, 2W doubles) when the
 * work runs, and the results are written to device memory
 * (out_dev = [nll, n_bad, grad 2W]; pwa_nll_async writes the first two).  The
 * call only enqueues kernels on hip_stream and returns: it allocates nothing,
 * records no memset or copy and touches no host memory, so it can be captured
 * and replayed, each replay reading the V then in v_dev.  Nothing is checked
 * on V (a non-finite V gives non-finite results).  A degenerate evaluation
 * has n_bad > 0, nll = +INFINITY and a NaN gradient.  All forms but the
 * 16-bit matrix forms.  Evaluations of one model share its scratch buffers:
 * they must be ordered on one stream (or captured in one graph branch), also
 * with respect to its synchronous calls.  A captured graph holds the model's
 * device buffers: while it may still be replayed, the model must not be freed
 * or re-shaped (pwa_set_amplitude_shape, pwa_tune_amplitude_shape).
 */
int pwa_nll_async(const pwa_model* model, const double* v_dev, double* out_dev,
                  void* hip_stream);
int pwa_nll_grad_async(const pwa_model* model, const double* v_dev, double* out_dev,
                       void* hip_stream);

/*
 * pwa_nll_batched -- many parameter sets, possibly on several models (fits
 * repeated from several starting points and several models tried, Sec. 2).
 *
 *   models       n_models model handles.
 *   k_per_model  K_m >= 0 parameter sets for model m.
 *   v            concatenation over m of K_m x 2W_m doubles.
 *   nll          sum_m K_m doubles (same order).
 *   grad         sum_m K_m x 2W_m doubles, or NULL for NLL only.
 *
 * Returns PWA_WARN_DEGENERATE if any evaluation is degenerate (those entries
 * are +INFINITY / NaN); other entries are valid.  The K_m evaluations of a
 * model are queued back to back and waited for once.  When every model is of
 * PWA_FORM_AMPLITUDE (and there are at least two evaluations), the call runs
 * as one work list replayed from a captured HIP graph: the plans (work list,
 * buffers, graph) of the 8 most recent distinct (model, K) lists are kept, so
 * that alternating model sets replay without a new capture; freeing or
 * re-shaping a model drops the plans that use it.
 */
int pwa_nll_batched(pwa_model* const* models, int32_t n_models, const int32_t* k_per_model,
                    const double* v, double* nll, double* grad, void* hip_stream);

/*
 * pwa_nll_batched_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the K-vector evaluation of pwa_nll_batched on one model of a
 * 16-bit amplitude form (PWA_FORM_AMPLITUDE_BF16 / _FP16), with every buffer
 * of its kernels in a static device array of 16 MiB that the library holds on
 * each device it runs on until the process ends.  It allocates nothing and
 * only enqueues kernels on hip_stream (no memset, no copy, no host memory
 * touched, no wait), so it can be captured and replayed.
 *
 *   k        1 <= k <= 1024 parameter vectors.
 *   v_dev    k x 2W doubles in device memory, read when the work runs.
 *   out_dev  k x (2 + 2W) doubles in device memory: per vector
 *            [nll, n_bad, grad 2W]; a degenerate evaluation has n_bad > 0,
 *            nll = +INFINITY and a NaN gradient.
 * Returns PWA_ERR_INVALID for another form, for k out of range, or when the k
 * vectors' buffers at this W exceed the static array (the split vector matrix
 * and the records of at least one event chunk must fit); nothing is enqueued
 * then.  When the records of the event chunks pwa_nll_batched would use fit,
 * the results equal pwa_nll_batched's bit for bit; otherwise the events are cut
 * into fewer chunks and the results agree within the FP32 accumulation error
 * of the longer chunks.  Every call on one device shares that device's array:
 * calls that overlap on one GPU (concurrent streams, or host threads without
 * stream order between them) race and give wrong results.
 */
int pwa_nll_batched_noalloc(const pwa_model* model, int32_t k, const double* v_dev,
                            double* out_dev, void* hip_stream);

/*
 * pwa_nll_grad_hess -- NLL, gradient and the FUMILI second-derivative matrix
 * in one call (the paper's fits use FUMILI with analytic derivatives and ship
 * likelihood, gradient and this matrix per iteration, Sec. 5).  Amplitude form
 * (PWA_FORM_AMPLITUDE) only.
 *
 *   hess  2W x 2W doubles, row-major, over theta = (Re V_0, Im V_0, Re V_1, ...):
 *         H = sum_i J_i J_i^T with J_i = grad_theta ln I_i, in FP64.  FUMILI
 *         replaces the Hessian of -ln L by these outer products, dropping the
 *         second derivatives of I_i; for the extended likelihood of Eq. 3 the
 *         dropped terms cancel the Hessian of the MC term on average over
 *         samples drawn from the model, so neither appears (H is the observed
 *         information, positive semidefinite, with the global-phase direction
 *         i V in its null space).
 * Degenerate events: as pwa_nll_grad, and hess is NaN.
 */
int pwa_nll_grad_hess(const pwa_model* model, const double* v, double* nll, double* grad,
                      double* hess, void* hip_stream);

/* pwa_free -- release a model and all device memory it owns.  NULL is ignored. */
void pwa_free(pwa_model* model);

/* pwa_last_error -- message for the last non-OK status of the calling thread. */
const char* pwa_last_error(void);

/*
 * Inspection.  pwa_model_info fills, in order: N, W, P, form flag,
 * bytes streamed from device memory per single-V evaluation by the main
 * kernel (the algorithmic traffic: table or amplitude bytes, padding
 * excluded), grid size of the main kernel, and the number of compute units.
 */
typedef struct pwa_info {
    int64_t n_data;
    int32_t n_waves;
    int32_t n_packed;
    uint32_t form;
    int64_t stream_bytes;
    int32_t grid_blocks;
    int32_t compute_units;
} pwa_info;
int pwa_model_info(const pwa_model* model, pwa_info* out);

/* Copy the model's table back in the canonical packed N x P layout (complex64
 * for PWA_FORM_TABLE, complex128 for the FP64 forms); for the amplitude forms,
 * the stored amplitudes as complex64, N x W row-major (widened from the
 * 16-bit forms). */
int pwa_copy_table(const pwa_model* model, void* out_host, void* hip_stream);

/*
 * Storage shape of a PWA_FORM_AMPLITUDE model (Eq. 1: S_i = sum_a V_a A_ia).
 * Each event's amplitudes are spread over lanes_per_event (1, 2, 4, 8 or 16)
 * neighbouring lanes of a wavefront, each holding waves_per_lane (even, 2..16)
 * of its waves; rows are padded with zero waves to lanes x waves_per_lane >= W.
 * pwa_build_table picks the shape with the fewest padded waves, counting rows
 * of more than 10 waves per lane 25 % longer (such lanes need more registers,
 * which halves the wavefronts in flight); among equal costs, the largest
 * waves_per_lane up to 10, else the smallest.
 *
 * pwa_set_amplitude_shape re-stores the amplitudes in another shape (device
 * memory for one extra N x W complex64 copy is taken while it runs); it
 * returns PWA_ERR_INVALID for a shape that does not hold W waves.  Results of
 * every shape agree to FP64 rounding; for a given shape they repeat bit for
 * bit.  pwa_tune_amplitude_shape times `evals` gradient evaluations of the
 * streaming kernel in each candidate shape (per lane count, the fewest waves
 * per lane that hold W, when the row is at most 25 % longer than the
 * shortest), three times over the candidates keeping each one's fastest and
 * slowest time; it leaves the default shape unless a candidate's fastest time
 * beats the default's by more than the spread (slowest minus fastest) of
 * either, leaves the model in the shape chosen and returns it (either output
 * pointer may be NULL).  Both synchronise hip_stream and must not run
 * concurrently with evaluations of the model; cached multi-model plans that
 * use the model are rebuilt at their next call.
 */
int pwa_get_amplitude_shape(const pwa_model* model, int32_t* lanes_per_event,
                            int32_t* waves_per_lane);
int pwa_set_amplitude_shape(pwa_model* model, int32_t lanes_per_event, int32_t waves_per_lane,
                            void* hip_stream);
int pwa_tune_amplitude_shape(pwa_model* model, int32_t evals, void* hip_stream,
                             int32_t* lanes_per_event, int32_t* waves_per_lane);

/* Copy M (W x W complex128, row-major) to host memory. */
int pwa_copy_mc_matrix(const pwa_model* model, double* out_host, void* hip_stream);

/* Replace M by a caller-supplied W x W complex128 Hermitian matrix (host). */
int pwa_set_mc_matrix(pwa_model* model, const double* m_host, void* hip_stream);

/*
 * Kernel timing: with enable = k > 0, every k-th evaluation (the first, then
 * every k-th after it; 1 = all) has the runtime stamp two HIP events with the
 * begin and end of the main (event-streaming) kernel's dispatch on the
 * evaluation's stream (for PWA_PRECISION_FP64_PLAIN, the begin of the first
 * pass and the end of the second); enable = 0 turns timing off.  A stamped
 * launch costs the evaluation some microseconds, so sampling every k-th keeps
 * a throughput measurement close to an untimed one.  The events are read back
 * lazily: pwa_get_timing returns the accumulated device time of the timed
 * kernels in milliseconds and their number, and resets both.
 */
int pwa_set_timing(pwa_model* model, int enable);
int pwa_get_timing(pwa_model* model, double* total_ms, int64_t* launches);

/*
 * Device time of the two build steps that bracket the fit (Sec. 5, Table 1:
 * the MC integral and the lookup-table creation), measured with HIP events
 * when the model was built, in milliseconds: table_ms covers the preparation
 * of the table (or the amplitude copy) from the device-resident input, mc_ms
 * the MC integral M (0 when n_mc_acc == 0).  Staging host inputs to the device
 * is not included.  For the table forms and the MC integral the interval
 * starts when the first kernel is dispatched (a first launch's host-side set-up
 * is not counted); for the other forms it starts with a plain event.
 */
int pwa_build_timing(const pwa_model* model, double* table_ms, double* mc_ms);

/*
 * Achievable read bandwidth on the model's stored data (the measurement
 * reference for the streaming kernels' HBM roofline).  For the tiled tables
 * (PWA_FORM_TABLE, PWA_PRECISION_FP64_FUSED) it runs the fused kernel's own
 * loads (same grid, block shape, sub-tile order and register double
 * buffering) with all arithmetic taken out; for the other forms a plain reader
 * (one 1024-thread block per compute unit, 1 KB per wavefront load, two
 * register buffers) that reads every stored byte once with the same
 * non-temporal 16-byte loads.  One untimed pass, then reps timed ones (HIP
 * events around the dispatch); *ms is the fastest, *bytes the bytes read per
 * pass.  Synchronises hip_stream; allocates a small device buffer for the
 * duration.
 */
int pwa_read_ceiling(const pwa_model* model, int32_t reps, void* hip_stream, double* ms,
                     int64_t* bytes);

/*
 * ---- Fit driver: limited-memory BFGS ---------------------------------------
 *
 * The fits of Sec. 2 minimise Eq. 3 with analytic derivatives, repeated from
 * several starting points.  pwa_lbfgs_minimize is a general minimiser (the
 * two-loop L-BFGS recursion with a strong Wolfe line search, Nocedal and
 * Wright, Numerical Optimization, Algorithms 7.4, 3.5 and 3.6) over a caller
 * objective; pwa_fit_lbfgs drives it with pwa_nll_grad on a model.
 *
 * pwa_objective: fills *f and g[n] at x[n]; returns 0, or a negative status
 * to abort the minimisation (returned unchanged).  A non-finite *f is taken as
 * a point outside the domain: the line search shortens the step.
 */
typedef int (*pwa_objective)(void* ctx, const double* x, double* f, double* g);

typedef struct pwa_lbfgs_options {
    int32_t max_iterations;  /* default 2000                                           */
    int32_t history;         /* correction pairs kept, default 10                      */
    double grad_tol;         /* stop when ||g||_2 <= grad_tol * max(1, |f|); 1e-9      */
    double rel_f_tol;        /* stop after 3 iterations each lowering f by at most
                                rel_f_tol * max(1, |f|); default 1e-15; 0 = off        */
    int32_t fixed_index;     /* coordinate held at its start value, or -1 (default)    */
} pwa_lbfgs_options;

enum {
    PWA_LBFGS_CONVERGED_GRADIENT = 0,
    PWA_LBFGS_CONVERGED_VALUE = 1,
    PWA_LBFGS_MAX_ITERATIONS = 2,
    PWA_LBFGS_LINE_SEARCH_FAILED = 3
};

typedef struct pwa_lbfgs_result {
    int32_t status;          /* PWA_LBFGS_*                                            */
    int32_t iterations;
    int32_t evaluations;     /* objective calls, line-search trials included           */
    double f;                /* objective at the returned x                            */
    double grad_norm;        /* ||g||_2 there (fixed coordinate excluded)              */
} pwa_lbfgs_result;

/* Fill `opt` with the defaults above. */
void pwa_lbfgs_default_options(pwa_lbfgs_options* opt);

/*
 * Minimise fn from x (n values, overwritten with the result).  options may be
 * NULL for the defaults.  Returns PWA_OK (then res->status says how it
 * stopped), PWA_WARN_DEGENERATE if f is not finite at the start,
 * PWA_ERR_INVALID for bad arguments, or the objective's negative status.
 */
int pwa_lbfgs_minimize(int32_t n, double* x, pwa_objective fn, void* ctx,
                       const pwa_lbfgs_options* options, pwa_lbfgs_result* res);

/*
 * Fit V on a model: minimise NLL(V) from v (2W doubles, host, overwritten with
 * the fitted V).  The NLL is invariant under a global phase of V, so the start
 * is first rotated to make V_0 real and non-negative and Im V_0 is then held
 * at zero (options->fixed_index is ignored); Re V_0 may change sign.  The
 * start is then scaled to the minimum of Eq. 3 along its ray, s^2 = N / mu(V),
 * when mu(V) > 0 (a start whose scale is far off otherwise takes the
 * minimiser through other basins of the likelihood).  Each objective call is
 * one pwa_nll_grad on hip_stream.
 */
int pwa_fit_lbfgs(const pwa_model* model, double* v, const pwa_lbfgs_options* options,
                  pwa_lbfgs_result* res, void* hip_stream);

/*
 * ---- Fit driver: damped Newton steps on the FUMILI matrix ------------------
 *
 * pwa_objective_hess fills *f and g[n] at x[n], and H[n x n] (row-major) when
 * H is not NULL; returns 0 or a negative status.  pwa_newton_minimize solves
 * (H + lambda diag H) d = -g by Cholesky (lambda raised until the matrix is
 * positive definite) and takes x + d when the decrease of f is at least 1e-4 of
 * the decrease the quadratic model predicts, -(g.d + d.H.d / 2); lambda is then
 * divided by 5 (ratio above 0.75) or multiplied by 4 (below 0.25); a step not
 * taken leaves x and multiplies lambda by 4 (Levenberg-Marquardt damping of the
 * Gauss-Newton steps that FUMILI takes).  Trial points are evaluated with
 * H = NULL; H is asked for at the points taken.  Options and result as for
 * L-BFGS (history is unused; evaluations counts both kinds of call).
 * pwa_fit_fumili fits V on an amplitude-form model with pwa_nll_grad at trial
 * points and pwa_nll_grad_hess at the points taken, with the gauge of
 * pwa_fit_lbfgs, after scaling the start to the minimum of Eq. 3 along its
 * ray, s^2 = N / mu(V) (the data term changes by -N ln s^2, the MC term by the
 * factor s^2), when mu(V) > 0: along V the FUMILI matrix has the curvature 4N
 * and Eq. 3 the curvature 2N + 2 mu(V), equal there.
 */
typedef int (*pwa_objective_hess)(void* ctx, const double* x, double* f, double* g, double* H);

int pwa_newton_minimize(int32_t n, double* x, pwa_objective_hess fn, void* ctx,
                        const pwa_lbfgs_options* options, pwa_lbfgs_result* res);

int pwa_fit_fumili(const pwa_model* model, double* v, const pwa_lbfgs_options* options,
                   pwa_lbfgs_result* res, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PWA_H */
