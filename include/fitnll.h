/*
 * fitnll.h -- C ABI of libfitnll.so, an unbinned maximum-likelihood engine for
 * AMD Instinct MI355X (gfx950).
 *
 * What it computes.  Fitting a probability density to a data sample spends
 * nearly all its time evaluating the density independently at every event of
 * the sample (GooFit 2.0, Sec. 1).  The library evaluates, for a model (a
 * composed density: basic components added with fractions, or a coherent sum
 * of complex resonance amplitudes whose magnitude squared is the density,
 * Sec. 1 and 5), a parameter vector theta and an event sample x_1..x_N:
 *
 *     NLL(theta) = - sum_i ln P~(x_i | theta) + N ln I(theta),
 *     I(theta)   = integral of P~ over the observable domain,
 *
 * and optionally dNLL/dtheta by a hand-written adjoint pass.  This is the
 * objective function the paper's fitters hand to Minuit (Sec. 4); the fitter
 * itself (a quasi-Newton minimizer) and many-fits-per-launch batching sit on
 * top of the same kernels.
 *
 * Conventions shared by every entry point:
 *  - Every call returns fn_status; FN_OK is 0, errors are negative.  On error
 *    fn_last_error() returns a message (thread-local, owned by the library,
 *    valid until the next fn_* call on the same thread).  The paper unified
 *    its errors in one exception type (Sec. 3); this is the C form of that.
 *  - Floating point is IEEE binary64 throughout.
 *  - Events are caller-owned DEVICE memory in structure-of-arrays layout:
 *    observable j of event i is at ev[j*ld + i], ld >= n.  The library never
 *    frees or writes them; they must stay valid until the stream work that
 *    reads them has completed.  (The paper credits its structure-of-arrays
 *    layout for speed, Sec. 4.)
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Entry
 *    points documented as synchronous return after the stream work is done;
 *    *_async ones only enqueue work.
 *  - A model may be used from one host thread and one stream at a time.
 *  - Results are deterministic: the event sum is a fixed two-level tree
 *    (a fixed chunk of events per workgroup, then a fixed-order sum of the
 *    chunk partials), so repeated calls, and the same fit alone or inside a
 *    batch, give bitwise identical values.
 *  - Non-finite or non-positive P~ at any event (or I <= 0) makes the NLL
 *    +inf, the gradient NaN, and the call returns FN_E_NONFINITE; a minimizer
 *    treats that as a rejected step.
 */
#ifndef FITNLL_H
#define FITNLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fn_status;
enum {
  FN_OK = 0,
  FN_E_INVALID = -1,   /* bad argument or malformed model description */
  FN_E_DOMAIN = -2,    /* events outside the observable domain */
  FN_E_NONFINITE = -3, /* NLL not finite (P~ <= 0, NaN parameters, I <= 0) */
  FN_E_NOMEM = -4,     /* device or pinned host allocation failed */
  FN_E_HIP = -5,       /* a HIP runtime call failed; message has its text */
  FN_E_BUDGET = -6,    /* request larger than the memory budget */
  FN_E_CANCELLED = -7  /* request cancelled before it finished */
};

/* Message for the last failing call on this thread ("" if none). */
const char* fn_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int32_t fn_version(void);

/* ---------------------------------------------------------------- context */
typedef struct fn_ctx fn_ctx;
/* One context per device; `device` is a HIP device ordinal.  The context owns
 * nothing but the device binding; models hold their own buffers. */
fn_status fn_ctx_create(int32_t device, fn_ctx** out);
fn_status fn_ctx_destroy(fn_ctx* ctx);

/* ------------------------------------------------------------------ model */
typedef struct fn_model fn_model;

/* Compile a model description (JSON text, UTF-8) into a device model.
 *
 * Models follow the paper's composition (Fig. 1): observables with ranges,
 * parameters addressed by index, components combined into one density.
 * Integers in the description are indices into theta.
 *
 *  kind "mix1d":  {"kind":"mix1d","lo":a,"hi":b,"n_params":P,
 *                  "components":[{"type":T,"params":[i,j]},...],"fracs":[...]}
 *     T in gauss(mu,sigma), exp(tau), argus(m0,c) [power 1/2, c<0, lo>=0],
 *     bw(m0,gamma) [non-relativistic].  K components take K-1 fractions; the
 *     last gets 1 - sum.  Each component is normalized analytically on
 *     [lo,b], so I = 1.  One observable.  Optional "yield": i makes the
 *     likelihood extended with expected count nu = theta[i] > 0: the NLL of
 *     N events gains nu - N ln nu, and binned data take nu as their total.
 *  kind "dalitz3": {"kind":"dalitz3","M":..,"m":[m1,m2,m3],"r_res":r,
 *                  "r_D":rD,"grid":[nx,ny],"free_lineshapes":bool,
 *                  "resonances":[{"pair":"12"|"13"|"23","L":0|1|2,
 *                                 "m0":..,"w0":..},...]}
 *     Two observables (s12, s13).  P~ = |sum_k c_k A_k|^2 with relativistic
 *     Breit-Wigner lineshapes (mass-dependent width, Blatt-Weisskopf
 *     barriers) times Zemach spin factors; I is the midpoint rule on an
 *     nx x ny grid over the Dalitz bounding box, cells counted when their
 *     centre is inside the physical region.  theta = (Re c_k, Im c_k)_k, then
 *     (m0_k, Gamma0_k)_k when free_lineshapes is true.  Up to 16 resonances.
 *     With fixed lineshapes the grid is reduced once to the Hermitian matrix
 *     M_ij = dA sum_cells A_i conj(A_j) and I = c^H M c afterwards (the
 *     paper's caching of partial results while parameters are unchanged,
 *     Sec. 4).
 *  kind "td4":   {"kind":"td4","M":..,"m":[m1,m2,m3,m4],"r_res":r,"tau":..,
 *                 "sigma_t":..,"r12":[{"L":0|1,"m0":..,"w0":..},...],
 *                 "r34":[...],"amps":[[i12,i34,type],...]}
 *     The time-dependent four-body amplitude model (the paper's four-body
 *     time-dependent analyses, Abstract and Sec. 5).  Six observables
 *     (m12, m34, cos theta12, cos theta34, phi, t).  Basis amplitudes
 *     B_k = a12[i12] a34[i34] Omega_type with relativistic Breit-Wigner
 *     lineshapes (m0 = 0 marks a flat non-resonant entry; L = 0 or 1; up to 4
 *     entries per pair) and helicity angular factors: type 0 -> 1, 1 -> c34,
 *     2 -> c12, 3 -> c12 c34, 4/5 -> sin12 sin34 exp(+-i phi) / 2.  A = sum c_k B_k,
 *     Abar = sum cbar_k B_k (up to 12 amplitudes); the rate mixes them with
 *     decay time through Gamma = 1/tau and mixing parameters x, y, convolved
 *     with a Gaussian time resolution of width sigma_t.  I is the average of
 *     the time-integrated rate over a phase-space sample that must be given
 *     with fn_model_set_norm_sample before the first evaluation.
 *     theta = (Re c_k, Im c_k)_k, (Re cbar_k, Im cbar_k)_k, x, y  (P = 4K + 2).
 *     The lineshape constants and sigma_t form the model's fixed-constant
 *     vector (fn_model_fixed): (m0, w0) of every r12 entry, of every r34
 *     entry, then sigma_t.
 *  Optional keys for every kind: "chunk" (events per workgroup, a multiple of
 *  256 in [256, 2^22], default chosen per kind) -- fixed per model, it
 *  defines the summation tree.  dalitz3 only: "events_per_thread" (1, the
 *  default, or 2: events each thread of the events passes evaluates per loop
 *  iteration; a thread adds its events in index order either way, so the
 *  results are bitwise the same).
 * Returns FN_E_INVALID with a message for a malformed description. */
fn_status fn_model_create(fn_ctx* ctx, const char* desc_json, fn_model** out);
/* Compile a description's structure-specialized kernels for the GPU
 * architecture `arch` (NULL or "" = "gfx950") without a device and without
 * loading them: the same runtime compilation fn_model_create performs (it
 * specializes the per-event passes of amplitude models to their structure).
 * Returns FN_E_INVALID with the compiler log for a description that does not
 * compile.  Needs no GPU. */
fn_status fn_model_check_compile(const char* desc_json, const char* arch);
/* Number of parameters, observables, and the summation chunk of a model. */
fn_status fn_model_info(const fn_model* m, int32_t* n_params, int32_t* n_obs, int32_t* chunk);
/* Frees the model's device memory.  Streams using it must be synchronised. */
fn_status fn_model_destroy(fn_model* m);
/* Autotuner of the summation chunk (events per workgroup; it also fixes the
 * order of the sums) and, for dalitz3, of the events per thread and loop
 * iteration of the events passes (1 or 2; the sums are bitwise the same):
 * times the full NLL + gradient evaluation at theta (host, P doubles) on the
 * caller's events (device, as fn_nll) for each candidate (3 warm-up calls,
 * then the median of reps timed calls, HIP events on `stream`; reps < 1 means
 * 20).  Among the candidates within 2% of the fastest it keeps one event per
 * thread if any has it, then the largest chunk; the choice becomes the
 * model's (reported by fn_model_info, used by every later evaluation and by
 * batches created afterwards) and is written to *chunk_out and *ept_out
 * (each may be NULL).  The chunk candidates are the powers of two 256 ..
 * 16384, then the multiples of 256 that give the sample j x (number of
 * compute units) workgroups, j = 1 .. 8 (workgroup counts that fill the
 * device's resident slots evenly), where they differ from the first.
 * chunks_out (NULL or FN_TUNE_MAX entries) receives the chunk candidates in
 * the order tried, unused entries 0; us_out (NULL or FN_TUNE_EPT x
 * FN_TUNE_MAX entries) their median times in microseconds, one event per
 * thread in entries 0 .. FN_TUNE_MAX - 1, two from FN_TUNE_MAX on, NaN where
 * nothing was timed.  The workgroup size is fixed (256 threads: the
 * two-level sums and their LDS layout are built for four wave64s).
 * Synchronous.  FN_E_INVALID for NULL theta, n < 1 or bad event arguments;
 * the model keeps its previous choice on any error. */
#define FN_TUNE_MAX 16
#define FN_TUNE_EPT 2
fn_status fn_model_autotune(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld,
                            int32_t reps, int32_t* chunk_out, int32_t* ept_out, int32_t* chunks_out, double* us_out,
                            void* stream);

/* Count events outside the observable domain (range for mix1d; bounding box
 * and physical region, with a relative tolerance of 1e-9, for dalitz3).
 * Out-of-range data checks are a paper feature (Sec. 4).  Synchronous.
 * Returns FN_E_DOMAIN when *n_bad > 0. */
fn_status fn_events_check(fn_model* m, const double* ev, int64_t n, int64_t ld,
                          int64_t* n_bad, void* stream);

/* NLL and, when grad_host != NULL, its gradient (P doubles), for host theta
 * (P doubles, copied before return): the objective a fit hands to the
 * minimizer (Sec. 4, the FCN given to Minuit), whose cost is the independent
 * evaluation of the density at every event (Sec. 1).  Synchronous.  n may be
 * 0 (NLL = 0).  FN_E_INVALID for NULL theta, n < 0, NULL events with n > 0,
 * or ld < n for a model with several observables. */
fn_status fn_nll(fn_model* m, const double* theta_host, const double* ev, int64_t n,
                 int64_t ld, double* nll_host, double* grad_host, void* stream);

/* Asynchronous form of fn_nll for device-resident loops (the direct FCN
 * access of Sec. 4 without a host round trip): theta_dev (P doubles) and
 * out_dev (1+P doubles: NLL then gradient; gradient entries untouched when
 * with_grad == 0) are device pointers, both read and written in stream
 * order.  No host synchronisation; no allocation after the first call of a
 * given size and kind (the first call may build the cached normalization
 * matrix), after which the call can be captured into a graph.  Non-finite
 * results are left in out_dev for the caller to inspect. */
fn_status fn_nll_async(fn_model* m, const double* theta_dev, const double* ev, int64_t n,
                       int64_t ld, double* out_dev, int32_t with_grad, void* stream);

/* fn_nll_async without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * fn_nll_async (bitwise), but the partial rows of the call (the events
 * pass's level-1 rows, and on the first call of a model whose cached
 * normalization is not built yet, or every call of a free-lineshape dalitz3
 * model, the normalization's rows) live in a static device array of the
 * library: 2^21 doubles (16 MiB) per device, whose address is looked up
 * when the device's context is created and which is held until the process
 * ends.  The call makes no hipMalloc, hipFree or other allocating call;
 * every row it reads was written earlier in the same call, so nothing needs
 * clearing between calls.  The array is shared by every call on one device:
 * calls that overlap on one device (different streams, models or host
 * threads) race and give wrong results; serialise them.  The event pass is
 * never timed by fn_model_timing.  FN_E_INVALID as fn_nll_async, and when
 * the rows do not fit (about 2^21 / (1 + P) chunks of the model's chunk
 * size: 123k chunks, 250M events at 2048 per chunk, for a 16-parameter
 * dalitz3 gradient); nothing is enqueued then except, possibly, the
 * parameter prologue. */
fn_status fn_nll_async_noalloc(fn_model* m, const double* theta_dev, const double* ev, int64_t n,
                               int64_t ld, double* out_dev, int32_t with_grad, void* stream);

/* Binned data of a mix1d model (the paper's binned DataSet, Fig. 1 and
 * Sec. 4): counts_dev holds n_bins >= 1 counts (device doubles, finite and
 * >= 0) of uniform bins on [lo, hi].  The expected count of bin b is
 * nu_b = N Delta P(x_b) at the bin centre x_b = lo + (b + 1/2) Delta,
 * Delta = (hi - lo)/n_bins, with N the yield parameter of an extended model,
 * otherwise the total count W.  stat 0: Poisson NLL sum_b (nu_b - n_b ln nu_b)
 * (the constant sum ln n_b! is omitted); stat 1: chi^2
 * sum_{b: n_b > 0} (n_b - nu_b)^2 / n_b.  value_host gets the statistic and
 * grad_host (may be NULL) its gradient (P doubles).  Synchronous.
 * FN_E_INVALID for another model kind, n_bins < 1, NULL counts or another
 * stat; FN_E_NONFINITE when the statistic is not finite (P = 0 in a filled
 * bin, invalid parameters, no events in a non-extended fit). */
fn_status fn_nll_binned(fn_model* m, const double* theta_host, const double* counts_dev, int64_t n_bins,
                        int32_t stat, double* value_host, double* grad_host, void* stream);

/* Normalization integral I(theta) and, when dnorm_host != NULL, dI/dtheta
 * (P doubles, host): the integral of P~ over the observable domain that
 * makes the composed density a probability density (Sec. 1; by Monte Carlo
 * over a phase-space sample for td4, Sec. 5).  theta_host: P doubles.
 * Synchronous.  mix1d: I = 1 (each component normalized analytically). */
fn_status fn_norm(fn_model* m, const double* theta_host, double* norm_host,
                  double* dnorm_host, void* stream);

/* Normalized density P~(x_i)/I per event into p_dev (n doubles, device,
 * caller-owned), the per-event function value of Sec. 1, for plots and tests.
 * theta_host: P doubles.  Synchronous.  FN_E_INVALID for tddp3 models and
 * for a NULL output with n > 0. */
fn_status fn_eval(fn_model* m, const double* theta_host, const double* ev, int64_t n,
                  int64_t ld, double* p_dev, void* stream);

/* td4 only: the phase-space sample that defines the normalization average
 * (the paper integrates four-body phase space by Monte Carlo, Sec. 5).
 * mc_dev: device memory, 5 rows (m12, m34, cos theta12, cos theta34, phi) of
 * n_mc unweighted points, row j at mc_dev[j*ld + i]; copied into model-owned
 * memory before return (the caller may free it).  Synchronous.  Replaces any
 * previous sample and invalidates the cached normalization matrix. */
fn_status fn_model_set_norm_sample(fn_model* m, const double* mc_dev, int64_t n_mc, int64_t ld, void* stream);
/* td4 only: the normalization sample generated on the device instead of
 * copied: n_mc unweighted four-body phase-space points, point i by
 * accept-reject with Philox4x32-10 counters (i, 100 + 3a, 2), (i, 101 + 3a, 2),
 * (i, 102 + 3a, 2) for attempt a under key (seed, fit): (m12, m34) uniform in
 * [m1+m2, M-m3-m4] x [m3+m4, M-m1-m2], kept when m12 + m34 < M and
 * u3 * wmax < q(M; m12, m34) q(m12; m1, m2) q(m34; m3, m4) (wmax: 1.05 x the
 * largest weight on an 801 x 801 grid of the box), then cos theta12 = 2 u4 - 1,
 * cos theta34 = 2 u5 - 1, phi = (2 u6 - 1) pi.  Synchronous; replaces any
 * previous sample.  FN_E_DOMAIN if a point is not resolved within 4096
 * attempts (the model then has no sample). */
fn_status fn_model_generate_norm_sample(fn_model* m, uint32_t seed, uint32_t fit, int64_t n_mc, void* stream);
/* td4 only: size of the fixed-constant vector and (fixed_host != NULL) the
 * values from the description. */
fn_status fn_model_fixed(const fn_model* m, int32_t* n_fixed, double* fixed_host);

/* Kernel timing (measurement support, not on the result path).  With
 * every = k >= 1, the 1st, (k+1)-th, (2k+1)-th ... per-event evaluation launch
 * of the model from this call on is timed: the dispatch itself records the
 * kernel's start and end times into a pair of HIP events
 * (hipExtModuleLaunchKernel / hipExtLaunchKernel; k = 1: every launch, a
 * large k keeps the timing work out of most of a timed loop); every = 0 turns
 * timing off.  every = -1 (dalitz3 models): every per-event launch from now
 * on, including launches captured into graphs while the mode is on and
 * replayed later, measures itself: each workgroup stores its start and end
 * on the device wall clock, and the level-2 kernel after it adds the
 * launch's span (last end - first start) to a device record.  This times
 * launches inside a timed loop of graph replays without HIP events.
 * Synchronous when set; the first launch of a larger sample than before in
 * this mode synchronizes the device (capture graphs after a warm-up call).
 * FN_E_INVALID if every < -1, or -1 for another model kind.
 * fn_model_kernel_time waits for the recorded events (span mode: for the
 * device), returns the summed duration in milliseconds and the number of
 * timed launches since the last query, and resets both. */
fn_status fn_model_timing(fn_model* m, int32_t every);
fn_status fn_model_kernel_time(fn_model* m, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------- fitting */
/* One fit by quasi-Newton minimization (BFGS with a line search satisfying
 * the strong Wolfe conditions) of the NLL on the device, replacing the
 * paper's FitManager + Minuit loop (Fig. 1, Sec. 4).
 *  theta0_host: start (P doubles).  free_mask: P int32, nonzero = free
 *  (NULL = all free).  grad_mode: 0 = adjoint gradient from the device,
 *  1 = central finite differences of the NLL (2 extra NLL calls per free
 *  parameter, step 1e-6 max(|theta|,1)).  Outputs (host, P doubles each,
 *  may be NULL): theta_out, err_out (sqrt of the diagonal of the inverse of
 *  the Hessian of NLL, which is the covariance for an NLL with error
 *  definition 1/2; fixed parameters get 0).  nll_out, n_iter, n_calls
 *  (NLL evaluations) may be NULL.  Convergence: estimated distance to
 *  minimum g^T H^-1 g / 2 < tol (tol <= 0 selects 1e-7), at most max_iter
 *  iterations (<= 0 selects 500).  Returns FN_OK when converged, FN_E_NONFINITE
 *  if the start point is not finite, FN_E_INVALID if it did not converge. */
fn_status fn_fit(fn_model* m, const double* theta0_host, const int32_t* free_mask,
                 const double* ev, int64_t n, int64_t ld, int32_t grad_mode, double tol,
                 int32_t max_iter, double* theta_out, double* err_out, double* nll_out,
                 int32_t* n_iter, int32_t* n_calls, void* stream);
/* The same fit of binned data (fn_nll_binned's counts, n_bins and stat);
 * value_out receives the minimum of the statistic, and errors use the error
 * definition of the statistic (1/2 for the Poisson NLL, 1 for chi^2). */
fn_status fn_fit_binned(fn_model* m, const double* theta0_host, const int32_t* free_mask,
                        const double* counts_dev, int64_t n_bins, int32_t stat, int32_t grad_mode, double tol,
                        int32_t max_iter, double* theta_out, double* err_out, double* value_out,
                        int32_t* n_iter, int32_t* n_calls, void* stream);

/* ------------------------------------------------- systematic variations
 * Many fits of one "td4" model to ONE event sample that differ in their fixed
 * constants (the model's fixed-constant vector: lineshape masses and widths,
 * time resolution) and start points -- the systematic-variation fits of a
 * time-dependent amplitude analysis (Sec. 5), advanced together on the
 * device.  Every step evaluates NLL + gradient for all running fits in one
 * events pass (one workgroup per (event chunk, fit)), then advances each
 * fit's BFGS / strong-Wolfe state machine (the minimizer of fn_fit, state in
 * device memory) by one evaluation.  Each fit's normalization matrix over the
 * model's phase-space sample is built once per batch and kept until its fixed
 * constants or the sample change.  A fit's NLL is bitwise the single-fit
 * fn_nll value of a model with the same constants.  A batch uses its own
 * stream, ordered after `stream` (the stream that produced the events);
 * calls are synchronous and must not overlap on one batch. */
typedef struct fn_vbatch fn_vbatch;
/* n_fits in [1, 4096]; every fit starts with the model's fixed constants. */
fn_status fn_vbatch_create(fn_model* m, int32_t n_fits, fn_vbatch** out);
fn_status fn_vbatch_destroy(fn_vbatch* b);
/* Fixed constants of fit `fit` (host, the model's fixed-constant vector
 * layout, see fn_model_fixed; NULL restores the model's).  FN_E_INVALID for
 * unphysical values (m0 at or below threshold, w0 <= 0, sigma_t <= 0). */
fn_status fn_vbatch_set_fixed(fn_vbatch* b, int32_t fit, const double* fixed_host);
/* NLL of every fit at theta_host (n_fits x P, row-major) into nll_host
 * (n_fits) and, when grad_host != NULL, gradients (n_fits x P).  One events
 * pass for all fits.  FN_E_NONFINITE if any fit's NLL is not finite (the
 * values are still written). */
fn_status fn_vbatch_nll(fn_vbatch* b, const double* theta_host, const double* ev, int64_t n, int64_t ld,
                        double* nll_host, double* grad_host, void* stream);
/* Minimize every fit from theta0_host (n_fits x P); free_mask (P int32, NULL =
 * all free) applies to all fits.  tol, max_iter as for fn_fit; use_graph != 0
 * replays one captured step graph.  Outputs (host, may be NULL): status
 * (n_fits, FN_FIT_*), theta and err (n_fits x P; err = sqrt of the diagonal of
 * the BFGS inverse-Hessian approximation, 0 for fixed parameters), nll,
 * iterations and evaluations (n_fits). */
fn_status fn_vbatch_fit(fn_vbatch* b, const double* theta0_host, const int32_t* free_mask, const double* ev,
                        int64_t n, int64_t ld, double tol, int32_t max_iter, int32_t use_graph, int32_t* status_out,
                        double* theta_out, double* err_out, double* nll_out, int32_t* iters_out,
                        int32_t* n_evals_out, void* stream);

/* Continuous serving of systematic-variation fits (the fits of one recorded
 * sample under varied fixed constants, Sec. 5) on the batch's slots: a
 * request carries its fixed constants and start point and arrives at
 * arrival_s seconds after the call starts.  At every step boundary the
 * arrivals visible by then are admitted, in arrival order, into free slots:
 * their fixed constants and start points are copied to the device and their
 * tables and normalization matrices built (one pass over the phase-space
 * sample for all fits admitted together); they then share every events pass
 * with the fits already running.  A fit that converges or fails retires at
 * the next poll (every poll_every steps) and frees its slot.  Device memory
 * is reserved per slot at fn_vbatch_create (state, table, matrix, partial
 * rows), so admission is by free slot; the events are the shared sample.  A
 * request's result is bitwise the same as when it runs alone in a batch.
 * Outputs are per request, in the order of reqs (host arrays of n_req, or
 * n_req x P for theta and err; any may be NULL); t_admit and t_done are
 * seconds after the call starts.  Synchronous.  The batch's fixed constants
 * afterwards are those of the last request each slot served.  FN_E_INVALID
 * for a request without a start point, a negative or non-finite arrival
 * time, or invalid fixed constants (nothing runs then). */
typedef struct {
  int64_t id;
  double arrival_s;
  const double* fixed;      /* host, fn_model_fixed layout; NULL = the model's constants */
  const double* theta0;     /* host, P doubles */
} fn_vrequest;
fn_status fn_vbatch_serve(fn_vbatch* b, const fn_vrequest* reqs, int32_t n_req, const int32_t* free_mask,
                          const double* ev, int64_t n, int64_t ld, double tol, int32_t max_iter, int32_t poll_every,
                          int32_t* status_out, double* theta_out, double* err_out, double* nll_out,
                          int32_t* iters_out, int32_t* n_evals_out, double* t_admit_out, double* t_done_out,
                          void* stream);

/* ---------------------------------------------------------------- batching
 * Many independent fits of one "mix1d" model advanced together on the device
 * (the paper's toy Monte Carlo studies: many fits of the same PDF to
 * different samples, Sec. 5).  Each fit occupies a slot; a step evaluates
 * NLL + gradient for every running slot at its trial point and advances that
 * slot's BFGS / strong-Wolfe line-search state machine by one evaluation
 * (the same minimizer as fn_fit, state kept in device memory).  Fits never
 * interact: a fit's result bits do not depend on the other slots.  Step
 * launches are captured once in a hipGraph on an internal stream and replayed;
 * the host reads back only the running-slot count between groups of steps.
 * A batch uses its own stream; calls on one batch must not overlap. */
typedef struct fn_batch fn_batch;
enum { FN_FIT_IDLE = 0, FN_FIT_RUNNING = 1, FN_FIT_CONVERGED = 2, FN_FIT_FAILED = 3 };

/* max_fits slots for a mix1d model with at most 24 parameters; events per fit
 * up to max_events_per_fit.  Allocates all device state up front. */
fn_status fn_batch_create(fn_model* m, int32_t max_fits, int64_t max_events_per_fit, fn_batch** out);
fn_status fn_batch_destroy(fn_batch* b);
/* Put a fit into slot `slot`: device events (n, caller-owned, valid until the
 * slot is cleared or the fit finishes), host start point theta0 (P doubles),
 * free mask (P int32, NULL = all free).  The slot becomes RUNNING. */
fn_status fn_batch_set_slot(fn_batch* b, int32_t slot, const double* ev, int64_t n, const double* theta0,
                            const int32_t* free_mask);
/* Mark a slot IDLE (frees it for reuse; its last results stay readable). */
fn_status fn_batch_clear_slot(fn_batch* b, int32_t slot);
/* Convergence tolerance on the estimated distance to minimum (<= 0: 1e-7)
 * and iteration limit (<= 0: 500) for fits set after this call. */
fn_status fn_batch_config(fn_batch* b, double tol, int32_t max_iter, int32_t use_graph);
/* Run up to max_steps steps (poll the running count every poll_every steps);
 * returns the number of steps run and the slots still running. */
fn_status fn_batch_run(fn_batch* b, int32_t max_steps, int32_t poll_every, int32_t* steps_done,
                       int32_t* n_running);
/* Array form of fn_batch_set_slot (the paper's FitManager handed many fits of
 * one PDF at once, Fig. 1 caption and Sec. 5): slots 0 .. n_fits-1 become
 * fresh RUNNING fits with all parameters free, slots n_fits .. max_fits-1
 * become IDLE.  Fit f reads n[f] device events at ev[f] (caller-owned, valid
 * until the fit finishes or the batch is set again; ev and n are host arrays
 * of n_fits entries); ld (host, may be NULL) gives each fit's leading
 * dimension, which must be >= n[f] (a mix1d model has one observable, so it
 * is only checked).  theta0_dev: device memory, n_fits x P start points,
 * row-major; it must be ready (its producer synchronised) and is read before
 * return.  Synchronous.  FN_E_INVALID for n_fits outside [0, max_fits], NULL
 * pointers, event counts outside [1, max_events_per_fit] or ld < n. */
fn_status fn_batch_set(fn_batch* b, int32_t n_fits, const double* const* ev, const int64_t* n, const int64_t* ld,
                       const double* theta0_dev);
/* One step of every running fit, enqueued on `stream` (the paper's direct
 * access to the FCN from the caller's own loop, Sec. 4): NLL + gradient at
 * each fit's trial point, then one BFGS / strong-Wolfe state-machine step.
 * No host synchronisation, no allocation and no memset: when `stream` is
 * being captured, the step's kernels are recorded into the caller's graph
 * (replaying it steps the batch); otherwise the batch's own step graph is
 * launched on `stream`.  Steps run on `stream` are ordered before later
 * fn_batch_* calls on the same batch (which wait for them); a caller that
 * replays a captured step synchronises its stream before reading status.
 * The same sequence of steps gives bitwise the results of fn_batch_run. */
fn_status fn_batch_step(fn_batch* b, void* stream);
/* Per-fit status (FN_FIT_*), theta (max_fits x P), NLL and errors
 * (max_fits x P: sqrt of the diagonal of the BFGS inverse-Hessian estimate,
 * 0 for fixed parameters) into host arrays (any may be NULL) after the steps
 * enqueued so far.  Synchronous. */
fn_status fn_batch_status(fn_batch* b, int32_t* status_host, double* theta_host, double* nll_host,
                          double* err_host);
/* Per-slot results (host arrays of max_fits entries; any may be NULL):
 * status, theta (max_fits x P), nll, errors (sqrt of the diagonal of the BFGS
 * inverse-Hessian estimate; 0 for fixed parameters), iterations, evaluations. */
fn_status fn_batch_results(fn_batch* b, int32_t* status, double* theta, double* nll, double* errors,
                           int32_t* iters, int32_t* n_evals);

/* Device toy generation (Philox4x32-10 counters (i, attempt, word) under key
 * (seed, fit)) of n events of the Gaussian(mu, sigma) fraction f + exponential
 * (tau) mixture on [lo, hi], theta_gen = (mu, sigma, tau, f) on the host,
 * into caller-owned device memory x (n doubles).  Synchronous. */
fn_status fn_generate_mix1d(uint32_t seed, uint32_t fit, int64_t n, const double* theta_gen, double lo, double hi,
                            double* x, void* stream);

/* Toy events of a dalitz3, tddp3 or td4 model at theta (host, P doubles) by
 * accept-reject on the device, for toy studies (the paper's Monte Carlo
 * generation with MCBooster, Sec. 5).  td4 (six rows m12, m34, cos theta12,
 * cos theta34, phi, t): attempt a draws a phase-space point as
 * fn_model_generate_norm_sample does with word 4 and streams 4a, 4a + 1,
 * 4a + 2, then (u7, u8) from (i, 4a + 3, 4): t = -ln(1 - u7)/lam and the
 * point is kept when u8 * envelope * exp(-lam t) < R, as for tddp3; the
 * automatic envelope is 1.2 x the largest (|A| + |Abar|)^2 over the model's
 * normalization sample (which must be set); Box-Muller from (i, 0, 5); at
 * most 65536 attempts per event.  tddp3 (three rows s12, s13, t): event
 * i, attempt a takes (u1, u2) from counter (i, 2a, 2) and (u3, u4) from
 * (i, 2a + 1, 2); the candidate point in the box below with
 * t = -ln(1 - u3)/lam, lam = (1 - |y|)/tau, is kept inside the region when
 * u4 * envelope * exp(-lam t) < R(s12, s13, t) (the unconvolved rate, which
 * is at most exp(-lam t) (|A| + |Abar|)^2), then t gains sigma_t times a
 * Box-Muller normal from counter (i, 0, 3); the automatic envelope is 1.2 x
 * the largest (|A| + |Abar|)^2 at the grid-cell centres; t goes to
 * ev_dev[2 ld + i].  dalitz3: event i, attempt a draws (u1, u2) from
 * Philox4x32-10 counter (i, 2a, 1) and u3 from (i, 2a + 1, 1) under key
 * (seed, fit); the
 * candidate s12 = lo12 + u1 (hi12 - lo12), s13 = lo13 + u2 (hi13 - lo13) in
 * the kinematic box [(m1+m2)^2, (M-m3)^2] x [(m1+m3)^2, (M-m2)^2] is kept when
 * it lies in the Dalitz region and u3 * envelope < P~(s12, s13) (the
 * unnormalized density |sum_k c_k A_k|^2), at most 4096 attempts.
 *  envelope: an upper bound of P~ over the region, or 0 for 1.2 x the largest
 *  P~ at the centres of the model's integration-grid cells; the value used is
 *  written to *envelope_used (may be NULL).
 *  ev_dev: caller-owned device memory, s12 at ev_dev[i], s13 at ev_dev[ld + i]
 *  (ld >= n).  Synchronous on `stream`.
 * FN_E_INVALID for another model kind, NULL pointers, ld < n, a negative or
 * non-finite envelope, invalid lineshape parameters, |y| >= 1 (tddp3), or a
 * density that vanishes on the grid; FN_E_DOMAIN if an accepted event lies
 * above the envelope (raise it) or an event was not accepted within the
 * attempts (it is NaN).  Event i depends only on (theta, seed, fit, envelope, i). */
fn_status fn_generate(fn_model* m, const double* theta_host, uint32_t seed, uint32_t fit, int64_t n,
                      double envelope, double* ev_dev, int64_t ld, double* envelope_used, void* stream);

/* ----------------------------------------------------------------- serving
 * A request loop over one batch: requests (toy-MC fits of a mix1d model, the
 * paper's toy Monte Carlo studies, Sec. 5) arrive at given times, are
 * admitted at step boundaries when a slot is free and their events fit the
 * device-memory budget, have their events generated on the device (or use
 * caller events), run inside the batch with the fits already on the GPU, and
 * retire when converged or failed, freeing slot and memory for queued
 * requests (continuous batching).  A request's result does not depend on
 * which other requests shared the batch.
 *
 * Budget: every admitted, unfinished request is charged 8 * n_events bytes,
 * whether its events are generated into the server's arena or owned by the
 * caller; a request is admitted only while the charges stay within
 * budget_bytes.  Admission follows arrival order with backfilling: a request
 * that does not fit the free budget does not hold back later arrivals that
 * do, until 256 requests have been admitted past it; then admission waits
 * until it fits.  A request larger than the whole budget completes at once
 * with status FN_E_BUDGET.
 *
 * Times: the server's clock starts with its first fn_server_run; arrival_s
 * and the result times are seconds on that clock. */
typedef struct fn_server fn_server;

typedef struct {
  int64_t id;
  int64_t n_events;
  uint32_t seed, fit;       /* generation key when events == NULL */
  const double* events;     /* optional caller-owned device events (n_events) */
  double theta_gen[4];      /* generation point (mu, sigma, tau, f) */
  double theta0[24];        /* start point, first P entries used */
  double arrival_s;         /* arrival time on the server clock */
} fn_request;

typedef struct {
  int64_t id;
  int32_t status;           /* FN_FIT_CONVERGED, FN_FIT_FAILED, or FN_E_BUDGET if it can never fit */
  int32_t iters, n_evals, pad;
  double nll;
  double theta[24], errors[24];
  double t_arrival, t_admit, t_done;  /* server clock */
} fn_result;

/* Server over a mix1d model whose components are (gauss, exp) when events are
 * generated: max_slots concurrent fits, at most max_events_per_fit events per
 * request, budget_bytes of device memory for request events. */
fn_status fn_server_create(fn_model* m, int32_t max_slots, int64_t max_events_per_fit, int64_t budget_bytes,
                           fn_server** out);
fn_status fn_server_destroy(fn_server* s);
/* Queue requests (copied). */
fn_status fn_server_submit(fn_server* s, const fn_request* reqs, int32_t n);
/* Serve every queued request, stepping the batch poll_every steps between
 * admission/retirement checks, until none is queued or running; with
 * max_seconds > 0 it returns after about that many seconds of this call
 * instead, and fits still running keep their slots, memory and state for the
 * next fn_server_run, which continues them.  *n_done: results so far.
 * Synchronous. */
fn_status fn_server_run(fn_server* s, int32_t poll_every, double max_seconds, int32_t* n_done);
/* Results of finished requests, in completion order; *n_out <= max. */
fn_status fn_server_results(fn_server* s, fn_result* out, int32_t max, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* FITNLL_H */
