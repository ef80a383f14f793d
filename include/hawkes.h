/*
 * hawkes.h -- C ABI of libhawkes, the MI355X (gfx950) evaluator of the exact O(N^2)
 * spatiotemporal Hawkes log-likelihood of arXiv 2005.10123 and of its gradient.
 *
 * Model (Section 2.1 "Model", the log-likelihood equation): for events (x_n, y_n, t_n), n = 1..N,
 * and parameters Theta = (mu0, tau_x, tau_t, theta, omega, h),
 *
 *   lambda_n = mu0 / (tau_x^2 tau_t) sum_{n'} phi2((x_n - x_n')/tau_x) phi1((t_n - t_n')/tau_t)
 *            + theta omega / h^2 sum_{n': t_n' < t_n} exp(-omega (t_n - t_n')) phi2((x_n - x_n')/h)
 *   Lambda_n = mu0 (Phi((T - t_n)/tau_t) - Phi(-t_n/tau_t)) - theta (exp(-omega (T - t_n)) - 1)
 *   ell      = sum_n (log lambda_n - Lambda_n),     T = max_n t_n,
 *
 * phi1/phi2 the standard normal densities in 1 and 2 dimensions, Phi the standard normal CDF.  The
 * background sum includes n' = n; the trigger indicator is strict (ties are not causal); the
 * trigger coefficient is theta*omega/h^2 (the reading under which the paper's closed-form
 * integral of the intensity holds).  The gradient is d ell / d Theta in the order of Theta.  The
 * self-excitation probability (the paper's probability equation) is pi_n = xi_n / lambda_n with
 * xi_n the trigger part of lambda_n.
 *
 * Conventions for every function:
 *   - the return value is a hawkes_status: HAWKES_OK (0) or a negative error code; no C++
 *     exception crosses this interface;
 *   - on failure hawkes_last_error() returns a message for the calling thread;
 *   - all pointers are host pointers unless the name says d_ (device memory of the context's GPU);
 *   - the library never keeps a caller pointer after a call returns.
 */
#ifndef HAWKES_H
#define HAWKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hawkes_ctx hawkes_ctx; /* opaque; owns every device allocation it makes */
typedef int32_t hawkes_status;

enum {
    HAWKES_OK = 0,
    HAWKES_EINVAL = -1,    /* invalid argument (null pointer, non-finite or out-of-domain value) */
    HAWKES_ENOMEM = -2,    /* over the context's HBM budget, or a device allocation failed */
    HAWKES_EBUSY = -3,     /* the dataset still has requests in flight */
    HAWKES_EAGAIN = -4,    /* hawkes_poll: nothing completed within the timeout */
    HAWKES_EDEVICE = -5,   /* a HIP runtime call failed; the context is unusable afterwards */
    HAWKES_ENOTFOUND = -6, /* unknown dataset id */
    HAWKES_ECANCELED = -7  /* request cancelled by hawkes_destroy */
};

/* Arithmetic of the pairwise pass.  Both paths keep log lambda_n, Lambda_n, the per-event
 * gradient and every cross-event reduction in binary64.
 *   HAWKES_FP64 : pair terms, exponentials and per-event sums in binary64.
 *   HAWKES_FP32C: pair terms in binary32 from exactly split (hi + lo) coordinates, exponentials by
 *                 the hardware base-2 exponential, per-event sums compensated (TwoSum). */
enum { HAWKES_FP64 = 0, HAWKES_FP32C = 1 };

/* Theta in the order of Section 2.1.  Domain: all finite; mu0, tau_x, tau_t, omega, h > 0 and at
 * most 1e12; theta >= 0 (theta = 0 is the background-only model). */
typedef struct {
    double mu0, tau_x, tau_t, theta, omega, h;
} hawkes_params;

/* Number of doubles per event written by hawkes_rows. */
#define HAWKES_ROW_FIELDS 10

/* Create a context on HIP device `device`.
 *   hbm_budget_bytes: upper bound on the device memory the context may hold (datasets plus
 *                     evaluation scratch); 0 means 90% of the device's free memory.
 *   hip_stream      : a hipStream_t the context launches its blocking and device calls on, or
 *                     NULL for a stream of its own.  The caller keeps ownership of a passed stream.
 * On success *out receives the context. */
hawkes_status hawkes_create(int device, size_t hbm_budget_bytes, void* hip_stream, hawkes_ctx** out);

/* Destroy a context: waits for the device, fails every pending or in-flight request with
 * HAWKES_ECANCELED (readable by no one afterwards) and frees all device memory.  NULL is allowed. */
hawkes_status hawkes_destroy(hawkes_ctx* ctx);

/* Register an event set (Section 2.1: x_n in R^2, t_n in R+).  x, y, t are n host doubles each,
 * in any order; they are copied, so the caller may free them when the call returns.  n >= 1,
 * every value finite, every t >= 0.  The library sorts by (t, input index), centres the
 * coordinates, splits them for the FP32C path and computes each event's causal count
 * #{n': t_n' < t_n}.  *out_id receives a non-negative dataset id. */
hawkes_status hawkes_dataset_create(hawkes_ctx* ctx, const double* x, const double* y, const double* t,
                                    int64_t n, int32_t* out_id);

/* Free a dataset.  HAWKES_EBUSY while submitted requests on it have not been polled. */
hawkes_status hawkes_dataset_destroy(hawkes_ctx* ctx, int32_t id);

/* Events and device bytes held by a dataset. */
hawkes_status hawkes_dataset_info(hawkes_ctx* ctx, int32_t id, int64_t* n, size_t* device_bytes);

/* Blocking log-likelihood ell(Theta) (the log-likelihood equation).  precision is HAWKES_FP64 or
 * HAWKES_FP32C.  Writes one double to *out_loglik. */
hawkes_status hawkes_loglik(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision,
                            double* out_loglik);

/* Blocking log-likelihood and gradient d ell / d Theta in one pairwise pass.  out_grad receives 6
 * doubles in the order of hawkes_params. */
hawkes_status hawkes_grad(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision,
                          double* out_loglik, double* out_grad);

/* Asynchronous variant of hawkes_grad for callers that own device memory (e.g. a tensor library):
 * enqueues the evaluation on hip_stream (a hipStream_t; NULL is the device's null stream, as in
 * HIP) and writes 7 doubles (ell, then the gradient) to d_out7, device memory of the context's GPU.
 * Returns once the work is enqueued; the result is valid when that stream reaches this point.  The
 * evaluation scratch is shared with the context's other blocking and device calls, which are
 * ordered after it by an event. */
hawkes_status hawkes_grad_device(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision,
                                 double* d_out7, void* hip_stream);

/* hawkes_grad_device for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels, plan and result
 * as hawkes_grad_device (bitwise), but the evaluation scratch is a fixed 256 MiB device array that
 * the library holds on every device it runs on until the process ends, not memory of the context:
 * this call makes no device or host allocation (its address is looked up once per device by
 * hawkes_create).  Limit: an evaluation whose scratch exceeds 256 MiB fails with HAWKES_ENOMEM
 * before anything is enqueued (symmetric enumeration: up to about 110,000 events with FP32C, about
 * 99,000 with FP64; the direct enumeration's scratch grows linearly in n).  Every call on one GPU,
 * from any context or thread, shares that array: calls whose device work overlaps (different
 * streams not ordered with each other, or another context on the same GPU) race and give wrong
 * results; calls on one stream, or on streams the caller orders, are safe.  The array keeps the
 * last call's contents; nothing in it needs clearing between calls. */
hawkes_status hawkes_grad_device_noalloc(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision,
                                         double* d_out7, void* hip_stream);

/* Blocking per-event results in the caller's original order: for event k, out_rows[10k + f] with
 * f = 0 lambda_k, 1 Lambda_k, 2 ell_k = log lambda_k - Lambda_k, 3 pi_k (self-excitation
 * probability), 4..9 d ell_k / d Theta.  out_rows holds n * HAWKES_ROW_FIELDS doubles. */
hawkes_status hawkes_rows(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision,
                          double* out_rows);

/* Log-likelihood and self-excitation probabilities for `count` parameter vectors over one dataset
 * (the paper evaluates pi_n for every event under each of 1,000 posterior samples of Theta,
 * Section 3.2).  thetas: count parameter vectors.  out_loglik: count doubles, or NULL.
 * out_pi: count * n doubles, or NULL; pi of event k under thetas[s] at out_pi[s * n + k], events in
 * the caller's original order.  At least one output must be requested.  FP32C shares each pair's
 * differences among four parameter vectors per pass; FP64 evaluates them one at a time. */
hawkes_status hawkes_loglik_multi(hawkes_ctx* ctx, int32_t id, const hawkes_params* thetas, int32_t count,
                                  int precision, double* out_loglik, double* out_pi);

/* ---- one dataset over several devices ----------------------------------------------------------
 * The log-likelihood equation needs, for every event n, six sums over the other events: the
 * background sums S_b = sum_n' B(n, n') (n' = n included), S_br = sum r^2 B, S_bt = sum dt^2 B and the
 * trigger sums S_e = sum_{t_n' < t_n} E(n, n'), S_et = sum dt E, S_er = sum r^2 E, with
 * B = exp(-r^2 / (2 tau_x^2) - dt^2 / (2 tau_t^2)), E = exp(-omega dt - r^2 / (2 h^2)), r and dt the
 * distance and time difference of the pair; lambda_n = c_b S_b + c_e S_e (Section 2.1).  The pairs
 * n' < n (in time order) are cut into `nshards` contiguous ranges of equal work; a device (one
 * context per device, the dataset registered in each) computes the sums over its range, the
 * per-event sums of all shards are added (e.g. by an all-reduce), and hawkes_finish turns the totals
 * into ell and its gradient.  Symmetric enumeration, whatever hawkes_set_pair_scheme chose. */

/* Per-event sums of shard `shard` (0 <= shard < nshards) of the pairwise pass.  out_sums: n * 6
 * doubles, event k (caller's order) at out_sums[6k .. 6k + 5] = (S_b, S_br, S_bt, S_e, S_et, S_er);
 * the diagonal term B(n, n) = 1 is in shard 0's S_b.  precision as for hawkes_grad. */
hawkes_status hawkes_shard_sums(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, int precision, int32_t shard,
                                int32_t nshards, double* out_sums);

/* ell and, if out_grad is not NULL, its gradient (6 doubles) from the per-event sums `sums` (n * 6
 * doubles in the layout of hawkes_shard_sums, added over all shards of the same parameters), in
 * binary64. */
hawkes_status hawkes_finish(hawkes_ctx* ctx, int32_t id, const hawkes_params* p, const double* sums,
                            double* out_loglik, double* out_grad);

/* ---- batched serving -------------------------------------------------------------------------
 * Requests from many concurrent samplers (the paper's Algorithm 1 evaluates the likelihood once
 * per Metropolis-Hastings step) are queued, admitted while evaluation slots and the HBM budget
 * allow, packed into shared device launches with the requests already running, and completed
 * independently.  The result of a request does not depend on what it was batched with. */
typedef struct {
    int32_t dataset;   /* dataset id */
    int32_t precision; /* HAWKES_FP64 or HAWKES_FP32C */
    int32_t want_grad; /* 0: log-likelihood only; 1: log-likelihood and gradient */
    int32_t _pad;
    hawkes_params p;
    uint64_t tag; /* returned unchanged in the result */
} hawkes_request;

typedef struct {
    uint64_t tag;
    hawkes_status status; /* HAWKES_OK, HAWKES_EINVAL (bad request), HAWKES_EDEVICE, ... */
    int32_t _pad;
    double loglik;
    double grad[6];        /* zeros when want_grad was 0 */
    uint64_t t_submit_ns;  /* steady-clock nanoseconds at hawkes_submit */
    uint64_t t_done_ns;    /* steady-clock nanoseconds when the device result was observed */
} hawkes_result;

/* Queue n requests; never blocks on the device.  A request with invalid parameters or an unknown
 * dataset completes with that error status instead of failing the call; the call itself fails
 * (HAWKES_EINVAL) only for a NULL ctx/reqs or n < 0.  Requests larger than the remaining budget
 * wait until memory frees up; one that can never fit completes with HAWKES_ENOMEM. */
hawkes_status hawkes_submit(hawkes_ctx* ctx, const hawkes_request* reqs, int32_t n);

/* Collect up to cap completed results into out (completion order).  Waits at most timeout_us
 * microseconds (0: do not wait; negative: wait until at least one result is ready or nothing is
 * outstanding).  *n_out receives the number written; HAWKES_EAGAIN when it is 0. */
hawkes_status hawkes_poll(hawkes_ctx* ctx, hawkes_result* out, int32_t cap, int32_t* n_out,
                          int64_t timeout_us);

/* Requests submitted but not yet returned by hawkes_poll. */
hawkes_status hawkes_outstanding(hawkes_ctx* ctx, int64_t* n);

/* ---- enumeration of the pair terms ----------------------------------------------------------
 * HAWKES_PAIRS_SYMMETRIC (default): each unordered pair once.  The background kernel of the
 *   log-likelihood equation is symmetric in (n, n'), so one evaluation of it feeds both lambda_n
 *   and lambda_n'; the trigger term feeds only the later event.  Same sums, about half the work.
 * HAWKES_PAIRS_DIRECT: every ordered pair (n, n'), the enumeration of the paper's Algorithm 3.
 * Both give the same result up to rounding; a context's choice applies to calls and requests
 * made after it is set. */
enum { HAWKES_PAIRS_SYMMETRIC = 0, HAWKES_PAIRS_DIRECT = 1 };
hawkes_status hawkes_set_pair_scheme(hawkes_ctx* ctx, int scheme);

/* Zero-tile skipping (enable = 1; 0, the default, turns it off).  Both kernels of the
 * log-likelihood equation decay in the time difference: the background term as
 * exp(-dt^2 / (2 tau_t^2)), the trigger term as exp(-omega dt).  Beyond a separation D(Theta) both
 * are exactly zero in the arithmetic of the chosen precision (binary32 exponentials below 2^-170
 * for HAWKES_FP32C, binary64 ones below 2^-1110 for HAWKES_FP64), so the pairs further apart add
 * nothing to any sum.  With skipping on, the symmetric enumeration leaves out every column tile
 * whose events all lie at least D before the first event of the row block against which it would
 * be evaluated, and the direct enumeration every tile all of whose events are at least D before or
 * after all of the row block's; on data spanning many multiples of tau_t and 1/omega most pairs
 * are such.  The
 * result is the same sum of the same non-zero terms; only its grouping into partial sums changes
 * (as it does with the device's number of compute units), so it agrees with the unskipped
 * evaluation to rounding.  Applies to hawkes_loglik, hawkes_grad, hawkes_grad_device, hawkes_rows,
 * hawkes_loglik_multi (a tile is left out when the terms of every parameter vector of its pass
 * vanish there) and submitted requests made after the call, with either enumeration; not to
 * hawkes_shard_sums. */
hawkes_status hawkes_set_zero_tile_skipping(hawkes_ctx* ctx, int enable);

/* Shared passes for served log-likelihoods (enable: 1, or 0, the default).  Chains of the paper's
 * sampler (Algorithm 1, step 5a) each ask for one log-likelihood per proposal, many of them on the
 * same dataset.  With shared passes on, submitted HAWKES_FP32C requests without the gradient are
 * evaluated by the multi-parameter pass of hawkes_loglik_multi: the requests of one launch on one
 * dataset share passes of up to 4 parameter vectors, each pair's differences formed once for all
 * of them.  A request's result is then bitwise hawkes_loglik_multi's value for its vector, the
 * same alone or grouped (which vectors share a pass does not change any vector's arithmetic), and
 * agrees with hawkes_loglik to rounding (a different grouping of the same binary32 terms).  With
 * zero-tile skipping on, each such request has a pass of its own (the tiles a pass leaves out
 * depend on all of its vectors).  With shared passes off, those requests are evaluated like
 * hawkes_loglik, bitwise.  Applies to requests admitted after the call.  Off by default: a request
 * that finds no companions has a pass of one vector, which costs more than the single-parameter
 * pass, and on MI355X the sharing gained little where groups formed. */
hawkes_status hawkes_set_shared_passes(hawkes_ctx* ctx, int enable);

/* ---- host evaluation ------------------------------------------------------------------------
 * The paper's multi-core CPU design (Section 2.3; its CPU algorithms for the log-likelihood and the
 * self-excitation probabilities): the events' rows are dealt to `threads` host threads, each
 * keeping its row's coordinates in registers and running SIMD-vectorised loops over the other
 * events (AVX-512, AVX2 or SSE2, chosen at load time) with running sums only; binary64 throughout,
 * every ordered pair evaluated.  A separate evaluation on the host's cores, needing no context or
 * device; no device entry point ever falls back to it.
 *   x, y, t : n events in any order (host memory, copied; t >= 0, all finite); n >= 1
 *   p       : Theta, validated as for hawkes_grad
 *   threads : host threads to use (<= 0: as many as the hardware reports)
 *   out7    : 7 doubles: ell, then d ell / d Theta
 *   out_pi  : n doubles (pi_k in the caller's order), or NULL
 * The result does not depend on `threads` (per-event terms summed in time order). */
hawkes_status hawkes_host_eval(const double* x, const double* y, const double* t, int64_t n, const hawkes_params* p,
                               int threads, double* out7, double* out_pi);

/* ---- diagnostics -------------------------------------------------------------------------- */

/* Thread-local message describing the calling thread's last failure ("" if none).  With the
 * environment variable HAWKES_LOG set (to anything but "0") each such message is also printed to
 * stderr when it is recorded. */
const char* hawkes_last_error(void);

/* Turn on (1) or off (0) device-event timing of the pairwise kernel on the launching stream, and
 * read the accumulated milliseconds and launch count since the last reset (reset = 1 clears). */
hawkes_status hawkes_profile(hawkes_ctx* ctx, int enable);
hawkes_status hawkes_kernel_time(hawkes_ctx* ctx, double* pair_ms, int64_t* pair_launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_H */
