// hawkes_runtime.hip -- host runtime behind include/hawkes.h: contexts, the dataset registry,
// parameter folding, evaluation plans, scratch and budget accounting, blocking and asynchronous
// evaluation.  The batched serving loop lives in hawkes_serving.hip.
#include "hawkes_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

namespace hawkes {

thread_local std::string g_last_error;

// HAWKES_LOG set to a non-empty value other than "0" also prints every failure to stderr.
static bool log_failures()
{
    static const bool on = [] {
        const char* v = std::getenv("HAWKES_LOG");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

hawkes_status fail(hawkes_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (log_failures()) std::fprintf(stderr, "libhawkes: status %d: %s\n", (int)code, buf);
    return code;
}

hawkes_status check_params(const hawkes_params* p)
{
    if (!p) return fail(HAWKES_EINVAL, "params is NULL");
    const double v[6] = {p->mu0, p->tau_x, p->tau_t, p->theta, p->omega, p->h};
    static const char* names[6] = {"mu0", "tau_x", "tau_t", "theta", "omega", "h"};
    for (int k = 0; k < 6; ++k) {
        if (!std::isfinite(v[k])) return fail(HAWKES_EINVAL, "%s is not finite", names[k]);
        if (v[k] > 1e12) return fail(HAWKES_EINVAL, "%s = %g exceeds 1e12", names[k], v[k]);
        if (k == 3 ? v[k] < 0.0 : v[k] <= 0.0)
            return fail(HAWKES_EINVAL, "%s = %g is outside its domain", names[k], v[k]);
    }
    return HAWKES_OK;
}

Plan make_plan(const hawkes_ctx* c, int64_t n, int npad, bool grad, int precision, int scheme, int shard, int nshards,
               bool zero_skip)
{
    Plan pl;
    pl.scheme = scheme;
    pl.precision = precision;
    pl.row_blocks = npad / kRowsPerBlock;
    pl.K = grad ? 6 : 2;
    pl.epi_blocks = (int)((n + kThreads - 1) / kThreads);
    if (scheme == kSymmetric) {
        // Contiguous ranges of lower-triangle work units, one range per resident block, their
        // lengths differing by at most one unit, so every block of a lone evaluation runs from
        // start to end together with the others and every resident slot is used.
        const long long TB = kRowsPerBlock / kTile;
        const long long T = pl.row_blocks;
        const long long all = TB * T * (T + 1) / 2;
        pl.ubegin = all * shard / nshards;
        pl.units = all * (shard + 1) / nshards - pl.ubegin;
        const long long slots = std::max(1, c->sym_slots[precision == kFP32C ? 1 : 0][grad ? 1 : 0]);
        pl.items = (int)std::min(slots, pl.units);
        pl.ubase = pl.items > 0 ? (int)(pl.units / pl.items) : 1;
        pl.urem = pl.items > 0 ? (int)(pl.units % pl.items) : 0;
        // Dynamic tail (walk_split): up to kDynChunksPerBlock chunks per block, each with row
        // partial slots of its own.
        pl.dchunks = pl.units >= kDynMinUnitsPerBlock * pl.items
                         ? (int)std::min<long long>(pl.units / kDynDiv, (long long)kDynChunksPerBlock * pl.items)
                         : 0;
        pl.part_doubles = (size_t)(pl.items + T + (pl.dchunks > 0 ? pl.dchunks + T : 0)) * pl.K * kRowsPerBlock;
        pl.col_stride = (long long)kRowsPerBlock * T * (T + 1) / 2;
        // The FP32C pass writes binary32 column partials (sums of binary32 terms over one row
        // block), the FP64 pass binary64 ones.
        const size_t col_elem = precision == kFP32C ? sizeof(float) : sizeof(double);
        pl.col_bytes = ((size_t)(grad ? 3 : 1) * pl.col_stride * col_elem + 7) & ~(size_t)7;
        if (zero_skip && shard == 0 && nshards == 1) {
            // Leaving tiles out only shortens the walk: the grid and the partial-sum slots stay
            // those of the whole triangle.
            pl.zskip = true;
            pl.zbytes = ((size_t)(T + 1) * sizeof(long long) + (size_t)T * sizeof(int) + 7) & ~(size_t)7;
        }
        return pl;
    }
    const int tiles = npad / kTile;
    // About eight blocks per compute unit: enough that the spread of per-block work (later rows
    // have more causal columns) leaves a short tail.
    const int target_blocks = 2048;
    int splits = (target_blocks + pl.row_blocks - 1) / pl.row_blocks;
    splits = std::max(1, std::min(splits, std::min(kMaxSplits, tiles)));
    pl.tiles_per_split = (tiles + splits - 1) / splits;
    pl.splits = (tiles + pl.tiles_per_split - 1) / pl.tiles_per_split;
    pl.items = pl.row_blocks * pl.splits;
    pl.part_doubles = (size_t)pl.splits * pl.K * npad;
    pl.zdirect = zero_skip && shard == 0 && nshards == 1;
    return pl;
}

size_t scratch_bytes(const Plan& pl, int64_t n, bool rows)
{
    size_t b = pl.part_doubles * sizeof(double) + pl.col_bytes + (size_t)pl.epi_blocks * 7 * sizeof(double) +
               8 * sizeof(double) + pl.zbytes;
    if (rows) b += (size_t)n * kRowOut * sizeof(double);
    return b;
}

// Base-2 exponent coefficients, negated: B = 2^(nab r^2 + nbb dt^2), E = 2^(nae r^2 + nbe dt).
void fold(const hawkes_params& p, PairReq& r)
{
    const double log2e = 1.44269504088896340736;
    r.nab64 = -log2e / (2.0 * p.tau_x * p.tau_x);
    r.nbb64 = -log2e / (2.0 * p.tau_t * p.tau_t);
    r.nae64 = -log2e / (2.0 * p.h * p.h);
    r.nbe64 = -log2e * p.omega;
    r.nab = (float)r.nab64;
    r.nae = (float)r.nae64;
    const double ts = std::sqrt(-r.nbb64);
    r.tsh = (float)ts;
    r.tsl = (float)(ts - (double)r.tsh);
    r.kte = (float)(r.nbe64 / ((double)r.tsh + (double)r.tsl));
}

void fill_epi(const hawkes_params& p, const Dataset& d, const Plan& pl, bool grad, int precision, const Carved& cv,
              EpiReq& e)
{
    const double two_pi = 6.28318530717958647693;
    e.ev64 = d.ev64;
    e.part = cv.part;
    e.colpart = cv.colpart;
    e.col_stride = pl.col_stride;
    e.colpart_f32 = (pl.scheme == kSymmetric && precision == kFP32C) ? 1 : 0;
    e.block_part = cv.block_part;
    e.out7 = cv.out7;
    e.rows_out = cv.rows;
    e.n = (int)d.n;
    e.npad = d.npad;
    e.splits = pl.splits;
    e.grad = grad ? 1 : 0;
    e.scheme = pl.scheme;
    e.row_blocks = pl.row_blocks;
    e.ubase = pl.ubase;
    e.urem = pl.urem;
    e.ubegin = pl.ubegin;
    e.uend = pl.ubegin + pl.units;
    e.add_diag = 1;
    e.nblocks = pl.epi_blocks;
    e.pair_items = pl.items;
    e.dchunks = pl.dchunks;
    e.zcum = cv.zcum;
    e.T = d.T;
    e.mu0 = p.mu0;
    e.tau_x = p.tau_x;
    e.tau_t = p.tau_t;
    e.theta = p.theta;
    e.omega = p.omega;
    e.h = p.h;
    e.cb = p.mu0 / (std::pow(two_pi, 1.5) * p.tau_x * p.tau_x * p.tau_t);
    e.ce = p.theta * p.omega / (two_pi * p.h * p.h);
    PairReq folded;
    fold(p, folded);
    e.t_scale = precision == kFP32C ? (double)folded.tsh + (double)folded.tsl : 1.0;
}

// Time separation from which both exponentials of a pair are exactly zero in the pass's
// arithmetic: the base-2 exponents nbb dt^2 (background) and nbe dt (trigger) are then at most
// -170, far below binary32's smallest subnormal 2^-149 (FP32C), or at most -1110, where the
// binary64 exponential is clamped to 2^-1100 = 0 (FP64).  The spatial parts only lower them.
void zero_gaps(const hawkes_params& p, int precision, double T, double& background, double& trigger)
{
    const double log2e = 1.44269504088896340736;
    const double c = precision == kFP32C ? 170.0 : 1110.0;
    background = p.tau_t * std::sqrt(2.0 * c / log2e);
    trigger = c / (p.omega * log2e);
    if (precision == kFP32C) {
        // The FP32C pass forms time differences from binary32 times (centred, |t - centre| <=
        // T / 2) and its kernel compares a binary32 gap with these: widen them by far more than
        // those roundings can move a difference, so every term left out would have been exactly
        // zero in that arithmetic too.
        const double widen = 1.0 + std::ldexp(1.0, -18), slack = std::ldexp(T, -18);
        background = background * widen + slack;
        trigger = trigger * widen + slack;
    }
}

double zero_separation(const hawkes_params& p, int precision, double T)
{
    double background, trigger;
    zero_gaps(p, precision, T, background, trigger);
    return std::max(background, trigger);
}

void fill_pair(const hawkes_params& p, const Dataset& d, const Plan& pl, const Carved& cv, PairReq& r)
{
    r.ev32 = d.ev32;
    r.ev64 = d.ev64;
    r.cut = d.cut;
    r.part = cv.part;
    r.colpart = cv.colpart;
    r.units = pl.units;
    r.col_stride = pl.col_stride;
    r.n = (int)d.n;
    r.npad = d.npad;
    r.row_blocks = pl.row_blocks;
    r.splits = pl.splits;
    r.tiles_per_split = pl.tiles_per_split;
    r.ubase = pl.ubase;
    r.urem = pl.urem;
    r.ubegin = pl.ubegin;
    r.items = pl.items;
    r.dchunks = pl.dchunks;
    r.ctr = cv.ctr;
    r.zcum = cv.zcum;
    r.zdirect = pl.zdirect ? 1 : 0;
    double gap_b, gap_e;
    zero_gaps(p, pl.precision, d.T, gap_b, gap_e);
    r.zero_dt = std::max(gap_b, gap_e);
    r.zero_gap_b = (float)gap_b;
    r.zero_gap_e = (float)gap_e;
    fold(p, r);
}

hawkes_status hip_fail(hipError_t e, const char* what)
{
    return fail(HAWKES_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Budgeted device allocation; `used` is the caller-held running total.
hawkes_status dev_alloc(hawkes_ctx* c, void** p, size_t bytes)
{
    if (c->used + bytes > c->budget)
        return fail(HAWKES_ENOMEM, "HBM budget exceeded: %zu used + %zu requested > %zu", c->used, bytes, c->budget);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(HAWKES_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    c->used += bytes;
    return HAWKES_OK;
}

void dev_free(hawkes_ctx* c, void* p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    c->used -= bytes;
}

// Blocking-call scratch: on budget exhaustion the serving pool's idle buffers are given back first.
hawkes_status reserve_blocking(hawkes_ctx* c, size_t need)
{
    hawkes_status st = c->blk.reserve(c, need);
    if (st == HAWKES_ENOMEM) {
        server_trim(c);
        st = c->blk.reserve(c, need);
    }
    if (st == HAWKES_ENOMEM && c->scheme == kSymmetric)
        // The symmetric enumeration's column partial sums grow as N^2 / 2048 values per quantity
        // (about 5.9 GB for the FP32C gradient at N = 10^6, binary32); the direct one needs O(N).
        g_last_error += " (the symmetric pair enumeration's scratch grows as N^2; "
                        "hawkes_set_pair_scheme(ctx, HAWKES_PAIRS_DIRECT) needs memory linear in N)";
    return st;
}

hawkes_status Scratch::reserve(hawkes_ctx* c, size_t need)
{
    if (need <= bytes) return HAWKES_OK;
    if (base) {
        // The previous user of this scratch may still run on the device.
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        dev_free(c, base, bytes);
        base = nullptr;
        bytes = 0;
    }
    void* p = nullptr;
    hawkes_status st = dev_alloc(c, &p, need);
    if (st != HAWKES_OK) return st;
    base = (char*)p;
    bytes = need;
    return HAWKES_OK;
}

void Scratch::release(hawkes_ctx* c)
{
    dev_free(c, base, bytes);
    base = nullptr;
    bytes = 0;
}

// Carve one evaluation's scratch: row partials, column partials, block partials, 7 result doubles,
// zero-tile skipping tables, per-row output.
Carved carve(char* base, const Plan& pl, bool rows)
{
    Carved cv;
    double* p = (double*)base;
    cv.part = p;
    p += pl.part_doubles;
    cv.colpart = pl.col_bytes ? p : nullptr;
    p += pl.col_bytes / sizeof(double);
    cv.block_part = p;
    p += (size_t)pl.epi_blocks * 7;
    cv.out7 = p;
    cv.ctr = (unsigned long long*)(p + 7);
    p += 8;
    cv.zcum = pl.zskip ? (long long*)p : nullptr;
    p += pl.zbytes / sizeof(double);
    cv.rows = rows ? p : nullptr;
    return cv;
}

hawkes_status enqueue_eval(hawkes_ctx* c, const Dataset& d, const hawkes_params& p, int precision, bool grad,
                           char* scratch, double* out7_override, double** out7_used, double** rows_out,
                           bool want_rows, hipStream_t s)
{
    const Plan pl = make_plan(c, d.n, d.npad, grad, precision, c->scheme, 0, 1, c->zero_skip);
    Carved cv = carve(scratch, pl, want_rows);
    if (out7_override) cv.out7 = out7_override;

    PairBatch pb;
    memset(&pb, 0, sizeof pb);
    fill_pair(p, d, pl, cv, pb.r[0]);
    pb.r[0].item_begin = 0;
    pb.r[0].balance = 1;
    pb.nreq = 1;
    pb.total_items = pl.items;

    EpiBatch eb;
    memset(&eb, 0, sizeof eb);
    fill_epi(p, d, pl, grad, precision, cv, eb.r[0]);
    eb.r[0].item_begin = 0;
    eb.nreq = 1;
    eb.total_items = pl.epi_blocks;

    hipError_t e;
    if (c->profile) {
        e = hipEventRecord(c->prof_ev[0], s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (pl.zskip) {
        e = launch_zero_prefix(pb, s);
        if (e != hipSuccess) return hip_fail(e, "zero-tile table launch");
    }
    e = launch_pair(pb, precision, grad, pl.scheme, pl.zskip, s);
    if (e != hipSuccess) return hip_fail(e, "pair kernel launch");
    if (c->profile) {
        e = hipEventRecord(c->prof_ev[1], s);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        c->prof_pending = true;
    }
    e = launch_epilogue(eb, s);
    if (e != hipSuccess) return hip_fail(e, "epilogue launch");
    e = launch_final(eb, s);
    if (e != hipSuccess) return hip_fail(e, "final reduction launch");
    if (out7_used) *out7_used = cv.out7;
    if (rows_out) *rows_out = cv.rows;
    return HAWKES_OK;
}

// Adds the last profiled pair-kernel time once the stream has passed it.
void collect_profile(hawkes_ctx* c)
{
    if (!c->prof_pending) return;
    float ms = 0.0f;
    if (hipEventSynchronize(c->prof_ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, c->prof_ev[0], c->prof_ev[1]) == hipSuccess) {
        c->pair_ms += ms;
        c->pair_launches += 1;
    }
    c->prof_pending = false;
}

hawkes_status begin_call(hawkes_ctx* c)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    if (c->poisoned) return fail(HAWKES_EDEVICE, "context is unusable after an earlier device failure");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return HAWKES_OK;
}

hawkes_status poison(hawkes_ctx* c, hawkes_status st)
{
    if (st == HAWKES_EDEVICE) c->poisoned = true;
    return st;
}

Dataset* find_dataset(hawkes_ctx* c, int32_t id)
{
    auto it = c->datasets.find(id);
    return it == c->datasets.end() ? nullptr : it->second.get();
}

// Shared body of the blocking calls.  Holds the context lock for the whole evaluation.
hawkes_status blocking_eval(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, bool grad,
                            double out7[7], double* host_rows)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if ((st = check_params(p)) != HAWKES_OK) return st;
    if (precision != HAWKES_FP64 && precision != HAWKES_FP32C)
        return fail(HAWKES_EINVAL, "precision %d is neither HAWKES_FP64 nor HAWKES_FP32C", precision);
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    const bool want_rows = host_rows != nullptr;
    const Plan pl = make_plan(c, d->n, d->npad, grad, precision, c->scheme, 0, 1, c->zero_skip);
    if ((st = reserve_blocking(c, scratch_bytes(pl, d->n, want_rows))) != HAWKES_OK) return st;
    hipStream_t s = c->stream;
    hipError_t e = hipStreamWaitEvent(s, c->blk_free, 0);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamWaitEvent"));
    double *dout7 = nullptr, *drows = nullptr;
    st = enqueue_eval(c, *d, *p, precision, grad, c->blk.base, nullptr, &dout7, &drows, want_rows, s);
    if (st != HAWKES_OK) return poison(c, st);
    e = hipMemcpyAsync(c->h_out7, dout7, 7 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipMemcpyAsync"));
    std::vector<double> sorted_rows;
    if (want_rows) {
        sorted_rows.resize((size_t)d->n * kRowOut);
        e = hipMemcpyAsync(sorted_rows.data(), drows, sorted_rows.size() * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return poison(c, hip_fail(e, "hipMemcpyAsync"));
    }
    e = hipEventRecord(c->blk_free, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamSynchronize"));
    collect_profile(c);
    memcpy(out7, c->h_out7, 7 * sizeof(double));
    if (want_rows)
        for (int64_t k = 0; k < d->n; ++k)
            memcpy(host_rows + (size_t)d->perm[k] * kRowOut, sorted_rows.data() + (size_t)k * kRowOut,
                   kRowOut * sizeof(double));
    return HAWKES_OK;
}

hawkes_status build_dataset(hawkes_ctx* c, const double* x, const double* y, const double* t, int64_t n,
                            std::unique_ptr<Dataset>& out)
{
    if (!x || !y || !t) return fail(HAWKES_EINVAL, "event pointer is NULL");
    if (n < 1) return fail(HAWKES_EINVAL, "n = %lld < 1", (long long)n);
    if (n > (int64_t)1 << 30) return fail(HAWKES_EINVAL, "n = %lld exceeds 2^30", (long long)n);
    for (int64_t k = 0; k < n; ++k) {
        if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || !std::isfinite(t[k]))
            return fail(HAWKES_EINVAL, "event %lld has a non-finite coordinate", (long long)k);
        if (t[k] < 0.0) return fail(HAWKES_EINVAL, "event %lld has t = %g < 0", (long long)k, t[k]);
        if (std::fabs(x[k]) > 1e15 || std::fabs(y[k]) > 1e15)
            return fail(HAWKES_EINVAL, "event %lld has |x| or |y| > 1e15", (long long)k);
    }
    auto d = std::make_unique<Dataset>();
    d->n = n;
    d->npad = (int)(((n + kPad - 1) / kPad) * kPad);
    d->perm.resize(n);
    std::iota(d->perm.begin(), d->perm.end(), 0);
    std::stable_sort(d->perm.begin(), d->perm.end(), [&](int a, int b) { return t[a] < t[b]; });

    double xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0], tmin = t[0], tmax = t[0];
    for (int64_t k = 1; k < n; ++k) {
        xmin = std::min(xmin, x[k]); xmax = std::max(xmax, x[k]);
        ymin = std::min(ymin, y[k]); ymax = std::max(ymax, y[k]);
        tmin = std::min(tmin, t[k]); tmax = std::max(tmax, t[k]);
    }
    d->T = tmax;
    const double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax), ctm = 0.5 * (tmin + tmax);

    const int np = d->npad;
    std::vector<float4> ev32((size_t)2 * np);
    std::vector<double4> ev64(np);
    std::vector<int> cut(np);
    auto split = [](double v, float& hi, float& lo) {
        hi = (float)v;
        lo = (float)(v - (double)hi);
    };
    int run_start = 0;
    for (int k = 0; k < np; ++k) {
        if (k < n) {
            const int src = d->perm[k];
            float xh, xl, yh, yl, th, tl;
            split(x[src] - cx, xh, xl);
            split(y[src] - cy, yh, yl);
            split(t[src] - ctm, th, tl);
            ev32[2 * k] = make_float4(xh, yh, th, 0.0f);
            ev32[2 * k + 1] = make_float4(xl, yl, tl, 0.0f);
            ev64[k] = make_double4(x[src], y[src], t[src], 0.0);
            if (k > 0 && t[src] != t[d->perm[k - 1]]) run_start = k;
            cut[k] = run_start;  // events before the first one with this time are exactly the earlier ones
        } else {
            ev32[2 * k] = make_float4((float)kSentinel, (float)kSentinel, 0.0f, 0.0f);
            ev32[2 * k + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            ev64[k] = make_double4(kSentinel, kSentinel, 0.0, 0.0);
            cut[k] = (int)n;
        }
    }
    const size_t b32 = ev32.size() * sizeof(float4), b64 = ev64.size() * sizeof(double4), bc = cut.size() * sizeof(int);
    void *p32 = nullptr, *p64 = nullptr, *pc = nullptr;
    hawkes_status st;
    if ((st = dev_alloc(c, &p32, b32)) != HAWKES_OK) return st;
    if ((st = dev_alloc(c, &p64, b64)) != HAWKES_OK) {
        dev_free(c, p32, b32);
        return st;
    }
    if ((st = dev_alloc(c, &pc, bc)) != HAWKES_OK) {
        dev_free(c, p32, b32);
        dev_free(c, p64, b64);
        return st;
    }
    d->ev32 = (float4*)p32;
    d->ev64 = (double4*)p64;
    d->cut = (int*)pc;
    d->bytes = b32 + b64 + bc;
    hipError_t e = hipMemcpy(p32, ev32.data(), b32, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p64, ev64.data(), b64, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pc, cut.data(), bc, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_dataset(c, *d);
        return hip_fail(e, "hipMemcpy (dataset upload)");
    }
    out = std::move(d);
    return HAWKES_OK;
}

void free_dataset(hawkes_ctx* c, Dataset& d)
{
    dev_free(c, d.ev32, (size_t)2 * d.npad * sizeof(float4));
    dev_free(c, d.ev64, (size_t)d.npad * sizeof(double4));
    dev_free(c, d.cut, (size_t)d.npad * sizeof(int));
    d.ev32 = nullptr;
    d.ev64 = nullptr;
    d.cut = nullptr;
}

}  // namespace hawkes

using namespace hawkes;

extern "C" {

const char* hawkes_last_error(void) { return g_last_error.c_str(); }

hawkes_status hawkes_create(int device, size_t hbm_budget_bytes, void* hip_stream, hawkes_ctx** out)
{
    if (!out) return fail(HAWKES_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(HAWKES_EINVAL, "device %d not in [0, %d)", device, ndev);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    auto c = std::make_unique<hawkes_ctx>();
    c->device = device;
    size_t free_b = 0, total_b = 0;
    if ((e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return hip_fail(e, "hipMemGetInfo");
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
        c->own_stream = true;
    }
    if ((e = hipEventCreateWithFlags(&c->blk_free, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->prof_ev[0])) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&c->prof_ev[1])) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipHostMalloc((void**)&c->h_out7, 8 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "hipHostMalloc");
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess)
        return hip_fail(e, "hipDeviceGetAttribute");
    for (int prec = 0; prec < 2; ++prec)
        for (int g = 0; g < 2; ++g) c->sym_slots[prec][g] = cus * sym_blocks_per_cu(prec, g != 0);
    c->multi_slots = cus * multi_blocks_per_cu();
    hawkes_status st = noalloc_init(device);
    if (st != HAWKES_OK) return st;
    st = server_start(c.get());
    if (st != HAWKES_OK) return st;
    *out = c.release();
    return HAWKES_OK;
}

hawkes_status hawkes_destroy(hawkes_ctx* c)
{
    if (!c) return HAWKES_OK;
    (void)hipSetDevice(c->device);
    server_stop(c);
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (auto& kv : c->datasets) free_dataset(c, *kv.second);
        c->datasets.clear();
        c->blk.release(c);
    }
    if (c->h_out7) (void)hipHostFree(c->h_out7);
    (void)hipEventDestroy(c->blk_free);
    (void)hipEventDestroy(c->prof_ev[0]);
    (void)hipEventDestroy(c->prof_ev[1]);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return HAWKES_OK;
}

hawkes_status hawkes_dataset_create(hawkes_ctx* c, const double* x, const double* y, const double* t, int64_t n,
                                    int32_t* out_id)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if (!out_id) return fail(HAWKES_EINVAL, "out_id is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    std::unique_ptr<Dataset> d;
    if ((st = build_dataset(c, x, y, t, n, d)) != HAWKES_OK) return poison(c, st);
    d->id = c->next_id++;
    *out_id = d->id;
    c->datasets[d->id] = std::move(d);
    return HAWKES_OK;
}

hawkes_status hawkes_dataset_destroy(hawkes_ctx* c, int32_t id)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    if (d->inflight > 0) return fail(HAWKES_EBUSY, "dataset %d has %d requests in flight", id, d->inflight);
    // Blocking and device calls may still read it on the device.
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipDeviceSynchronize"));
    free_dataset(c, *d);
    c->datasets.erase(id);
    return HAWKES_OK;
}

hawkes_status hawkes_dataset_info(hawkes_ctx* c, int32_t id, int64_t* n, size_t* device_bytes)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    if (n) *n = d->n;
    if (device_bytes) *device_bytes = d->bytes;
    return HAWKES_OK;
}

hawkes_status hawkes_loglik(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, double* out_loglik)
{
    if (!out_loglik) return fail(HAWKES_EINVAL, "out_loglik is NULL");
    double o[7];
    hawkes_status st = blocking_eval(c, id, p, precision, false, o, nullptr);
    if (st == HAWKES_OK) *out_loglik = o[0];
    return st;
}

hawkes_status hawkes_grad(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, double* out_loglik,
                          double* out_grad)
{
    if (!out_loglik || !out_grad) return fail(HAWKES_EINVAL, "output pointer is NULL");
    double o[7];
    hawkes_status st = blocking_eval(c, id, p, precision, true, o, nullptr);
    if (st == HAWKES_OK) {
        *out_loglik = o[0];
        memcpy(out_grad, o + 1, 6 * sizeof(double));
    }
    return st;
}

hawkes_status hawkes_rows(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, double* out_rows)
{
    if (!out_rows) return fail(HAWKES_EINVAL, "out_rows is NULL");
    double o[7];
    return blocking_eval(c, id, p, precision, true, o, out_rows);
}

hawkes_status hawkes_grad_device(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, double* d_out7,
                                 void* hip_stream)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if (!d_out7) return fail(HAWKES_EINVAL, "d_out7 is NULL");
    if ((st = check_params(p)) != HAWKES_OK) return st;
    if (precision != HAWKES_FP64 && precision != HAWKES_FP32C)
        return fail(HAWKES_EINVAL, "precision %d is neither HAWKES_FP64 nor HAWKES_FP32C", precision);
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    const Plan pl = make_plan(c, d->n, d->npad, true, precision, c->scheme, 0, 1, c->zero_skip);
    if ((st = reserve_blocking(c, scratch_bytes(pl, d->n, false))) != HAWKES_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;  // NULL: the null stream
    // The scratch is shared with every other blocking or device call of this context.
    hipError_t e = hipStreamWaitEvent(s, c->blk_free, 0);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamWaitEvent"));
    st = enqueue_eval(c, *d, *p, precision, true, c->blk.base, d_out7, nullptr, nullptr, false, s);
    if (st != HAWKES_OK) return poison(c, st);
    e = hipEventRecord(c->blk_free, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
    c->prof_pending = false;  // not waited for here; device calls are not profiled
    return HAWKES_OK;
}

hawkes_status hawkes_set_pair_scheme(hawkes_ctx* c, int scheme)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    if (scheme != HAWKES_PAIRS_SYMMETRIC && scheme != HAWKES_PAIRS_DIRECT)
        return fail(HAWKES_EINVAL, "unknown pair scheme %d", scheme);
    std::lock_guard<std::mutex> lk(c->mu);
    c->scheme = scheme == HAWKES_PAIRS_DIRECT ? kDirect : kSymmetric;
    return HAWKES_OK;
}

hawkes_status hawkes_set_zero_tile_skipping(hawkes_ctx* c, int enable)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(HAWKES_EINVAL, "enable must be 0 or 1, not %d", enable);
    std::lock_guard<std::mutex> lk(c->mu);
    c->zero_skip = enable != 0;
    return HAWKES_OK;
}

hawkes_status hawkes_set_shared_passes(hawkes_ctx* c, int enable)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(HAWKES_EINVAL, "enable must be 0 or 1, not %d", enable);
    std::lock_guard<std::mutex> lk(c->mu);
    c->shared_passes = enable != 0;
    return HAWKES_OK;
}

hawkes_status hawkes_profile(hawkes_ctx* c, int enable)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    c->profile = enable != 0;
    return HAWKES_OK;
}

hawkes_status hawkes_kernel_time(hawkes_ctx* c, double* pair_ms, int64_t* pair_launches, int reset)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    if (pair_ms) *pair_ms = c->pair_ms;
    if (pair_launches) *pair_launches = c->pair_launches;
    if (reset) {
        c->pair_ms = 0.0;
        c->pair_launches = 0;
    }
    return HAWKES_OK;
}

}  // extern "C"
