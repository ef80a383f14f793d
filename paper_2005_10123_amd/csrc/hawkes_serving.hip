// hawkes_serving.hip -- continuous batching of likelihood / gradient requests (hawkes_submit /
// hawkes_poll).
//
// Many samplers each ask for one evaluation per proposal (the likelihood step of the paper's
// Algorithm 1).  A scheduler thread per context:
//   * admits queued requests in arrival order while launch slots and the HBM budget allow; each
//     admitted request gets a scratch buffer from a pool (its partial sums and block partials);
//   * packs admitted requests of one kind (precision, with/without gradient) into one launch of
//     the three evaluation kernels -- the work items of all requests in a launch share the grid;
//   * evaluates FP32C log-likelihood requests (no gradient: the requests of Algorithm 1's chains)
//     through the multi-parameter pass when hawkes_set_shared_passes turned that on: the launch's requests on one dataset share passes of up to
//     kMultiTheta parameter vectors (each pair's differences formed once for all of them), and every
//     such request, alone or grouped, gets that pass's result for its vector, which does not depend
//     on the vectors sharing the pass (with zero-tile skipping on, which tiles a pass leaves out
//     depends on all its vectors, so each request then has a pass of its own);
//   * issues each launch on the next of several streams, so a launch built from requests that
//     arrived while earlier ones were running overlaps them on the device;
//   * reaps finished launches by event query, returns the scratch to the pool and publishes the
//     results for hawkes_poll.
// Every request is evaluated with the plan of its own (n, gradient) and its own scratch (or its
// pass's), so its result is bitwise the same alone or in any mix: with the gradient, and in FP64,
// the blocking call's; FP32C log-likelihoods, hawkes_loglik_multi's for that vector (equal to the
// blocking call's to rounding).
#include "hawkes_runtime.h"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace hawkes {

namespace {

constexpr int kStreams = 3;
constexpr int kMaxLaunches = 8;
constexpr int kMaxAdmitted = 64;

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Pending {
    hawkes_request req;
    uint64_t t_submit;
};

struct PoolBuf {
    Scratch s;
    bool busy = false;
};

struct Launch {
    bool busy = false;
    bool failed = false;  // an enqueue step failed: complete every request with HAWKES_EDEVICE
    hipEvent_t done = nullptr;
    double* d_out = nullptr;  // kMaxBatch x 8 doubles
    double* h_out = nullptr;  // pinned mirror
    int nreq = 0;
    Pending req[kMaxBatch];
    int buf[kMaxBatch];
};

}  // namespace

struct Server {
    std::mutex mu;  // pending, done, outstanding, stop
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> pending;
    std::deque<hawkes_result> done;
    int64_t outstanding = 0;
    bool stop = false;
    std::thread th;
    hipStream_t streams[kStreams] = {};
    int next_stream = 0;
    // Scheduler-thread state (pool buffers are allocated under the context lock).
    std::vector<PoolBuf> pool;
    Launch launches[kMaxLaunches];
    int admitted = 0;
};

namespace {

hawkes_result make_result(const Pending& p, hawkes_status st)
{
    hawkes_result r;
    memset(&r, 0, sizeof r);
    r.tag = p.req.tag;
    r.status = st;
    r.t_submit_ns = p.t_submit;
    r.t_done_ns = now_ns();
    return r;
}

void publish(Server* sv, const hawkes_result* r, int n)
{
    std::lock_guard<std::mutex> lk(sv->mu);
    for (int k = 0; k < n; ++k) sv->done.push_back(r[k]);
    sv->cv_done.notify_all();
}

// Pool buffer of at least `need` bytes, or -1 if the budget cannot provide one right now.
// Caller holds c->mu.
int get_buffer(hawkes_ctx* c, Server* sv, size_t need)
{
    int best = -1;
    for (int k = 0; k < (int)sv->pool.size(); ++k) {
        const PoolBuf& b = sv->pool[k];
        if (!b.busy && b.s.bytes >= need && (best < 0 || b.s.bytes < sv->pool[best].s.bytes)) best = k;
    }
    if (best >= 0) return best;
    const size_t round = (size_t)1 << 20;
    const size_t want = (need + round - 1) / round * round;
    if (c->used + want > c->budget) {
        // Give back idle buffers (too small for this request) before giving up.  Entries stay in
        // the pool so the indices held by running launches remain valid.
        for (auto& b : sv->pool)
            if (!b.busy && b.s.base) b.s.release(c);
        if (c->used + want > c->budget) return -1;
    }
    int slot = -1;
    for (int k = 0; k < (int)sv->pool.size(); ++k)
        if (!sv->pool[k].busy && !sv->pool[k].s.base) slot = k;
    if (slot < 0) {
        sv->pool.push_back(PoolBuf());
        slot = (int)sv->pool.size() - 1;
    }
    if (sv->pool[slot].s.reserve(c, want) != HAWKES_OK) return -1;
    return slot;
}

void reap(hawkes_ctx* c, Server* sv)
{
    for (auto& L : sv->launches) {
        if (!L.busy) continue;
        hipError_t e = L.failed ? hipSuccess : hipEventQuery(L.done);
        if (e == hipErrorNotReady) continue;
        hawkes_result res[kMaxBatch];
        const hawkes_status st = (e == hipSuccess && !L.failed) ? HAWKES_OK : HAWKES_EDEVICE;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            for (int k = 0; k < L.nreq; ++k) {
                res[k] = make_result(L.req[k], st);
                if (st == HAWKES_OK) {
                    res[k].loglik = L.h_out[8 * k];
                    if (L.req[k].req.want_grad)
                        for (int p = 0; p < 6; ++p) res[k].grad[p] = L.h_out[8 * k + 1 + p];
                }
                sv->pool[L.buf[k]].busy = false;
                if (Dataset* d = find_dataset(c, L.req[k].req.dataset)) d->inflight -= 1;
            }
            if (st != HAWKES_OK) c->poisoned = true;
        }
        sv->admitted -= L.nreq;
        L.busy = false;
        publish(sv, res, L.nreq);
    }
}

int free_launch(Server* sv)
{
    for (int k = 0; k < kMaxLaunches; ++k)
        if (!sv->launches[k].busy) return k;
    return -1;
}

bool any_busy(Server* sv)
{
    for (auto& L : sv->launches)
        if (L.busy) return true;
    return false;
}

// Launch FP32C log-likelihood requests (`cand`, arrival order) as multi-parameter passes: requests
// on one dataset in groups of up to kMultiTheta (one without zero-tile skipping), each group with
// one pool buffer, its requests contiguous in L.req and their results at d_out + 8 k.  Returns false
// when the launch could not start everything (requests waiting for memory go back to the queue).
bool admit_shared(hawkes_ctx* c, Server* sv, Launch& L, const std::vector<Pending>& cand)
{
    struct Group {
        Dataset* d = nullptr;
        int first = 0, count = 0, buf = -1;
        hawkes_params th[kMultiTheta];
    };
    std::vector<Group> groups;
    std::vector<Pending> back;
    std::vector<hawkes_result> failed;
    int nb = 0;
    bool zero_skip = false;
    hipStream_t s = sv->streams[sv->next_stream];
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        zero_skip = c->zero_skip;
        const int per_pass = zero_skip ? 1 : kMultiTheta;
        // Group by dataset, keeping arrival order within each dataset.
        std::vector<std::vector<const Pending*>> by_ds;
        std::vector<Dataset*> ds;
        for (const Pending& p : cand) {
            Dataset* d = find_dataset(c, p.req.dataset);
            if (!d) {
                failed.push_back(make_result(p, HAWKES_ENOTFOUND));
                continue;
            }
            size_t k = 0;
            while (k < ds.size() && ds[k] != d) ++k;
            if (k == ds.size()) {
                ds.push_back(d);
                by_ds.emplace_back();
            }
            by_ds[k].push_back(&p);
        }
        for (size_t k = 0; k < ds.size(); ++k)
            for (size_t a = 0; a < by_ds[k].size(); a += per_pass) {
                Group g;
                g.d = ds[k];
                g.count = (int)std::min<size_t>(per_pass, by_ds[k].size() - a);
                const size_t need = multi_scratch_bytes(c, *g.d, zero_skip, false);
                g.buf = back.empty() ? get_buffer(c, sv, need) : -1;
                if (g.buf < 0) {
                    for (int q = 0; q < g.count; ++q) {
                        const Pending& p = *by_ds[k][a + q];
                        if (!back.empty() || nb > 0 || sv->admitted > 0 || any_busy(sv)) {
                            back.push_back(p);  // wait for memory held by running work
                        } else {
                            g.d->inflight -= 1;
                            failed.push_back(make_result(p, HAWKES_ENOMEM));
                        }
                    }
                    continue;
                }
                sv->pool[g.buf].busy = true;
                g.first = nb;
                for (int q = 0; q < g.count; ++q) {
                    L.req[nb] = *by_ds[k][a + q];
                    L.buf[nb] = g.buf;
                    g.th[q] = L.req[nb].req.p;
                    ++nb;
                }
                groups.push_back(g);
            }
        for (const Group& g : groups) {
            e = enqueue_multi_fp32c(c, *g.d, g.th, g.count, sv->pool[g.buf].s.base, zero_skip, L.d_out + 8 * g.first, 8,
                                    nullptr, s);
            if (e != hipSuccess) break;
        }
    }
    if (!failed.empty()) publish(sv, failed.data(), (int)failed.size());
    if (!back.empty()) {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto it = back.rbegin(); it != back.rend(); ++it) sv->pending.push_front(*it);
    }
    if (nb == 0) return back.empty();
    sv->next_stream = (sv->next_stream + 1) % kStreams;
    if (e == hipSuccess) e = hipMemcpyAsync(L.h_out, L.d_out, (size_t)nb * 8 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(L.done, s);
    L.nreq = nb;
    sv->admitted += nb;
    L.busy = true;
    L.failed = e != hipSuccess;  // reaped as a device failure on the next pass
    if (L.failed) (void)hipStreamSynchronize(s);
    return back.empty();
}

// Admit and launch as much queued work as slots and budget allow.
void admit(hawkes_ctx* c, Server* sv)
{
    while (true) {
        const int li = free_launch(sv);
        if (li < 0 || sv->admitted >= kMaxAdmitted) return;
        Launch& L = sv->launches[li];
        bool shared = false, zero_skip_now = false;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            shared = c->shared_passes;
            zero_skip_now = c->zero_skip;
        }
        std::vector<Pending> cand;
        bool shared_kind = false;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->pending.empty()) return;
            // The head request decides the kind of this launch; later requests of the same kind
            // join it (up to kMaxBatch); requests of other kinds keep their place in the queue.
            // For shared passes, a queued request joins its dataset's pass while that holds fewer
            // than kMultiTheta vectors, and starts a new one only while the launch has room.
            const int prec = sv->pending.front().req.precision, grad = sv->pending.front().req.want_grad;
            shared_kind = shared && prec == HAWKES_FP32C && !grad;
            const int per_pass = zero_skip_now ? 1 : kMultiTheta;
            std::vector<std::pair<int32_t, int>> passes;  // (dataset, requests in its open pass)
            int slots = 0;                                 // requests the launch's passes can hold
            for (auto it = sv->pending.begin(); it != sv->pending.end();) {
                bool take = false;
                if (it->req.precision == prec && it->req.want_grad == grad &&
                    sv->admitted + (int)cand.size() < kMaxAdmitted) {
                    if (!shared_kind) {
                        take = (int)cand.size() < kMaxBatch;
                    } else {
                        auto ps = std::find_if(passes.begin(), passes.end(), [&](const std::pair<int32_t, int>& q) {
                            return q.first == it->req.dataset && q.second < per_pass;
                        });
                        if (ps != passes.end()) {
                            ps->second += 1;
                            take = true;
                        } else if (slots + per_pass <= kMaxBatch) {
                            passes.emplace_back(it->req.dataset, 1);
                            slots += per_pass;
                            take = true;
                        }
                    }
                }
                if (take) {
                    cand.push_back(*it);
                    it = sv->pending.erase(it);
                } else {
                    ++it;
                }
                if (!shared_kind && (int)cand.size() >= kMaxBatch) break;
            }
        }
        if (shared_kind && !cand.empty()) {
            if (!admit_shared(c, sv, L, cand)) return;
            continue;
        }
        PairBatch pb;
        EpiBatch eb;
        memset(&pb, 0, sizeof pb);
        memset(&eb, 0, sizeof eb);
        int nb = 0, items = 0, epi_items = 0;
        std::vector<Pending> back;  // could not get memory now: return to the queue front
        std::vector<hawkes_result> failed;
        int scheme = kSymmetric;
        bool zero_skip = false;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            scheme = c->scheme;
            zero_skip = c->zero_skip;
            for (size_t k = 0; k < cand.size(); ++k) {
                const Pending& p = cand[k];
                Dataset* d = find_dataset(c, p.req.dataset);
                if (!d) {
                    failed.push_back(make_result(p, HAWKES_ENOTFOUND));
                    continue;
                }
                const bool grad = p.req.want_grad != 0;
                const Plan pl = make_plan(c, d->n, d->npad, grad, p.req.precision, scheme, 0, 1, zero_skip);
                const size_t need = scratch_bytes(pl, d->n, false);
                int bi = back.empty() ? get_buffer(c, sv, need) : -1;
                if (bi < 0) {
                    if (!back.empty() || sv->admitted + nb > 0 || any_busy(sv)) {
                        back.push_back(p);  // wait for memory held by running work
                    } else {
                        d->inflight -= 1;
                        failed.push_back(make_result(p, HAWKES_ENOMEM));
                    }
                    continue;
                }
                sv->pool[bi].busy = true;
                Carved cv = carve(sv->pool[bi].s.base, pl, false);
                cv.out7 = L.d_out + 8 * nb;
                fill_pair(p.req.p, *d, pl, cv, pb.r[nb]);
                pb.r[nb].item_begin = items;
                pb.r[nb].balance = 0;  // launches overlap here; later batches fill the CUs
                items += pl.items;
                fill_epi(p.req.p, *d, pl, grad, p.req.precision, cv, eb.r[nb]);
                eb.r[nb].item_begin = epi_items;
                epi_items += pl.epi_blocks;
                L.req[nb] = p;
                L.buf[nb] = bi;
                ++nb;
            }
        }
        if (!failed.empty()) publish(sv, failed.data(), (int)failed.size());
        if (!back.empty()) {
            std::lock_guard<std::mutex> lk(sv->mu);
            for (auto it = back.rbegin(); it != back.rend(); ++it) sv->pending.push_front(*it);
        }
        if (nb == 0) return;
        pb.nreq = eb.nreq = nb;
        pb.total_items = items;
        eb.total_items = epi_items;
        hipStream_t s = sv->streams[sv->next_stream];
        sv->next_stream = (sv->next_stream + 1) % kStreams;
        const int prec = L.req[0].req.precision;
        const bool grad = L.req[0].req.want_grad != 0;
        hipError_t e = hipSuccess;
        if (zero_skip && scheme == kSymmetric) e = launch_zero_prefix(pb, s);
        if (e == hipSuccess) e = launch_pair(pb, prec, grad, scheme, zero_skip && scheme == kSymmetric, s);
        if (e == hipSuccess) e = launch_epilogue(eb, s);
        if (e == hipSuccess) e = launch_final(eb, s);
        if (e == hipSuccess) e = hipMemcpyAsync(L.h_out, L.d_out, (size_t)nb * 8 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(L.done, s);
        L.nreq = nb;
        sv->admitted += nb;
        L.busy = true;
        L.failed = e != hipSuccess;  // reaped as a device failure on the next pass
        if (L.failed) {
            // Let the device finish whatever was enqueued before the scratch is reused.
            (void)hipStreamSynchronize(s);
        }
        if (!back.empty()) return;
    }
}

void scheduler(hawkes_ctx* c)
{
    Server* sv = c->server;
    (void)hipSetDevice(c->device);
    while (true) {
        reap(c, sv);
        admit(c, sv);
        std::unique_lock<std::mutex> lk(sv->mu);
        if (sv->stop) break;
        if (any_busy(sv)) {
            // Launches in flight: look again soon (completion is observed by event query).
            sv->cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
        }
        if (sv->stop) break;
    }
}

}  // namespace

hawkes_status server_start(hawkes_ctx* c)
{
    auto sv = std::make_unique<Server>();
    hipError_t e;
    for (auto& s : sv->streams)
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
    for (auto& L : sv->launches) {
        if ((e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
        if ((e = hipMalloc((void**)&L.d_out, kMaxBatch * 8 * sizeof(double))) != hipSuccess) return hip_fail(e, "hipMalloc");
        if ((e = hipHostMalloc((void**)&L.h_out, kMaxBatch * 8 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
            return hip_fail(e, "hipHostMalloc");
    }
    c->server = sv.release();
    c->server->th = std::thread(scheduler, c);
    return HAWKES_OK;
}

void server_trim(hawkes_ctx* c)
{
    Server* sv = c->server;
    if (!sv) return;
    for (auto& b : sv->pool)
        if (!b.busy && b.s.base) b.s.release(c);
}

void server_stop(hawkes_ctx* c)
{
    Server* sv = c->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (auto& b : sv->pool) b.s.release(c);
    }
    for (auto& L : sv->launches) {
        (void)hipEventDestroy(L.done);
        (void)hipFree(L.d_out);
        (void)hipHostFree(L.h_out);
    }
    for (auto& s : sv->streams) (void)hipStreamDestroy(s);
    c->server = nullptr;
    delete sv;
}

}  // namespace hawkes

using namespace hawkes;

extern "C" {

hawkes_status hawkes_submit(hawkes_ctx* c, const hawkes_request* reqs, int32_t n)
{
    if (!c) return fail(HAWKES_EINVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && !reqs)) return fail(HAWKES_EINVAL, "bad request array");
    if (c->poisoned) return fail(HAWKES_EDEVICE, "context is unusable after an earlier device failure");
    Server* sv = c->server;
    const uint64_t t = now_ns();
    std::vector<Pending> ok;
    std::vector<hawkes_result> bad;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (int k = 0; k < n; ++k) {
            Pending p{reqs[k], t};
            hawkes_status st = check_params(&reqs[k].p);
            if (st == HAWKES_OK && reqs[k].precision != HAWKES_FP64 && reqs[k].precision != HAWKES_FP32C)
                st = HAWKES_EINVAL;
            if (st == HAWKES_OK && reqs[k].want_grad != 0 && reqs[k].want_grad != 1) st = HAWKES_EINVAL;
            Dataset* d = st == HAWKES_OK ? find_dataset(c, reqs[k].dataset) : nullptr;
            if (st == HAWKES_OK && !d) st = HAWKES_ENOTFOUND;
            if (st != HAWKES_OK) {
                bad.push_back(make_result(p, st));
                continue;
            }
            d->inflight += 1;
            ok.push_back(p);
        }
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto& p : ok) sv->pending.push_back(p);
        for (auto& r : bad) sv->done.push_back(r);
        sv->outstanding += n;
        sv->cv_work.notify_all();
        if (!bad.empty()) sv->cv_done.notify_all();
    }
    return HAWKES_OK;
}

hawkes_status hawkes_poll(hawkes_ctx* c, hawkes_result* out, int32_t cap, int32_t* n_out, int64_t timeout_us)
{
    if (!c || !n_out || cap < 0 || (cap > 0 && !out)) return fail(HAWKES_EINVAL, "bad poll arguments");
    *n_out = 0;
    Server* sv = c->server;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return !sv->done.empty() || sv->stop; };
    if (timeout_us > 0)
        sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    else if (timeout_us < 0)
        sv->cv_done.wait(lk, [&] { return ready() || sv->outstanding == 0; });
    int32_t k = 0;
    while (k < cap && !sv->done.empty()) {
        out[k++] = sv->done.front();
        sv->done.pop_front();
    }
    sv->outstanding -= k;
    *n_out = k;
    if (k == 0) {
        g_last_error = "no completed request";  // an ordinary outcome: not logged as a failure
        return HAWKES_EAGAIN;
    }
    return HAWKES_OK;
}

hawkes_status hawkes_outstanding(hawkes_ctx* c, int64_t* n)
{
    if (!c || !n) return fail(HAWKES_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> lk(c->server->mu);
    *n = c->server->outstanding;
    return HAWKES_OK;
}

}  // extern "C"
