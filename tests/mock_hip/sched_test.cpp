// Scheduler and host-runtime scenarios of libhawkes run against the CPU test double of the device
// (mock_device.cpp), built and run by tests/test_scheduler_cpu.py, also under ThreadSanitizer and
// AddressSanitizer.  Each scenario prints "PASS <name>" or "FAIL <name>: <reason>"; the exit status
// is the number of failed scenarios.
//
// The stand-in device writes loglik = n + mu0 and grad = Theta (zeros without the gradient), so a
// result can be matched to its own request.
#include <hawkes.h>

#include "hawkes_runtime.h"

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

extern "C" {
void mock_set_latency_us(int us);
void mock_fail_launches(int k);
int mock_stamp_errors();
long long mock_device_bytes();
long long mock_peak_device_bytes();
void mock_reset_peak();
void mock_multi_counts(int* passes, int* vectors, int* max_nth);
}

namespace {

int g_failed = 0;

struct Fail {
    std::string why;
};

void check(bool ok, const std::string& why)
{
    if (!ok) throw Fail{why};
}

void run(const char* name, void (*fn)())
{
    try {
        fn();
        std::printf("PASS %s\n", name);
    } catch (const Fail& f) {
        std::printf("FAIL %s: %s (last error: %s)\n", name, f.why.c_str(), hawkes_last_error());
        ++g_failed;
    }
    std::fflush(stdout);
}

int32_t make_dataset(hawkes_ctx* c, int64_t n, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::vector<double> x(n), y(n), t(n);
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 10.0 * u(rng);
        y[i] = 10.0 * u(rng);
        t[i] = 1000.0 * u(rng);
    }
    int32_t id = -1;
    check(hawkes_dataset_create(c, x.data(), y.data(), t.data(), n, &id) == HAWKES_OK, "dataset_create");
    return id;
}

hawkes_params theta(double jitter)
{
    return hawkes_params{1.0 + jitter, 0.5, 20.0, 0.3, 0.5, 0.1};
}

hawkes_request request(int32_t ds, int prec, int grad, double jitter, uint64_t tag)
{
    hawkes_request r;
    std::memset(&r, 0, sizeof r);
    r.dataset = ds;
    r.precision = prec;
    r.want_grad = grad;
    r.p = theta(jitter);
    r.tag = tag;
    return r;
}

// Result of a request as the stand-in device computes it.
bool matches(const hawkes_result& res, const hawkes_request& req, int64_t n)
{
    if (res.status != HAWKES_OK || res.tag != req.tag) return false;
    if (res.loglik != (double)n + req.p.mu0) return false;
    const double th[6] = {req.p.mu0, req.p.tau_x, req.p.tau_t, req.p.theta, req.p.omega, req.p.h};
    for (int k = 0; k < 6; ++k)
        if (res.grad[k] != (req.want_grad ? th[k] : 0.0)) return false;
    return res.t_done_ns >= res.t_submit_ns;
}

// Poll until `count` results arrived (or the deadline passes).
std::vector<hawkes_result> collect(hawkes_ctx* c, size_t count, double seconds = 120.0)
{
    std::vector<hawkes_result> got;
    const auto end = std::chrono::steady_clock::now() + std::chrono::duration<double>(seconds);
    hawkes_result buf[64];
    while (got.size() < count && std::chrono::steady_clock::now() < end) {
        int32_t k = 0;
        const hawkes_status st = hawkes_poll(c, buf, 64, &k, 20000);
        check(st == HAWKES_OK || st == HAWKES_EAGAIN, "poll status");
        got.insert(got.end(), buf, buf + k);
    }
    return got;
}

void basic_mix()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int64_t sizes[3] = {3000, 8000, 16000};
    int32_t ds[3];
    for (int k = 0; k < 3; ++k) ds[k] = make_dataset(c, sizes[k], 10 + k);
    std::mt19937 rng(1);
    std::map<uint64_t, std::pair<hawkes_request, int64_t>> want;
    std::vector<hawkes_request> reqs;
    for (uint64_t tag = 0; tag < 300; ++tag) {
        const int d = rng() % 3;
        reqs.push_back(request(ds[d], rng() % 2, rng() % 2, 1e-3 * tag, tag));
        want[tag] = {reqs.back(), sizes[d]};
    }
    for (size_t k = 0; k < reqs.size(); k += 37)
        check(hawkes_submit(c, reqs.data() + k, (int32_t)std::min<size_t>(37, reqs.size() - k)) == HAWKES_OK, "submit");
    const auto got = collect(c, reqs.size());
    check(got.size() == reqs.size(), "all results arrived");
    std::set<uint64_t> seen;
    for (const auto& r : got) {
        check(seen.insert(r.tag).second, "each tag once");
        check(matches(r, want[r.tag].first, want[r.tag].second), "result matches its request");
    }
    int64_t out = -1;
    check(hawkes_outstanding(c, &out) == HAWKES_OK && out == 0, "nothing outstanding");
    check(mock_stamp_errors() == 0, "scratch of each request is its own");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

// FP32C log-likelihood requests share multi-parameter passes: queued behind a slow launch, 40
// requests over two datasets go out in passes of up to four vectors of one dataset; with shared
// passes off they take the single-parameter path; with zero-tile skipping on, one pass each.
void shared_passes()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int64_t sizes[2] = {4000, 9000};
    const int32_t ds[2] = {make_dataset(c, sizes[0], 30), make_dataset(c, sizes[1], 31)};
    mock_set_latency_us(2000);
    check(hawkes_set_shared_passes(c, 1) == HAWKES_OK, "shared on");
    int p0 = 0, v0 = 0, m0 = 0;
    mock_multi_counts(&p0, &v0, &m0);
    std::vector<hawkes_request> reqs;
    reqs.push_back(request(ds[1], HAWKES_FP32C, 1, 0.0, 0));  // occupies the device first
    for (uint64_t tag = 1; tag <= 40; ++tag) reqs.push_back(request(ds[tag % 2], HAWKES_FP32C, 0, 1e-3 * tag, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    auto got = collect(c, reqs.size());
    check(got.size() == reqs.size(), "all results arrived");
    for (const auto& r : got) check(matches(r, reqs[r.tag], sizes[reqs[r.tag].dataset == ds[1]]), "shared result");
    int p1 = 0, v1 = 0, m1 = 0;
    mock_multi_counts(&p1, &v1, &m1);
    check(v1 - v0 == 40, "every log-likelihood request went through a shared pass");
    check(p1 - p0 < 40 && m1 <= 4 && m1 >= 2, "requests grouped, at most four per pass");
    // Shared passes off: the single-parameter path.
    check(hawkes_set_shared_passes(c, 0) == HAWKES_OK, "shared off");
    reqs.clear();
    for (uint64_t tag = 0; tag < 10; ++tag) reqs.push_back(request(ds[tag % 2], HAWKES_FP32C, 0, 1e-3 * tag, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    got = collect(c, reqs.size());
    for (const auto& r : got) check(matches(r, reqs[r.tag], sizes[reqs[r.tag].dataset == ds[1]]), "unshared result");
    int p2 = 0, v2 = 0, m2 = 0;
    mock_multi_counts(&p2, &v2, &m2);
    check(v2 == v1, "no shared pass with shared passes off");
    // Zero-tile skipping on: one vector per pass.
    check(hawkes_set_shared_passes(c, 1) == HAWKES_OK && hawkes_set_zero_tile_skipping(c, 1) == HAWKES_OK, "settings");
    reqs.clear();
    reqs.push_back(request(ds[1], HAWKES_FP32C, 1, 0.0, 0));
    for (uint64_t tag = 1; tag <= 12; ++tag) reqs.push_back(request(ds[tag % 2], HAWKES_FP32C, 0, 1e-3 * tag, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    got = collect(c, reqs.size());
    for (const auto& r : got) check(matches(r, reqs[r.tag], sizes[reqs[r.tag].dataset == ds[1]]), "skipping result");
    int p3 = 0, v3 = 0, m3 = 0;
    mock_multi_counts(&p3, &v3, &m3);
    check(v3 - v2 == 12 && p3 - p2 == 12, "one vector per pass with zero-tile skipping");
    mock_set_latency_us(200);
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void blocking_beside_serving()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t a = make_dataset(c, 12000, 3), b = make_dataset(c, 5000, 4);
    std::vector<hawkes_request> reqs;
    for (uint64_t tag = 0; tag < 100; ++tag) reqs.push_back(request(a, 1, 1, 0.0, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    for (int k = 0; k < 20; ++k) {
        const hawkes_params p = theta(0.01 * k);
        double ell = 0, g[6];
        check(hawkes_grad(c, b, &p, k % 2, &ell, g) == HAWKES_OK, "blocking grad");
        check(ell == 5000 + p.mu0 && g[1] == p.tau_x, "blocking result");
        check(hawkes_loglik(c, b, &p, k % 2, &ell) == HAWKES_OK && ell == 5000 + p.mu0, "blocking loglik");
    }
    const auto got = collect(c, reqs.size());
    check(got.size() == reqs.size(), "served results arrived");
    for (const auto& r : got) check(matches(r, reqs[r.tag], 12000), "served result");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

// Device bytes one served request of this dataset and kind takes, measured on a roomy context.
long long request_bytes(int64_t n)
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, n, 5);
    const long long before = mock_device_bytes();
    mock_reset_peak();
    hawkes_request r = request(d, 1, 1, 0.0, 0);
    check(hawkes_submit(c, &r, 1) == HAWKES_OK, "submit");
    check(collect(c, 1).size() == 1, "result");
    const long long need = mock_peak_device_bytes() - before;
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
    return need;
}

void tiny_budget_queues()
{
    const int64_t n = 12000;
    const long long need = request_bytes(n);
    hawkes_ctx* c = nullptr;
    // Room for the dataset and for one request's scratch at a time, not two.
    hawkes_ctx* probe = nullptr;
    check(hawkes_create(0, 0, nullptr, &probe) == HAWKES_OK, "create probe");
    const int32_t pd = make_dataset(probe, n, 6);
    size_t ds_bytes = 0;
    int64_t nn = 0;
    check(hawkes_dataset_info(probe, pd, &nn, &ds_bytes) == HAWKES_OK, "dataset_info");
    check(hawkes_destroy(probe) == HAWKES_OK, "destroy probe");
    const size_t budget = ds_bytes + (size_t)(1.5 * need);
    check(hawkes_create(0, budget, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, n, 6);
    const long long base = mock_device_bytes();
    mock_reset_peak();
    std::vector<hawkes_request> reqs;
    for (uint64_t tag = 0; tag < 60; ++tag) reqs.push_back(request(d, 1, 1, 1e-3 * tag, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    const auto got = collect(c, reqs.size());
    check(got.size() == reqs.size(), "every request completes (queued, not refused)");
    for (const auto& r : got) check(matches(r, reqs[r.tag], n), "result under a tiny budget");
    check(mock_peak_device_bytes() - base <= (long long)(1.5 * need), "one request's scratch at a time");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

// The FP32C symmetric pass writes binary32 column partials, the FP64 one binary64: an evaluation's
// scratch holds 4 (FP32C) or 8 (FP64) bytes per column value, carved in that order, and a budget
// sized for k FP32C gradient requests admits k of them at once.
void column_scratch_by_precision()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int64_t n = 50000;
    const int npad = (int)((n + hawkes::kPad - 1) / hawkes::kPad * hawkes::kPad);
    const long long T = npad / hawkes::kRowsPerBlock;
    const long long stride = (long long)hawkes::kRowsPerBlock * T * (T + 1) / 2;
    for (int prec = 0; prec < 2; ++prec)
        for (int grad = 0; grad < 2; ++grad) {
            const hawkes::Plan pl = hawkes::make_plan(c, n, npad, grad != 0, prec, hawkes::kSymmetric);
            const size_t elem = prec == HAWKES_FP32C ? sizeof(float) : sizeof(double);
            const size_t col = ((size_t)(grad ? 3 : 1) * stride * elem + 7) / 8 * 8;
            check(pl.col_stride == stride, "values per column-sum quantity");
            check(pl.col_bytes == col, "column partials sized by the pass's element type");
            const size_t want = pl.part_doubles * sizeof(double) + col + (size_t)pl.epi_blocks * 7 * sizeof(double) +
                                8 * sizeof(double);
            check(hawkes::scratch_bytes(pl, n, false) == want, "scratch bytes of one evaluation");
            std::vector<char> buf(want);
            const hawkes::Carved cv = hawkes::carve(buf.data(), pl, false);
            check((char*)cv.colpart - buf.data() == (ptrdiff_t)(pl.part_doubles * sizeof(double)), "column partials carved after the row partials");
            check((char*)cv.block_part - (char*)cv.colpart == (ptrdiff_t)col, "block partials carved after the column partials");
            check((char*)(cv.out7 + 8) - buf.data() == (ptrdiff_t)want, "the carve fills the scratch exactly");
        }
    // Budget admission: room for the dataset and four FP32C gradient requests (the pool rounds
    // each buffer up to a MiB), not five.
    const hawkes::Plan pl = hawkes::make_plan(c, n, npad, true, HAWKES_FP32C, hawkes::kSymmetric);
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
    const size_t mib = (size_t)1 << 20;
    const size_t per = (hawkes::scratch_bytes(pl, n, false) + mib - 1) / mib * mib;
    hawkes_ctx* probe = nullptr;
    check(hawkes_create(0, 0, nullptr, &probe) == HAWKES_OK, "create probe");
    size_t ds_bytes = 0;
    int64_t nn = 0;
    check(hawkes_dataset_info(probe, make_dataset(probe, n, 16), &nn, &ds_bytes) == HAWKES_OK, "dataset_info");
    check(hawkes_destroy(probe) == HAWKES_OK, "destroy probe");
    mock_set_latency_us(3000);
    check(hawkes_create(0, ds_bytes + 4 * per + per / 2, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, n, 16);
    const long long base = mock_device_bytes();
    mock_reset_peak();
    std::vector<hawkes_request> reqs;
    for (uint64_t tag = 0; tag < 24; ++tag) reqs.push_back(request(d, HAWKES_FP32C, 1, 1e-3 * tag, tag));
    check(hawkes_submit(c, reqs.data(), (int32_t)reqs.size()) == HAWKES_OK, "submit");
    const auto got = collect(c, reqs.size());
    mock_set_latency_us(200);
    check(got.size() == reqs.size(), "every request completes");
    for (const auto& r : got) check(matches(r, reqs[r.tag], n), "result");
    check(mock_peak_device_bytes() - base == (long long)(4 * per), "four FP32C requests' scratch at once");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void too_large_fails_alone()
{
    hawkes_ctx* probe = nullptr;
    check(hawkes_create(0, 0, nullptr, &probe) == HAWKES_OK, "create probe");
    size_t big_bytes = 0, small_bytes = 0;
    int64_t nn = 0;
    check(hawkes_dataset_info(probe, make_dataset(probe, 30000, 7), &nn, &big_bytes) == HAWKES_OK, "info");
    check(hawkes_dataset_info(probe, make_dataset(probe, 2000, 8), &nn, &small_bytes) == HAWKES_OK, "info");
    check(hawkes_destroy(probe) == HAWKES_OK, "destroy probe");
    // The datasets fit, a 30,000-event request's scratch (tens of MB) does not; a 2,000-event one does.
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, big_bytes + small_bytes + (4 << 20), nullptr, &c) == HAWKES_OK, "create");
    const int32_t big = make_dataset(c, 30000, 7), small = make_dataset(c, 2000, 8);
    hawkes_request r[2] = {request(big, 1, 1, 0.0, 1), request(small, 1, 1, 0.0, 2)};
    check(hawkes_submit(c, r, 2) == HAWKES_OK, "submit");
    const auto got = collect(c, 2);
    check(got.size() == 2, "both complete");
    for (const auto& x : got) {
        if (x.tag == 1) check(x.status == HAWKES_ENOMEM, "the request that can never fit gets ENOMEM");
        else check(matches(x, r[1], 2000), "the small request is served");
    }
    check(hawkes_dataset_destroy(c, big) == HAWKES_OK, "dataset with no request in flight can go");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void invalid_requests_fail_alone()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, 4000, 9);
    std::vector<hawkes_request> r;
    r.push_back(request(d, 1, 1, 0.0, 0));
    r.push_back(request(d, 1, 1, 0.0, 1));
    r.back().p.mu0 = NAN;
    r.push_back(request(d, 1, 1, 0.0, 2));
    r.back().p.tau_x = -1.0;
    r.push_back(request(d, 5, 1, 0.0, 3));
    r.push_back(request(d, 1, 2, 0.0, 4));
    r.push_back(request(999, 1, 1, 0.0, 5));
    r.push_back(request(d, 0, 0, 0.0, 6));
    check(hawkes_submit(c, r.data(), (int32_t)r.size()) == HAWKES_OK, "submit");
    check(hawkes_submit(c, nullptr, 1) == HAWKES_EINVAL, "NULL request array");
    const auto got = collect(c, r.size());
    check(got.size() == r.size(), "all complete");
    for (const auto& x : got) {
        if (x.tag == 0 || x.tag == 6) check(matches(x, r[x.tag], 4000), "valid request served");
        else if (x.tag == 5) check(x.status == HAWKES_ENOTFOUND, "unknown dataset");
        else check(x.status == HAWKES_EINVAL, "invalid request");
    }
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void busy_dataset()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, 8000, 11);
    std::vector<hawkes_request> r;
    for (uint64_t tag = 0; tag < 20; ++tag) r.push_back(request(d, 1, 1, 0.0, tag));
    check(hawkes_submit(c, r.data(), (int32_t)r.size()) == HAWKES_OK, "submit");
    check(hawkes_dataset_destroy(c, d) == HAWKES_EBUSY, "EBUSY while requests are in flight");
    check(collect(c, r.size()).size() == r.size(), "all complete");
    check(hawkes_dataset_destroy(c, d) == HAWKES_OK, "destroyed once polled");
    check(hawkes_dataset_destroy(c, d) == HAWKES_ENOTFOUND, "gone");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void many_threads()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int64_t sizes[2] = {4000, 12000};
    const int32_t ds[2] = {make_dataset(c, sizes[0], 12), make_dataset(c, sizes[1], 13)};
    constexpr int kThreadsN = 8, kPer = 100;
    std::mutex mu;
    std::map<uint64_t, hawkes_result> got;
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int w = 0; w < kThreadsN; ++w)
        th.emplace_back([&, w] {
            std::mt19937 rng(100 + w);
            for (int k = 0; k < kPer; k += 10) {
                hawkes_request r[10];
                for (int q = 0; q < 10; ++q) {
                    const uint64_t tag = (uint64_t)w * kPer + k + q;
                    r[q] = request(ds[tag % 2], rng() % 2, rng() % 2, 1e-4 * tag, tag);
                }
                if (hawkes_submit(c, r, 10) != HAWKES_OK) bad += 1;
                hawkes_result buf[16];
                int32_t n = 0;
                if (hawkes_poll(c, buf, 16, &n, 1000) == HAWKES_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    for (int q = 0; q < n; ++q)
                        if (!got.emplace(buf[q].tag, buf[q]).second) bad += 1;
                }
            }
        });
    for (auto& t : th) t.join();
    for (const auto& r : collect(c, kThreadsN * kPer - got.size()))
        if (!got.emplace(r.tag, r).second) bad += 1;
    check(bad == 0, "submits succeed and no tag arrives twice");
    check(got.size() == (size_t)kThreadsN * kPer, "every request completes");
    for (const auto& kv : got) {
        const uint64_t tag = kv.first;
        const hawkes_result& r = kv.second;
        check(r.status == HAWKES_OK && r.loglik == (double)sizes[tag % 2] + theta(1e-4 * tag).mu0, "result matches its request");
    }
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void device_failure_poisons()
{
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, 5000, 14);
    mock_fail_launches(1);
    std::vector<hawkes_request> r;
    for (uint64_t tag = 0; tag < 4; ++tag) r.push_back(request(d, 1, 1, 0.0, tag));
    check(hawkes_submit(c, r.data(), (int32_t)r.size()) == HAWKES_OK, "submit");
    const auto got = collect(c, r.size());
    mock_fail_launches(0);
    check(got.size() == r.size(), "all complete");
    int failed = 0;
    for (const auto& x : got) failed += x.status == HAWKES_EDEVICE;
    check(failed >= 1, "the failed launch's requests report HAWKES_EDEVICE");
    check(hawkes_submit(c, r.data(), 1) == HAWKES_EDEVICE, "the context is unusable afterwards");
    double ell = 0;
    check(hawkes_loglik(c, d, &r[0].p, 1, &ell) == HAWKES_EDEVICE, "blocking calls too");
    check(hawkes_destroy(c) == HAWKES_OK, "destroy");
}

void destroy_in_flight()
{
    const long long before = mock_device_bytes();
    mock_set_latency_us(2000);
    hawkes_ctx* c = nullptr;
    check(hawkes_create(0, 0, nullptr, &c) == HAWKES_OK, "create");
    const int32_t d = make_dataset(c, 8000, 15);
    std::vector<hawkes_request> r;
    for (uint64_t tag = 0; tag < 200; ++tag) r.push_back(request(d, tag % 2, 1, 0.0, tag));
    check(hawkes_submit(c, r.data(), (int32_t)r.size()) == HAWKES_OK, "submit");
    std::this_thread::sleep_for(std::chrono::milliseconds(3));
    check(hawkes_destroy(c) == HAWKES_OK, "destroy with requests pending and in flight");
    mock_set_latency_us(200);
    check(mock_device_bytes() == before, "every device allocation freed");
}

}  // namespace

int main()
{
    run("basic_mix", basic_mix);
    run("blocking_beside_serving", blocking_beside_serving);
    run("shared_passes", shared_passes);
    run("tiny_budget_queues", tiny_budget_queues);
    run("column_scratch_by_precision", column_scratch_by_precision);
    run("too_large_fails_alone", too_large_fails_alone);
    run("invalid_requests_fail_alone", invalid_requests_fail_alone);
    run("busy_dataset", busy_dataset);
    run("many_threads", many_threads);
    run("device_failure_poisons", device_failure_poisons);
    run("destroy_in_flight", destroy_in_flight);
    if (mock_stamp_errors() != 0) {
        std::printf("FAIL scratch: %d evaluations read another request's partial sums\n", mock_stamp_errors());
        ++g_failed;
    }
    return g_failed;
}
