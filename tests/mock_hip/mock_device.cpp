// Test double of the device side of libhawkes, for building its host runtime and scheduler on the
// CPU (tests/test_scheduler_cpu.py).  Not a production path: nothing here computes the
// likelihood.
//
// * "Device" memory is host memory; copies happen when they are enqueued.
// * Every stream keeps the time until which its enqueued work runs; each pairwise launch adds a
//   fixed latency to it, and an event recorded on the stream completes at that time.  Launches
//   therefore stay in flight for a while, as on the device, and several streams overlap.
// * The pairwise launch stamps each request's row partials with a value derived from that
//   request; the epilogue checks the stamp (a scratch buffer shared by two requests of a batch
//   would fail it) and the final step writes a stand-in result: loglik = n + mu0 and, with the
//   gradient, grad = (mu0, tau_x, tau_t, theta, omega, h).
// * mock_fail_launches(k) makes the next k pairwise launches fail, as a device error would.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

#include "hawkes_internal.h"
#include "hawkes_runtime.h"

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

std::atomic<int64_t> g_latency_ns{200000};
std::atomic<int> g_fail_launches{0};
std::atomic<int> g_stamp_errors{0};
std::atomic<int64_t> g_device_bytes{0};
std::atomic<int64_t> g_peak_device_bytes{0};
constexpr size_t kTotalBytes = (size_t)64 << 30;

void wait_until(int64_t t)
{
    const int64_t now = now_ns();
    if (t > now) std::this_thread::sleep_for(std::chrono::nanoseconds(t - now));
}

// Allocations carry their size in a header, for the device-memory accounting.
void* alloc_tracked(size_t bytes)
{
    char* p = (char*)std::malloc(bytes + 64);
    if (!p) return nullptr;
    std::memcpy(p, &bytes, sizeof bytes);
    std::memset(p + 64, 0xff, bytes);  // NaN in every double: results never come from stale memory
    const int64_t used = g_device_bytes += (int64_t)bytes;
    int64_t peak = g_peak_device_bytes.load();
    while (used > peak && !g_peak_device_bytes.compare_exchange_weak(peak, used)) {
    }
    return p + 64;
}

void free_tracked(void* q)
{
    if (!q) return;
    char* p = (char*)q - 64;
    size_t bytes;
    std::memcpy(&bytes, p, sizeof bytes);
    g_device_bytes -= (int64_t)bytes;
    std::free(p);
}

}  // namespace

struct MockStream {
    std::mutex mu;
    int64_t busy_until = 0;
    int64_t advance(int64_t latency)
    {
        std::lock_guard<std::mutex> lk(mu);
        busy_until = std::max(busy_until, now_ns()) + latency;
        return busy_until;
    }
    int64_t until()
    {
        std::lock_guard<std::mutex> lk(mu);
        return busy_until;
    }
};

struct MockEvent {
    std::atomic<int64_t> ready_ns{0};
    std::atomic<int64_t> record_ns{0};
};

namespace {

MockStream g_null_stream;
std::mutex g_streams_mu;
MockStream* g_streams[256];
int g_nstreams = 0;

MockStream* stream_of(hipStream_t s) { return s ? s : &g_null_stream; }

}  // namespace

extern "C" {
std::atomic<int> g_multi_passes{0}, g_multi_vectors{0}, g_multi_max_nth{0};
void mock_multi_counts(int* passes, int* vectors, int* max_nth)
{
    *passes = g_multi_passes.load();
    *vectors = g_multi_vectors.load();
    *max_nth = g_multi_max_nth.load();
}
void mock_set_latency_us(int us) { g_latency_ns = (int64_t)us * 1000; }
void mock_fail_launches(int k) { g_fail_launches = k; }
int mock_stamp_errors() { return g_stamp_errors.load(); }
long long mock_device_bytes() { return (long long)g_device_bytes.load(); }
long long mock_peak_device_bytes() { return (long long)g_peak_device_bytes.load(); }
void mock_reset_peak() { g_peak_device_bytes = g_device_bytes.load(); }
}

hipError_t hipGetDeviceCount(int* n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t, int)
{
    *value = 256;
    return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* free_bytes, size_t* total_bytes)
{
    *total_bytes = kTotalBytes;
    *free_bytes = kTotalBytes - (size_t)g_device_bytes.load();
    return hipSuccess;
}
hipError_t hipDeviceSynchronize()
{
    int64_t t = g_null_stream.until();
    {
        std::lock_guard<std::mutex> lk(g_streams_mu);
        for (int k = 0; k < g_nstreams; ++k)
            if (g_streams[k]) t = std::max(t, g_streams[k]->until());
    }
    wait_until(t);
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock device error"; }

hipError_t hipMalloc(void** p, size_t bytes)
{
    *p = alloc_tracked(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p)
{
    free_tracked(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned)
{
    *p = std::malloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p)
{
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind)
{
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t)
{
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned)
{
    *s = new MockStream;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    for (int k = 0; k < g_nstreams; ++k)
        if (!g_streams[k]) {
            g_streams[k] = *s;
            return hipSuccess;
        }
    if (g_nstreams == 256) return hipErrorOutOfMemory;
    g_streams[g_nstreams++] = *s;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    {
        std::lock_guard<std::mutex> lk(g_streams_mu);
        for (int k = 0; k < g_nstreams; ++k)
            if (g_streams[k] == s) g_streams[k] = nullptr;
    }
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    wait_until(stream_of(s)->until());
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    MockStream* st = stream_of(s);
    std::lock_guard<std::mutex> lk(st->mu);
    st->busy_until = std::max(st->busy_until, e->ready_ns.load());
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e)
{
    *e = new MockEvent;
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    const int64_t t = stream_of(s)->until();
    e->record_ns = std::max(t, now_ns());
    e->ready_ns = std::max(t, now_ns());
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) { return now_ns() >= e->ready_ns.load() ? hipSuccess : hipErrorNotReady; }
hipError_t hipEventSynchronize(hipEvent_t e)
{
    wait_until(e->ready_ns.load());
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    *ms = (float)((b->ready_ns.load() - a->record_ns.load()) * 1e-6);
    return hipSuccess;
}

namespace hawkes {

namespace {

double stamp(int n, double nab64) { return (double)n + nab64; }

}  // namespace

hipError_t launch_pair(const PairBatch& b, int, bool, int, bool, hipStream_t s)
{
    if (g_fail_launches.load() > 0 && g_fail_launches.fetch_sub(1) > 0) return hipErrorLaunchFailure;
    for (int k = 0; k < b.nreq; ++k) b.r[k].part[0] = stamp(b.r[k].n, b.r[k].nab64);
    stream_of(s)->advance(g_latency_ns.load());
    return hipSuccess;
}

hipError_t launch_zero_prefix(const PairBatch&, hipStream_t) { return hipSuccess; }

int sym_blocks_per_cu(int precision, bool) { return precision == 0 ? 2 : 3; }

int multi_blocks_per_cu() { return 2; }

// The fixed-scratch entry point (hawkes_noalloc.hip) is device code only; its set-up call is a no-op here.
hawkes_status noalloc_init(int) { return HAWKES_OK; }

hipError_t launch_epilogue(const EpiBatch& b, hipStream_t)
{
    const double log2e = 1.44269504088896340736;
    for (int k = 0; k < b.nreq; ++k) {
        const EpiReq& e = b.r[k];
        const double nab64 = -log2e / (2.0 * e.tau_x * e.tau_x);
        if (e.part[0] != stamp(e.n, nab64)) g_stamp_errors += 1;
        if (e.rows_out)
            for (long long i = 0; i < (long long)e.n * kRowOut; ++i) e.rows_out[i] = 0.0;
        if (e.sums_out)
            for (long long i = 0; i < (long long)e.n * 6; ++i) e.sums_out[i] = 0.0;
    }
    return hipSuccess;
}

// The multi-parameter pass: its scratch is one stamped row-partial area per pass; the stand-in
// result of vector q (ell = n + mu0) goes to out[q * out_stride].
size_t multi_scratch_bytes(const hawkes_ctx*, const Dataset& d, bool, bool) { return (size_t)(d.n + 64) * sizeof(double); }

hipError_t enqueue_multi_fp32c(const hawkes_ctx*, const Dataset& d, const hawkes_params* th, int nth, char* scratch,
                               bool, double* out, int out_stride, double*, hipStream_t s)
{
    if (g_fail_launches.load() > 0 && g_fail_launches.fetch_sub(1) > 0) return hipErrorLaunchFailure;
    g_multi_passes += 1;
    g_multi_vectors += nth;
    int m = g_multi_max_nth.load();
    while (nth > m && !g_multi_max_nth.compare_exchange_weak(m, nth)) {
    }
    double* part = (double*)scratch;
    part[0] = stamp((int)d.n, th[0].mu0);
    stream_of(s)->advance(g_latency_ns.load());
    if (part[0] != stamp((int)d.n, th[0].mu0)) g_stamp_errors += 1;
    for (int q = 0; q < nth; ++q) out[(size_t)q * out_stride] = (double)d.n + th[q].mu0;
    return hipSuccess;
}

hipError_t launch_final(const EpiBatch& b, hipStream_t)
{
    for (int k = 0; k < b.nreq; ++k) {
        const EpiReq& e = b.r[k];
        if (e.sums_out) continue;
        e.out7[0] = e.n + e.mu0;
        const double th[6] = {e.mu0, e.tau_x, e.tau_t, e.theta, e.omega, e.h};
        for (int p = 0; p < 6; ++p) e.out7[1 + p] = e.grad ? th[p] : 0.0;
    }
    return hipSuccess;
}

}  // namespace hawkes
