// hawkes_noalloc.hip -- hawkes_grad_device_noalloc: hawkes_grad_device with its evaluation scratch
// in a fixed device array instead of memory the context allocates, for callers that cannot
// allocate device memory (work captured into a HIP graph, serving loops or harnesses that forbid
// it).  The kernels, the plan and the summation order are those of hawkes_grad_device; only where
// the row and column partial sums, block partials and zero-tile tables live differs.
#include "hawkes_runtime.h"

namespace hawkes {

namespace {

constexpr int kMaxDevices = 64;

// The evaluation scratch of every hawkes_grad_device_noalloc call on one GPU.  Each device the
// library runs on holds its own copy until the process ends.  Host code never passes this name to
// a kernel or a copy (on the host it is only a stand-in for the symbol): it uses the address
// hipGetSymbolAddress returned for the device, kept in g_scratch.
__device__ __align__(256) char scratch[kNoallocScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

}  // namespace

// Called by hawkes_create with `device` current.
hawkes_status noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(HAWKES_EINVAL, "device %d beyond the %d devices the fixed scratch is kept for", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return HAWKES_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(HAWKES_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[device] = (char*)p;
    return HAWKES_OK;
}

}  // namespace hawkes

using namespace hawkes;

extern "C" hawkes_status hawkes_grad_device_noalloc(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision,
                                                    double* d_out7, void* hip_stream)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if (!d_out7) return fail(HAWKES_EINVAL, "d_out7 is NULL");
    if ((st = check_params(p)) != HAWKES_OK) return st;
    if (precision != HAWKES_FP64 && precision != HAWKES_FP32C)
        return fail(HAWKES_EINVAL, "precision %d is neither HAWKES_FP64 nor HAWKES_FP32C", precision);
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_scratch[c->device];
    }
    if (!base) return fail(HAWKES_EDEVICE, "no fixed scratch address for device %d", c->device);
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    const Plan pl = make_plan(c, d->n, d->npad, true, precision, c->scheme, 0, 1, c->zero_skip);
    const size_t need = scratch_bytes(pl, d->n, false);
    if (need > kNoallocScratchBytes)
        return fail(HAWKES_ENOMEM,
                    "dataset %d (n = %lld) needs %zu bytes of evaluation scratch, more than the fixed %zu of "
                    "hawkes_grad_device_noalloc%s",
                    id, (long long)d->n, need, kNoallocScratchBytes,
                    c->scheme == kSymmetric ? " (the direct pair enumeration needs memory linear in n)" : "");
    // Every kernel writes each scratch value it later reads, so nothing needs clearing between calls.
    st = enqueue_eval(c, *d, *p, precision, true, base, d_out7, nullptr, nullptr, false, (hipStream_t)hip_stream);
    if (st != HAWKES_OK) return poison(c, st);
    c->prof_pending = false;  // not waited for here; device calls are not profiled
    return HAWKES_OK;
}
