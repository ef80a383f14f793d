// hawkes_runtime.h -- host-side state of a libhawkes context (not part of the public ABI).
#pragma once

#include "../../include/hawkes.h"
#include "hawkes_internal.h"

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace hawkes {

struct Dataset {
    int32_t id = -1;
    int64_t n = 0;
    int npad = 0;
    float4* ev32 = nullptr;
    double4* ev64 = nullptr;
    int* cut = nullptr;
    size_t bytes = 0;
    std::vector<int> perm;  // sorted position -> caller index
    double T = 0.0;         // largest event time
    int inflight = 0;       // submitted requests not yet completed
};

// How one evaluation is cut into blocks; a function of the dataset's size, the kind of evaluation
// and the context's settings only, so a request's arithmetic is identical whether it runs alone,
// blocking, or batched with others.
struct Plan {
    int scheme = kSymmetric;
    int precision = kFP64;
    int row_blocks = 0, splits = 0, tiles_per_split = 0, K = 0, epi_blocks = 0;
    int items = 0;            // blocks of the pairwise kernel
    int ubase = 0, urem = 0;  // symmetric: block b walks ubase + (b < urem) work units
    long long units = 0;      // symmetric: (row block, column tile) units this evaluation walks
    long long ubegin = 0;     // symmetric: first of them in the row-major order of the lower triangle
    long long col_stride = 0; // symmetric: values per column-sum quantity
    int dchunks = 0;          // symmetric: chunks of the walk's dynamic tail (dev::walk_split)
    size_t part_doubles = 0;  // row partial sums
    size_t col_bytes = 0;     // symmetric: column partial sums (binary32 values for FP32C, binary64
                              // for FP64), rounded up to a multiple of 8 bytes
    bool zskip = false;       // symmetric: zero-tile skipping (tables zcum, zskip in the scratch)
    bool zdirect = false;     // direct: zero-tile skipping (each row block walks its window only)
    size_t zbytes = 0;        // bytes of those tables
};

// One evaluation's scratch carved out of a buffer.
struct Carved {
    double *part = nullptr, *colpart = nullptr, *block_part = nullptr, *out7 = nullptr, *rows = nullptr;
    long long* zcum = nullptr;  // zero-tile skipping tables, when the plan uses them
    unsigned long long* ctr = nullptr;  // the dynamic tail's chunk counter (the 8th double of the
                                        // scratch's result slot, which holds 7 results)
};

struct Scratch {
    char* base = nullptr;
    size_t bytes = 0;
    hawkes_status reserve(hawkes_ctx* c, size_t need);
    void release(hawkes_ctx* c);
};

struct Server;  // hawkes_serving.hip

}  // namespace hawkes

struct hawkes_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    size_t used = 0;  // device bytes held (datasets + scratch); guarded by mu
    std::mutex mu;    // datasets, budget, blocking scratch, profiling
    std::map<int32_t, std::unique_ptr<hawkes::Dataset>> datasets;
    int32_t next_id = 0;
    hawkes::Scratch blk;       // scratch of blocking and device calls
    hipEvent_t blk_free = nullptr;  // recorded after the last use of blk
    double* h_out7 = nullptr;  // pinned
    std::atomic<bool> poisoned{false};  // set after a device failure; read by every call, without mu
    bool profile = false;
    bool prof_pending = false;
    hipEvent_t prof_ev[2] = {nullptr, nullptr};
    double pair_ms = 0.0;
    int64_t pair_launches = 0;
    hawkes::Server* server = nullptr;
    int scheme = hawkes::kSymmetric;  // how pair terms are enumerated (hawkes_set_pair_scheme)
    bool zero_skip = false;           // zero-tile skipping (hawkes_set_zero_tile_skipping)
    bool shared_passes = false;       // served FP32C log-likelihoods in multi-parameter passes
    int sym_slots[2][2] = {{0, 0}, {0, 0}};  // [precision][grad] resident blocks of the symmetric kernel
    int multi_slots = 0;                     // resident blocks of the multi-parameter kernel
};

namespace hawkes {

extern thread_local std::string g_last_error;
hawkes_status fail(hawkes_status code, const char* fmt, ...);
hawkes_status hip_fail(hipError_t e, const char* what);
hawkes_status check_params(const hawkes_params* p);
// shard / nshards: the evaluation walks the shard-th of nshards contiguous, equal ranges of the
// symmetric work units (symmetric scheme only; 0 / 1 is the whole triangle).  zero_skip: leave out
// the column tiles whose pair terms are all exactly zero (the whole evaluation only, not a shard).
Plan make_plan(const hawkes_ctx* c, int64_t n, int npad, bool grad, int precision, int scheme, int shard = 0,
               int nshards = 1, bool zero_skip = false);
size_t scratch_bytes(const Plan& pl, int64_t n, bool rows);
// Time separation from which a pair's background and trigger exponentials are both exactly zero
// in the arithmetic of `precision` (zero-tile skipping).
// T: the dataset's largest time (for the binary32 rounding of the FP32C pass's times).
double zero_separation(const hawkes_params& p, int precision, double T);
// Its two parts: the separations from which every background / every trigger term is zero.
void zero_gaps(const hawkes_params& p, int precision, double T, double& background, double& trigger);
void fill_pair(const hawkes_params& p, const Dataset& d, const Plan& pl, const Carved& cv, PairReq& r);
void fill_epi(const hawkes_params& p, const Dataset& d, const Plan& pl, bool grad, int precision, const Carved& cv,
              EpiReq& e);
Carved carve(char* base, const Plan& pl, bool rows);
hawkes_status dev_alloc(hawkes_ctx* c, void** p, size_t bytes);
void dev_free(hawkes_ctx* c, void* p, size_t bytes);
Dataset* find_dataset(hawkes_ctx* c, int32_t id);
void free_dataset(hawkes_ctx* c, Dataset& d);

hawkes_status begin_call(hawkes_ctx* c);
// Marks the context unusable after a device failure (HAWKES_EDEVICE); returns st.
hawkes_status poison(hawkes_ctx* c, hawkes_status st);
// Adds the last profiled pair-kernel time once the stream has passed it.
void collect_profile(hawkes_ctx* c);
hawkes_status reserve_blocking(hawkes_ctx* c, size_t need);
// Enqueue one evaluation (pairwise pass, epilogue, final reduction) on stream s with its scratch
// carved from `scratch`; out7_override (device, 7 doubles) replaces the scratch's result slot.
hawkes_status enqueue_eval(hawkes_ctx* c, const Dataset& d, const hawkes_params& p, int precision, bool grad,
                           char* scratch, double* out7_override, double** out7_used, double** rows_out,
                           bool want_rows, hipStream_t s);
hawkes_status blocking_eval(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, bool grad,
                            double out7[7], double* host_rows);
int multi_blocks_per_cu();
// The FP32C multi-parameter pass (hawkes_multi.hip): up to kMultiTheta parameter vectors share each
// pair's differences; a vector's result does not depend on the vectors sharing its pass.
constexpr int kMultiTheta = 4;
size_t multi_scratch_bytes(const hawkes_ctx* c, const Dataset& d, bool zero_skip, bool want_pi);
// One pass over nth (1 to kMultiTheta) vectors on stream s: ell of vector q to out[q * out_stride]
// (device), pi (sorted order) to pi_out[q * n + i] when pi_out is set.
hipError_t enqueue_multi_fp32c(const hawkes_ctx* c, const Dataset& d, const hawkes_params* th, int nth, char* scratch,
                               bool zero_skip, double* out, int out_stride, double* pi_out, hipStream_t s);

// hawkes_grad_device_noalloc: the fixed device array holding its evaluation scratch (256 MiB on
// every device the library runs on), and the per-device lookup of that array's address, done once
// per device by hawkes_create with the device current.
constexpr size_t kNoallocScratchBytes = (size_t)256 << 20;
hawkes_status noalloc_init(int device);

hawkes_status server_start(hawkes_ctx* c);
void server_stop(hawkes_ctx* c);
// Free the serving pool's idle scratch buffers (caller holds c->mu).
void server_trim(hawkes_ctx* c);

}  // namespace hawkes
