// hawkes_shard.hip -- evaluation of one dataset split over several devices: per-event sums of a
// shard of the symmetric pairwise pass (hawkes_shard_sums) and the log-likelihood and gradient
// from the per-event sums added over all shards (hawkes_finish).
#include "hawkes_runtime.h"

#include <cstring>
#include <vector>

using namespace hawkes;

extern "C" {

hawkes_status hawkes_shard_sums(hawkes_ctx* c, int32_t id, const hawkes_params* p, int precision, int32_t shard,
                                int32_t nshards, double* out_sums)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if ((st = check_params(p)) != HAWKES_OK) return st;
    if (precision != HAWKES_FP64 && precision != HAWKES_FP32C)
        return fail(HAWKES_EINVAL, "precision %d is neither HAWKES_FP64 nor HAWKES_FP32C", precision);
    if (nshards < 1 || shard < 0 || shard >= nshards)
        return fail(HAWKES_EINVAL, "shard %d of %d is not a shard", shard, nshards);
    if (!out_sums) return fail(HAWKES_EINVAL, "out_sums is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    const Plan pl = make_plan(c, d->n, d->npad, true, precision, kSymmetric, shard, nshards);
    const size_t base_bytes = scratch_bytes(pl, d->n, false);
    const size_t sums_bytes = (size_t)d->n * 6 * sizeof(double);
    if ((st = reserve_blocking(c, base_bytes + sums_bytes)) != HAWKES_OK) return st;
    hipStream_t s = c->stream;
    hipError_t e = hipStreamWaitEvent(s, c->blk_free, 0);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamWaitEvent"));
    const Carved cv = carve(c->blk.base, pl, false);
    double* dsums = (double*)(c->blk.base + base_bytes);

    PairBatch pb;
    memset(&pb, 0, sizeof pb);
    fill_pair(*p, *d, pl, cv, pb.r[0]);
    pb.r[0].item_begin = 0;
    pb.r[0].balance = 1;
    pb.nreq = 1;
    pb.total_items = pl.items;
    EpiBatch eb;
    memset(&eb, 0, sizeof eb);
    fill_epi(*p, *d, pl, true, precision, cv, eb.r[0]);
    eb.r[0].item_begin = 0;
    eb.r[0].add_diag = shard == 0 ? 1 : 0;
    eb.r[0].sums_out = dsums;
    eb.nreq = 1;
    eb.total_items = pl.epi_blocks;

    if (c->profile) {
        e = hipEventRecord(c->prof_ev[0], s);
        if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
    }
    e = launch_pair(pb, precision, true, kSymmetric, false, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "pair kernel launch"));
    if (c->profile) {
        e = hipEventRecord(c->prof_ev[1], s);
        if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
        c->prof_pending = true;
    }
    e = launch_epilogue(eb, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "epilogue launch"));
    std::vector<double> sorted((size_t)d->n * 6);
    e = hipMemcpyAsync(sorted.data(), dsums, sums_bytes, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipMemcpyAsync"));
    e = hipEventRecord(c->blk_free, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamSynchronize"));
    collect_profile(c);
    for (int64_t k = 0; k < d->n; ++k)
        memcpy(out_sums + (size_t)d->perm[k] * 6, sorted.data() + (size_t)k * 6, 6 * sizeof(double));
    return HAWKES_OK;
}

hawkes_status hawkes_finish(hawkes_ctx* c, int32_t id, const hawkes_params* p, const double* sums,
                            double* out_loglik, double* out_grad)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if ((st = check_params(p)) != HAWKES_OK) return st;
    if (!sums) return fail(HAWKES_EINVAL, "sums is NULL");
    if (!out_loglik) return fail(HAWKES_EINVAL, "out_loglik is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    const Plan pl = make_plan(c, d->n, d->npad, true, HAWKES_FP64, kSymmetric);
    const size_t head = ((size_t)pl.epi_blocks * 7 + 8) * sizeof(double);
    const size_t sums_bytes = (size_t)d->n * 6 * sizeof(double);
    if ((st = reserve_blocking(c, head + sums_bytes)) != HAWKES_OK) return st;
    hipStream_t s = c->stream;
    hipError_t e = hipStreamWaitEvent(s, c->blk_free, 0);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamWaitEvent"));
    Carved cv;
    cv.block_part = (double*)c->blk.base;
    cv.out7 = cv.block_part + (size_t)pl.epi_blocks * 7;
    double* dsums = (double*)(c->blk.base + head);
    std::vector<double> sorted((size_t)d->n * 6);
    for (int64_t k = 0; k < d->n; ++k)
        memcpy(sorted.data() + (size_t)k * 6, sums + (size_t)d->perm[k] * 6, 6 * sizeof(double));
    e = hipMemcpyAsync(dsums, sorted.data(), sums_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipMemcpyAsync"));

    EpiBatch eb;
    memset(&eb, 0, sizeof eb);
    fill_epi(*p, *d, pl, true, HAWKES_FP64, cv, eb.r[0]);
    eb.r[0].item_begin = 0;
    eb.r[0].sums_in = dsums;
    eb.nreq = 1;
    eb.total_items = pl.epi_blocks;
    e = launch_epilogue(eb, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "epilogue launch"));
    e = launch_final(eb, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "final reduction launch"));
    e = hipMemcpyAsync(c->h_out7, cv.out7, 7 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipMemcpyAsync"));
    e = hipEventRecord(c->blk_free, s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipEventRecord"));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return poison(c, hip_fail(e, "hipStreamSynchronize"));
    *out_loglik = c->h_out7[0];
    if (out_grad) memcpy(out_grad, c->h_out7 + 1, 6 * sizeof(double));
    return HAWKES_OK;
}

}  // extern "C"
