// hawkes_epilogue.hip -- the per-event epilogue and the final reduction of an evaluation (gfx950).
//
//  epilogue -- per event, in binary64: combine the pairwise pass's partial sums in a fixed order
//     into S_b, S_br, S_bt, S_e, S_et, S_er, then lambda_i = c_b S_b + c_e S_e, Lambda_i (closed
//     form of Section 2.1), ell_i = log lambda_i - Lambda_i and the six gradient terms; then a
//     fixed-shape tree reduction per block.
//  final -- one block per request sums the block partials in a fixed order (the paper's second
//     kernel, Algorithm 3 step 2, made deterministic).
#include "hawkes_device.h"

namespace hawkes {
namespace {

using namespace dev;

__device__ __forceinline__ double std_normal_cdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }
__device__ __forceinline__ double std_normal_pdf(double z) { return exp(-0.5 * z * z) * 0.39894228040143267794; }

// Fixed-shape tree over the block: v[m] of every thread summed into thread 0's v[m].
__device__ __forceinline__ void block_sum7(double (&v)[7], double (*red)[kThreads])
{
#pragma unroll
    for (int m = 0; m < 7; ++m) red[m][threadIdx.x] = v[m];
    __syncthreads();
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
#pragma unroll
            for (int m = 0; m < 7; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + stride];
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) v[m] = red[m][0];
}

// Adds to S[0..KC) one event's column partial sums (pc: its entry in row block 0's layout,
// quantities `stride` apart) over row blocks [J0, J1): per quantity four running sums taking row
// blocks in turn, combined in a fixed order; every quantity's loads of a step are issued together.
template <int KC, typename T>
__device__ __forceinline__ void column_totals(const T* __restrict__ pc, long long stride, int J0, int J1, double (&S)[6])
{
    double acc[KC][4];
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[q][u] = 0.0;
    int J = J0;
    for (; J + 3 < J1; J += 4) {
        T v[4][KC];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < KC; ++q) v[u][q] = pc[q * stride + (long long)kRowsPerBlock * (J + u) * (J + u + 1) / 2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < KC; ++q) acc[q][u] += (double)v[u][q];
    }
    for (; J < J1; ++J)
#pragma unroll
        for (int q = 0; q < KC; ++q) acc[q][0] += (double)pc[q * stride + (long long)kRowsPerBlock * J * (J + 1) / 2];
#pragma unroll
    for (int q = 0; q < KC; ++q) S[q] += (acc[q][0] + acc[q][1]) + (acc[q][2] + acc[q][3]);
}

// The walk positions [lo, hi) of row block I's units in the symmetric pass (the walked units with
// zero-tile skipping), the walk's split, and the dynamic-tail chunks [cf, cl] holding some of them
// (cl < cf: none).
struct RowBlockWalk {
    long long lo, hi;
    WalkSplit ws;
    long long cf, cl;
};

__device__ __forceinline__ RowBlockWalk row_block_walk(const EpiReq& rq, int I)
{
    constexpr long long TB = kRowsPerBlock / kTile;
    RowBlockWalk r;
    long long units;
    if (rq.zcum) {
        units = rq.zcum[rq.row_blocks];
        r.lo = rq.zcum[I];
        r.hi = rq.zcum[I + 1];
    } else {
        units = rq.uend - rq.ubegin;
        r.lo = max(TB * I * (I + 1) / 2, rq.ubegin) - rq.ubegin;
        r.hi = min(TB * (I + 1) * (I + 2) / 2, rq.uend) - rq.ubegin;
    }
    r.ws = walk_split(units, rq.pair_items, rq.dchunks);
    r.cf = 0;
    r.cl = -1;
    const long long dlo = max(r.lo, r.ws.sunits);
    if (dlo < r.hi) {
        r.cf = split_block(dlo - r.ws.sunits, r.ws.cbase, r.ws.crem);
        r.cl = split_block(r.hi - 1 - r.ws.sunits, r.ws.cbase, r.ws.crem);
    }
    return r;
}

// Row partials of the dynamic-tail chunks: per row block that several chunks walked, their sums
// in chunk order are folded into the first chunk's slot, so the epilogue reads one slot for them.
// A block takes one (row block, quantity, 64 rows): its kFoldWaves waves take every
// kFoldWaves-th chunk (four running sums each, combined in a fixed order), lanes are consecutive
// rows (coalesced), and the waves' sums are added in wave order.  Every element is read and
// written by one block only, so the fold is in place; the result depends only on the plan.
constexpr int kFoldWaves = 8;
constexpr int kFoldGroups = kRowsPerBlock / 64;

__global__ __launch_bounds__(kFoldWaves * 64) void dyn_fold(const EpiReq rq, int first_row_block)
{
    __shared__ double wsum[kFoldWaves][64];
    const int K = rq.grad ? 6 : 2;
    const int per_block = kFoldGroups * K;
    const int I = first_row_block + (int)blockIdx.x / per_block;
    const int k = ((int)blockIdx.x % per_block) / kFoldGroups, g = (int)blockIdx.x % kFoldGroups;
    const RowBlockWalk rw = row_block_walk(rq, I);
    if (rw.cl <= rw.cf) return;  // no chunk, or one: nothing to fold (uniform over the block)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const size_t stride = (size_t)K * kRowsPerBlock;
    const double* src = rq.part + (size_t)(rq.pair_items + rq.row_blocks + I) * stride + (size_t)k * kRowsPerBlock +
                        g * 64 + lane;  // + c * stride: chunk c's value
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    long long c = rw.cf + w;
    constexpr int W = kFoldWaves;
    for (; c + 3 * W <= rw.cl; c += 4 * W) {
        const double v0 = src[(size_t)c * stride], v1 = src[(size_t)(c + W) * stride];
        const double v2 = src[(size_t)(c + 2 * W) * stride], v3 = src[(size_t)(c + 3 * W) * stride];
        a0 += v0;
        a1 += v1;
        a2 += v2;
        a3 += v3;
    }
    for (; c <= rw.cl; c += W) a0 += src[(size_t)c * stride];
    wsum[w][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (w == 0) {
        double t = wsum[0][lane];
#pragma unroll
        for (int v = 1; v < kFoldWaves; ++v) t += wsum[v][lane];
        const_cast<double*>(src)[(size_t)rw.cf * stride] = t;
    }
}

__global__ __launch_bounds__(kThreads) void epilogue(const EpiBatch batch)
{
    __shared__ double red[7][kThreads];
    const int q = find_request(batch.r, batch.nreq, (int)blockIdx.x);
    const EpiReq& rq = batch.r[q];
    const int blk = (int)blockIdx.x - rq.item_begin;
    const int i = blk * kThreads + threadIdx.x;
    const int K = rq.grad ? 6 : 2;

    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < rq.n) {
        double S[6] = {0, 0, 0, 0, 0, 0};  // Sb, Sbr, Sbt, Se, Set, Ser
        if (rq.sums_in) {
#pragma unroll
            for (int k = 0; k < 6; ++k) S[k] = rq.sums_in[(size_t)i * 6 + k];
        } else if (rq.scheme == kSymmetric) {
            // Row sums: one partial per static range (block) that walked a unit of this row block,
            // in block order, then the dynamic-tail chunks' (folded into the first one's slot).
            const int I = i / kRowsPerBlock, rho = i % kRowsPerBlock;
            const RowBlockWalk rw = row_block_walk(rq, I);
            const long long shi = min(rw.hi, rw.ws.sunits);
            long long nslot = 0;
            long long slots[2] = {0, 0};  // static: [bf, bl] + I; then the folded dynamic slot
            long long bf = 0, bl = -1;
            if (rw.lo < shi) {
                bf = split_block(rw.lo, rw.ws.sbase, rw.ws.srem);
                bl = split_block(shi - 1, rw.ws.sbase, rw.ws.srem);
            }
            if (rw.cl >= rw.cf) slots[nslot++] = rq.pair_items + rq.row_blocks + rw.cf + I;
            for (long long m = 0; m < (bl - bf + 1) + nslot; ++m) {
                const long long slot = m <= bl - bf ? bf + m + I : slots[m - (bl - bf + 1)];
                const double* ps = rq.part + (size_t)slot * K * kRowsPerBlock + rho;
                if (rq.grad) {
#pragma unroll
                    for (int q6 = 0; q6 < 6; ++q6) S[q6] += ps[(size_t)q6 * kRowsPerBlock];
                } else {
                    S[0] += ps[0];
                    S[3] += ps[kRowsPerBlock];
                }
            }
            // Column sums: the background terms with every later event, by row block J >= I, from
            // the units (J, tile of i) that were walked, gathered four row blocks at a time into
            // four partial sums combined in a fixed order (four independent loads in flight).
            const long long tile_i = i / kTile;
            int J0, J1;
            if (rq.zcum) {
                // Row blocks from the first whose skipped prefix covers this event's tile on
                // did not walk it (the prefixes grow with the row block).
                const int* zskip = zero_skip_tiles(rq.zcum, rq.row_blocks);
                int a = I, b = rq.row_blocks;
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (zskip[mid] > tile_i)
                        b = mid;
                    else
                        a = mid + 1;
                }
                J0 = I;
                J1 = a;
            } else {
                J0 = max(I, sym_first_block_from(rq.ubegin - tile_i));
                J1 = min(rq.row_blocks, sym_first_block_from(rq.uend - tile_i));
            }
            if (rq.colpart_f32) {
                const float* pc = reinterpret_cast<const float*>(rq.colpart) + i;
                if (rq.grad)
                    column_totals<3>(pc, rq.col_stride, J0, J1, S);
                else
                    column_totals<1>(pc, rq.col_stride, J0, J1, S);
            } else {
                const double* pc = rq.colpart + i;
                if (rq.grad)
                    column_totals<3>(pc, rq.col_stride, J0, J1, S);
                else
                    column_totals<1>(pc, rq.col_stride, J0, J1, S);
            }
            if (rq.add_diag) S[0] += 1.0;  // the diagonal term B_ii = 1
        } else {
            for (int s = 0; s < rq.splits; ++s) {
                const double* ps = rq.part + (size_t)s * K * rq.npad + i;
                if (rq.grad) {
#pragma unroll
                    for (int k = 0; k < 6; ++k) S[k] += ps[(size_t)k * rq.npad];
                } else {
                    S[0] += ps[0];
                    S[3] += ps[rq.npad];
                }
            }
        }
        // Moments in dt were summed in scaled time dt' = t_scale dt.
        S[2] /= rq.t_scale * rq.t_scale;
        S[4] /= rq.t_scale;
        if (rq.sums_out) {
#pragma unroll
            for (int k = 0; k < 6; ++k) rq.sums_out[(size_t)i * 6 + k] = S[k];
        } else {
            const double ti = rq.ev64[i].z;
            const double mu0 = rq.mu0, tx = rq.tau_x, tt = rq.tau_t, th = rq.theta, om = rq.omega, h = rq.h;
            const double lam = rq.cb * S[0] + rq.ce * S[3];
            const double u = rq.T - ti;
            const double bg_int = std_normal_cdf(u / tt) - std_normal_cdf(-ti / tt);
            const double Lam = mu0 * bg_int - th * expm1(-om * u);
            const double ell = log(lam) - Lam;
            v[0] = ell;
            double g[6] = {0, 0, 0, 0, 0, 0};
            if (rq.grad) {
                const double inv = 1.0 / lam;
                const double k2pih2 = 1.0 / (6.28318530717958647693 * h * h);
                g[0] = rq.cb * S[0] / mu0 * inv - bg_int;
                g[1] = rq.cb * (-2.0 * S[0] / tx + S[1] / (tx * tx * tx)) * inv;
                g[2] = rq.cb * (-S[0] / tt + S[2] / (tt * tt * tt)) * inv
                     + (mu0 / (tt * tt)) * (u * std_normal_pdf(u / tt) + ti * std_normal_pdf(ti / tt));
                g[3] = om * k2pih2 * S[3] * inv + expm1(-om * u);
                g[4] = th * k2pih2 * (S[3] - om * S[4]) * inv - th * u * exp(-om * u);
                g[5] = rq.ce * (-2.0 * S[3] / h + S[5] / (h * h * h)) * inv;
#pragma unroll
                for (int p = 0; p < 6; ++p) v[1 + p] = g[p];
            }
            if (rq.rows_out) {
                double* o = rq.rows_out + (size_t)i * kRowOut;
                o[0] = lam;
                o[1] = Lam;
                o[2] = ell;
                o[3] = rq.ce * S[3] / lam;
#pragma unroll
                for (int p = 0; p < 6; ++p) o[4 + p] = g[p];
            }
        }
    }
    block_sum7(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < 7; ++m) rq.block_part[(size_t)blk * 7 + m] = v[m];
}

__global__ __launch_bounds__(kThreads) void final_sum(const EpiBatch batch)
{
    __shared__ double red[7][kThreads];
    const EpiReq& rq = batch.r[blockIdx.x];
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < rq.nblocks; b += kThreads)
#pragma unroll
        for (int m = 0; m < 7; ++m) v[m] += rq.block_part[(size_t)b * 7 + m];
    block_sum7(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < 7; ++m) rq.out7[m] = v[m];
}

}  // namespace

hipError_t launch_epilogue(const EpiBatch& b, hipStream_t s)
{
    if (b.total_items <= 0) return hipSuccess;
    for (int q = 0; q < b.nreq; ++q) {
        const EpiReq& r = b.r[q];
        if (r.scheme != kSymmetric || r.dchunks <= 0 || r.sums_in) continue;
        // Row blocks that may hold dynamic-tail chunks: with zero-tile skipping any (the walked
        // units are known on the device only); otherwise those ending after the static part.
        int first = 0;
        if (!r.zcum) {
            constexpr long long TB = kRowsPerBlock / kTile;
            const WalkSplit ws = walk_split(r.uend - r.ubegin, r.pair_items, r.dchunks);
            while (first < r.row_blocks && TB * (first + 1) * (first + 2) / 2 - r.ubegin <= ws.sunits) ++first;
        }
        if (first >= r.row_blocks) continue;
        const int K = r.grad ? 6 : 2;
        dyn_fold<<<dim3((r.row_blocks - first) * kFoldGroups * K), dim3(kFoldWaves * 64), 0, s>>>(r, first);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    epilogue<<<dim3(b.total_items), dim3(kThreads), 0, s>>>(b);
    return hipGetLastError();
}

hipError_t launch_final(const EpiBatch& b, hipStream_t s)
{
    if (b.nreq <= 0) return hipSuccess;
    final_sum<<<dim3(b.nreq), dim3(kThreads), 0, s>>>(b);
    return hipGetLastError();
}

}  // namespace hawkes
