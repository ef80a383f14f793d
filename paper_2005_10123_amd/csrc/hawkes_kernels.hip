// hawkes_kernels.hip -- gfx950 kernels of the exact O(N^2) spatiotemporal Hawkes log-likelihood
// (arXiv 2005.10123, Section 2.1, the log-likelihood equation) and its gradient.
//
// The pairwise pass, one launch per evaluation or batch of requests (the epilogue and the final
// reduction are in hawkes_epilogue.hip).  For every row (event) i it sums over the columns j the
// unnormalised background kernel B_ij = exp(-r^2/(2 tau_x^2) - dt^2/(2 tau_t^2)) (j = i included)
// and, for causal columns j < cut[i] (t_j < t_i), the unnormalised trigger
// E_ij = exp(-omega dt - r^2/(2 h^2)); with the gradient also r^2 B, dt^2 B, dt E and r^2 E.
// Running sums only, never the N x N terms (the paper's fourth rule of thumb, Section 2.3).
// Rows live in registers (kRowsPerLane per lane), column tiles of kTile events are staged in LDS
// and read as broadcasts.  Every block writes its own partial sums, so the result never depends
// on scheduling.  Because rows and columns are time-sorted, a whole tile is either fully causal
// for a wave (no mask), fully non-causal (no trigger work) or straddles the wave's rows (masked
// exponent).  Two enumerations: the direct one (every ordered pair, column ranges split over
// blocks) and the symmetric one (each unordered pair once, below).
//
// The exponentials are base 2 with log2(e) folded into the coefficients: the FP32C path uses the
// hardware v_exp_f32, the FP64 path the exp2 below.  There is no matrix-core work: with two
// spatial dimensions the pair terms are not a dense contraction.
#include "hawkes_device.h"

namespace hawkes {
namespace {

using namespace dev;

// ------------------------------------------------------------------------------------------------
// FP32C pairwise pass.
//
// Each lane holds kRowsPerLane consecutive rows.  Space: dx = (x_i,hi - x_j,hi) + (x_i,lo - x_j,lo)
// gives the difference to binary32 precision of the difference itself.  Time: every lane measures
// times from its own first row t0 = t0_hi + t0_lo and scales them by s = sqrt(-nbb), so a column's
// time tj = s ((tj_hi - t0_hi) + (tj_lo - t0_lo)) is formed once per column per lane and shared by
// the lane's rows, and dt = ti - tj costs one subtraction per pair.  Its error is of order
// 2^-24 (|dt| + s |t_row - t0|), with the lane's rows only a few events apart.  The scale turns
// the background exponent into nab r^2 - dt^2; the epilogue divides the dt-moments by s and s^2.
// s is applied as s_hi + s_lo: a binary32 s alone would perturb every background exponent by the
// same relative amount (up to 2^-23), a bias that does not average out over the sum.
// EXACT: the time difference of each pair from the hi/lo parts of both events (th, tl: the rows'
// times), for tiles near the rows; otherwise from the lane's first row (ti, t0h, t0l).
template <int MODE, bool EXACT, bool GRAD>
__device__ __forceinline__ void chunk_fp32(const float4* __restrict__ sj, int jbase,
                                           const float (&xh)[kRowsPerLane], const float (&yh)[kRowsPerLane],
                                           const float (&xl)[kRowsPerLane], const float (&yl)[kRowsPerLane],
                                           const float (&ti)[kRowsPerLane], const float (&th)[kRowsPerLane],
                                           const float (&tl)[kRowsPerLane], const int (&ct)[kRowsPerLane],
                                           float t0h, float t0l, float tsh, float tsl, float nab, float nae, float kte,
                                           float (&p)[6][kRowsPerLane])
{
    constexpr int R = kRowsPerLane;
#pragma unroll 2
    for (int jj = 0; jj < kChunk; ++jj) {
        const float4 hi = sj[2 * jj];
        const float4 lo = sj[2 * jj + 1];
        float tj = 0.0f;
        if (!EXACT) {
            const float tu = (hi.z - t0h) + (lo.z - t0l);
            tj = fmaf(tu, tsh, tu * tsl);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = (xh[r] - hi.x) + (xl[r] - lo.x);
            const float dy = (yh[r] - hi.y) + (yl[r] - lo.y);
            float dt;
            if (EXACT) {
                const float du = (th[r] - hi.z) + (tl[r] - lo.z);
                dt = fmaf(du, tsh, du * tsl);
            } else {
                dt = ti[r] - tj;
            }
            const float r2 = fmaf(dx, dx, dy * dy);
            const float dt2 = dt * dt;
            const float b = __builtin_amdgcn_exp2f(fmaf(r2, nab, -dt2));
            p[0][r] += b;
            if (GRAD) {
                p[1][r] = fmaf(r2, b, p[1][r]);
                p[2][r] = fmaf(dt2, b, p[2][r]);
            }
            if (MODE != kNone) {
                float ae = fmaf(r2, nae, dt * kte);
                if (MODE == kMask) ae = (jbase + jj < ct[r]) ? ae : -INFINITY;
                const float e = __builtin_amdgcn_exp2f(ae);
                const int ke = GRAD ? 3 : 1;
                p[ke][r] += e;
                if (GRAD) {
                    p[4][r] = fmaf(dt, e, p[4][r]);
                    p[5][r] = fmaf(r2, e, p[5][r]);
                }
            }
        }
    }
}

// Column tiles [t0, t1) walked by split sp of row block rb in the direct enumeration: all tiles
// cut into ranges of tiles_per_split; with zero-tile skipping (zdirect), only the tiles that hold an
// event less than zero_dt from one of the row block's events (a window, the events being
// time-sorted; tiles of padding only are left out too), cut into `splits` near-equal ranges.
__device__ __forceinline__ void direct_range(const PairReq& rq, int rb, int sp, int& t0, int& t1)
{
    const int tiles = rq.npad / kTile;
    if (!rq.zdirect) {
        t0 = sp * rq.tiles_per_split;
        t1 = min(t0 + rq.tiles_per_split, tiles);
        return;
    }
    const int n = rq.n;
    const double t_first = rq.ev64[(size_t)rb * kRowsPerBlock].z;
    const double t_last = rq.ev64[(size_t)min(rb * kRowsPerBlock + kRowsPerBlock - 1, n - 1)].z;
    // lo: whole tiles ending at least zero_dt before the row block's first event.
    int lo = 0, hi = n / kTile;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (t_first - rq.ev64[(size_t)mid * kTile + kTile - 1].z >= rq.zero_dt)
            lo = mid + 1;
        else
            hi = mid;
    }
    // end: the first tile starting at least zero_dt after the row block's last event.
    int a = lo, end = (n + kTile - 1) / kTile;
    while (a < end) {
        const int mid = (a + end) >> 1;
        if (rq.ev64[(size_t)mid * kTile].z - t_last >= rq.zero_dt)
            end = mid;
        else
            a = mid + 1;
    }
    const long long len = end - lo;
    t0 = lo + (int)(len * sp / rq.splits);
    t1 = lo + (int)(len * (sp + 1) / rq.splits);
}

template <bool GRAD>
__global__ __launch_bounds__(kThreads) void pair_fp32c(const PairBatch batch)
{
    constexpr int R = kRowsPerLane;
    constexpr int K = GRAD ? 6 : 2;
    __shared__ float4 sj[2 * kTile];

    const int q = find_request(batch.r, batch.nreq, (int)blockIdx.x);
    const PairReq& rq = batch.r[q];
    const int local = (int)blockIdx.x - rq.item_begin;
    const int rb = rq.row_blocks - 1 - local / rq.splits;  // latest (heaviest) rows first
    const int sp = local % rq.splits;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = rq.n;
    const int wrow0 = rb * kRowsPerBlock + wave * (64 * R);
    const int lrow0 = wrow0 + R * lane;  // this lane's rows: lrow0 .. lrow0 + R - 1
    const bool active = wrow0 < n;       // wave-uniform

    const float tsh = in_vgpr(rq.tsh), tsl = in_vgpr(rq.tsl), nab = in_vgpr(rq.nab);
    const float nae = in_vgpr(rq.nae), kte = in_vgpr(rq.kte);
    float xh[R], yh[R], xl[R], yl[R], ti[R], th[R], tl[R];
    int ct[R];
    float t0h = 0.0f, t0l = 0.0f, lane_span = 0.0f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lrow0 + r;
        const float4 a = rq.ev32[2 * (size_t)i];
        const float4 b = rq.ev32[2 * (size_t)i + 1];
        if (r == 0) {
            t0h = a.z;
            t0l = b.z;
        }
        xh[r] = a.x; yh[r] = a.y; xl[r] = b.x; yl[r] = b.y;
        th[r] = a.z; tl[r] = b.z;
        const float tu = (a.z - t0h) + (b.z - t0l);
        ti[r] = fmaf(tu, tsh, tu * tsl);
        ct[r] = rq.cut[i];
        if (i < n) lane_span = tu;  // rows are time-sorted: the last valid row is the latest
    }
    // Rows are time-sorted, so the causal counts of the wave's rows lie in [clo, chi].
    const int clo = __builtin_amdgcn_readfirstlane(rq.cut[min(wrow0, n - 1)]);
    const int chi = __builtin_amdgcn_readfirstlane(rq.cut[min(wrow0 + 64 * R - 1, n - 1)]);
    // Causal tiles closer in time to the wave's first row than kNearSpans lane spans, and tiles
    // straddling the causal counts, take exact time differences (kNearSpans in hawkes_device.h).
    const float span = uniform(wave_max(lane_span));
    const float t_first = uniform(rq.ev32[2 * (size_t)min(wrow0, n - 1)].z + rq.ev32[2 * (size_t)min(wrow0, n - 1) + 1].z);

    float s[K][R], c[K][R];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) s[k][r] = c[k][r] = 0.0f;

    int t0, t1;
    direct_range(rq, rb, sp, t0, t1);
    for (int tile = t0; tile < t1; ++tile) {
        const int j0 = tile * kTile;
        __syncthreads();
        const float4* src = rq.ev32 + 2 * (size_t)(j0 + threadIdx.x);
        sj[2 * threadIdx.x] = src[0];
        sj[2 * threadIdx.x + 1] = src[1];
        __syncthreads();
        if (!active) continue;
        int mode = (j0 + kTile <= clo) ? kFull : (j0 >= chi ? kNone : kMask);
        if (mode == kFull && !far_tile(sj, t_first, span))
            mode = kMask;  // near: the masked path (exact times), whose causal mask passes every pair
        for (int ch = 0; ch < kTile; ch += kChunk) {
            float p[6][R];
#pragma unroll
            for (int k = 0; k < 6; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) p[k][r] = 0.0f;
            const float4* tj = sj + 2 * ch;
            if (mode == kNone)
                chunk_fp32<kNone, false, GRAD>(tj, j0 + ch, xh, yh, xl, yl, ti, th, tl, ct, t0h, t0l, tsh, tsl, nab, nae, kte, p);
            else if (mode == kFull)
                chunk_fp32<kFull, false, GRAD>(tj, j0 + ch, xh, yh, xl, yl, ti, th, tl, ct, t0h, t0l, tsh, tsl, nab, nae, kte, p);
            else
                chunk_fp32<kMask, true, GRAD>(tj, j0 + ch, xh, yh, xl, yl, ti, th, tl, ct, t0h, t0l, tsh, tsl, nab, nae, kte, p);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) two_sum_into(s[k][r], c[k][r], p[k][r]);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r)
            rq.part[((size_t)sp * K + k) * rq.npad + lrow0 + r] = (double)s[k][r] + (double)c[k][r];
}

// ------------------------------------------------------------------------------------------------
// FP64 pairwise pass: same decomposition, binary64 throughout, plain running sums.
template <int MODE, bool GRAD>
__device__ __forceinline__ void tile_fp64(const double4* __restrict__ sj, int jbase,
                                          const double (&x)[kRowsPerLane], const double (&y)[kRowsPerLane],
                                          const double (&t)[kRowsPerLane], const int (&ct)[kRowsPerLane],
                                          double nab, double nbb, double nae, double nbe,
                                          double (&a)[6][kRowsPerLane])
{
    constexpr int R = kRowsPerLane;
#pragma unroll 1
    for (int jj = 0; jj < kTile; ++jj) {
        const double4 e = sj[jj];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = x[r] - e.x;
            const double dy = y[r] - e.y;
            const double dt = t[r] - e.z;
            const double r2 = fma(dx, dx, dy * dy);
            const double dt2 = dt * dt;
            const double b = exp2_f64(fma(r2, nab, dt2 * nbb));
            a[0][r] += b;
            if (GRAD) {
                a[1][r] = fma(r2, b, a[1][r]);
                a[2][r] = fma(dt2, b, a[2][r]);
            }
            if (MODE != kNone) {
                double ae = fma(r2, nae, dt * nbe);
                if (MODE == kMask) ae = (jbase + jj < ct[r]) ? ae : -INFINITY;
                const double ex = exp2_f64(ae);
                const int ke = GRAD ? 3 : 1;
                a[ke][r] += ex;
                if (GRAD) {
                    a[4][r] = fma(dt, ex, a[4][r]);
                    a[5][r] = fma(r2, ex, a[5][r]);
                }
            }
        }
    }
}

template <bool GRAD>
__global__ __launch_bounds__(kThreads) void pair_fp64(const PairBatch batch)
{
    constexpr int R = kRowsPerLane;
    constexpr int K = GRAD ? 6 : 2;
    __shared__ double4 sj[kTile];

    const int q = find_request(batch.r, batch.nreq, (int)blockIdx.x);
    const PairReq& rq = batch.r[q];
    const int local = (int)blockIdx.x - rq.item_begin;
    const int rb = rq.row_blocks - 1 - local / rq.splits;
    const int sp = local % rq.splits;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = rq.n;
    const int wrow0 = rb * kRowsPerBlock + wave * (64 * R);
    const bool active = wrow0 < n;

    double x[R], y[R], t[R];
    int ct[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = wrow0 + 64 * r + lane;
        const double4 e = rq.ev64[i];
        x[r] = e.x; y[r] = e.y; t[r] = e.z;
        ct[r] = rq.cut[i];
    }
    const int clo = __builtin_amdgcn_readfirstlane(rq.cut[min(wrow0, n - 1)]);
    const int chi = __builtin_amdgcn_readfirstlane(rq.cut[min(wrow0 + 64 * R - 1, n - 1)]);

    double a[6][R];
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) a[k][r] = 0.0;

    int t0, t1;
    direct_range(rq, rb, sp, t0, t1);
    for (int tile = t0; tile < t1; ++tile) {
        const int j0 = tile * kTile;
        __syncthreads();
        sj[threadIdx.x] = rq.ev64[j0 + threadIdx.x];
        __syncthreads();
        if (!active) continue;
        const int mode = (j0 + kTile <= clo) ? kFull : (j0 >= chi ? kNone : kMask);
        if (mode == kNone)
            tile_fp64<kNone, GRAD>(sj, j0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a);
        else if (mode == kFull)
            tile_fp64<kFull, GRAD>(sj, j0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a);
        else
            tile_fp64<kMask, GRAD>(sj, j0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ka = GRAD ? k : (k == 0 ? 0 : 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = wrow0 + 64 * r + lane;
            rq.part[((size_t)sp * K + k) * rq.npad + i] = a[ka][r];
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Symmetric pairwise pass: every unordered pair j < i (time-sorted indices) once.
//
// A block walks a contiguous range of work units (row block I, column tile t) in row-major order
// over the lower triangle.  For each tile a lane forms its rows' pair terms with each column; the
// background term B and its moments go both to the lane's row sums (registers) and to the
// column's sums; the trigger term only to the row (the column is the earlier event).  Column sums
// are reduced over the 64 lanes 4 columns at a time (column_sums4: through LDS, then DPP row
// rotations), combined over the block's waves in LDS in a fixed order, and written once per
// (row block, column).  Row sums are written once per (block, row block) the block touched.
// Tiles below a wave's rows need no mask for B; tiles straddling them mask j >= i; tiles above
// are skipped.

// One tile of the FP32C symmetric pass for one wave.
template <int MODE, bool GRAD, int R, int NT>
__device__ __forceinline__ void sym_tile_fp32(const float4* __restrict__ sj, int j0, int lrow0,
                                              const float (&xh)[R], const float (&yh)[R],
                                              const float (&xl)[R], const float (&yl)[R],
                                              const float (&ti)[R], const float (&th)[R], const float (&tl)[R],
                                              const int (&ct)[R], float tsh, float tsl, float nab, float nae,
                                              float kte, float (&s)[6][R], volatile lds_float* comp,
                                              float* __restrict__ colw, float* __restrict__ red, int lane)
{
    constexpr int K = GRAD ? 6 : 2;
    constexpr int KC = GRAD ? 3 : 1;
    // Tiles far before the rows measure times from the tile's first event (rows: ti; columns: the
    // staged .w); the others take every time difference from the hi/lo parts of the two events.
    constexpr bool FAR = MODE == kFullLow || MODE == kFullLowB || MODE == kFullLowE;
    constexpr bool EXACT = !FAR;
    constexpr bool DO_B = MODE != kFullLowE;  // background terms (and the column sums)
    constexpr bool DO_E = MODE != kFullLowB;  // trigger terms
    if (!DO_B)
#pragma unroll
        for (int qq = 0; qq < KC; ++qq)
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0f;
    for (int ch = 0; ch < kTile; ch += kChunk) {
        float p[6][R];
#pragma unroll
        for (int k = 0; k < 6; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) p[k][r] = 0.0f;
#pragma unroll 1
        for (int g = ch; g < ch + kChunk; g += 4) {
            float cp[3][4];  // set by each column's first row (no additions of zero)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const float4 hi = sj[2 * (g + cc)];
                const float4 lo = sj[2 * (g + cc) + 1];
                const float tj = EXACT ? 0.0f : hi.w;
                const int j = j0 + g + cc;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = (xh[r] - hi.x) + (xl[r] - lo.x);
                    const float dy = (yh[r] - hi.y) + (yl[r] - lo.y);
                    float dt;
                    if (EXACT) {
                        const float du = (th[r] - hi.z) + (tl[r] - lo.z);
                        dt = fmaf(du, tsh, du * tsl);
                    } else {
                        dt = ti[r] - tj;
                    }
                    const float r2 = fmaf(dx, dx, dy * dy);
                    if (DO_B) {
                        const float dt2 = dt * dt;
                        float ab = fmaf(r2, nab, -dt2);
                        if (MODE == kDiag) ab = (j < lrow0 + r) ? ab : -INFINITY;
                        const float b = __builtin_amdgcn_exp2f(ab);
                        p[0][r] += b;
                        if (GRAD) {
                            p[1][r] = fmaf(r2, b, p[1][r]);
                            p[2][r] = fmaf(dt2, b, p[2][r]);
                        }
                        if (r == 0) {
                            cp[0][cc] = b;
                            if (GRAD) {
                                cp[1][cc] = r2 * b;
                                cp[2][cc] = dt2 * b;
                            }
                        } else {
                            cp[0][cc] += b;
                            if (GRAD) {
                                cp[1][cc] = fmaf(r2, b, cp[1][cc]);
                                cp[2][cc] = fmaf(dt2, b, cp[2][cc]);
                            }
                        }
                    }
                    if (DO_E) {
                        float ae = fmaf(r2, nae, dt * kte);
                        if (!FAR) ae = (j < ct[r]) ? ae : -INFINITY;
                        const float e = __builtin_amdgcn_exp2f(ae);
                        const int ke = GRAD ? 3 : 1;
                        p[ke][r] += e;
                        if (GRAD) {
                            p[4][r] = fmaf(dt, e, p[4][r]);
                            p[5][r] = fmaf(r2, e, p[5][r]);
                        }
                    }
                }
            }
            if (DO_B) {
                float v[3];
                column_sums4<KC>(cp, red, lane, v);
                if ((lane & 15) == 0)
#pragma unroll
                    for (int q = 0; q < KC; ++q) colw[q * kTile + g + (lane >> 4)] = v[q];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // Quantities 0 .. K/2 - 1 are background sums, the rest trigger sums; the kernel a mode
            // leaves out adds exact zeros, which the compensated sums would not change.
            if ((k < K / 2 && !DO_B) || (k >= K / 2 && !DO_E)) continue;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float cc = comp[(k * R + r) * NT];
                two_sum_into(s[k][r], cc, p[k][r]);
                comp[(k * R + r) * NT] = cc;
            }
        }
    }
}

// Shape of the FP32C symmetric pass: kSymRows rows per lane; a block's threads together hold one
// row block of the walk.
constexpr int kSymRows = 4;
constexpr int kSymThreads = kRowsPerBlock / kSymRows;
constexpr int kSymWaves = kSymThreads / 64;
// Waves per SIMD the register budget is sized for: three with the gradient (168 VGPRs, three
// blocks per CU); four for the log-likelihood alone (128 VGPRs), which measures faster there.
template <bool GRAD>
constexpr int kSymWavesPerSimd = GRAD ? 3 : 4;
static_assert(kSymThreads % 64 == 0 && kTile % kSymThreads == 0, "symmetric FP32C block shape");

// The rows' times (hi th, lo tl) since the staged tile's first event (hi c0h, lo c0l), scaled by
// s = tsh + tsl like the columns' staged times.
template <int R>
__device__ __forceinline__ void tile_times(const float (&th)[R], const float (&tl)[R], float c0h, float c0l,
                                           float tsh, float tsl, float (&ti)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float tu = (th[r] - c0h) + (tl[r] - c0l);
        ti[r] = fmaf(tu, tsh, tu * tsl);
    }
}

// The compensation terms of the row sums are touched once per 64 columns, so they live in LDS
// (one float per thread per accumulator, thread-contiguous) rather than in registers.
// ZSKIP: the variant for zero-tile skipping (PairReq::zcum set): row blocks' walked tiles in the
// order of walk_tile, and far tiles where one kernel's terms are all exactly zero forming only the
// other's (modes kFullLowB, kFullLowE).
template <bool GRAD, bool ZSKIP>
__global__ __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(kSymWavesPerSimd<GRAD>))) void pair_sym_fp32c(const PairBatch batch)
{
    constexpr int R = kSymRows;
    constexpr int NT = kSymThreads;
    constexpr int K = GRAD ? 6 : 2;
    constexpr int KC = GRAD ? 3 : 1;
    constexpr int TB = kRowsPerBlock / kTile;
    __shared__ float4 sj[2 * kTile];
    __shared__ float colred[kSymWaves][KC][kTile];
    __shared__ float comp_lds[K * R * NT];
    __shared__ float red_lds[kSymWaves][4 * 64];
    volatile lds_float* comp = (lds_float*)comp_lds + threadIdx.x;
    __shared__ long long next_chunk;

    const int q = find_request(batch.r, batch.nreq, (int)blockIdx.x);
    const PairReq& rq = batch.r[q];
    const int blk = (int)blockIdx.x - rq.item_begin;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = rq.n;
    // Walk positions: without zero-tile skipping, units ubegin + position of the lower triangle;
    // with it, the walked units (zcum) from 0.  The block's static range first, then chunks of the
    // dynamic tail (walk_split) while any are left.
    const long long walk0 = ZSKIP ? 0 : rq.ubegin;
    const WalkSplit ws = walk_split(ZSKIP ? rq.zcum[rq.row_blocks] : rq.units, rq.items, rq.dchunks);
    long long r0 = split_begin(blk, ws.sbase, ws.srem), r1 = split_begin(blk + 1, ws.sbase, ws.srem);
    const long long static_len = r1 - r0;
    int slot0 = blk;  // row partials of row block I go to slot slot0 + I
    int prio = -1;

    const float tsh = in_vgpr(rq.tsh), tsl = in_vgpr(rq.tsl), nab = in_vgpr(rq.nab);
    const float nae = in_vgpr(rq.nae), kte = in_vgpr(rq.kte);
    float xh[R], yh[R], xl[R], yl[R];
    float s[6][R];
    int cur = -1, w0 = 0, lrow0 = 0, clo = 0;
    bool active = false;
    float t_first = 0.0f;  // centred time of the wave's first row
    float ti[R];           // the rows' times since the current far tile's first event
    float th[R], tl[R];    // the rows' hi/lo times (kept across tiles without the gradient)

    for (long long chunk = -1;;) {
        long long u = walk0 + r0;
        const long long uend = walk0 + r1;
        int I = 0, kw = 0;  // the current unit: the kw-th walked tile of row block I
        if (u < uend) {
            if (ZSKIP) {
                I = zero_row_block(rq.zcum, rq.row_blocks, u);
                kw = (int)(u - rq.zcum[I]);
            } else {
                I = sym_row_block(u);
                kw = (int)(u - sym_unit0(I));
            }
        }
        cur = -1;
        for (; u < uend; ++u) {
            // Static range: priority from the block's progress through it; dynamic chunks: lowest.
            if (rq.balance) progress_priority(chunk < 0 ? u - walk0 - r0 : static_len, static_len, prio);
            if (I != cur) {
                if (cur >= 0) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            rq.part[((size_t)(slot0 + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] =
                                (double)s[k][r] + (double)comp[(k * R + r) * NT];
                }
                cur = I;
                w0 = I * kRowsPerBlock + wave * (64 * R);
                lrow0 = w0 + R * lane;
                active = w0 < n;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int i = lrow0 + r;
                    const float4 a = rq.ev32[2 * (size_t)i];
                    const float4 b = rq.ev32[2 * (size_t)i + 1];
                    xh[r] = a.x; yh[r] = a.y; xl[r] = b.x; yl[r] = b.y;
                    th[r] = a.z;
                    tl[r] = b.z;
                }
                t_first = uniform(rq.ev32[2 * (size_t)min(w0, n - 1)].z + rq.ev32[2 * (size_t)min(w0, n - 1) + 1].z);
                clo = __builtin_amdgcn_readfirstlane(rq.cut[min(w0, n - 1)]);
#pragma unroll
                for (int k = 0; k < 6; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) s[k][r] = 0.0f;
#pragma unroll
                for (int k = 0; k < K * R; ++k) comp[k * NT] = 0.0f;
            }
            const int tile = ZSKIP ? walk_tile(rq.zcum, rq.row_blocks, I, kw) : kw;
            const int j0 = tile * kTile;
            __syncthreads();
            {
                // Each column's scaled time since the tile's first event goes into the .w of its hi
                // part (read by far tiles only).
                const float c0h = rq.ev32[2 * (size_t)j0].z, c0l = rq.ev32[2 * (size_t)j0 + 1].z;
#pragma unroll
                for (int c = threadIdx.x; c < kTile; c += NT) {
                    const float4* src = rq.ev32 + 2 * (size_t)(j0 + c);
                    float4 hi = src[0];
                    const float4 lo = src[1];
                    const float tu = (hi.z - c0h) + (lo.z - c0l);
                    hi.w = fmaf(tu, tsh, tu * tsl);
                    sj[2 * c] = hi;
                    sj[2 * c + 1] = lo;
                }
            }
            __syncthreads();
            int mode;
            if (!active || j0 >= w0 + 64 * R) mode = kSkip;
            else if (j0 + kTile <= w0) mode = (j0 + kTile <= clo) ? kFullLow : kMaskLow;
            else mode = kDiag;
            float* colw = &colred[wave][0][0];
            if (mode == kSkip) {
#pragma unroll
                for (int qq = 0; qq < KC; ++qq)
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0f;
            } else if (mode == kFullLow && far_tile_by_span(sj, t_first)) {
                if (GRAD) {  // short of registers: the row times are reloaded rather than kept
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        th[r] = rq.ev32[2 * (size_t)(lrow0 + r)].z;
                        tl[r] = rq.ev32[2 * (size_t)(lrow0 + r) + 1].z;
                    }
                }
                tile_times(th, tl, sj[0].z, sj[1].z, tsh, tsl, ti);
                const int ct[R] = {};  // not read: every column of the tile is causal for every row
                int far_mode = kFullLow;
                if (ZSKIP) {
                    // Every pair of the tile is at least `gap` apart in time.
                    const float gap = uniform(t_first - (sj[2 * (kTile - 1)].z + sj[2 * (kTile - 1) + 1].z));
                    const bool no_b = gap >= rq.zero_gap_b, no_e = gap >= rq.zero_gap_e;
                    far_mode = no_b ? (no_e ? kSkip : kFullLowE) : (no_e ? kFullLowB : kFullLow);
                }
                if (far_mode == kFullLow)
                    sym_tile_fp32<kFullLow, GRAD, R, NT>(sj, j0, lrow0, xh, yh, xl, yl, ti, ti, ti, ct, tsh, tsl,
                                                         nab, nae, kte, s, comp, colw, red_lds[wave], lane);
                else if (far_mode == kFullLowB)
                    sym_tile_fp32<kFullLowB, GRAD, R, NT>(sj, j0, lrow0, xh, yh, xl, yl, ti, ti, ti, ct, tsh, tsl,
                                                          nab, nae, kte, s, comp, colw, red_lds[wave], lane);
                else if (far_mode == kFullLowE)
                    sym_tile_fp32<kFullLowE, GRAD, R, NT>(sj, j0, lrow0, xh, yh, xl, yl, ti, ti, ti, ct, tsh, tsl,
                                                          nab, nae, kte, s, comp, colw, red_lds[wave], lane);
                else
#pragma unroll
                    for (int qq = 0; qq < KC; ++qq)
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0f;
            } else {
                // Tiles that straddle the rows' causal counts or their own positions, and causal tiles
                // closer in time to the rows than kNearTiles tile spans (taken by the masked path, whose
                // masks then pass every pair): exact time differences, from the row times loaded here.
                int ct[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    ct[r] = rq.cut[lrow0 + r];
                    if (GRAD) {  // short of registers: reloaded here rather than kept
                        th[r] = rq.ev32[2 * (size_t)(lrow0 + r)].z;
                        tl[r] = rq.ev32[2 * (size_t)(lrow0 + r) + 1].z;
                    }
                }
                if (mode == kDiag)
                    sym_tile_fp32<kDiag, GRAD, R, NT>(sj, j0, lrow0, xh, yh, xl, yl, th, th, tl, ct, tsh, tsl, nab,
                                                      nae, kte, s, comp, colw, red_lds[wave], lane);
                else
                    sym_tile_fp32<kMaskLow, GRAD, R, NT>(sj, j0, lrow0, xh, yh, xl, yl, th, th, tl, ct, tsh, tsl,
                                                         nab, nae, kte, s, comp, colw, red_lds[wave], lane);
            }
            __syncthreads();
            // Column totals of this tile over the block's waves, in wave order (binary32: each is a
            // sum of binary32 terms; the epilogue adds them over row blocks in binary64).
            float* colpart32 = reinterpret_cast<float*>(rq.colpart);
#pragma unroll
            for (int c = threadIdx.x; c < kTile; c += NT) {
                const long long cb = (long long)kRowsPerBlock * I * (I + 1) / 2 + j0 + c;
#pragma unroll
                for (int qq = 0; qq < KC; ++qq) {
                    double v = 0.0;
#pragma unroll
                    for (int w = 0; w < kSymWaves; ++w) v += (double)colred[w][qq][c];
                    colpart32[qq * rq.col_stride + cb] = (float)v;
                }
            }
            if (++kw == (ZSKIP ? walk_units(rq.zcum, rq.row_blocks, I) : TB * (I + 1))) {
                ++I;
                kw = 0;
            }
        }
        if (cur >= 0) {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    rq.part[((size_t)(slot0 + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] =
                        (double)s[k][r] + (double)comp[(k * R + r) * NT];
        }
        // Next chunk of the dynamic tail (the counter starts at zero; every block stops at the first
        // number beyond the last chunk).
        if (ws.chunks == 0) break;
        if (threadIdx.x == 0) next_chunk = (long long)atomicAdd(rq.ctr, 1ULL);
        __syncthreads();
        chunk = next_chunk;
        __syncthreads();
        if (chunk >= ws.chunks) break;
        r0 = ws.sunits + split_begin(chunk, ws.cbase, ws.crem);
        r1 = ws.sunits + split_begin(chunk + 1, ws.cbase, ws.crem);
        slot0 = rq.items + rq.row_blocks + (int)chunk;
    }
}

// Zero-tile skipping tables of one request (one block): for each row block I, zskip[I] = the
// number of leading column tiles t < TB I whose last event is at least zero_dt before the row
// block's first event (a prefix: the events are time-sorted), then zcum = the exclusive prefix sum
// of the walked units TB (I + 1) - zskip[I] in row-block order.  Every pair of a skipped tile is
// separated by at least zero_dt, for which the host guarantees that both the background and the
// trigger exponentials are exactly zero in the pass's arithmetic.
__global__ __launch_bounds__(kThreads) void zero_prefix(const PairBatch batch)
{
    constexpr int TB = kRowsPerBlock / kTile;
    __shared__ long long part[kThreads];
    const PairReq& rq = batch.r[blockIdx.x];
    if (!rq.zcum) return;
    const int RB = rq.row_blocks;
    int* zskip = zero_skip_tiles(rq.zcum, RB);
    const int per = (RB + kThreads - 1) / kThreads;
    const int I0 = min(RB, (int)threadIdx.x * per), I1 = min(RB, I0 + per);
    long long walked = 0;
    for (int I = I0; I < I1; ++I) {
        const double t_first = rq.ev64[(size_t)I * kRowsPerBlock].z;
        int lo = 0, hi = TB * I;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (t_first - rq.ev64[(size_t)mid * kTile + kTile - 1].z >= rq.zero_dt)
                lo = mid + 1;
            else
                hi = mid;
        }
        zskip[I] = lo;
        walked += TB * (I + 1) - lo;
    }
    part[threadIdx.x] = walked;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int k = 0; k < kThreads; ++k) {
            const long long v = part[k];
            part[k] = acc;
            acc += v;
        }
    }
    __syncthreads();
    long long acc = part[threadIdx.x];
    for (int I = I0; I < I1; ++I) {
        rq.zcum[I] = acc;
        acc += TB * (I + 1) - zskip[I];
    }
    if (I0 < I1 && I1 == RB) rq.zcum[RB] = acc;
}

// FP64 symmetric pass: same walk, binary64 pair terms and plain binary64 sums.
template <int MODE, bool GRAD>
__device__ __forceinline__ void sym_tile_fp64(const double4* __restrict__ sj, int j0, int lrow0,
                                              const double (&x)[kRowsPerLane], const double (&y)[kRowsPerLane],
                                              const double (&t)[kRowsPerLane], const int (&ct)[kRowsPerLane],
                                              double nab, double nbb, double nae, double nbe,
                                              double (&a)[6][kRowsPerLane], double* __restrict__ colw,
                                              double* __restrict__ red, int lane)
{
    constexpr int R = kRowsPerLane;
    constexpr int KC = GRAD ? 3 : 1;
    constexpr bool FAR = MODE == kFullLow || MODE == kFullLowB || MODE == kFullLowE;  // unmasked
    constexpr bool DO_B = MODE != kFullLowE;  // background terms (and the column sums)
    constexpr bool DO_E = MODE != kFullLowB;  // trigger terms
    if (!DO_B)
#pragma unroll
        for (int qq = 0; qq < KC; ++qq)
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0;
#pragma unroll 1
    for (int g = 0; g < kTile; g += 4) {
        double cp[3][4];  // set by each column's first row (no additions of zero)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const double4 e = sj[g + cc];
            const int j = j0 + g + cc;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double dx = x[r] - e.x;
                const double dy = y[r] - e.y;
                const double dt = t[r] - e.z;
                const double r2 = fma(dx, dx, dy * dy);
                if (DO_B) {
                    const double dt2 = dt * dt;
                    double ab = fma(r2, nab, dt2 * nbb);
                    if (MODE == kDiag) ab = (j < lrow0 + r) ? ab : -INFINITY;
                    const double b = exp2_f64(ab);
                    a[0][r] += b;
                    if (GRAD) {
                        a[1][r] = fma(r2, b, a[1][r]);
                        a[2][r] = fma(dt2, b, a[2][r]);
                    }
                    if (r == 0) {
                        cp[0][cc] = b;
                        if (GRAD) {
                            cp[1][cc] = r2 * b;
                            cp[2][cc] = dt2 * b;
                        }
                    } else {
                        cp[0][cc] += b;
                        if (GRAD) {
                            cp[1][cc] = fma(r2, b, cp[1][cc]);
                            cp[2][cc] = fma(dt2, b, cp[2][cc]);
                        }
                    }
                }
                if (DO_E) {
                    double ae = fma(r2, nae, dt * nbe);
                    if (!FAR) ae = (j < ct[r]) ? ae : -INFINITY;
                    const double ex = exp2_f64(ae);
                    const int ke = GRAD ? 3 : 1;
                    a[ke][r] += ex;
                    if (GRAD) {
                        a[4][r] = fma(dt, ex, a[4][r]);
                        a[5][r] = fma(r2, ex, a[5][r]);
                    }
                }
            }
        }
        if (DO_B) {
            double v[3];
            column_sums4<KC>(cp, red, lane, v);
            if ((lane & 15) == 0)
#pragma unroll
                for (int q = 0; q < KC; ++q) colw[q * kTile + g + (lane >> 4)] = v[q];
        }
    }
}

template <bool GRAD, bool ZSKIP>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void pair_sym_fp64(const PairBatch batch)
{
    constexpr int R = kRowsPerLane;
    constexpr int K = GRAD ? 6 : 2;
    constexpr int KC = GRAD ? 3 : 1;
    constexpr int TB = kRowsPerBlock / kTile;
    __shared__ double4 sj[kTile];
    __shared__ double colred[4][KC][kTile];
    __shared__ double red_lds[4][4 * 64];

    __shared__ long long next_chunk;
    const int q = find_request(batch.r, batch.nreq, (int)blockIdx.x);
    const PairReq& rq = batch.r[q];
    const int blk = (int)blockIdx.x - rq.item_begin;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = rq.n;
    // The walk of pair_sym_fp32c: the block's static range, then chunks of the dynamic tail.
    const long long walk0 = ZSKIP ? 0 : rq.ubegin;
    const WalkSplit ws = walk_split(ZSKIP ? rq.zcum[rq.row_blocks] : rq.units, rq.items, rq.dchunks);
    long long r0 = split_begin(blk, ws.sbase, ws.srem), r1 = split_begin(blk + 1, ws.sbase, ws.srem);
    const long long static_len = r1 - r0;
    int slot0 = blk;  // row partials of row block I go to slot slot0 + I
    int prio = -1;

    double x[R], y[R], t[R];
    int ct[R];
    double a[6][R];
    int cur = -1, w0 = 0, lrow0 = 0, clo = 0;
    bool active = false;

    for (long long chunk = -1;;) {
        long long u = walk0 + r0;
        const long long uend = walk0 + r1;
        int I = 0, kw = 0;  // the current unit: the kw-th walked tile of row block I
        if (u < uend) {
            if (ZSKIP) {
                I = zero_row_block(rq.zcum, rq.row_blocks, u);
                kw = (int)(u - rq.zcum[I]);
            } else {
                I = sym_row_block(u);
                kw = (int)(u - sym_unit0(I));
            }
        }
        cur = -1;
        for (; u < uend; ++u) {
            if (rq.balance) progress_priority(chunk < 0 ? u - walk0 - r0 : static_len, static_len, prio);
            if (I != cur) {
                if (cur >= 0) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const int ka = GRAD ? k : (k == 0 ? 0 : 1);
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            rq.part[((size_t)(slot0 + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] = a[ka][r];
                    }
                }
                cur = I;
                w0 = I * kRowsPerBlock + wave * (64 * R);
                lrow0 = w0 + R * lane;
                active = w0 < n;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double4 e = rq.ev64[lrow0 + r];
                    x[r] = e.x; y[r] = e.y; t[r] = e.z;
                    ct[r] = rq.cut[lrow0 + r];
                }
                clo = __builtin_amdgcn_readfirstlane(rq.cut[min(w0, n - 1)]);
#pragma unroll
                for (int k = 0; k < 6; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) a[k][r] = 0.0;
            }
            const int tile = ZSKIP ? walk_tile(rq.zcum, rq.row_blocks, I, kw) : kw;
            const int j0 = tile * kTile;
            __syncthreads();
            sj[threadIdx.x] = rq.ev64[j0 + threadIdx.x];
            __syncthreads();
            int mode;
            if (!active || j0 >= w0 + 64 * R) mode = kSkip;
            else if (j0 + kTile <= w0) mode = (j0 + kTile <= clo) ? kFullLow : kMaskLow;
            else mode = kDiag;
            double* colw = &colred[wave][0][0];
            if (mode == kSkip) {
#pragma unroll
                for (int qq = 0; qq < KC; ++qq)
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0;
            } else if (mode == kFullLow) {
                int far_mode = kFullLow;
                if (ZSKIP) {
                    // Every pair of the tile is at least `gap` apart in time.
                    const double gap = uniform(rq.ev64[min(w0, n - 1)].z - sj[kTile - 1].z);
                    const bool no_b = gap >= (double)rq.zero_gap_b, no_e = gap >= (double)rq.zero_gap_e;
                    far_mode = no_b ? (no_e ? kSkip : kFullLowE) : (no_e ? kFullLowB : kFullLow);
                }
                if (far_mode == kFullLow)
                    sym_tile_fp64<kFullLow, GRAD>(sj, j0, lrow0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a, colw,
                                                  red_lds[wave], lane);
                else if (far_mode == kFullLowB)
                    sym_tile_fp64<kFullLowB, GRAD>(sj, j0, lrow0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a, colw,
                                                   red_lds[wave], lane);
                else if (far_mode == kFullLowE)
                    sym_tile_fp64<kFullLowE, GRAD>(sj, j0, lrow0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a, colw,
                                                   red_lds[wave], lane);
                else
#pragma unroll
                    for (int qq = 0; qq < KC; ++qq)
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4) colw[qq * kTile + 4 * lane + k4] = 0.0;
            } else if (mode == kMaskLow) {
                sym_tile_fp64<kMaskLow, GRAD>(sj, j0, lrow0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a, colw, red_lds[wave], lane);
            } else {
                sym_tile_fp64<kDiag, GRAD>(sj, j0, lrow0, x, y, t, ct, rq.nab64, rq.nbb64, rq.nae64, rq.nbe64, a, colw, red_lds[wave], lane);
            }
            __syncthreads();
            const long long cb = (long long)kRowsPerBlock * I * (I + 1) / 2 + j0 + threadIdx.x;
#pragma unroll
            for (int qq = 0; qq < KC; ++qq)
                rq.colpart[qq * rq.col_stride + cb] = colred[0][qq][threadIdx.x] + colred[1][qq][threadIdx.x] +
                                                      colred[2][qq][threadIdx.x] + colred[3][qq][threadIdx.x];
            if (++kw == (ZSKIP ? walk_units(rq.zcum, rq.row_blocks, I) : TB * (I + 1))) {
                ++I;
                kw = 0;
            }
        }
        if (cur >= 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int ka = GRAD ? k : (k == 0 ? 0 : 1);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    rq.part[((size_t)(slot0 + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] = a[ka][r];
            }
        }
        if (ws.chunks == 0) break;
        if (threadIdx.x == 0) next_chunk = (long long)atomicAdd(rq.ctr, 1ULL);
        __syncthreads();
        chunk = next_chunk;
        __syncthreads();
        if (chunk >= ws.chunks) break;
        r0 = ws.sunits + split_begin(chunk, ws.cbase, ws.crem);
        r1 = ws.sunits + split_begin(chunk + 1, ws.cbase, ws.crem);
        slot0 = rq.items + rq.row_blocks + (int)chunk;
    }
}

// Zero the dynamic-tail counters of the launch's requests (before their symmetric pass).
__global__ __launch_bounds__(64) void walk_reset(const PairBatch batch)
{
    const int k = threadIdx.x;
    if (k < batch.nreq && batch.r[k].dchunks > 0) *batch.r[k].ctr = 0ULL;
}

}  // namespace

hipError_t launch_zero_prefix(const PairBatch& b, hipStream_t s)
{
    if (b.nreq <= 0) return hipSuccess;
    zero_prefix<<<dim3(b.nreq), dim3(kThreads), 0, s>>>(b);
    return hipGetLastError();
}

hipError_t launch_pair(const PairBatch& b, int precision, bool grad, int scheme, bool zskip, hipStream_t s)
{
    if (b.total_items <= 0) return hipSuccess;
    const dim3 grid(b.total_items), block(kThreads);
    if (scheme == kSymmetric) {
        bool dynamic_tail = false;
        for (int k = 0; k < b.nreq; ++k) dynamic_tail = dynamic_tail || b.r[k].dchunks > 0;
        if (dynamic_tail) {
            walk_reset<<<dim3(1), dim3(64), 0, s>>>(b);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (precision == kFP32C) {
            if (zskip) {
                if (grad) pair_sym_fp32c<true, true><<<grid, dim3(kSymThreads), 0, s>>>(b);
                else pair_sym_fp32c<false, true><<<grid, dim3(kSymThreads), 0, s>>>(b);
            } else {
                if (grad) pair_sym_fp32c<true, false><<<grid, dim3(kSymThreads), 0, s>>>(b);
                else pair_sym_fp32c<false, false><<<grid, dim3(kSymThreads), 0, s>>>(b);
            }
        } else if (zskip) {
            if (grad) pair_sym_fp64<true, true><<<grid, block, 0, s>>>(b);
            else pair_sym_fp64<false, true><<<grid, block, 0, s>>>(b);
        } else {
            if (grad) pair_sym_fp64<true, false><<<grid, block, 0, s>>>(b);
            else pair_sym_fp64<false, false><<<grid, block, 0, s>>>(b);
        }
    } else if (precision == kFP32C) {
        if (grad) pair_fp32c<true><<<grid, block, 0, s>>>(b);
        else pair_fp32c<false><<<grid, block, 0, s>>>(b);
    } else {
        if (grad) pair_fp64<true><<<grid, block, 0, s>>>(b);
        else pair_fp64<false><<<grid, block, 0, s>>>(b);
    }
    return hipGetLastError();
}

int sym_blocks_per_cu(int precision, bool grad)
{
    int nb = 0;
    hipError_t e;
    if (precision == kFP32C)
        e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_fp32c<true, false>, kSymThreads, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_fp32c<false, false>, kSymThreads, 0);
    else
        e = grad ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_fp64<true, false>, kThreads, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_sym_fp64<false, false>, kThreads, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace hawkes
