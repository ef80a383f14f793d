// hawkes_multi.hip -- the log-likelihood and the self-excitation probabilities for many parameter
// vectors over one dataset (arXiv 2005.10123, Section 2.1: the log-likelihood equation and the
// probability equation pi_n = xi_n / lambda_n; Section 3.2 evaluates pi for 1,000 posterior samples
// of Theta).
//
// FP32C: the symmetric lower-triangle walk of the single-Theta pass, but each pair's differences,
// r^2 and dt^2 are formed once and shared by kMultiTheta parameter vectors, each with its own two
// exponentials and running sums (log-likelihood terms only: S_b, S_e).  Time differences are taken
// from each lane's own first row without a Theta-dependent scale.  FP64: one FP64 evaluation per
// parameter vector.
#include "hawkes_device.h"
#include "hawkes_runtime.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace hawkes {

// Shape of the FP32C multi-parameter pass: kMultiRows rows per lane; a block's threads together hold
// one row block of the walk; the register budget is sized for kMultiWavesPerSimd waves per SIMD.
constexpr int kMultiRows = 4;
constexpr int kMultiThreads = kRowsPerBlock / kMultiRows;
constexpr int kMultiWaves = kMultiThreads / 64;
constexpr int kMultiWavesPerSimd = 2;
static_assert(kMultiThreads % 64 == 0 && kMultiThreads >= kTile, "multi-parameter block shape");

struct MultiReq {
    const float4* ev32;
    const int* cut;
    double* part;     // [blocks + row_blocks][2 * kMultiTheta][kRowsPerBlock]
    double* colpart;  // [kMultiTheta][col_stride]
    long long* zcum;  // zero-tile skipping tables (as in PairReq) for all vectors of the pass, or nullptr
    long long units, col_stride, ubegin;
    int n, npad, row_blocks, ubase, urem, items;
    float nab[kMultiTheta], nbb[kMultiTheta], nae[kMultiTheta], nbe[kMultiTheta];
};

struct MultiEpi {
    const double4* ev64;
    const double* part;
    const double* colpart;
    const long long* zcum;  // as in MultiReq
    int items;              // blocks of the pairwise pass
    double* pi_out;      // [nth][n] in sorted order, or nullptr
    double* block_part;  // [nblocks][kMultiTheta]
    double* out;         // log-likelihood of vector q at out[q * out_stride]
    int out_stride;
    long long col_stride;
    int n, npad, row_blocks, ubase, urem, nth, nblocks;
    double T;
    double mu0[kMultiTheta], tau_t[kMultiTheta], theta[kMultiTheta], omega[kMultiTheta];
    double cb[kMultiTheta], ce[kMultiTheta];
};

namespace {

using namespace dev;

template <int MODE, int KT>
__device__ __forceinline__ void multi_tile(const float4* __restrict__ sj, int j0, int lrow0,
                                           const float (&xh)[kMultiRows], const float (&yh)[kMultiRows],
                                           const float (&xl)[kMultiRows], const float (&yl)[kMultiRows],
                                           const float (&ti)[kMultiRows], const float (&th)[kMultiRows],
                                           const float (&tl)[kMultiRows], const int (&ct)[kMultiRows],
                                           float t0h, float t0l, const float (&nab)[KT],
                                           const float (&nbb)[KT], const float (&nae)[KT],
                                           const float (&nbe)[KT], float (&s)[2 * KT][kMultiRows],
                                           volatile lds_float* comp, float* __restrict__ colw,
                                           float* __restrict__ red, int lane)
{
    constexpr int R = kMultiRows;
    // Far tiles measure times from the lane's first row; masked and near ones take each pair's time
    // difference from the hi/lo parts of both events (see kNearSpans).
    constexpr bool EXACT = MODE != kFullLow;
    for (int ch = 0; ch < kTile; ch += kChunk) {
        float p[2 * KT][R];
#pragma unroll
        for (int k = 0; k < 2 * KT; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) p[k][r] = 0.0f;
#pragma unroll 1
        for (int g = ch; g < ch + kChunk; g += 4) {
            float cp[KT][4];  // set by each column's first row (no additions of zero)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const float4 hi = sj[2 * (g + cc)];
                const float4 lo = sj[2 * (g + cc) + 1];
                const float tj = EXACT ? 0.0f : (hi.z - t0h) + (lo.z - t0l);
                const int j = j0 + g + cc;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = (xh[r] - hi.x) + (xl[r] - lo.x);
                    const float dy = (yh[r] - hi.y) + (yl[r] - lo.y);
                    const float dt = EXACT ? (th[r] - hi.z) + (tl[r] - lo.z) : ti[r] - tj;
                    const float r2 = fmaf(dx, dx, dy * dy);
                    const float dt2 = dt * dt;
                    const bool below = MODE != kDiag || j < lrow0 + r;
                    const bool causal = MODE == kFullLow || j < ct[r];
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        float ab = fmaf(r2, nab[q], dt2 * nbb[q]);
                        if (MODE == kDiag) ab = below ? ab : -INFINITY;
                        const float b = __builtin_amdgcn_exp2f(ab);
                        p[2 * q][r] += b;
                        cp[q][cc] = r == 0 ? b : cp[q][cc] + b;
                        float ae = fmaf(r2, nae[q], dt * nbe[q]);
                        if (MODE != kFullLow) ae = causal ? ae : -INFINITY;
                        p[2 * q + 1][r] += __builtin_amdgcn_exp2f(ae);
                    }
                }
            }
            float v[KT];
            column_sums4<KT>(cp, red, lane, v);
            if ((lane & 15) == 0)
#pragma unroll
                for (int q = 0; q < KT; ++q) colw[q * kTile + g + (lane >> 4)] = v[q];
        }
#pragma unroll
        for (int k = 0; k < 2 * KT; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float cc = comp[(k * R + r) * kMultiThreads];
                two_sum_into(s[k][r], cc, p[k][r]);
                comp[(k * R + r) * kMultiThreads] = cc;
            }
    }
}

// KT parameter vectors per pass (1 to kMultiTheta); a vector's arithmetic is the same for every KT,
// so its results do not depend on the vectors it shares a pass with.
template <int KT>
__global__ __launch_bounds__(kMultiThreads) __attribute__((amdgpu_waves_per_eu(kMultiWavesPerSimd))) void pair_multi_fp32c(const MultiReq rq)
{
    constexpr int R = kMultiRows;
    constexpr int K = 2 * KT;
    constexpr int TB = kRowsPerBlock / kTile;
    __shared__ float4 sj[2 * kTile];
    __shared__ float colred[kMultiWaves][KT][kTile];
    __shared__ float comp_lds[K * R * kMultiThreads];
    __shared__ float red_lds[kMultiWaves][4 * 64];
    volatile lds_float* comp = (lds_float*)comp_lds + threadIdx.x;

    const int blk = (int)blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = rq.n;
    const SymWalk walk = sym_walk_begin(rq, blk);
    long long u = walk.u;
    const long long uend = walk.uend;
    const long long ubeg = u;
    int prio = -1;
    int I = walk.I;
    int kw = walk.k;  // position of the current unit among row block I's walked tiles

    float nab[KT], nbb[KT], nae[KT], nbe[KT];
#pragma unroll
    for (int q = 0; q < KT; ++q) {
        nab[q] = in_vgpr(rq.nab[q]);
        nbb[q] = in_vgpr(rq.nbb[q]);
        nae[q] = in_vgpr(rq.nae[q]);
        nbe[q] = in_vgpr(rq.nbe[q]);
    }
    float xh[R], yh[R], xl[R], yl[R];
    float s[K][R];
    int cur = -1, w0 = 0, lrow0 = 0, clo = 0;
    bool active = false;
    float t_first = 0.0f;  // centred time of the wave's first row
    float span = 0.0f;     // largest time spanned by one lane's rows in the wave

    for (; u < uend; ++u) {
        progress_priority(u - ubeg, uend - ubeg, prio);
        if (I != cur) {
            if (cur >= 0) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        rq.part[((size_t)(blk + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] =
                            (double)s[k][r] + (double)comp[(k * R + r) * kMultiThreads];
            }
            cur = I;
            w0 = I * kRowsPerBlock + wave * (64 * R);
            lrow0 = w0 + R * lane;
            active = w0 < n;
            float lane_span = 0.0f, t0h = 0.0f, t0l = 0.0f;
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
                if (i < n) lane_span = (a.z - t0h) + (b.z - t0l);  // time-sorted: the last valid row is the latest
            }
            span = uniform(wave_max(lane_span));
            t_first = uniform(rq.ev32[2 * (size_t)min(w0, n - 1)].z + rq.ev32[2 * (size_t)min(w0, n - 1) + 1].z);
            clo = __builtin_amdgcn_readfirstlane(rq.cut[min(w0, n - 1)]);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    s[k][r] = 0.0f;
                    comp[(k * R + r) * kMultiThreads] = 0.0f;
                }
        }
        const int tile = (rq.zcum != nullptr) ? walk_tile(rq.zcum, rq.row_blocks, I, kw) : kw;
        const int j0 = tile * kTile;
        __syncthreads();
        for (int c = threadIdx.x; c < kTile; c += kMultiThreads) {
            const float4* src = rq.ev32 + 2 * (size_t)(j0 + c);
            sj[2 * c] = src[0];
            sj[2 * c + 1] = src[1];
        }
        __syncthreads();
        int mode;
        if (!active || j0 >= w0 + 64 * R) mode = kSkip;
        else if (j0 + kTile <= w0) mode = (j0 + kTile <= clo) ? kFullLow : kMaskLow;
        else mode = kDiag;
        float* colw = &colred[wave][0][0];
        if (mode == kSkip) {
#pragma unroll
            for (int q = 0; q < KT; ++q)
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) colw[q * kTile + 4 * lane + k4] = 0.0f;
        } else if (mode == kFullLow && far_tile(sj, t_first, span)) {
            // Row times from the lane's first row, formed per tile rather than kept live.
            float ti[R];
            const float t0h = rq.ev32[2 * (size_t)lrow0].z, t0l = rq.ev32[2 * (size_t)lrow0 + 1].z;
#pragma unroll
            for (int r = 0; r < R; ++r)
                ti[r] = (rq.ev32[2 * (size_t)(lrow0 + r)].z - t0h) + (rq.ev32[2 * (size_t)(lrow0 + r) + 1].z - t0l);
            const int ct[R] = {};  // not read: every column of the tile is causal for every row
            multi_tile<kFullLow, KT>(sj, j0, lrow0, xh, yh, xl, yl, ti, ti, ti, ct, t0h, t0l, nab, nbb, nae, nbe, s, comp, colw,
                                 red_lds[wave], lane);
        } else {
            // Straddling tiles and near causal ones (the masked path; its causal mask then passes
            // every pair): exact time differences from the rows' hi/lo times.
            int ct[R];
            float th[R], tl[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                ct[r] = rq.cut[lrow0 + r];
                th[r] = rq.ev32[2 * (size_t)(lrow0 + r)].z;
                tl[r] = rq.ev32[2 * (size_t)(lrow0 + r) + 1].z;
            }
            if (mode == kDiag)
                multi_tile<kDiag, KT>(sj, j0, lrow0, xh, yh, xl, yl, th, th, tl, ct, 0.0f, 0.0f, nab, nbb, nae, nbe, s, comp, colw,
                                  red_lds[wave], lane);
            else
                multi_tile<kMaskLow, KT>(sj, j0, lrow0, xh, yh, xl, yl, th, th, tl, ct, 0.0f, 0.0f, nab, nbb, nae, nbe, s, comp,
                                     colw, red_lds[wave], lane);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < kTile; c += kMultiThreads) {
            const long long cb = (long long)kRowsPerBlock * I * (I + 1) / 2 + j0 + c;
#pragma unroll
            for (int q = 0; q < KT; ++q) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < kMultiWaves; ++w) v += (double)colred[w][q][c];
                rq.colpart[q * rq.col_stride + cb] = v;
            }
        }
        if (++kw == ((rq.zcum != nullptr) ? walk_units(rq.zcum, rq.row_blocks, I) : TB * (I + 1))) {
            ++I;
            kw = 0;
        }
    }
    if (cur >= 0) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r)
                rq.part[((size_t)(blk + cur) * K + k) * kRowsPerBlock + wave * 64 * R + R * lane + r] =
                    (double)s[k][r] + (double)comp[(k * R + r) * kMultiThreads];
    }
}

__device__ __forceinline__ double normal_cdf(double z) { return 0.5 * erfc(-z * 0.70710678118654752440); }

// Per event and parameter vector: lambda, Lambda, ell_i and pi_i (binary64); block sums of ell.
template <int KT>
__global__ __launch_bounds__(kThreads) void epilogue_multi(const MultiEpi e)
{
    constexpr long long TB = kRowsPerBlock / kTile;
    __shared__ double red[KT][kThreads];
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double v[KT] = {};
    if (i < e.n) {
        const int I = i / kRowsPerBlock, rho = i % kRowsPerBlock;
        long long bf, bl;
        int J1 = e.row_blocks;
        if (e.zcum) {  // zero-tile skipping: the walked units, split evenly; see the single-Theta epilogue
            const long long units = e.zcum[e.row_blocks];
            const long long base = units / e.items, rem = units % e.items;
            bf = split_block(e.zcum[I], base, rem);
            bl = split_block(e.zcum[I + 1] - 1, base, rem);
            const int* zskip = zero_skip_tiles(e.zcum, e.row_blocks);
            const int tile_i = i / kTile;
            int a = I;
            while (a < J1) {
                const int mid = (a + J1) >> 1;
                if (zskip[mid] > tile_i)
                    J1 = mid;
                else
                    a = mid + 1;
            }
        } else {
            bf = split_block(TB * I * (I + 1) / 2, e.ubase, e.urem);
            bl = split_block(TB * (I + 1) * (I + 2) / 2 - 1, e.ubase, e.urem);
        }
        double Sb[KT] = {}, Se[KT] = {};
        for (long long b = bf; b <= bl; ++b) {
            const double* ps = e.part + (size_t)(b + I) * 2 * KT * kRowsPerBlock + rho;
#pragma unroll
            for (int q = 0; q < KT; ++q) {
                Sb[q] += ps[(size_t)(2 * q) * kRowsPerBlock];
                Se[q] += ps[(size_t)(2 * q + 1) * kRowsPerBlock];
            }
        }
        for (int J = I; J < J1; ++J) {
            const double* pc = e.colpart + (long long)kRowsPerBlock * J * (J + 1) / 2 + i;
#pragma unroll
            for (int q = 0; q < KT; ++q) Sb[q] += pc[q * e.col_stride];
        }
        const double ti = e.ev64[i].z;
        const double u = e.T - ti;
#pragma unroll
        for (int q = 0; q < KT; ++q) {
            if (q >= e.nth) break;
            const double lam = e.cb[q] * (Sb[q] + 1.0) + e.ce[q] * Se[q];
            const double Lam = e.mu0[q] * (normal_cdf(u / e.tau_t[q]) - normal_cdf(-ti / e.tau_t[q])) -
                               e.theta[q] * expm1(-e.omega[q] * u);
            v[q] = log(lam) - Lam;
            if (e.pi_out) e.pi_out[(size_t)q * e.n + i] = e.ce[q] * Se[q] / lam;
        }
    }
#pragma unroll
    for (int q = 0; q < KT; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
#pragma unroll
            for (int q = 0; q < KT; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < KT; ++q) e.block_part[(size_t)blockIdx.x * KT + q] = red[q][0];
}

template <int KT>
__global__ __launch_bounds__(kThreads) void final_multi(const MultiEpi e)
{
    __shared__ double red[KT][kThreads];
    double v[KT] = {};
    for (int b = threadIdx.x; b < e.nblocks; b += kThreads)
#pragma unroll
        for (int q = 0; q < KT; ++q) v[q] += e.block_part[(size_t)b * KT + q];
#pragma unroll
    for (int q = 0; q < KT; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int stride = kThreads / 2; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride)
#pragma unroll
            for (int q = 0; q < KT; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + stride];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < KT; ++q) e.out[(size_t)q * e.out_stride] = red[q][0];
}

}  // namespace

int multi_blocks_per_cu()
{
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pair_multi_fp32c<kMultiTheta>, kMultiThreads, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

// Split and scratch layout of the FP32C multi-parameter pass over one dataset.  They do not depend
// on the number of vectors in a pass (the grid is sized for kMultiTheta), so a vector's result is the
// same whichever vectors share its pass.
struct MultiPlan {
    long long T = 0, units = 0, col_stride = 0;
    int items = 0, ubase = 0, urem = 0, nblocks = 0;
    size_t part_d = 0, col_d = 0, z_d = 0;  // doubles
};

static MultiPlan multi_plan(const hawkes_ctx* c, const Dataset& d, bool zero_skip)
{
    constexpr int KT = kMultiTheta;
    const long long TB = kRowsPerBlock / kTile;
    MultiPlan m;
    m.T = d.npad / kRowsPerBlock;
    m.units = TB * m.T * (m.T + 1) / 2;
    const long long slots = std::max(1, c->multi_slots);
    m.items = (int)std::min(slots, m.units);
    m.ubase = (int)(m.units / m.items);
    m.urem = (int)(m.units % m.items);
    m.col_stride = (long long)kRowsPerBlock * m.T * (m.T + 1) / 2;
    m.nblocks = (int)((d.n + kThreads - 1) / kThreads);
    m.part_d = (size_t)(m.items + m.T) * 2 * KT * kRowsPerBlock;
    m.col_d = (size_t)KT * m.col_stride;
    m.z_d = zero_skip ? ((size_t)(m.T + 1) * sizeof(long long) + (size_t)m.T * sizeof(int) + 7) / 8 : 0;
    return m;
}

// Scratch of one pass: row partials, column partials, block partials, 8 result doubles, zero-tile
// tables, then (want_pi) kMultiTheta x n probabilities.
size_t multi_scratch_bytes(const hawkes_ctx* c, const Dataset& d, bool zero_skip, bool want_pi)
{
    const MultiPlan m = multi_plan(c, d, zero_skip);
    const size_t pi_d = want_pi ? (size_t)kMultiTheta * d.n : 0;
    return (m.part_d + m.col_d + (size_t)m.nblocks * kMultiTheta + 8 + m.z_d + pi_d) * sizeof(double);
}

template <int KT>
static hipError_t launch_multi(const MultiReq& r, const MultiEpi& e, int items, int nblocks, hipStream_t s)
{
    pair_multi_fp32c<KT><<<dim3(items), dim3(kMultiThreads), 0, s>>>(r);
    epilogue_multi<KT><<<dim3(nblocks), dim3(kThreads), 0, s>>>(e);
    final_multi<KT><<<dim3(1), dim3(kThreads), 0, s>>>(e);
    return hipGetLastError();
}

// Enqueue one pass over nth (1 to kMultiTheta) parameter vectors on stream s: ell of vector q to
// out[q * out_stride] (device memory), pi of event i (sorted order) to pi_out[q * n + i] when pi_out
// is set.  The scratch is laid out as multi_scratch_bytes describes.
hipError_t enqueue_multi_fp32c(const hawkes_ctx* c, const Dataset& d, const hawkes_params* th, int nth, char* scratch,
                               bool zero_skip, double* out, int out_stride, double* pi_out, hipStream_t s)
{
    constexpr int KT = kMultiTheta;
    const MultiPlan m = multi_plan(c, d, zero_skip);
    double* base = (double*)scratch;
    MultiReq r;
    memset(&r, 0, sizeof r);
    r.ev32 = d.ev32;
    r.cut = d.cut;
    r.part = base;
    r.colpart = base + m.part_d;
    r.units = m.units;
    r.col_stride = m.col_stride;
    r.n = (int)d.n;
    r.npad = d.npad;
    r.row_blocks = (int)m.T;
    r.ubase = m.ubase;
    r.urem = m.urem;
    r.items = m.items;
    MultiEpi e;
    memset(&e, 0, sizeof e);
    e.ev64 = d.ev64;
    e.part = r.part;
    e.colpart = r.colpart;
    e.block_part = base + m.part_d + m.col_d;
    e.out = out;
    e.out_stride = out_stride;
    e.pi_out = pi_out;
    r.zcum = zero_skip ? (long long*)(e.block_part + (size_t)m.nblocks * KT + 8) : nullptr;
    e.zcum = r.zcum;
    e.items = m.items;
    e.col_stride = m.col_stride;
    e.n = (int)d.n;
    e.npad = d.npad;
    e.row_blocks = (int)m.T;
    e.ubase = m.ubase;
    e.urem = m.urem;
    e.nblocks = m.nblocks;
    e.T = d.T;
    e.nth = nth;
    const double log2e = 1.44269504088896340736, two_pi = 6.28318530717958647693;
    for (int q = 0; q < nth; ++q) {
        const hawkes_params& p = th[q];
        r.nab[q] = (float)(-log2e / (2.0 * p.tau_x * p.tau_x));
        r.nbb[q] = (float)(-log2e / (2.0 * p.tau_t * p.tau_t));
        r.nae[q] = (float)(-log2e / (2.0 * p.h * p.h));
        r.nbe[q] = (float)(-log2e * p.omega);
        e.mu0[q] = p.mu0;
        e.tau_t[q] = p.tau_t;
        e.theta[q] = p.theta;
        e.omega[q] = p.omega;
        e.cb[q] = p.mu0 / (std::pow(two_pi, 1.5) * p.tau_x * p.tau_x * p.tau_t);
        e.ce[q] = p.theta * p.omega / (two_pi * p.h * p.h);
    }
    hipError_t err = hipSuccess;
    if (zero_skip) {
        // Zero-tile tables of the pass: the tiles where the pair terms of all its vectors vanish.
        PairBatch zb;
        memset(&zb, 0, sizeof zb);
        zb.nreq = 1;
        zb.r[0].ev64 = d.ev64;
        zb.r[0].row_blocks = (int)m.T;
        zb.r[0].zcum = r.zcum;
        double zdt = 0.0;
        for (int q = 0; q < nth; ++q) zdt = std::max(zdt, zero_separation(th[q], kFP32C, d.T));
        zb.r[0].zero_dt = zdt;
        if ((err = launch_zero_prefix(zb, s)) != hipSuccess) return err;
    }
    switch (nth) {
    case 1: return launch_multi<1>(r, e, m.items, m.nblocks, s);
    case 2: return launch_multi<2>(r, e, m.items, m.nblocks, s);
    case 3: return launch_multi<3>(r, e, m.items, m.nblocks, s);
    default: return launch_multi<4>(r, e, m.items, m.nblocks, s);
    }
}

// FP32C: up to kMultiTheta parameter vectors per pass.  Caller holds c->mu.
static hawkes_status multi_fp32c(hawkes_ctx* c, const Dataset& d, const hawkes_params* th, int S, double* out_ll,
                                 double* out_pi)
{
    constexpr int KT = kMultiTheta;
    const bool zero_skip = c->zero_skip;
    const MultiPlan m = multi_plan(c, d, zero_skip);
    hawkes_status st = reserve_blocking(c, multi_scratch_bytes(c, d, zero_skip, out_pi != nullptr));
    if (st != HAWKES_OK) return st;
    double* out = (double*)c->blk.base + m.part_d + m.col_d + (size_t)m.nblocks * KT;
    double* pi_dev = out_pi ? out + 8 + m.z_d : nullptr;
    std::vector<double> host_out(8);
    std::vector<double> host_pi(out_pi ? (size_t)KT * d.n : 0);
    hipStream_t s = c->stream;
    hipError_t err = hipStreamWaitEvent(s, c->blk_free, 0);
    for (int s0 = 0; s0 < S && err == hipSuccess; s0 += KT) {
        const int nth = std::min(KT, S - s0);
        err = enqueue_multi_fp32c(c, d, th + s0, nth, c->blk.base, zero_skip, out, 1, pi_dev, s);
        if (err == hipSuccess) err = hipMemcpyAsync(host_out.data(), out, nth * sizeof(double), hipMemcpyDeviceToHost, s);
        if (err == hipSuccess && out_pi)
            err = hipMemcpyAsync(host_pi.data(), pi_dev, (size_t)nth * d.n * sizeof(double), hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) break;
        for (int q = 0; q < nth; ++q) {
            if (out_ll) out_ll[s0 + q] = host_out[q];
            if (out_pi)
                for (int64_t k = 0; k < d.n; ++k) out_pi[(size_t)(s0 + q) * d.n + d.perm[k]] = host_pi[(size_t)q * d.n + k];
        }
    }
    if (err == hipSuccess) err = hipEventRecord(c->blk_free, s);
    if (err != hipSuccess) {
        c->poisoned = true;
        return hip_fail(err, "multi-parameter evaluation");
    }
    return HAWKES_OK;
}

}  // namespace hawkes

using namespace hawkes;

extern "C" hawkes_status hawkes_loglik_multi(hawkes_ctx* c, int32_t id, const hawkes_params* thetas, int32_t count,
                                             int precision, double* out_loglik, double* out_pi)
{
    hawkes_status st = begin_call(c);
    if (st != HAWKES_OK) return st;
    if (count < 0 || (count > 0 && !thetas)) return fail(HAWKES_EINVAL, "bad parameter array");
    if (!out_loglik && !out_pi) return fail(HAWKES_EINVAL, "no output requested");
    if (precision != HAWKES_FP64 && precision != HAWKES_FP32C)
        return fail(HAWKES_EINVAL, "precision %d is neither HAWKES_FP64 nor HAWKES_FP32C", precision);
    for (int k = 0; k < count; ++k)
        if ((st = check_params(&thetas[k])) != HAWKES_OK) return st;
    if (count == 0) return HAWKES_OK;
    if (precision == HAWKES_FP64) {
        // One binary64 evaluation per parameter vector (per-event results give pi).
        int64_t n = 0;
        if ((st = hawkes_dataset_info(c, id, &n, nullptr)) != HAWKES_OK) return st;
        std::vector<double> rows((size_t)n * kRowOut);
        for (int k = 0; k < count; ++k) {
            double o7[7];
            if ((st = blocking_eval(c, id, &thetas[k], HAWKES_FP64, false, o7, rows.data())) != HAWKES_OK) return st;
            if (out_loglik) out_loglik[k] = o7[0];
            if (out_pi)
                for (int64_t e = 0; e < n; ++e) out_pi[(size_t)k * n + e] = rows[(size_t)e * kRowOut + 3];
        }
        return HAWKES_OK;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    Dataset* d = find_dataset(c, id);
    if (!d) return fail(HAWKES_ENOTFOUND, "no dataset %d", id);
    return multi_fp32c(c, *d, thetas, count, out_loglik, out_pi);
}
