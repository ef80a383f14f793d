// hawkes_device.h -- device helpers shared by the pairwise kernels of libhawkes (gfx950).
#pragma once

#include "hawkes_internal.h"

#include <math.h>

namespace hawkes {
namespace dev {

// A float in LDS, addressed as such (accesses through it stay LDS instructions even when the
// pointer is volatile).
using lds_float = __attribute__((address_space(3))) float;

constexpr int kChunk = 64;  // pair terms summed plainly in binary32 before a compensated merge

enum Mode : int { kNone = 0, kFull = 1, kMask = 2 };

// The request of a batched launch that work item `item` belongs to (items are numbered
// consecutively over the requests, request k starting at r[k].item_begin).
template <typename Req>
__device__ __forceinline__ int find_request(const Req* r, int nreq, int item)
{
    int q = 0;
#pragma unroll 1
    for (int k = 1; k < nreq; ++k)
        if (item >= r[k].item_begin) q = k;
    return q;
}

// Keep a wave-uniform constant in a vector register: two-operand VALU ops whose operands are all
// VGPRs issue faster on gfx950 than ones reading a scalar register.
__device__ __forceinline__ float in_vgpr(float v)
{
    float r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// s + c += p with the rounding error of s + p kept exactly in c (Knuth's TwoSum).
__device__ __forceinline__ void two_sum_into(float& s, float& c, float p)
{
    const float t = s + p;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (p - bp);
    s = t;
    c += err;
}

// 2^a in binary64 for a <= 0 (a = -inf allowed).  Range reduction a = k + f, k = rint(a),
// |f| <= 1/2, then 2^f by the degree-10 polynomial that minimises the maximal relative error on
// [-1/2, 1/2] (Remez exchange, exp2_minimax.py; 2.8e-16 relative with the coefficients rounded to
// binary64, about the rounding of the Horner evaluation itself), scaled by 2^k.  Arguments below
// -1100 give exactly 0.
__device__ __forceinline__ double exp2_f64(double a)
{
    a = fmax(a, -1100.0);
    const double k = rint(a);
    const double f = a - k;
    double p = 7.03735743919096230754e-09;
    p = fma(p, f, 1.02085352821412315164e-07);
    p = fma(p, f, 1.32156624055817323250e-06);
    p = fma(p, f, 1.52526581335867644459e-05);
    p = fma(p, f, 1.54035299619204323106e-04);
    p = fma(p, f, 1.33335582285240734912e-03);
    p = fma(p, f, 9.61812910803399277737e-03);
    p = fma(p, f, 5.55041086644591438737e-02);
    p = fma(p, f, 2.40226506959087704463e-01);
    p = fma(p, f, 6.93147180559949727119e-01);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)k);
}

// Symmetric-pass tile modes.  kFullLowB / kFullLowE: an unmasked far tile where every trigger /
// every background term is exactly zero (zero-tile skipping), so only the other kernel is formed.
enum SymMode : int { kSkip = 0, kFullLow = 1, kMaskLow = 2, kDiag = 3, kFullLowB = 4, kFullLowE = 5 };

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v)
{
    const uint2 u = __builtin_bit_cast(uint2, v);
    return __builtin_bit_cast(double, make_uint2((unsigned)__builtin_amdgcn_readfirstlane((int)u.x),
                                                 (unsigned)__builtin_amdgcn_readfirstlane((int)u.y)));
}

// Largest v over the 64 lanes of the wave (every lane receives it).
__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Time differences in the FP32C passes.  Measuring times from a lane's first row makes a column's
// time one value shared by the lane's rows (one subtraction per pair), at an absolute error of a
// few binary32 ulps of the time the lane's rows span.  For a column at least kNearSpans such spans
// before the rows that is at most 2^-23 / kNearSpans of the difference itself; nearer columns,
// where the trigger term and the dt-moments of close pairs are decided, take the difference from
// the hi/lo parts of both events instead (error a binary32 ulp of the difference).
constexpr float kNearSpans = 8.0f;

// Whether a causal tile staged in LDS (sj: hi, lo float4 pairs of kTile events, time in .z) lies at
// least kNearSpans lane spans before the wave's first row (t_first: its centred time, hi + lo).
// Uniform over the wave.
__device__ __forceinline__ bool far_tile(const float4* __restrict__ sj, float t_first, float span)
{
    const float t_last = sj[2 * (kTile - 1)].z + sj[2 * (kTile - 1) + 1].z;
    return uniform(t_first - t_last) >= kNearSpans * span;
}

// The symmetric FP32C pass measures far tiles' times from the staged tile's first event instead:
// a column's time since that event (scaled, formed once when the tile is staged and kept in the
// otherwise unused .w of its hi part) serves every row of the block, and a row's time since it is
// formed once per tile.  With u the binary32 unit roundoff, S the tile's span and d a pair's
// difference, the computed difference is off by at most about u (3 d + 4 S): the rounding of each
// time since the origin and of their difference.  Tiles at least kNearTiles tile spans before the
// wave's first row (S <= d / 2) keep it within 5 u d; nearer ones take the exact path.  (A wider
// near zone, 8 tile spans, puts ~5 % of the tiles at N = 85,000 over 1,000 days on the masked path,
// whose tiles gather at the end of each row block, and was measured 7 % slower.)
constexpr float kNearTiles = 2.0f;

// Whether a causal tile staged in LDS lies at least kNearTiles of its own spans before the wave's
// first row (t_first: its centred time, hi + lo).  Uniform over the wave.
__device__ __forceinline__ bool far_tile_by_span(const float4* __restrict__ sj, float t_first)
{
    const float t_origin = sj[0].z + sj[1].z;
    const float t_last = sj[2 * (kTile - 1)].z + sj[2 * (kTile - 1) + 1].z;
    return uniform(t_first - t_last) >= kNearTiles * uniform(t_last - t_origin);
}

// Lane-rotated copy of v within each 16-lane row (DPP control CTRL, e.g. 0x128 = row_ror:8).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const uint2 u = __builtin_bit_cast(uint2, v);
    uint2 r;
    // No "old" operand: a rotation reads a valid lane everywhere, and an old value of zero would
    // cost a move per half and level (binary64 additions take no DPP operand to fuse it into).
    r.x = (unsigned)__builtin_amdgcn_mov_dpp((int)u.x, CTRL, 0xF, 0xF, false);
    r.y = (unsigned)__builtin_amdgcn_mov_dpp((int)u.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}

// Column sums of one group of four columns over the 64 lanes of a wave, through a wave-private
// LDS area `red` of 4 x 64 values: each lane stores its partial sums of the four columns, reads
// back the values of four consecutive lanes of one column (lane l: column l / 16), adds them,
// and a rotation tree over the 16 lanes of its DPP row finishes the sum, so every lane of row c
// holds the total of column c.  One quantity at a time; out[q] is valid in every lane.  Cheaper
// on the VALU than an all-register transposing tree, whose cross-half lane exchanges
// (v_permlane32/16_swap) issue at half rate.  LDS operations of one wave complete in order, so
// the area is reused without waits.
template <int KC, int NQ>
__device__ __forceinline__ void column_sums4(const float (&cp)[NQ][4], float* __restrict__ red, int lane, float (&out)[NQ])
{
#pragma unroll
    for (int q = 0; q < KC; ++q) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) red[cc * 64 + lane] = cp[q][cc];
        __builtin_amdgcn_wave_barrier();
        const float4 v = *reinterpret_cast<const float4*>(red + (lane >> 4) * 64 + (lane & 15) * 4);
        __builtin_amdgcn_wave_barrier();
        float z = (v.x + v.y) + (v.z + v.w);
        z += dpp_f<0x128>(z);  // row_ror:8
        z += dpp_f<0x124>(z);  // row_ror:4
        z += dpp_f<0x122>(z);  // row_ror:2
        z += dpp_f<0x121>(z);  // row_ror:1
        // Callers store the total from one lane per row; without this the compiler moves the
        // last addition under that lane mask, where its DPP operand can no longer be fused into it
        // (three instructions instead of one).  Not volatile: a volatile statement would also fix
        // its place and serialise the quantities' reductions (measured 3.6 % slower).
        asm("" : "+v"(z));
        out[q] = z;
    }
}

template <int KC, int NQ>
__device__ __forceinline__ void column_sums4(const double (&cp)[NQ][4], double* __restrict__ red, int lane, double (&out)[NQ])
{
#pragma unroll
    for (int q = 0; q < KC; ++q) {
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) red[cc * 64 + lane] = cp[q][cc];
        __builtin_amdgcn_wave_barrier();
        const double* src = red + (lane >> 4) * 64 + (lane & 15) * 4;
        const double2 v0 = *reinterpret_cast<const double2*>(src);
        const double2 v1 = *reinterpret_cast<const double2*>(src + 2);
        __builtin_amdgcn_wave_barrier();
        double z = (v0.x + v0.y) + (v1.x + v1.y);
        z += dpp_d<0x128>(z);
        z += dpp_d<0x124>(z);
        z += dpp_d<0x122>(z);
        z += dpp_d<0x121>(z);
        out[q] = z;
    }
}

// Wave priority from a block's progress through its range of work units.  The hardware issues
// from the oldest ready wave first, so blocks with equal work that share a CU finish far apart
// and the CU runs its last block alone, at one wave per SIMD, which cannot keep the VALU busy.
// Blocks that are behind issue first instead: level 3 below 70 % of the range, then 2, 1 and 0
// from 70, 85 and 95 %.  `level` is the wave's current level (-1 before the first call); every
// argument is uniform over the block.
__device__ __forceinline__ void progress_priority(long long done, long long total, int& level)
{
    const long long d = 20 * done;
    const int want = d >= 19 * total ? 0 : d >= 17 * total ? 1 : d >= 14 * total ? 2 : 3;
    if (want == level) return;
    level = want;
    switch (want) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Even split of the work units over the blocks of a launch: block b walks units
// [split_begin(b), split_begin(b + 1)), the first `rem` blocks one unit more than the others.
__device__ __forceinline__ long long split_begin(long long b, long long base, long long rem)
{
    return b * base + (b < rem ? b : rem);
}

// The block whose range holds unit u.
__device__ __forceinline__ long long split_block(long long u, long long base, long long rem)
{
    const long long big = rem * (base + 1);
    return u < big ? u / (base + 1) : rem + (u - big) / base;
}

// First work unit of each row block: u(I, 0) = TB I (I + 1) / 2, TB tiles per row block.
__device__ __forceinline__ long long sym_unit0(int I)
{
    constexpr long long TB = kRowsPerBlock / kTile;
    return TB * (long long)I * (I + 1) / 2;
}

__device__ __forceinline__ int sym_row_block(long long u);

// The first row block J with sym_unit0(J) >= target.
__device__ __forceinline__ int sym_first_block_from(long long target)
{
    return target <= 0 ? 0 : sym_row_block(target - 1) + 1;
}

__device__ __forceinline__ int sym_row_block(long long u)
{
    constexpr double TB = kRowsPerBlock / kTile;
    int I = (int)((sqrt(8.0 * (double)u / TB + 1.0) - 1.0) * 0.5);
    while (sym_unit0(I + 1) <= u) ++I;
    while (sym_unit0(I) > u) --I;
    return I;
}

// Start of the symmetric walk of block blk: it walks units [u, uend) in order, the first being the
// k-th walked tile of row block I (walk_tile); after the last of row block I comes row block I + 1
// at k = 0.  Without zero-tile skipping the units are the lower triangle's (row block, tile) pairs
// in row-major order, split evenly by the host (ubase, urem); with it they are the same pairs minus
// each row block's zskip[I] leading tiles, split evenly here.
struct SymWalk {
    long long u, uend;
    int I, k;  // the current unit: the k-th walked tile of row block I
};

// Tile of the k-th walked unit of row block I.  Without skipping: tile k.  With zero-tile
// skipping the row block's walked tiles [zskip[I], TB (I + 1)) are visited outside-in (first,
// last, second, second-to-last, ...): the far tiles at one end, which skipping leaves cheap (one
// kernel only), and the near, masked ones at the other, which cost most, alternate, so the short
// contiguous unit ranges of the blocks carry similar work.
__device__ __forceinline__ int walk_tile(const long long* zcum, int row_blocks, int I, int k)
{
    constexpr int TB = kRowsPerBlock / kTile;
    const int first = zero_skip_tiles(zcum, row_blocks)[I];
    const int n = TB * (I + 1) - first;
    return first + ((k & 1) ? n - 1 - (k >> 1) : (k >> 1));
}

// Walked units of row block I.
__device__ __forceinline__ int walk_units(const long long* zcum, int row_blocks, int I)
{
    constexpr int TB = kRowsPerBlock / kTile;
    return TB * (I + 1) - (zcum ? zero_skip_tiles(zcum, row_blocks)[I] : 0);
}

// The row block holding walked unit u under zero-tile skipping: the largest I with zcum[I] <= u.
__device__ __forceinline__ int zero_row_block(const long long* zcum, int row_blocks, long long u)
{
    int lo = 0, hi = row_blocks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (zcum[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename Req>
__device__ __forceinline__ SymWalk sym_walk_begin(const Req& rq, int blk)
{
    SymWalk w;
    if (rq.zcum) {
        const long long units = rq.zcum[rq.row_blocks];
        const long long base = units / rq.items, rem = units % rq.items;
        w.u = split_begin(blk, base, rem);
        w.uend = split_begin(blk + 1, base, rem);
        w.I = zero_row_block(rq.zcum, rq.row_blocks, w.u < units ? w.u : units - 1);
        w.k = (int)(w.u - rq.zcum[w.I]);
    } else {
        w.u = rq.ubegin + split_begin(blk, rq.ubase, rq.urem);
        w.uend = rq.ubegin + split_begin(blk + 1, rq.ubase, rq.urem);
        w.I = sym_row_block(w.u);
        w.k = (int)(w.u - sym_unit0(w.I));
    }
    return w;
}

}  // namespace dev
}  // namespace hawkes
