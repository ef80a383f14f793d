// hawkes_device.h -- device helpers shared by the pairwise kernels of libhawkes (gfx950).
#pragma once

#include "hawkes_internal.h"

#include <math.h>

namespace hawkes {
namespace dev {

constexpr int kChunk = 64;  // pair terms summed plainly in binary32 before a compensated merge

enum Mode : int { kNone = 0, kFull = 1, kMask = 2 };

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
// |f| <= 1/2, then 2^f = exp(f ln 2) by its Taylor polynomial of degree 12 (truncation error
// below 2e-16 relative on |f ln 2| <= 0.347), scaled by 2^k.  Arguments below -1100 give exactly 0.
__device__ __forceinline__ double exp2_f64(double a)
{
    a = fmax(a, -1100.0);
    const double k = rint(a);
    const double f = a - k;
    double p = 2.5678435993488205142e-11;
    p = fma(p, f, 4.4455382718708114976e-10);
    p = fma(p, f, 7.0549116208011233299e-09);
    p = fma(p, f, 1.0178086009239699727e-07);
    p = fma(p, f, 1.3215486790144309488e-06);
    p = fma(p, f, 1.5252733804059840280e-05);
    p = fma(p, f, 1.5403530393381609954e-04);
    p = fma(p, f, 1.3333558146428443423e-03);
    p = fma(p, f, 9.6181291076284771620e-03);
    p = fma(p, f, 5.5504108664821579953e-02);
    p = fma(p, f, 2.4022650695910071233e-01);
    p = fma(p, f, 6.9314718055994530942e-01);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)k);
}

enum SymMode : int { kSkip = 0, kFullLow = 1, kMaskLow = 2, kDiag = 3 };

// v_permlane32_swap exchanges the upper 32 lanes of the first register with the lower 32 lanes
// of the second; v_permlane16_swap exchanges the odd 16-lane rows of the first with the even rows
// of the second.  Written as inline assembly with both registers as outputs (the compiler
// builtin's second result is not reliable); the s_nop covers the hazard of a VALU write
// immediately followed by a permlane read of the same register.
__device__ __forceinline__ void swap32(float& a, float& b)
{
    asm("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap16(float& a, float& b)
{
    asm("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
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
    r.x = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.x, CTRL, 0xF, 0xF, false);
    r.y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)u.y, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ void swap32(double& a, double& b)
{
    uint2 ua = __builtin_bit_cast(uint2, a), ub = __builtin_bit_cast(uint2, b);
    asm("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\tv_permlane32_swap_b32 %2, %3"
        : "+v"(ua.x), "+v"(ub.x), "+v"(ua.y), "+v"(ub.y));
    a = __builtin_bit_cast(double, ua);
    b = __builtin_bit_cast(double, ub);
}
__device__ __forceinline__ void swap16(double& a, double& b)
{
    uint2 ua = __builtin_bit_cast(uint2, a), ub = __builtin_bit_cast(uint2, b);
    asm("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\tv_permlane16_swap_b32 %2, %3"
        : "+v"(ua.x), "+v"(ub.x), "+v"(ua.y), "+v"(ub.y));
    a = __builtin_bit_cast(double, ua);
    b = __builtin_bit_cast(double, ub);
}

// Sum over the 64 lanes of v0..v3 (four columns); lane l receives the total of column l / 16.
// The swaps pair lane l with l + 32 (then l + 16) while handing half of the columns to each side,
// so the two exchange steps cost one add per column pair; rotations by 8, 4, 2, 1 within each
// 16-lane row finish the sum.  10 operations per four columns.
template <typename T>
__device__ __forceinline__ T reduce4(T v0, T v1, T v2, T v3)
{
    swap32(v0, v2);
    swap32(v1, v3);
    T a0 = v0 + v2, a1 = v1 + v3;
    swap16(a0, a1);
    T z = a0 + a1;
    if constexpr (sizeof(T) == 4) {
        z += dpp_f<0x128>(z);  // row_ror:8
        z += dpp_f<0x124>(z);  // row_ror:4
        z += dpp_f<0x122>(z);  // row_ror:2
        z += dpp_f<0x121>(z);  // row_ror:1
    } else {
        z += dpp_d<0x128>(z);
        z += dpp_d<0x124>(z);
        z += dpp_d<0x122>(z);
        z += dpp_d<0x121>(z);
    }
    return z;
}

// reduce4 for KC quantities at once, step by step interleaved so that each dependent DPP step
// of one quantity is separated by the others' (hides the DPP read-after-write wait states).
template <int KC, int NQ, typename T>
__device__ __forceinline__ void reduce4_multi(T (&cp)[NQ][4], T (&out)[NQ])
{
    T a0[KC], a1[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
        swap32(cp[q][0], cp[q][2]);
        swap32(cp[q][1], cp[q][3]);
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
        a0[q] = cp[q][0] + cp[q][2];
        a1[q] = cp[q][1] + cp[q][3];
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) swap16(a0[q], a1[q]);
#pragma unroll
    for (int q = 0; q < KC; ++q) out[q] = a0[q] + a1[q];
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_f<0x128>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_f<0x124>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_f<0x122>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_f<0x121>(out[q]);
    } else {
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_d<0x128>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_d<0x124>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_d<0x122>(out[q]);
#pragma unroll
        for (int q = 0; q < KC; ++q) out[q] += dpp_d<0x121>(out[q]);
    }
}

// First work unit of each row block: u(I, 0) = TB I (I + 1) / 2, TB tiles per row block.
__device__ __forceinline__ long long sym_unit0(int I)
{
    constexpr long long TB = kRowsPerBlock / kTile;
    return TB * (long long)I * (I + 1) / 2;
}

__device__ __forceinline__ int sym_row_block(long long u)
{
    constexpr double TB = kRowsPerBlock / kTile;
    int I = (int)((sqrt(8.0 * (double)u / TB + 1.0) - 1.0) * 0.5);
    while (sym_unit0(I + 1) <= u) ++I;
    while (sym_unit0(I) > u) --I;
    return I;
}

}  // namespace dev
}  // namespace hawkes
