// hawkes_internal.h -- types shared by the host runtime and the gfx950 kernels of libhawkes.
//
// Device layout of one dataset (events sorted by (t, input index), padded to a multiple of
// kPad with sentinel events that contribute exactly zero):
//   ev32[2*i], ev32[2*i+1] : float4 (x_hi, y_hi, t_hi, 0), float4 (x_lo, y_lo, t_lo, 0) where
//                            v_hi = fl32(v - c), v_lo = fl32((v - c) - v_hi), c = centring offset
//   ev64[i]                : double4 (x, y, t, 0), the caller's values unchanged
//   cut[i]                 : #{j : t_j < t_i} -- the events j < cut[i] are exactly the causal ones
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hawkes {

constexpr int kThreads = 256;          // threads per block of every kernel (4 waves of 64)
constexpr int kTile = 256;             // events per LDS tile of the pairwise pass
constexpr int kRowsPerLane = 4;        // rows held in registers by each lane
constexpr int kRowsPerBlock = kThreads * kRowsPerLane;  // 1024
constexpr int kPad = kRowsPerBlock;    // event arrays are padded to a multiple of this
constexpr int kMaxBatch = 16;          // requests per batched launch
constexpr int kMaxSplits = 32;         // column (j) splits of one evaluation
constexpr int kRowOut = 10;            // doubles per event in per-row output
// Sentinel padding event: so far away that every background term underflows to exactly 0 while
// r^2 stays finite in binary32 (2 * (1e18)^2 < FLT_MAX); it is never causal (index >= n).
constexpr double kSentinel = 1.0e18;

enum Precision : int { kFP64 = 0, kFP32C = 1 };

// One evaluation's view of its dataset and scratch, passed by value in the kernel arguments.
struct PairReq {
    const float4* ev32;
    const double4* ev64;
    const int* cut;
    double* part;         // [splits][K][npad] per-row partial sums, K = 6 (grad) or 2
    int n, npad;
    int row_blocks;       // npad / kRowsPerBlock
    int splits;           // column ranges the j loop is cut into
    int tiles_per_split;  // kTile-event tiles in each column range
    int item_begin;       // first work item (block) of this request in the launch
    // Negated base-2 exponent coefficients: B = 2^(nab r^2 + nbb dt^2), E = 2^(nae r^2 + nbe dt).
    // The FP32C pass works in scaled time dt' = ts dt with ts = tsh + tsl = sqrt(-nbb):
    // B = 2^(nab r^2 - dt'^2), E = 2^(nae r^2 + kte dt') with kte = nbe / ts.
    float nab, nae, tsh, tsl, kte;
    double nab64, nbb64, nae64, nbe64;
};

struct PairBatch {
    PairReq r[kMaxBatch];
    int nreq;
    int total_items;
};

struct EpiReq {
    const double4* ev64;
    const double* part;
    double* rows_out;     // [n][kRowOut] in sorted order, or nullptr
    double* block_part;   // [nblocks][7]
    double* out7;         // 7 doubles: ell, gradient
    int n, npad, splits, grad;
    int nblocks;          // ceil(n / kThreads)
    int item_begin;
    double T;             // largest event time
    double mu0, tau_x, tau_t, theta, omega, h;
    double cb, ce;        // background and trigger coefficients
    double t_scale;       // time scale of the dt-moments in the partial sums (1 for FP64)
};

struct EpiBatch {
    EpiReq r[kMaxBatch];
    int nreq;
    int total_items;
};

// Kernel launchers (hawkes_kernels.hip).  Each returns the launch's hipError_t.
hipError_t launch_pair(const PairBatch& b, int precision, bool grad, hipStream_t s);
hipError_t launch_epilogue(const EpiBatch& b, hipStream_t s);
hipError_t launch_final(const EpiBatch& b, hipStream_t s);

}  // namespace hawkes
