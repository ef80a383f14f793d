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

// How the pair terms are enumerated.
//   kDirect   : every ordered pair (i, j), as in the paper's Algorithm 3; column ranges of a row
//               block are split over blocks and each writes per-row partial sums.
//   kSymmetric: every unordered pair j < i once (lower triangle).  The background kernel B_ij and
//               its moments are symmetric, so one evaluation feeds both row i and row j; the
//               trigger term only ever feeds the later event i.  Work units are (row block I,
//               column tile t <= diagonal) in row-major order, dealt out in contiguous ranges
//               whose lengths differ by at most one to a grid of the device's resident blocks.
enum Scheme : int { kDirect = 0, kSymmetric = 1 };

// One evaluation's view of its dataset and scratch, passed by value in the kernel arguments.
struct PairReq {
    const float4* ev32;
    const double4* ev64;
    const int* cut;
    double* part;         // direct: [splits][K][npad]; symmetric: [blocks + row_blocks][K][kRowsPerBlock]
    double* colpart;      // symmetric: [KC][col_stride] column sums of row block I at RB*I(I+1)/2 + j
                          // (binary32 values in the FP32C pass)
    long long units;      // symmetric: work units walked, from ubegin on, of the
                          // row_blocks (row_blocks + 1) / 2 * (kRowsPerBlock / kTile) of the triangle
    long long ubegin;     // symmetric: first work unit walked
    long long col_stride; // symmetric: kRowsPerBlock * row_blocks (row_blocks + 1) / 2
    int n, npad;
    int row_blocks;       // npad / kRowsPerBlock
    int splits;           // direct: column ranges the j loop is cut into
    int tiles_per_split;  // direct: kTile-event tiles in each column range
    int ubase, urem;      // symmetric: block b walks ubase + (b < urem) units (even split)
    int item_begin;       // first work item (block) of this request in the launch
    int items;            // work items (blocks) of this request
    int balance;          // symmetric: 1 when the launch has the device to itself (progress priority)
    // Symmetric: the walk's dynamic tail (dev::walk_split): at most dchunks chunks taken from the
    // counter *ctr (zero when the pass starts; 0 chunks: a static split only).
    int dchunks;
    unsigned long long* ctr;
    // Zero-tile skipping (symmetric scheme; nullptr when off): zcum[I], I <= row_blocks, is the
    // number of walked units in the row blocks before I, followed by zskip[I] (int), the leading
    // column tiles of row block I that are not walked: every pair term there is exactly zero
    // because each of its events is at least zero_dt (time units of the data) after the tile's
    // last event.  Filled by the zero_prefix kernel.
    long long* zcum;
    double zero_dt;
    int zdirect;  // direct enumeration: walk only the column tiles within zero_dt of the row block
    // With zcum set, the FP32C pass also drops one kernel on far tiles at least zero_gap_b (every
    // background term zero) or zero_gap_e (every trigger term zero) time units before the rows.
    float zero_gap_b, zero_gap_e;
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
    const double* colpart;  // symmetric scheme only (binary32 values when colpart_f32)
    long long col_stride;
    int colpart_f32;
    double* rows_out;     // [n][kRowOut] in sorted order, or nullptr
    double* block_part;   // [nblocks][7]
    double* out7;         // 7 doubles: ell, gradient
    int n, npad, splits, grad;
    int scheme, row_blocks, ubase, urem;
    long long ubegin, uend;  // symmetric: work units the pairwise pass walked
    int add_diag;            // add the diagonal background term B_ii = 1
    double* sums_out;        // if set: write the six per-event sums [n][6] (sorted order) and stop
    const double* sums_in;   // if set: read the six per-event sums [n][6] instead of partials
    int nblocks;          // ceil(n / kThreads)
    int item_begin;
    int pair_items;          // blocks of the pairwise pass (symmetric: the walk's split)
    int dchunks;             // symmetric: the walk's dynamic tail, as in PairReq
    const long long* zcum;   // zero-tile skipping: as in PairReq, or nullptr
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

// Dynamic tail of the symmetric walk.  Run-time speed differs between compute units (the
// graphics clock of each XCD, the waves sharing a SIMD), so an even static split of the work units
// leaves some units idle at the end.  The last 1/kDynDiv of the walked units are cut into at most
// PairReq::dchunks contiguous chunks that blocks take from a counter once their own static range
// is done.  Each chunk writes its own row partial sums (slot items + row_blocks + c + I for chunk c
// and row block I; a static range b writes slot b + I), so which block runs a chunk changes neither
// the arithmetic nor the summation order, and the result stays deterministic.
constexpr long long kDynDiv = 8;
constexpr long long kDynMinUnitsPerBlock = 4;  // smaller walks keep the static split only
constexpr int kDynChunksPerBlock = 32;         // the host plan's cap on dchunks, per block

struct WalkSplit {
    long long sunits;       // walk positions [0, sunits) are dealt statically: block b walks
    long long sbase, srem;  // [b sbase + min(b, srem), (b + 1) sbase + min(b + 1, srem))
    long long chunks;       // positions [sunits, units) in `chunks` chunks, split the same way
    long long cbase, crem;
};

__host__ __device__ inline WalkSplit walk_split(long long units, int items, int dchunks)
{
    WalkSplit w = {0, 0, 0, 0, 0, 0};
    if (items <= 0 || units <= 0) return w;
    long long d = (dchunks > 0 && units >= kDynMinUnitsPerBlock * items) ? units / kDynDiv : 0;
    const long long ch = d < (long long)dchunks ? d : (long long)dchunks;
    if (ch <= 0) d = 0;
    w.sunits = units - d;
    w.sbase = w.sunits / items;
    w.srem = w.sunits % items;
    if (ch > 0) {
        w.chunks = ch;
        w.cbase = d / ch;
        w.crem = d % ch;
    }
    return w;
}

// Kernel arguments are passed by value; keep them within 4 KiB.
static_assert(sizeof(PairBatch) <= 4096 && sizeof(EpiBatch) <= 4096, "kernel argument block too large");

// The leading column tiles of each row block that zero-tile skipping leaves out (see PairReq).
__host__ __device__ inline int* zero_skip_tiles(long long* zcum, int row_blocks) { return (int*)(zcum + row_blocks + 1); }
__host__ __device__ inline const int* zero_skip_tiles(const long long* zcum, int row_blocks)
{
    return (const int*)(zcum + row_blocks + 1);
}

// Kernel launchers (hawkes_kernels.hip).  Each returns the launch's hipError_t.
// zskip: the requests use zero-tile skipping (PairReq::zcum set), served by its own variant of the
// symmetric kernels.
hipError_t launch_pair(const PairBatch& b, int precision, bool grad, int scheme, bool zskip, hipStream_t s);
// Zero-tile skipping tables (zcum, zskip) of the requests that use it; one block per request.
hipError_t launch_zero_prefix(const PairBatch& b, hipStream_t s);
// Resident blocks per CU of the symmetric pairwise kernel (for sizing its grid).
int sym_blocks_per_cu(int precision, bool grad);
hipError_t launch_epilogue(const EpiBatch& b, hipStream_t s);
hipError_t launch_final(const EpiBatch& b, hipStream_t s);

}  // namespace hawkes
