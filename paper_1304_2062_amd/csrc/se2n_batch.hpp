// Batched inpainting: the device-side item table and the persistent pass
// kernels' launch interface (FP32).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"

namespace se2n {

// One image of a batch as the kernels see it.  Pointers are refreshed on the
// device whenever a call passes different buffers; the rest is fixed per
// batch plan.
struct BItem {
    const float* f;
    const uint8_t* mask;
    uint8_t* rmap;     // orientation map (caller's rmap_out or workspace)
    float* out;
    C2<float>* spec;   // half-spectrum volume [N][M/2+1][M] (workspace)
    C2<float>* blk;    // row-blocked second volume between the inverse passes
                       // (sides with batch_two_buf, else null; workspace)
    unsigned* enc;     // max-combining buffer [M][M] (workspace)
    const float* P;    // propagator table of (M, N, T, beta, n, scheme)
    const C2<float>* tw;  // quarter-wave twiddles of M
    int M, N, K, rows, cols, ocols, pcols, proj, groups, Q, FS;
    int imask;  // 1: the inverse column pass takes negligible modes as zero, and the solve stores none
    float ocoef, oscale;  // orientation: -2 pi^2 sigma^2 / M^2 and sqrt(M)/M^2
    FftPlan planH, planM;
};

// Passes of a batch, in launch order.
enum BatchKind {
    BK_ORIENT_ROW = 0,
    BK_ORIENT_COL,
    BK_ORIENT_INV,
    BK_LIFT_ROW,
    BK_COL_FWD,
    BK_SOLVE,
    BK_COL_INV,
    BK_FILL,
    BK_ROW_INV_MAX,
    BK_ROW_INV_MEAN,
    BK_DECODE,
    BK_ORIENT_STENCIL,  // one launch per (M, sigma): `cls` is the radius, the taps are arguments
    BK_COUNT
};

constexpr int kBatchThreads = 512;  // block size of the generic and elementwise batched kernels
constexpr int kBatchMaxM = 1024;    // largest M the batched kernels are built for

// Threads per block of a pass (the solve's depends on N).
int batch_threads(int kind, int N);
// Size classes of the batched row and column kernels: class c > 0 runs the
// bodies compiled for side kBatchSides[c] (with that side's own thread
// counts), class 0 the generic body for every other side.
constexpr int kBatchClasses = 8;
constexpr int kBatchSides[kBatchClasses] = {0, 128, 192, 256, 384, 512, 768, 1024};
inline int batch_class(int M) {
    for (int c = 1; c < kBatchClasses; ++c)
        if (kBatchSides[c] == M) return c;
    return 0;
}
// Sides whose batched row passes run their stages between two row buffers
// with the stage twiddles in registers (the single-image kernels' form); their
// row passes take a second row buffer of LDS.  The other classes keep one
// buffer: with the tile loop's state the second one makes them spill.
template <int MS>
constexpr bool kBatchTwoBuf = MS == 512 || MS == 1024;
inline bool batch_two_buf(int M) { return M == 512 || M == 1024; }
// Sides whose inverse passes go through a row-blocked second volume (as the
// single-image path does): the inverse column pass writes it, the inverse
// row pass reads it in 64-byte pieces of consecutive lines.
template <int MS>
constexpr bool kBatchBlocked = MS == 512 || MS == 768 || MS == 1024;
inline bool batch_blocked(int M) { return M == 512 || M == 768 || M == 1024; }
static_assert(512 % kRowBlk == 0 && 768 % kRowBlk == 0 && 1024 % kRowBlk == 0, "row blocks of the blocked sides");

// Launch one pass (size class `cls`, solve instance N): `grid` workgroups
// walk tiles[0..ntiles) with stride grid.
hipError_t launch_batch(int kind, int N, int cls, const BItem* items, const int4* tiles, int ntiles, int grid,
                        size_t lds, hipStream_t st, const OrientTaps* taps = nullptr);
// Resident workgroups per compute unit of a pass's kernel with `lds` bytes.
hipError_t batch_occupancy(int kind, int N, int cls, size_t lds, int* per_cu);

}  // namespace se2n
