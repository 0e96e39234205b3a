// Persistent batched kernels (FP32): every pass of the inpainting path as one
// launch over the tiles of many images.  A workgroup walks the pass's tile
// list with stride gridDim.x; a tile {item, a, b, c} names its image and the
// part of that image's work (row block and slice range, first column, class
// block, pixel range).  The image's twiddle table is expanded into LDS only
// when the previous tile of the workgroup belonged to an image of another
// table.  The tile bodies are the ones the single-image kernels run; images
// of side 512 and 1024 use the bodies compiled for those sizes.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_batch.hpp"
#include "se2n_fft.hpp"
#include "se2n_internal.hpp"
#include "se2n_orient.hpp"
#include "se2n_passes.hpp"

namespace se2n {

namespace {

constexpr int BT = kBatchThreads;

// Threads of the row and column kernels of a size class (MS = 0: generic).
template <int MS>
constexpr int row_nt() { return MS ? geom_core<float>(MS).row_threads : BT; }
template <int MS>
constexpr int col_nt() { return MS ? geom_core<float>(MS).col_threads : BT; }
template <int MS>
constexpr int pcol_nt() { return MS ? geom_core<float>(MS).pcol_threads : BT; }
static_assert(row_nt<1024>() <= BT && row_nt<768>() <= BT && row_nt<192>() <= BT && col_nt<192>() <= BT,
              "no batched kernel exceeds the launch bound");

using C = C2<float>;

// Rows per row tile of a compiled side (where its second row buffer starts).
template <int MS>
constexpr int kBatchRows = geom_core<float>(MS ? MS : 16).rows;

// The thread index, hidden from loop-invariant code motion: the tile bodies
// derive many per-thread addresses from it, and hoisting them out of the
// tile loop would keep all of them live across it.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ const BItem& item_of(const BItem* __restrict__ items, int idx) {
    return items[__builtin_amdgcn_readfirstlane(idx)];
}

// Expand the image's quarter table into LDS unless it is already there.
// Called right after a barrier, so no thread still reads the old table.
template <bool FULL>
__device__ __forceinline__ void ensure_twiddles(C* tw, const C* src, int M, const C*& cur, int nthr) {
    if (src != cur) {
        load_twiddles<float>(tw, src, M >> 2, FULL, threadIdx.x, nthr);
        cur = src;
    }
}

// Uniform copy of a value loaded from the item table (kept in scalar registers).
template <class T>
__device__ __forceinline__ T uni(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values only");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// The row and column kernels come in three size classes, each launched over
// the tiles of its own images: MS = 1024 and MS = 512 run the bodies compiled
// for that side, MS = 0 the generic body for every other side.
template <int SRC, int MS>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4))) void kb_row_fwd(const BItem* __restrict__ items, const int4* __restrict__ tiles,
                                                 int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C* tw = reinterpret_cast<C*>(smem_raw);
    const C* cur = nullptr;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        const int M = MS ? MS : uni(d.M);
        C* buf = tw + tw_elems(M, true);
        __syncthreads();
        ensure_twiddles<true>(tw, uni(d.tw), M, cur, row_nt<MS>());
        // (the 512 class keeps its twiddles in LDS: with the tile loop's
        // state, the register copy makes it spill)
        row_fwd_tile<float, SRC, 8, true, MS, kBatchTwoBuf<MS> && MS != 512>(
            uni(d.f), uni(d.mask), SRC == SRC_LIFT ? uni(d.rmap) : nullptr, nullptr, uni(d.spec), M, uni(d.rows), BT,
            tl.y, tl.z, tl.w, d.planH, tw, buf, opaque_tid(), kBatchTwoBuf<MS> ? buf + row_buf_elems(M, kBatchRows<MS>) : nullptr);
    }
}

template <bool INV, int MS>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4))) void kb_col_fft(const BItem* __restrict__ items, const int4* __restrict__ tiles,
                                                 int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C* tw = reinterpret_cast<C*>(smem_raw);
    const C* cur = nullptr;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        const int M = MS ? MS : uni(d.M);
        C* buf = tw + tw_elems(M, false);
        const long ncols = (long)uni(d.N) * (M / 2 + 1);
        __syncthreads();
        ensure_twiddles<false>(tw, uni(d.tw), M, cur, col_nt<MS>());
        // forward: the modes of the item's negligible classes are not stored
        // (its solve, the next pass, overwrites them unread)
        col_fft_tile<float, INV, 8, false, MS>(uni(d.spec), ncols, M, uni(d.cols), BT, tl.y, d.planM, tw, buf,
                                               opaque_tid(), INV ? nullptr : table_flags(uni(d.P), M, uni(d.N), 4),
                                               uni(d.FS));
    }
}

// Inverse column pass on column pairs with the pairing step of the real
// inverse row transform (tile = linear pair-block index within the image).
template <int MS>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4))) void kb_col_inv_paired(
    const BItem* __restrict__ items, const int4* __restrict__ tiles, int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C* tw = reinterpret_cast<C*>(smem_raw);
    const C* cur = nullptr;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        const int M = MS ? MS : uni(d.M);
        C* buf = tw + tw_elems(M, false);
        __syncthreads();
        ensure_twiddles<false>(tw, uni(d.tw), M, cur, pcol_nt<MS>());
        // the blocked sides write the row-blocked volume blk
        col_inv_paired_tile<float, 8, MS, false, NoPre, kBatchBlocked<MS>>(
            uni(d.spec), M, uni(d.pcols), BT, tl.y, d.planM, tw, buf, opaque_tid(), 0,
            uni(d.imask) ? table_flags(uni(d.P), M, uni(d.N), 4) : nullptr, uni(d.FS), NoPre{}, -1,
            kBatchBlocked<MS> ? uni(d.blk) : nullptr);
    }
}

__global__ __launch_bounds__(BT) void kb_col_orient(const BItem* __restrict__ items, const int4* __restrict__ tiles,
                                                    int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C* tw = reinterpret_cast<C*>(smem_raw);
    const C* cur = nullptr;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        const int M = uni(d.M);
        C* buf = tw + tw_elems(M, false);
        __syncthreads();
        ensure_twiddles<false>(tw, uni(d.tw), M, cur, BT);
        col_orient_tile<float, 8, false>(uni(d.spec), M, uni(d.ocols), BT, tl.y, d.planM, tw, buf, uni(d.ocoef),
                                         uni(d.oscale), opaque_tid());
    }
}

// Orientation stencil over the tiles of images that share (M, sigma), hence
// the taps.
template <int RAD>
__global__ __launch_bounds__(kOrientNT) void kb_orient_stencil(const BItem* __restrict__ items,
                                                               const int4* __restrict__ tiles, int ntiles,
                                                               OrientTaps taps) {
    __shared__ float sa[orient_lds_floats<RAD>()];
    __shared__ float sb[orient_lds_floats<RAD>()];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        __syncthreads();
        orient_stencil_tile<RAD>(uni(d.f), uni(d.mask), uni(d.rmap), uni(d.M), uni(d.N), tl.y, taps, sa, sb,
                                 opaque_tid());
    }
}

// Inverse row pass: orientation binning (DST_ORIENT), max projection
// (DST_MAX: written directly with one slice group, else combined through the
// item's atomic buffer) or mean projection (DST_SUM, one slice group).
template <int DST, int MS, bool PAIRED = false>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(4))) void kb_row_inv(const BItem* __restrict__ items, const int4* __restrict__ tiles,
                                                 int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    C* tw = reinterpret_cast<C*>(smem_raw);
    const C* cur = nullptr;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        const int M = MS ? MS : uni(d.M);
        const int N = uni(d.N);
        C* buf = tw + tw_elems(M, true);
        __syncthreads();
        ensure_twiddles<true>(tw, uni(d.tw), M, cur, row_nt<MS>());
        unsigned* enc = (DST == DST_MAX && uni(d.groups) > 1) ? uni(d.enc) : nullptr;
        const float sc = DST == DST_SUM ? 1.0f / (float)N : 1.0f;
        constexpr bool TWO = kBatchTwoBuf<MS> && PAIRED;
        constexpr bool BLK = kBatchBlocked<MS> && PAIRED;
        // the paired passes of the blocked sides read the row-blocked volume
        row_inv_tile<float, DST, 8, true, MS, PAIRED, BLK, TWO>(
            BLK ? uni(d.blk) : uni(d.spec), DST == DST_ORIENT ? nullptr : uni(d.out), enc,
            DST == DST_ORIENT ? uni(d.rmap) : nullptr, M,
            uni(d.rows), BT, tl.y, tl.z, tl.w, N, sc, d.planH, tw, buf, opaque_tid(),
            TWO ? buf + row_buf_elems(M, kBatchRows<MS>) : nullptr);
    }
}

// Clear (DECODE = false) or decode into the output (DECODE = true) the
// max-combining buffer over pixels [b, b + c) of an image.
template <bool DECODE>
__global__ __launch_bounds__(BT) void kb_enc(const BItem* __restrict__ items, const int4* __restrict__ tiles,
                                             int ntiles) {
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        unsigned* enc = uni(d.enc);
        float* out = uni(d.out);
        for (int e = threadIdx.x; e < tl.z; e += BT) {
            const long p = (long)tl.y + e;
            if (DECODE) out[p] = Enc<float>::decode(enc[p]);
            else enc[p] = 0u;
        }
    }
}

template <int N, int CLS, int WAVES>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WAVES))) void kb_solve(
    const BItem* __restrict__ items, const int4* __restrict__ tiles, int ntiles) {
    extern __shared__ unsigned char smem_raw[];
    float* Ps = reinterpret_cast<float*>(smem_raw);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int4 tl = tiles[t];
        const BItem& d = item_of(items, tl.x);
        __syncthreads();
        solve_tile<float, N, CLS>(uni(d.spec), uni(d.P), uni(d.M), uni(d.Q), uni(d.FS), tl.y, tl.z, Ps,
                                  opaque_tid(), uni(d.imask) == 0);
    }
}

template <int N>
struct SolveCfg {
    static constexpr int CLS = solve_cls<float, N>();
    static constexpr int WAVES = (N * 4) <= 160 ? 4 : 2;
    static constexpr int THREADS = 16 * CLS < 512 ? 16 * CLS : 512;
};

// Calls f(kernel pointer, threads) for the kernel of a pass; `cls` selects
// the size class of the row and column kernels (kBatchSides), N the solve
// instance.
#define SE2N_BY_CLASS(KT, NT)                                                          \
    switch (cls) {                                                                     \
        case 1: return f((const void*)KT(128), NT<128>());                             \
        case 2: return f((const void*)KT(192), NT<192>());                             \
        case 3: return f((const void*)KT(256), NT<256>());                             \
        case 4: return f((const void*)KT(384), NT<384>());                             \
        case 5: return f((const void*)KT(512), NT<512>());                             \
        case 6: return f((const void*)KT(768), NT<768>());                             \
        case 7: return f((const void*)KT(1024), NT<1024>());                           \
        default: return f((const void*)KT(0), NT<0>());                                \
    }
static_assert(kBatchClasses == 8 && kBatchSides[1] == 128 && kBatchSides[7] == 1024, "class table");

template <class F>
hipError_t with_kernel(int kind, int N, int cls, F&& f) {
    switch (kind) {
        case BK_ORIENT_ROW: {
#define K_(m) kb_row_fwd<SRC_IMAGE, m>
            SE2N_BY_CLASS(K_, row_nt)
#undef K_
        }
        case BK_LIFT_ROW: {
#define K_(m) kb_row_fwd<SRC_LIFT, m>
            SE2N_BY_CLASS(K_, row_nt)
#undef K_
        }
        case BK_ORIENT_COL: return f((const void*)kb_col_orient, BT);
        case BK_ORIENT_INV: {
#define K_(m) kb_row_inv<DST_ORIENT, m>
            SE2N_BY_CLASS(K_, row_nt)
#undef K_
        }
        case BK_ROW_INV_MAX: {
#define K_(m) kb_row_inv<DST_MAX, m, true>
            SE2N_BY_CLASS(K_, row_nt)
#undef K_
        }
        case BK_ROW_INV_MEAN: {
#define K_(m) kb_row_inv<DST_SUM, m, true>
            SE2N_BY_CLASS(K_, row_nt)
#undef K_
        }
        case BK_COL_FWD: {
#define K_(m) kb_col_fft<false, m>
            SE2N_BY_CLASS(K_, col_nt)
#undef K_
        }
        case BK_COL_INV: {
#define K_(m) kb_col_inv_paired<m>
            SE2N_BY_CLASS(K_, pcol_nt)
#undef K_
        }
        case BK_ORIENT_STENCIL:
            switch (cls) {
                case 8: return f((const void*)kb_orient_stencil<8>, kOrientNT);
                case 12: return f((const void*)kb_orient_stencil<12>, kOrientNT);
                case 16: return f((const void*)kb_orient_stencil<16>, kOrientNT);
                case 20: return f((const void*)kb_orient_stencil<20>, kOrientNT);
                case 24: return f((const void*)kb_orient_stencil<24>, kOrientNT);
                case 32: return f((const void*)kb_orient_stencil<32>, kOrientNT);
                default: return hipErrorInvalidValue;
            }
        case BK_FILL: return f((const void*)kb_enc<false>, BT);
        case BK_DECODE: return f((const void*)kb_enc<true>, BT);
        case BK_SOLVE:
            switch (N) {
#define SE2N_BCASE(n)                                                                                     \
    case n:                                                                                               \
        return f((const void*)kb_solve<n, SolveCfg<n>::CLS, SolveCfg<n>::WAVES>, SolveCfg<n>::THREADS);
                SE2N_BCASE(4) SE2N_BCASE(6) SE2N_BCASE(8) SE2N_BCASE(10) SE2N_BCASE(12) SE2N_BCASE(14)
                SE2N_BCASE(16) SE2N_BCASE(18) SE2N_BCASE(20) SE2N_BCASE(22) SE2N_BCASE(24) SE2N_BCASE(26)
                SE2N_BCASE(28) SE2N_BCASE(30) SE2N_BCASE(32) SE2N_BCASE(34) SE2N_BCASE(36) SE2N_BCASE(38)
                SE2N_BCASE(40) SE2N_BCASE(42) SE2N_BCASE(44) SE2N_BCASE(46) SE2N_BCASE(48) SE2N_BCASE(50)
                SE2N_BCASE(52) SE2N_BCASE(54) SE2N_BCASE(56) SE2N_BCASE(58) SE2N_BCASE(60) SE2N_BCASE(62)
                SE2N_BCASE(64)
#undef SE2N_BCASE
                default: return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
}
#undef SE2N_BY_CLASS

}  // namespace

int batch_threads(int kind, int N) {
    int threads = 0;
    (void)with_kernel(kind, N, 0, [&](const void*, int th) {
        threads = th;
        return hipSuccess;
    });
    return threads;
}

hipError_t launch_batch(int kind, int N, int cls, const BItem* items, const int4* tiles, int ntiles, int grid,
                        size_t lds, hipStream_t st, const OrientTaps* taps) {
    if (ntiles <= 0) return hipSuccess;
    if (kind == BK_ORIENT_STENCIL && !taps) return hipErrorInvalidValue;
    OrientTaps tv{};
    if (taps) tv = *taps;
    return with_kernel(kind, N, cls, [&](const void* fn, int threads) {
        void* args[] = {(void*)&items, (void*)&tiles, (void*)&ntiles, (void*)&tv};
        return hipLaunchKernel(fn, dim3((unsigned)grid), dim3((unsigned)threads), args, lds, st);
    });
}

hipError_t batch_occupancy(int kind, int N, int cls, size_t lds, int* per_cu) {
    return with_kernel(kind, N, cls, [&](const void* fn, int threads) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, threads, lds);
    });
}

}  // namespace se2n
