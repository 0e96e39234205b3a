// Workgroup-level bodies of the passes of one diffusion, shared by the
// single-image kernels (one workgroup per tile, tile from blockIdx) and the
// batched persistent kernels (each workgroup walks a list of tiles of many
// images).  A body receives its tile, the image's sizes and the LDS twiddle
// table already loaded; it leaves LDS free for the next tile only after the
// caller's next barrier.
//
// Spectral layout (see the kernels file): spec[r][kx][ky], kx in [0, M/2],
// ky in [0, M) contiguous.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"

namespace se2n {

// Maximum of two values.  FP32 takes the IEEE maximum (one instruction; a
// NaN propagates); fmax would first quieten its loop-carried operand on
// every call.
template <class R>
__device__ __forceinline__ R vmax(R a, R b) {
    if constexpr (sizeof(R) == 4) return __builtin_elementwise_maximum(a, b);
    else return fmax(a, b);
}

// (q, r) = divmod(tid + i*nthr, d) without a per-element division when nthr
// is a multiple of d or d of nthr (uniform branches); inv_d = 1/d in float.
__device__ __forceinline__ void split_index(int tid, int i, int nthr, int d, float inv_d, int& q, int& r) {
    if (nthr % d == 0) {
        const int qt = tid / d;
        q = qt + i * (nthr / d);
        r = tid - qt * d;
    } else if (d % nthr == 0) {
        const int b = tid + i * nthr;
        const int per = d / nthr;
        q = i / per;
        r = b - q * d;
    } else {
        const int b = tid + i * nthr;
        q = fdiv(b, inv_d);
        r = b - q * d;
    }
}

// ---------------------------------------------------------------------------
// Row pass, forward: lift + R2C along x of `rows` image rows starting at
// y0 = rb*rows, for slices [s_begin, s_end), written transposed.
// ---------------------------------------------------------------------------
// A real row x[0..M) is transformed as the half-length complex sequence
// z[n] = x[2n] + i x[2n+1]:  with Z = FFT_H(z), H = M/2,
//   X[k] = (Z[k] + conj Z[H-k])/2 + w_M^k (Z[k] - conj Z[H-k])/(2i),  k = 0..H.
// MS != 0: compiled for M = MS with the geometry geom_core<R>(MS).
// TWC: the fixed-size two-buffer stages keep their twiddles in registers
// (StageTw), read once per tile (the caller has put the table in LDS).
template <class R, int SRC, int EPT, bool TWF, int MS, bool TWC = false>
__device__ __forceinline__ void row_fwd_tile(const R* __restrict__ f, const uint8_t* __restrict__ mask,
                                             const uint8_t* __restrict__ rmap, const R* __restrict__ vol,
                                             C2<R>* __restrict__ spec, int M_, int rows_, int nthr_, int rb,
                                             int s_begin, int s_end, const FftPlan& planH, const C2<R>* tw,
                                             C2<R>* buf, int tid, C2<R>* buf2 = nullptr) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    const int nthr = MS ? GC.row_threads : nthr_;
    const int M4 = M >> 2;
    const int H = M >> 1;
    const int K = H + 1;
    const int S = H + 2;  // LDS row stride: 8 rows of the transposed phase fall in distinct banks
    const int y0 = rb * rows;
    const int nel = rows * H;
    const float inv_H = 1.0f / (float)H;

    // Lift sources are read once per tile and kept in registers: element i
    // of the thread is (row, pixel pair n) of its first-stage butterfly inputs
    // (fixed-size transforms, which take them from registers) or of the
    // natural order e = tid + i*nthr (else).
    // registers per thread: EPT, or the first stage's input slots if more
    constexpr int NIN = MS != 0 && static_in_slots(MS ? MS / 2 : 8, GC.rows, GC.row_threads) > EPT
                            ? static_in_slots(MS ? MS / 2 : 8, GC.rows, GC.row_threads)
                            : EPT;
    auto elem = [&](int i, int& row, int& n) {
        if constexpr (MS != 0) {
            return static_in_pos<MS / 2, GC.rows, GC.row_threads>(tid, i, row, n);
        } else {
            split_index(tid, i, nthr, H, inv_H, row, n);
            return tid + i * nthr < nel;
        }
    };
    R fc0[NIN], fc1[NIN];
    uint8_t rm0[NIN], rm1[NIN];
    if (SRC != SRC_VOLUME) {
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            fc0[i] = R(0);
            fc1[i] = R(0);
            rm0[i] = 0xff;
            rm1[i] = 0xff;
            int row, n;
            if (elem(i, row, n)) {
                const size_t p = (size_t)(y0 + row) * M + 2 * n;
                const C2<R> fv = *reinterpret_cast<const C2<R>*>(f + p);
                const uint16_t mv = *reinterpret_cast<const uint16_t*>(mask + p);
                fc0[i] = (mv & 0xff) ? R(0) : fv.x;
                fc1[i] = (mv >> 8) ? R(0) : fv.y;
                if (SRC == SRC_LIFT) {
                    const uint16_t rv = *reinterpret_cast<const uint16_t*>(rmap + p);
                    rm0[i] = (uint8_t)(rv & 0xff);
                    rm1[i] = (uint8_t)(rv >> 8);
                }
            }
        }
    }

    // Fixed-size transforms with a second buffer (buf2) run their stages
    // between the two; bx is the buffer the next first stage may fill.
    const bool pp = MS != 0 && buf2 != nullptr;
    C2<R>* bx = buf;
    C2<R>* by = buf2;
    using TwC = StageTw<R, false, TWF, MS ? MS / 2 : 8, GC.rows, GC.row_threads, MS ? MS : 16,
                        MS != 0 && TWC ? static_nstages(MS ? MS / 2 : 8) : 1>;
    TwC twc;
    if constexpr (MS != 0 && TWC) {
        __syncthreads();  // the twiddle table is in LDS
        twc.load(tw, tid);
    }
    for (int s = s_begin; s < s_end; ++s) {
        // input element i of this slice (zero where unused)
        auto input = [&](int i) {
            C2<R> z = cmk<R>(R(0), R(0));
            int row, n;
            if (elem(i, row, n)) {
                if (SRC == SRC_VOLUME) {
                    z = *reinterpret_cast<const C2<R>*>(vol + ((size_t)s * M + y0 + row) * M + 2 * n);
                } else if (SRC == SRC_LIFT) {
                    z.x = (rm0[i] == s) ? fc0[i] : R(0);
                    z.y = (rm1[i] == s) ? fc1[i] : R(0);
                } else {
                    z.x = fc0[i];
                    z.y = fc1[i];
                }
            }
            return z;
        };
        C2<R>* res = buf;
        if constexpr (MS != 0) {
            if (pp) {
                if constexpr (TWC)
                    res = fft_static_in_pp<R, false, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(
                        bx, by, tw, tid, input, twc);
                else
                    res = fft_static_in_pp<R, false, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(
                        bx, by, tw, tid, input);
            }
            else
                fft_static_in<R, false, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(buf, tw, tid, input);
        } else {
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                int row, n;
                if (elem(i, row, n)) buf[lds_pad(row * S + n)] = input(i);
            }
            __syncthreads();
            fft_lds<R, false, EPT, TWF>(buf, planH, rows, S, tw, M4, tid, nthr);
        }
        // Unpack the real transform and write (r, kx, y0..y0+rows) segments.
        // One unit (row, k), k = 0 .. H/2, gives two outputs from a = Z[k] and
        // b = Z[(H - k) mod H] and one twiddle (w_M^{H-k} = -conj w_M^k):
        //   s = a + conj b,  u = w_M^k (a - conj b) / 2,
        //   X[k] = s/2 - i u,  X[H - k] = conj(s/2 + i u)
        // (k = 0 gives X[0] and X[H]; k = H/2 gives X[H/2] once).  On the
        // compiled sides a lane takes two adjacent rows of a column, so four
        // lanes write one 64-byte segment; the generic loop takes unit e as
        // (row e mod rows, k = e / rows).
        C2<R>* out = spec + (size_t)s * K * M + y0;
        const int H2 = H >> 1;
        const int rshift = __ffs(rows) - 1;  // rows is a power of two
        auto pair_out = [&](C2<R> a, C2<R> b, C2<R> w, C2<R>& xk, C2<R>& xh) {
            const R sx = a.x + b.x, sy = a.y - b.y;
            const R dx = R(0.5) * (a.x - b.x), dy = R(0.5) * (a.y + b.y);
            const R ux = w.x * dx - w.y * dy, uy = w.x * dy + w.y * dx;
            xk = cmk<R>(R(0.5) * sx + uy, R(0.5) * sy - ux);
            xh = cmk<R>(R(0.5) * sx - uy, R(-0.5) * sy - ux);
        };
        // twiddles w_M^k, k <= M/4, are in the quarter table as well
        constexpr int KSTEP = MS != 0 ? GC.row_threads / GC.rows : 1;
        constexpr bool LINU = MS != 0 && GC.row_threads % GC.rows == 0 && KSTEP % kLdsPadPeriod == 0 &&
                              KSTEP % (1 << SE2N_TW_PAD_SHIFT) == 0;
        // row pairs: a lane takes rows 2p and 2p + 1 of its columns, whose
        // outputs are adjacent, so it writes them with one 16-byte store
        // and reads one twiddle for both
        constexpr int NRP = MS != 0 ? GC.rows / 2 : 1;
        constexpr int KSTEP2 = MS != 0 ? GC.row_threads / NRP : 1;
        constexpr bool PAIRS = LINU && sizeof(R) == 4 && GC.rows % 2 == 0 &&
                               GC.row_threads % NRP == 0 && KSTEP2 % kLdsPadPeriod == 0 &&
                               KSTEP2 % (1 << SE2N_TW_PAD_SHIFT) == 0;
        if constexpr (PAIRS) {
            typedef R v4_t __attribute__((ext_vector_type(4)));
            constexpr int NU = NRP * (MS / 4 + 1);
            constexpr int FULLIT = NU / GC.row_threads;
            constexpr int LSTEP = KSTEP2 + KSTEP2 / kLdsPadPeriod;
            constexpr int TSTEP = KSTEP2 + (KSTEP2 >> SE2N_TW_PAD_SHIFT);
            const int rp = tid & (NRP - 1);
            const int k0 = tid / NRP;
            const int r0 = 2 * rp;
            const C2<R>* pa0 = res + lds_pad(r0 * S + k0);
            const C2<R>* pa1 = res + lds_pad((r0 + 1) * S + k0);
            const C2<R>* pb0 = res + lds_pad(r0 * S + H - k0);
            const C2<R>* pb1 = res + lds_pad((r0 + 1) * S + H - k0);
            const C2<R>* pz0 = k0 == 0 ? pa0 : pb0;  // Z[H] is Z[0]
            const C2<R>* pz1 = k0 == 0 ? pa1 : pb1;
            const C2<R>* pw = tw + tw_pos(k0);
            v4_t* ok = reinterpret_cast<v4_t*>(out + (size_t)k0 * MS + r0);
            v4_t* oh = reinterpret_cast<v4_t*>(out + (size_t)(H - k0) * MS + r0);
            constexpr long LB = (long)KSTEP2 * MS / 2;  // 16-byte units between a thread's output lines
            auto unit = [&](int it, bool both) {
                const C2<R> w = pw[it * TSTEP];
                C2<R> xk0, xh0, xk1, xh1;
                pair_out(pa0[it * LSTEP], it == 0 ? pz0[0] : pb0[-it * LSTEP], w, xk0, xh0);
                pair_out(pa1[it * LSTEP], it == 0 ? pz1[0] : pb1[-it * LSTEP], w, xk1, xh1);
                v4_t a, b;
                a.x = xk0.x; a.y = xk0.y; a.z = xk1.x; a.w = xk1.y;
                b.x = xh0.x; b.y = xh0.y; b.z = xh1.x; b.w = xh1.y;
                ok[it * LB] = a;
                if (both) oh[-it * LB] = b;
            };
#pragma unroll
            for (int it = 0; it < FULLIT; ++it) unit(it, true);
            if (tid + FULLIT * GC.row_threads < NU) {
                // k = k0 + FULLIT KSTEP2 <= H/2; the unit k = H/2 writes X[H/2] once
                unit(FULLIT, k0 + FULLIT * KSTEP2 != H2);
            }
        } else {
            for (int e = tid; e < rows * (H2 + 1); e += nthr) {
                const int k = e >> rshift;
                const int row = e & (rows - 1);
                const C2<R> a = res[lds_pad(row * S + k)];
                const C2<R> b = res[lds_pad(row * S + (k == 0 ? 0 : H - k))];
                C2<R> xk, xh;
                pair_out(a, b, tw[tw_pos(k)], xk, xh);
                out[(size_t)k * M + row] = xk;
                if (k != H2) out[(size_t)(H - k) * M + row] = xh;
            }
        }
        if (pp) {
            // the next first stage fills the buffer nobody reads any more
            by = res;
            bx = (res == buf) ? buf2 : buf;
        } else {
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Column pass: FFT along y of the columns [c0, c0 + ncb) (each M contiguous
// values), ncb = min(cols_per_tile, ncols - c0).
// ---------------------------------------------------------------------------
// With `negf` set (the negligible-class flags of the propagator table that
// the solve applies next, rows of FS bytes), the modes of negligible classes
// are not stored: the solve overwrites each of them with zero without reading
// it, and lines that hold no live mode never reach HBM.  Columns are
// c = r * (M/2 + 1) + kx; mode (kx, ky) belongs to class (fold kx, fold ky).
// This applies to full tiles of the compiled sizes whose thread count nthr
// divides M and either divides M/2 or is a multiple of it.  Thread tid then
// stores, in column q, the rows ky = tid + k nthr (k < M / nthr); the class
// index of a row depends only on u = ky mod M/2 (it is u for u <= M/4, else
// M/2 - u), and u takes U = max(1, M / (2 nthr)) values per column, so a
// thread needs U flags per column of its tile.  A per-element fold costs more
// VALU than the skipped stores save.
template <class R, int MS>
struct ColSkip {
    static constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    static constexpr int NT = GC.col_threads;
    static constexpr int H = MS / 2;
    static constexpr bool ok = col_skip_shape(MS, NT);
    static constexpr int CPT = ok ? MS / NT : 1;           // chunks of nthr rows per column
    static constexpr int U = ok && NT <= H ? H / NT : 1;   // values of ky mod M/2 per column
    static constexpr int EPT = GC.cols * CPT;              // elements a thread stores
    static_assert(!ok || EPT <= 16, "flags per thread");
};

// `pre` runs once before the tile's first LDS write, after its own global
// loads are issued (callers fetch the twiddles there, overlapping the two).
struct NoPre {
    __device__ void operator()() const {}
};

template <class R, bool INV, int EPT, bool TWF, int MS, class Pre = NoPre>
__device__ __forceinline__ void col_fft_tile(C2<R>* __restrict__ spec, long ncols, int M_, int cols_,
                                             int nthr_, long c0, const FftPlan& planM, const C2<R>* tw,
                                             C2<R>* buf, int tid, const uint8_t* __restrict__ negf = nullptr,
                                             int FS = 0, Pre pre = Pre{}) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int cols_per_tile = MS ? GC.cols : cols_;
    const int nthr = MS ? GC.col_threads : nthr_;
    const int M4 = M >> 2;
    const int ncb = (int)min((long)cols_per_tile, ncols - c0);
    const int nel = ncb * M;
    C2<R>* base = spec + c0 * M;
    using CS_ = ColSkip<R, MS>;
    // negligible flag of the element tid + j * nthr: loaded ahead of the
    // tile, used only by the stores after the transform, so their latency
    // hides behind it
    const bool skip = CS_::ok && negf != nullptr && ncb == cols_per_tile;
    uint8_t fb[CS_::ok ? CS_::EPT : 1];
    if constexpr (CS_::ok) {
        if (skip) {
            constexpr int H = CS_::H;
#pragma unroll
            for (int q = 0; q < GC.cols; ++q) {
                const int kx = ((int)c0 + q) % (H + 1);
                const uint8_t* row = negf + (size_t)(kx <= M4 ? kx : H - kx) * FS;
                uint8_t fu[CS_::U];
#pragma unroll
                for (int v = 0; v < CS_::U; ++v) {
                    const int u = (tid + v * CS_::NT) % H;
                    fu[v] = row[u <= M4 ? u : H - u];
                }
#pragma unroll
                for (int k = 0; k < CS_::CPT; ++k) fb[q * CS_::CPT + k] = fu[k % CS_::U];
            }
        }
    }
    // full tiles of a compiled size: element tid + i nthr sits at
    // lds_pad(tid) + i (nthr + nthr/32) when nthr is a multiple of the
    // padding period, so one base and immediate offsets serve every element
    constexpr bool LINT = MS != 0 && GC.col_threads % kLdsPadPeriod == 0 && (GC.cols * MS) % GC.col_threads == 0;
    constexpr int LEPT = LINT ? GC.cols * MS / GC.col_threads : 1;
    constexpr int LSTEP = GC.col_threads + GC.col_threads / kLdsPadPeriod;
    if (LINT && ncb == cols_per_tile) {
        const C2<R>* gb = base + tid;
        C2<R> v[LEPT];
#pragma unroll
        for (int i = 0; i < LEPT; ++i) v[i] = gb[i * GC.col_threads];
        pre();
        C2<R>* lb = buf + lds_pad(tid);
#pragma unroll
        for (int i = 0; i < LEPT; ++i) lb[i * LSTEP] = v[i];
    } else {
        pre();
        for (int e = tid; e < nel; e += nthr) buf[lds_pad(e)] = base[e];
    }
    __syncthreads();
    if constexpr (MS != 0) {
        if (ncb == GC.cols) fft_static<R, INV, TWF, MS, GC.cols, MS, GC.col_threads, MS>(buf, tw, tid);
        else fft_lds<R, INV, EPT, TWF>(buf, planM, ncb, M, tw, M4, tid, nthr);
    } else {
        fft_lds<R, INV, EPT, TWF>(buf, planM, ncb, M, tw, M4, tid, nthr);
    }
    if constexpr (CS_::ok) {
        if (skip) {
            // a wavefront stores 64 consecutive elements; a line is skipped only
            // when none of its modes is live (a partly written line still
            // reaches HBM)
            constexpr int LPL = 128 / (int)sizeof(C2<R>);  // lanes per 128-byte line
            constexpr unsigned long long LMASK = (1ull << LPL) - 1;
            const int lane = tid & 63;
            static_assert(!CS_::ok || (LINT && CS_::EPT == LEPT), "skip tiles are linear tiles");
            const C2<R>* lb = buf + lds_pad(tid);
            C2<R>* gb = base + tid;
#pragma unroll
            for (int j = 0; j < CS_::EPT; ++j) {
                const unsigned long long live = __ballot(!fb[j]);
                if ((live >> (lane & ~(LPL - 1))) & LMASK) gb[j * GC.col_threads] = lb[j * LSTEP];
            }
            return;
        }
    }
    if (LINT && ncb == cols_per_tile) {
        const C2<R>* lb = buf + lds_pad(tid);
        C2<R>* gb = base + tid;
#pragma unroll
        for (int i = 0; i < LEPT; ++i) gb[i * GC.col_threads] = lb[i * LSTEP];
        return;
    }
    for (int e = tid; e < nel; e += nthr) base[e] = buf[lds_pad(e)];
}

// The paired inverse tile holds the pairs (k, M/2 - k), k = p0 .. p0+P-1:
// both columns of a pair belong to class row fold(k), and the rows a thread
// loads meet the same U values of ky mod M/2 as above.
template <class R, int MS>
struct ColInvSkip {
    static constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    static constexpr int NT = GC.pcol_threads;
    static constexpr int H = MS / 2;
    static constexpr int P = GC.pcols / 2;
    static constexpr bool ok = col_skip_shape(MS, NT);
    static constexpr int CPT = ok ? MS / NT : 1;
    static constexpr int U = ok && NT <= H ? H / NT : 1;
    static constexpr int EPT = 2 * P * CPT;
    static_assert(!ok || EPT <= 16, "flags per thread");
};

// Class index of ky (or kx) for a side M: ky for ky <= M/4, folded back from
// M/2 and M otherwise.
__device__ __forceinline__ int fold_class(int k, int M) {
    const int H = M >> 1, M4 = M >> 2;
    return k <= M4 ? k : (k <= H ? H - k : (k <= H + M4 ? k - H : M - k));
}

// ---------------------------------------------------------------------------
// Inverse column pass on column pairs, then the pairing step of the real
// inverse row transform.  Tile `tile` of slice r = tile / tiles_per_slice
// holds the pairs (k, H-k), k = p0 .. p0+np-1 of that slice (H = M/2, pairs
// k = 0 .. H/2).  After the inverse FFT along y of both columns, for every y
//   Z[k]   = (X[k] + conj X[H-k]) + i w_M^{-k} (X[k] - conj X[H-k]),
//   Z[H-k] = (X[H-k] + conj X[k]) + i w_M^{-(H-k)} (X[H-k] - conj X[k])
// overwrite columns k and H-k (column H is left alone: the row pass reads
// Z[0 .. H-1] only).  The inverse FFT_H of Z along x is then M (x[2n] + i x[2n+1]).
// ---------------------------------------------------------------------------
//
// With `negf` set (the flags of the propagators the solve applied), the modes
// of negligible classes are taken as zero and not read: the solve then need
// not store them, and lines that hold no live mode are never fetched.
//
// tile2 >= 0 (same pair block as `tile`; the caller requests it only where
// every tile takes the flag-reading fast path): the workgroup also
// transforms that tile, reusing the flags and twiddles and holding its input
// in registers while the first tile is transformed.
//
// BLK: the result goes to `blk` (same slice stride as spec) in the
// row-blocked layout (row_blk_index) instead of back into the tile's columns.
template <class R, int EPT, int MS, bool HINTS = false, class Pre = NoPre, bool BLK = false>
__device__ __forceinline__ void col_inv_paired_tile(C2<R>* __restrict__ spec, int M_, int pcols_, int nthr_,
                                                    int tile, const FftPlan& planM, const C2<R>* tw, C2<R>* buf,
                                                    int tid, int nslices = 0,
                                                    const uint8_t* __restrict__ negf = nullptr, int FS = 0,
                                                    Pre pre = Pre{}, int tile2 = -1,
                                                    C2<R>* __restrict__ blk = nullptr) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int pc = MS ? GC.pcols : pcols_;
    const int nthr = MS ? GC.pcol_threads : nthr_;
    const int H = M >> 1;
    const int K = H + 1;
    const int M4 = M >> 2;
    const int P = pc >> 1;
    const int npair = H / 2 + 1;
    const int tps = (npair + P - 1) / P;
    const int r = tile / tps;
    const int p0 = (tile - r * tps) * P;
    const int np = min(P, npair - p0);
    C2<R>* base = spec + (size_t)r * K * M;
    const int r2 = tile2 >= 0 ? tile2 / tps : r;
    C2<R>* const base2 = spec + (size_t)r2 * K * M;
    // where output (column k, row y) of the current tile goes
    C2<R>* obase = BLK ? blk + (size_t)r * K * M : base;
    auto dst = [&](int k, int y) {
        if constexpr (BLK) return obase + row_blk_index(k, y, H);
        else return obase + (size_t)k * M + y;
    };
    const float inv_M = 1.0f / (float)M;
    const int nel = 2 * np * M;
    // LDS column q < np holds column k = p0 + q, column np + q its partner
    // H - k: the tile reads two contiguous runs, columns p0 .. p0+np-1 and
    // H-p0-np+1 .. H-p0 (the self-paired column M/4 is read twice).
    const int half = np * M;
    const int c2 = H - p0 - np + 1;
    // With HINTS (single-image pass, nslices slices): the input is read
    // non-temporally (its last use), and the slices below nslices/2, which
    // the inverse row pass reaches last (it walks slices downwards), are
    // stored non-temporally, which leaves the memory-side cache to the rest.
    typedef R v2_t __attribute__((ext_vector_type(2)));
    auto ld = [&](const C2<R>* p) {
        if constexpr (HINTS) {
            const v2_t v = __builtin_nontemporal_load(reinterpret_cast<const v2_t*>(p));
            return cmk<R>(v.x, v.y);
        } else {
            return *p;
        }
    };
    bool nts = HINTS && 2 * r < nslices;
    auto st = [&](C2<R>* p, C2<R> v) {
        if (nts) {
            v2_t w;
            w.x = v.x;
            w.y = v.y;
            __builtin_nontemporal_store(w, reinterpret_cast<v2_t*>(p));
        } else {
            *p = v;
        }
    };
    // transform the tile in LDS and store its pairs (the input is in LDS)
    auto finish = [&]() {
        __syncthreads();
        if constexpr (MS != 0) {
            if (np == P) fft_static<R, true, false, MS, GC.pcols, MS, GC.pcol_threads, MS>(buf, tw, tid);
            else fft_lds<R, true, EPT, false>(buf, planM, 2 * np, M, tw, M4, tid, nthr);
        } else {
            fft_lds<R, true, EPT, false>(buf, planM, 2 * np, M, tw, M4, tid, nthr);
        }
        if constexpr (MS != 0 && GC.pcol_threads <= MS && MS % GC.pcol_threads == 0) {
            if (np == P) {
                // full tile of a compiled size: element tid + i nthr lies in pair
                // i nthr / M, a constant of the unrolled loop, so each thread
                // reads the two twiddles of each pair once
                constexpr int NTc = GC.pcol_threads;
                constexpr int PP = GC.pcols / 2;
                C2<R> wk[PP], wkk[PP];
    #pragma unroll
                for (int q = 0; q < PP; ++q) {
                    wk[q] = cconj<R>(tw_get<R, false>(tw, p0 + q, M4));
                    wkk[q] = cconj<R>(tw_get<R, false>(tw, H - p0 - q, M4));
                }
    #pragma unroll
                for (int i = 0; i < PP * MS / NTc; ++i) {
                    const int q = i * NTc / MS;
                    const int y = i * NTc - q * MS + tid;
                    const int k = p0 + q;
                    const int kk = H - k;
                    const C2<R>* lb = buf + lds_pad(tid);  // slot of q M + y is lds_pad(tid) + pad_offset(1, i nthr)
                    const C2<R> a = lb[pad_offset(1, i * NTc)];
                    const C2<R> b = lb[pad_offset(1, PP * MS + i * NTc)];
                    const C2<R> sa = cmk<R>(a.x + b.x, a.y - b.y);  // a + conj b
                    const C2<R> da = cmk<R>(a.x - b.x, a.y + b.y);  // a - conj b
                    const C2<R> ta = cmul<R>(wk[q], da);
                    st(dst(k, y), cmk<R>(sa.x - ta.y, sa.y + ta.x));  // sa + i ta
                    if (k != 0 && kk != k) {
                        const C2<R> sb = cmk<R>(b.x + a.x, b.y - a.y);
                        const C2<R> db = cmk<R>(b.x - a.x, b.y + a.y);
                        const C2<R> tb = cmul<R>(wkk[q], db);
                        st(dst(kk, y), cmk<R>(sb.x - tb.y, sb.y + tb.x));
                    }
                }
                return;
            }
        }
        for (int e = tid; e < np * M; e += nthr) {
            const int q = fdiv(e, inv_M);
            const int y = e - q * M;
            const int k = p0 + q;
            const int kk = H - k;
            const C2<R> a = buf[lds_pad(q * M + y)];
            const C2<R> b = buf[lds_pad(half + q * M + y)];
            const C2<R> sa = cmk<R>(a.x + b.x, a.y - b.y);  // a + conj b
            const C2<R> da = cmk<R>(a.x - b.x, a.y + b.y);  // a - conj b
            const C2<R> ta = cmul<R>(cconj<R>(tw_get<R, false>(tw, k, M4)), da);
            st(dst(k, y), cmk<R>(sa.x - ta.y, sa.y + ta.x));  // sa + i ta
            if (k != 0 && kk != k) {
                const C2<R> sb = cmk<R>(b.x + a.x, b.y - a.y);
                const C2<R> db = cmk<R>(b.x - a.x, b.y + a.y);
                const C2<R> tb = cmul<R>(cconj<R>(tw_get<R, false>(tw, kk, M4)), db);
                st(dst(kk, y), cmk<R>(sb.x - tb.y, sb.y + tb.x));
            }
        }
    };
    using CI = ColInvSkip<R, MS>;
    if constexpr (CI::ok) {
        if (negf != nullptr && np == CI::P) {
            // U flags per pair of the tile, then element tid + j nthr: column
            // j / CPT of the first run (pair j / CPT) or of the second (pair
            // P - 1 - (j - P CPT) / CPT), row ky with ky mod M/2 the
            // ((j mod CPT) mod U)-th value
            uint8_t fu[CI::P][CI::U];
#pragma unroll
            for (int qq = 0; qq < CI::P; ++qq) {
                const uint8_t* row = negf + (size_t)fold_class(p0 + qq, M) * FS;
#pragma unroll
                for (int v = 0; v < CI::U; ++v) fu[qq][v] = row[fold_class((tid + v * CI::NT) % H, M)];
            }
            pre();  // overlaps the flag loads, which the data loads below wait for
            // element tid + j nthr: LDS slot lds_pad(tid) plus a compile-time
            // offset (nthr, M and the run length are multiples of the padding
            // period), global address run base + tid plus a constant
            static_assert(CI::NT % kLdsPadPeriod == 0 && MS % kLdsPadPeriod == 0, "linear slots");
            constexpr int F = CI::P * CI::CPT;  // elements of the first run per thread
            C2<R>* lb = buf + lds_pad(tid);
            // load the live elements of a tile whose slice starts at bse
            auto load_tile = [&](const C2<R>* bse, C2<R>* v) {
                const C2<R>* g1 = bse + (size_t)p0 * M + tid;
                const C2<R>* g2 = bse + (size_t)c2 * M + tid;
#pragma unroll
                for (int j = 0; j < CI::EPT; ++j) {
                    v[j] = cmk<R>(R(0), R(0));
                    const int pq = j < F ? j / CI::CPT : CI::P - 1 - (j - F) / CI::CPT;  // pair of element j
                    if (!fu[pq][(j % CI::CPT) % CI::U]) v[j] = ld(j < F ? g1 + j * CI::NT : g2 + (j - F) * CI::NT);
                }
            };
            auto to_lds = [&](const C2<R>* v) {
#pragma unroll
                for (int j = 0; j < CI::EPT; ++j) {
                    if (j < F) {
                        lb[pad_offset(j, CI::NT)] = v[j];
                    } else {
                        const int cm = (j - F) / CI::CPT;  // memory column c2 + cm, pair P - 1 - cm
                        const int yo = ((j - F) % CI::CPT) * CI::NT;  // row offset within the column
                        lb[pad_offset(1, CI::P * MS + (CI::P - 1 - cm) * MS + yo)] = v[j];
                    }
                }
            };
            C2<R> v1[CI::EPT], v2[CI::EPT];
            load_tile(base, v1);
            if (tile2 >= 0) load_tile(base2, v2);
            to_lds(v1);
            finish();
            if (tile2 >= 0) {
                __syncthreads();  // every thread is done with the first tile's LDS
                to_lds(v2);
                base = base2;
                obase = BLK ? blk + (size_t)r2 * K * M : base2;
                nts = HINTS && 2 * r2 < nslices;
                finish();
            }
            return;
        }
    }
    // generic path: element by element, the flags (if any) looked up per element
    auto load_generic = [&]() {
        for (int e = tid; e < nel; e += nthr) {
            C2<R> v = cmk<R>(R(0), R(0));
            if (e < half) {
                const int q = fdiv(e, inv_M);
                if (negf == nullptr || !negf[(size_t)fold_class(p0 + q, M) * FS + fold_class(e - q * M, M)])
                    v = ld(base + (size_t)p0 * M + e);
                buf[lds_pad(e)] = v;
            } else {
                const int e2 = e - half;
                const int cm = fdiv(e2, inv_M);           // memory column c2 + cm = H - p0 - q
                const int y = e2 - cm * M;
                const int q = np - 1 - cm;
                if (negf == nullptr || !negf[(size_t)fold_class(p0 + q, M) * FS + fold_class(y, M)])
                    v = ld(base + (size_t)c2 * M + e2);
                buf[lds_pad(half + q * M + y)] = v;
            }
        }
    };
    // (a second tile is only ever requested for full fast-path tiles, above)
    pre();
    load_generic();
    finish();
}

// ---------------------------------------------------------------------------
// Orientation: column FFT of the corrupted image's row spectrum F[kx][ky]
// (slice 0) for kx in [c0, c0 + ncb), multiplication by the smoothed
// central-difference symbols and inverse column FFTs.  Writes G_x into
// slice 0 and G_y into slice 1.
//   G_x = F * i sqrt(M) s_kx g(kx) g(ky) / M^2,  G_y likewise with s_ky,
//   s_k = sin(2 pi k/M), g(k) = exp(-2 pi^2 sigma^2 kbar^2 / M^2).
// (The 1/M^2 only keeps magnitudes moderate; the angle ignores it.)
// ---------------------------------------------------------------------------
template <class R, int EPT, bool TWF>
__device__ __forceinline__ void col_orient_tile(C2<R>* __restrict__ spec, int M, int cols_per_tile, int nthr,
                                                int c0, const FftPlan& planM, const C2<R>* tw, C2<R>* buf,
                                                R neg_two_pi2_sigma2_over_M2, R scale, int tid) {
    const int M4 = M >> 2;
    const int H = M >> 1;
    const int K = H + 1;
    const int ncb = min(cols_per_tile, K - c0);
    const int nel = ncb * M;
    C2<R>* gx = spec + (size_t)c0 * M;
    C2<R>* gy = spec + ((size_t)K + c0) * M;
    for (int e = tid; e < nel; e += nthr) buf[lds_pad(e)] = gx[e];
    __syncthreads();
    fft_lds<R, false, EPT, TWF>(buf, planM, ncb, M, tw, M4, tid, nthr);
    const float inv_M = 1.0f / (float)M;
    for (int e = tid; e < nel; e += nthr) {
        const int col = fdiv(e, inv_M);
        const int ky = e - col * M;
        const int kx = c0 + col;
        const R skx = -tw_get<R, TWF>(tw, kx, M4).y;
        const R sky = -tw_get<R, TWF>(tw, ky, M4).y;
        const R kxb = (R)kx;  // kx <= M/2; (M/2)^2 = (-M/2)^2
        const R kyb = (R)(ky < H ? ky : ky - M);
        const R g = exp(neg_two_pi2_sigma2_over_M2 * (kxb * kxb + kyb * kyb)) * scale;
        const C2<R> F = buf[lds_pad(e)];
        const C2<R> iF = cmk<R>(-F.y, F.x);
        buf[lds_pad(e)] = cmk<R>(iF.x * skx * g, iF.y * skx * g);
        buf[lds_pad(nel + e)] = cmk<R>(iF.x * sky * g, iF.y * sky * g);
    }
    __syncthreads();
    fft_lds<R, true, EPT, TWF>(buf, planM, 2 * ncb, M, tw, M4, tid, nthr);
    for (int e = tid; e < nel; e += nthr) {
        gx[e] = buf[lds_pad(e)];
        gy[e] = buf[lds_pad(nel + e)];
    }
}

// ---------------------------------------------------------------------------
// Row pass, inverse: C2R along x of rows y0 = rb*rows .. y0+rows from the
// transposed half spectrum of slices [s_begin, s_end), then projection over
// those slices (max / sum), the real volume, or the orientation binning
// (slices 0, 1 = g_x, g_y).  DST_MAX combines slice groups through `enc`
// (order-preserving integer atomics) when it is not null, else writes `out`.
// With Z[k] = (X[k] + conj X[H-k]) + i w_M^{-k} (X[k] - conj X[H-k]), k < H,
// the unnormalised inverse FFT_H of Z is M (x[2n] + i x[2n+1]).
// ---------------------------------------------------------------------------
// TWC: as for row_fwd_tile (twiddles of every stage in registers).
template <class R, int DST, int EPT, bool TWF, int MS, bool PAIRED = false, bool BLK = false, bool TWC = false>
__device__ __forceinline__ void row_inv_tile(const C2<R>* __restrict__ spec, R* __restrict__ out,
                                             typename Enc<R>::U* __restrict__ enc, uint8_t* __restrict__ rmap,
                                             int M_, int rows_, int nthr_, int rb, int s_begin, int s_end, int N,
                                             R out_scale, const FftPlan& planH, const C2<R>* tw, C2<R>* buf,
                                             int tid, C2<R>* buf2 = nullptr) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    const int nthr = MS ? GC.row_threads : nthr_;
    const int M4 = M >> 2;
    const int H = M >> 1;
    const int K = H + 1;
    const int S = H + 2;  // LDS row stride: 8 rows of the transposed phase fall in distinct banks
    const int y0 = rb * rows;
    const int nel = rows * H;
    const float inv_H = 1.0f / (float)H;

    // accumulators per thread: EPT, or the last stage's output slots if more
    constexpr int NOUT = MS != 0 && static_out_slots(MS ? MS / 2 : 8, GC.rows, GC.row_threads) > EPT
                             ? static_out_slots(MS ? MS / 2 : 8, GC.rows, GC.row_threads)
                             : EPT;
    C2<R> acc[NOUT], acc2[NOUT];
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        const R init = (DST == DST_MAX) ? -INFINITY : R(0);
        acc[i] = cmk<R>(init, init);
        acc2[i] = cmk<R>(R(0), R(0));
    }

    // The next slice's (kx, row) segments are loaded into registers while the
    // current slice is transformed.  Thread t reads row t mod rows of columns
    // kx = t/rows + i*kstep (rows and nthr are multiples of each other).
    constexpr int MAXL = EPT + 2;
    const int rshift = __ffs(rows) - 1;  // rows is a power of two
    const int row_t = tid & (rows - 1);
    const int kx_t = tid >> rshift;
    const int kstep = nthr >> rshift;
    const int KL = PAIRED ? H : K;       // columns the transform reads
    // held as native two-element vectors: an array of the C2 class type is
    // kept in memory by the FP64 build (scratch), a vector array is not
    typedef R pv_t __attribute__((ext_vector_type(2)));
    pv_t pre[MAXL];
    auto pv = [](C2<R> z) { pv_t v; v.x = z.x; v.y = z.y; return v; };
    auto cv = [](pv_t v) { return cmk<R>(v.x, v.y); };
    // Fixed-size paired transforms take the first stage's inputs straight
    // from the prefetch registers: slot i holds (row t, column n) of the
    // thread's first-stage butterfly, rows fastest across lanes so that 8
    // lanes read one 64-byte (slice, column) segment.
    constexpr bool DIRECT = MS != 0 && PAIRED;
    // the row-blocked input is read by the direct first stage only
    static_assert(!BLK || DIRECT, "row-blocked input needs the compiled paired pass");
    if constexpr (DIRECT)
        static_assert(static_in_slots(MS / 2, GC.rows, GC.row_threads) <= MAXL, "one register per input");
#define SE2N_FETCH(SL)                                                                                  \
    do {                                                                                               \
        if constexpr (DIRECT) {                                                                        \
            _Pragma("unroll") for (int i = 0; i < static_in_slots(MS / 2, GC.rows, GC.row_threads); ++i) { \
                int t_, n_;                                                                            \
                if (static_in_pos<MS / 2, GC.rows, GC.row_threads, true>(tid, i, t_, n_))              \
                    pre[i] = pv(spec[(size_t)(SL) * K * M +                                            \
                                     (BLK ? row_blk_index(n_, y0 + t_, H) : (long)n_ * M + y0 + t_)]); \
            }                                                                                          \
        } else {                                                                                       \
            const C2<R>* in_ = spec + (size_t)(SL) * K * M + (size_t)kx_t * M + y0 + row_t;            \
            static_for<MAXL>([&](auto I) {                                                             \
                if (kx_t + I * kstep < KL) pre[I] = pv(in_[(size_t)(I * kstep) * M]);                  \
            });                                                                                        \
        }                                                                                              \
    } while (0)
    // Fixed-size paired transforms with a second buffer (buf2) run their
    // stages between the two; bx is the buffer the next first stage may fill.
    const bool pp = DIRECT && buf2 != nullptr;
    C2<R>* bx = buf;
    C2<R>* by = buf2;
    // (not for the orientation pass: two slices only, and no registers to spare)
    constexpr bool CACHE = DIRECT && TWC && DST != DST_ORIENT;
    using TwC = StageTw<R, true, TWF, MS ? MS / 2 : 8, GC.rows, GC.row_threads, MS ? MS : 16,
                        CACHE ? static_nstages(MS ? MS / 2 : 8) : 1>;
    TwC twc;
    if constexpr (CACHE) {
        __syncthreads();  // the twiddle table is in LDS
        twc.load(tw, tid);
    }
    // consume output element i (row, pixel pair n) of slice s
    auto take = [&](int s, int i, int row, int n, C2<R> z) {
        if (DST == DST_VOLUME) {
            *reinterpret_cast<C2<R>*>(out + ((size_t)s * M + y0 + row) * M + 2 * n) =
                cmk<R>(z.x * out_scale, z.y * out_scale);
        } else if (DST == DST_MAX) {
            acc[i].x = vmax<R>(acc[i].x, z.x);
            acc[i].y = vmax<R>(acc[i].y, z.y);
        } else if (DST == DST_SUM) {
            acc[i].x += z.x;
            acc[i].y += z.y;
        } else {  // DST_ORIENT
            if (s == 0) acc[i] = z;
            else acc2[i] = z;
        }
    };
    // Slices are taken from the last to the first: the pass before this one
    // wrote the high slices last, so they are the ones still held by the
    // memory-side cache when this pass starts.
    SE2N_FETCH(s_end - 1);
    for (int s = s_end - 1; s >= s_begin; --s) {
      if constexpr (DIRECT) {
        fft_static_first<R, true, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, true>(
            pp ? bx : buf, tid, [&](int i) { return cv(pre[i]); });
        if (s > s_begin) SE2N_FETCH(s - 1);
      } else {
        static_for<MAXL>([&](auto I) {
            const int kx = kx_t + I * kstep;
            if (kx < KL) buf[lds_pad(row_t * S + kx)] = cv(pre[I]);
        });
        __syncthreads();
        if (s > s_begin) SE2N_FETCH(s - 1);
        if constexpr (!PAIRED) {
        // pairing step of the real inverse transform:
        //   Z[k] = (X[k] + conj X[H-k]) + i w_M^{-k} (X[k] - conj X[H-k]),  k < H
        const int npair = H / 2 + 1;
        const float inv_npair = 1.0f / (float)npair;
        for (int e = tid; e < rows * npair; e += nthr) {
            const int row = fdiv(e, inv_npair);
            const int k = e - row * npair;
            const int kk = H - k;
            const C2<R> a = buf[lds_pad(row * S + k)];
            const C2<R> b = buf[lds_pad(row * S + kk)];
            const C2<R> sa = cmk<R>(a.x + b.x, a.y - b.y);  // a + conj b
            const C2<R> da = cmk<R>(a.x - b.x, a.y + b.y);  // a - conj b
            const C2<R> ta = cmul<R>(cconj<R>(tw_get<R, TWF>(tw, k, M4)), da);
            const C2<R> sb = cmk<R>(b.x + a.x, b.y - a.y);
            const C2<R> db = cmk<R>(b.x - a.x, b.y + a.y);
            const C2<R> tb = cmul<R>(cconj<R>(tw_get<R, TWF>(tw, kk, M4)), db);
            buf[lds_pad(row * S + k)] = cmk<R>(sa.x - ta.y, sa.y + ta.x);  // sa + i ta
            if (kk != k) buf[lds_pad(row * S + kk)] = cmk<R>(sb.x - tb.y, sb.y + tb.x);
        }
        __syncthreads();
        }
      }
        if constexpr (DIRECT) {
            // stages 2.. with the last stage's outputs going to the accumulators
            constexpr int R0 = static_radix(MS / 2, 0);
            if (pp) {
                C2<R>* last = fft_static_out_pp<R, true, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS, 1, R0>(
                    bx, by, tw, tid, [&](int slot, int t, int n, C2<R> z) { take(s, slot, t, n, z); }, twc);
                // the last stage may still be reading `last`: the next first stage fills the other one
                by = last;
                bx = (last == buf) ? buf2 : buf;
            } else {
                fft_static_out<R, true, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS, 1, R0>(
                    buf, tw, tid, [&](int slot, int t, int n, C2<R> z) { take(s, slot, t, n, z); });
            }
        } else if constexpr (MS != 0) {
            // the last stage's outputs go straight to the accumulators
            fft_static_out<R, true, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(
                buf, tw, tid, [&](int slot, int t, int n, C2<R> z) { take(s, slot, t, n, z); });
        } else {
            fft_lds<R, true, EPT, TWF>(buf, planH, rows, S, tw, M4, tid, nthr);
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int e = tid + i * nthr;
                if (e < nel) {
                    int row, n;
                    split_index(tid, i, nthr, H, inv_H, row, n);
                    take(s, i, row, n, buf[lds_pad(row * S + n)]);
                }
            }
            __syncthreads();
        }
    }
#undef SE2N_FETCH

    if (DST == DST_VOLUME) return;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        int row, n;
        bool valid;
        if constexpr (MS != 0) {
            valid = static_out_pos<MS / 2, GC.rows, GC.row_threads>(tid, i, row, n);
        } else {
            valid = tid + i * nthr < nel;
            split_index(tid, i, nthr, H, inv_H, row, n);
        }
        if (valid) {
            const size_t p = (size_t)(y0 + row) * M + 2 * n;
            if (DST == DST_MAX) {
                if (enc) {
                    atomicMax(enc + p, Enc<R>::encode(acc[i].x));
                    atomicMax(enc + p + 1, Enc<R>::encode(acc[i].y));
                } else {
                    *reinterpret_cast<C2<R>*>(out + p) = acc[i];
                }
            } else if (DST == DST_SUM) {
                *reinterpret_cast<C2<R>*>(out + p) = cmk<R>(acc[i].x * out_scale, acc[i].y * out_scale);
            } else {  // orientation bins of pixels 2n and 2n+1
                const R two_pi = R(6.283185307179586476925);
                const R half_pi = R(1.570796326794896619231);
                R t0 = (atan2(acc2[i].x, acc[i].x) + half_pi) * (R)N / two_pi + R(0.5);
                R t1 = (atan2(acc2[i].y, acc[i].y) + half_pi) * (R)N / two_pi + R(0.5);
                // floor(t) lies in [-N/4, 3N/4] (atan2 in [-pi, pi]): one wrap
                int b0 = (int)floor(t0);
                int b1 = (int)floor(t1);
                if (b0 < 0) b0 += N;
                if (b1 < 0) b1 += N;
                const uint16_t packed = (uint16_t)((unsigned)b0 | ((unsigned)b1 << 8));
                *reinterpret_cast<uint16_t*>(rmap + p) = packed;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-mode solve: psi_hat(kx,ky) <- P(kx,ky) psi_hat(kx,ky).
// ---------------------------------------------------------------------------
// The potential M (cos e_r s_kx + sin e_r s_ky)^2 has period N/2 in r, so in
// the basis p_j = x_j + x_{j+N/2}, q_j = x_j - x_{j+N/2} (j < N/2) the N x N
// propagator is two symmetric N/2 x N/2 blocks (periodic and antiperiodic
// coupling).  The table holds, per frequency class (lx, ly) with
// |s_kx| = sin(2 pi lx/M), |s_ky| = sin(2 pi ly/M), lx, ly in [0, M/4], the
// packed upper triangles of both blocks, scaled by 1/(2 M^2), laid out as
// P[lx][element][ly] with a line-aligned ly stride.
//
// The members of class (lx, ly) in the half spectrum are kx in {lx, M/2-lx}
// and ky in {ly, M/2-ly, M/2+ly, M-ly}.  Where s_kx s_ky < 0 (ky > M/2) the
// potential is the class potential with r -> -r, so the propagator is the
// class one conjugated by that permutation: the kernel loads and stores
// through the mirrored orientation index.
//
// A workgroup takes one lx and CLS consecutive ly, stages their propagators
// in LDS once (one contiguous run of the class-major table), and applies them
// to all 8 members of each class.  Each mode is handled by a pair of adjacent
// lanes: the even lane loads x_j and the odd lane x_{j+N/2} (j < N/2); one
// DPP swap gives the even lane p = x_j + x_{j+N/2} and the odd lane
// q = x_j - x_{j+N/2}; each applies its block (periodic / antiperiodic) and a
// second swap forms x'_j = y_p + y_q (even) and x'_{j+N/2} = y_p - y_q (odd).
// A wavefront covers 32 consecutive classes of one member (CLS >= 32), or
// CLS classes of each of 32/CLS members: runs of consecutive (or reversed)
// ky of one column per orientation plane.
__device__ __forceinline__ float swap_pair(float v) {
    // lanes (0,1)(2,3)...: quad_perm [1,0,3,2]
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_pair(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffff), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// zfill: store the zeros of negligible classes (off when the inverse column
// pass takes them as zero without reading them).
// With 4 | N the classes with lx > ly of the block use the slot of (ly, lx),
// read through its reflection (table_slot).
template <class R, int N, int CLS>
__device__ __forceinline__ void solve_tile(C2<R>* __restrict__ spec, const R* __restrict__ P, int M, int Q,
                                           int FS, int lx, int ly0, R* Ps, int tid, bool zfill = true) {
    constexpr int h = N / 2;
    constexpr int Eh = h * (h + 1) / 2;
    constexpr int E = 2 * Eh;
    constexpr int CS = table_class_stride(N, (int)sizeof(R));  // reals per class in the table
    constexpr int S = solve_lds_stride(N, (int)sizeof(R));     // and in LDS
    constexpr int OQ = solve_q_offset(N);                      // LDS offset of the antiperiodic block
    static_assert(CLS <= 64, "one flag bit per class in a wavefront mask");
    const int H = M >> 1;
    constexpr int NT = 16 * CLS < 512 ? 16 * CLS : 512;  // blockDim.x: two lanes per mode
    const int nthr = NT;
    const int ncls = min(CLS, Q - ly0);
    // One byte per class after the table (rows of FS bytes): 1 where the
    // class's propagator is negligible (every entry below 2^-30 in FP32,
    // 2^-60 in FP64, before the 1/(2M^2) scaling), so its modes are zero at
    // time T to within the rounding of the result.  Each wavefront gathers
    // the block's flags into a mask, bit c for class ly0 + c; classes past
    // the last one count as negligible (nothing is read for them).
    uint64_t negm;
    {
        const uint8_t* __restrict__ flags =
            reinterpret_cast<const uint8_t*>(P + table_slots(M, N) * CS) + (size_t)lx * FS + ly0;
        const int l = tid & 63;
        negm = __ballot(l >= ncls || flags[l] != 0);
    }
    // every class negligible and no zeros to store: nothing to do (negm is
    // the same in every wavefront, so the whole workgroup returns)
    if (!zfill && negm == ~0ull) return;
    // Stage the block's propagators, class c at Ps + c * S: 16-byte chunks
    // of the contiguous run, every load of a thread issued before the first
    // is waited on.  Chunks of negligible classes are not read; they and the
    // classes past the last one are zeroed (their modes are multiplied by
    // zeros, never by stale LDS).
    auto stage = [&]() {
        constexpr int VEC = 16 / (int)sizeof(R);
        typedef R vec_t __attribute__((ext_vector_type(VEC)));
        constexpr int CPC = CS / VEC;  // chunks per class
        constexpr int CH = CLS * CPC;
        constexpr int NST = (CH + NT - 1) / NT;
        constexpr int BATCH = NST < 8 ? NST : 8;  // loads in flight per thread
        // the block's slots: one contiguous run, except where classes share
        // the slots of (ly, lx) (one slot per class, in rows ly < lx of the
        // triangle)
        for (int k0 = 0; k0 < NST; k0 += BATCH) {
            vec_t v[BATCH];
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int i = tid + (k0 + k) * NT;
                v[k] = vec_t(0);
                // non-temporal: each propagator is read once per call, and
                // keeping the table out of the caches leaves them to the
                // spectrum, which the next pass reads again
                if (i < CH && !((negm >> (i / CPC)) & 1)) {
                    const int c = i / CPC;
                    const R* a = P + table_slot(lx, ly0 + c, Q, N) * CS + (size_t)(i - c * CPC) * VEC;
                    v[k] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(a));
                }
            }
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int i = tid + (k0 + k) * NT;
                if (i < CH) {
                    const int c = i / CPC;
                    const int f = (i - c * CPC) * VEC;
#pragma unroll
                    for (int q = 0; q < VEC; ++q) {
                        const int e = f + q;
                        if (e < E) Ps[c * S + (e < Eh ? e : e + (OQ - Eh))] = v[k][q];
                    }
                }
            }
        }
    };
    const size_t plane = (size_t)(H + 1) * M;
    const int odd = tid & 1;
    // A wavefront holds 32 pairs; with CLS >= 32 they all belong to one member,
    // so the member, its column kx and its orientation mirroring are uniform
    // across the wavefront (the slot reflection, per class, is not).
    constexpr bool UNIFORM = CLS >= 32;
    // The mode of lane pair `pair`: its class c, row ky and column, whether it
    // exists (live), is read, is mirrored in orientation (perm) and shares
    // the slot of its transposed class (tr).
    struct Mode {
        int c, ky;
        bool live, read, perm, tr;
        C2<R>* colbase;
    };
    auto mode_of = [&](int pair) {
        Mode md;
        int m = pair / CLS;
        if (UNIFORM) m = __builtin_amdgcn_readfirstlane(m);
        md.c = pair - m * CLS;
        const int ly = ly0 + md.c;
        const int a = m >> 2;
        const int b = m & 3;
        bool live = md.c < ncls;
        live = live && !(a == 1 && 2 * lx == H);           // kx = M/4 is its own mirror
        live = live && !(ly == 0 && b >= 2);               // ky in {0, M/2} only
        live = live && !(2 * ly == H && (b & 1));          // ky in {M/4, 3M/4} only
        md.live = live;
        md.read = live && !((negm >> md.c) & 1);           // negligible classes: zeros, nothing read
        const int kx = a ? H - lx : lx;
        int ky = b == 0 ? ly : (b == 1 ? H - ly : (b == 2 ? H + ly : M - ly));
        md.ky = live ? ky : 0;  // harmless in-range address; nothing is stored
        // s_ky < 0 exactly for the live members b = 2, 3 (ky in (M/2, M))
        md.perm = b >= 2;
        // a class sharing the slot of (ly, lx) is read through its reflection
        md.tr = table_transposed(lx, ly, N);
        md.colbase = spec + (size_t)kx * M;
        return md;
    };
    // Orientation plane of logical index r: the mirror r -> -r for s_ky < 0,
    // and for a class read through its slot's reflection (tr) that
    // reflection composed with it, r -> N/4 - r, or r -> r - N/4 under the
    // mirror.
    auto plane_of = [&](bool perm, bool tr, int r) {
        if (table_sym(N) && tr) return perm ? (r + 3 * (N / 4)) % N : (N / 4 + N - r) % N;
        return perm ? (r == 0 ? 0 : N - r) : r;
    };
    // this lane's half of the orientation vector (lanes of dead or negligible
    // modes read nothing and hold zeros)
    auto load_half = [&](const Mode& md, C2<R>* x) {
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int r0 = j, r1 = j + h;
            const int a0 = plane_of(md.perm, md.tr, r0);
            const int a1 = plane_of(md.perm, md.tr, r1);
            const C2<R>* pl0 = md.colbase + (size_t)a0 * plane;
            const C2<R>* pl1 = md.colbase + (size_t)a1 * plane;
            C2<R> v = cmk<R>(R(0), R(0));
            if (md.read) v = odd ? pl1[md.ky] : pl0[md.ky];
            x[j] = v;
        }
    };
    // apply the class's blocks to the mode and store it
    auto apply_store = [&](const Mode& md, C2<R>* x) {
        const R* Pc = Ps + md.c * S + odd * OQ;
        // even lane: p = x_j + x_{j+h};  odd lane: q = x_j - x_{j+h}
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const R ox = swap_pair(x[j].x);
            const R oy = swap_pair(x[j].y);
            x[j] = odd ? cmk<R>(ox - x[j].x, oy - x[j].y) : cmk<R>(x[j].x + ox, x[j].y + oy);
        }
        C2<R> y[h];
#pragma unroll
        for (int j = 0; j < h; ++j) y[j] = cmk<R>(R(0), R(0));
        {
            int e = 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
#pragma unroll
                for (int j = i; j < h; ++j) {
                    const R w = Pc[e];
                    y[i].x += w * x[j].x;
                    y[i].y += w * x[j].y;
                    if (j != i) {
                        y[j].x += w * x[i].x;
                        y[j].y += w * x[i].y;
                    }
                    ++e;
                }
                // keep each row's LDS reads next to their use (bounded registers)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // even lane: y_p + y_q -> x'_j;  odd lane: y_p - y_q -> x'_{j+h}
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const R ox = swap_pair(y[j].x);
            const R oy = swap_pair(y[j].y);
            y[j] = odd ? cmk<R>(ox - y[j].x, oy - y[j].y) : cmk<R>(y[j].x + ox, y[j].y + oy);
        }
        if (md.live && (zfill || md.read)) {  // negligible classes store the zeros they were given, if asked
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const int r0 = j, r1 = j + h;
                const int a0 = plane_of(md.perm, md.tr, r0);
                const int a1 = plane_of(md.perm, md.tr, r1);
                C2<R>* pl = md.colbase + (size_t)(odd ? a1 : a0) * plane;
                pl[md.ky] = y[j];
            }
        }
    };
    if constexpr (NT / 2 == 8 * CLS) {
        // one mode per lane pair: its spectrum loads do not depend on the
        // table, so they go out before the staging and the two memory round
        // trips overlap
        const Mode md = mode_of(tid >> 1);
        C2<R> x[h];
        load_half(md, x);
        stage();
        __syncthreads();
        // a wavefront with nothing to read and no zeros to store has no work
        if (!zfill && __ballot(md.read) == 0) return;
        apply_store(md, x);
    } else {
        stage();
        __syncthreads();
        // every lane of a pair runs the same iterations, so the swaps always meet
#pragma unroll 1
        for (int pair = tid >> 1; pair < 8 * CLS; pair += nthr >> 1) {
            const Mode md = mode_of(pair);
            // (the loop bounds are the same for every lane of a wavefront)
            if (!zfill && __ballot(md.read) == 0) continue;
            C2<R> x[h];
            load_half(md, x);
            apply_store(md, x);
        }
    }
}

template <class R, int N>
constexpr int solve_cls() {
    return solve_classes(N, (int)sizeof(R));
}

}  // namespace se2n
