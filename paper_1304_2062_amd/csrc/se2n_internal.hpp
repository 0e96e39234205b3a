// Internal declarations shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"

namespace se2n {

enum { SRC_LIFT = 0, SRC_VOLUME = 1, SRC_IMAGE = 2 };
enum { DST_MAX = 0, DST_SUM = 1, DST_VOLUME = 2, DST_ORIENT = 3 };

// Order-preserving map of a real value to an unsigned integer, so that a
// maximum over workgroups can be taken with integer atomics.  0 is below the
// image of every real value.
template <class R>
struct Enc;
template <>
struct Enc<float> {
    using U = unsigned int;
    __device__ static U encode(float v) {
        const U u = __float_as_uint(v);
        return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    }
    __device__ static float decode(U e) {
        return __uint_as_float((e & 0x80000000u) ? (e ^ 0x80000000u) : ~e);
    }
};
template <>
struct Enc<double> {
    using U = unsigned long long;
    __device__ static U encode(double v) {
        const U u = (U)__double_as_longlong(v);
        return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
    }
    __device__ static double decode(U e) {
        return __longlong_as_double((long long)((e & 0x8000000000000000ull) ? (e ^ 0x8000000000000000ull) : ~e));
    }
};

// Launch geometry of one plan (chosen on the host from M and the dtype).
// Each FFT workgroup holds its transforms in LDS; every thread stages at most
// `ept` (8 or 16) complex elements of a stage in registers.
struct LaunchGeom {
    int rows;         // image rows per row-pass workgroup
    int row_threads;  // threads of a row-pass workgroup
    int row_ept;
    int row_slices;   // orientation slices per row-pass workgroup (forward)
    int inv_slices;   // orientation slices per row-pass workgroup (inverse, max projection)
    int cols;         // columns per column-pass workgroup
    int col_threads;
    int col_ept;
    int ocols;        // columns per orientation column workgroup
    int ocol_threads;
    int ocol_ept;
    int pcols;        // columns per paired inverse column workgroup (even: pairs kx, M/2-kx)
    int pcol_threads;
    int pcol_ept;
    int xcd_pair;     // pair adjacent row blocks on one XCD (row passes)
    int tw_full;      // row passes: full-period twiddle table in LDS (else the quarter table)
    int tw_full_col;  // column passes: the same choice
    int static_ok;    // use the kernels compiled for a fixed M when M has one
};

// The size-dependent part of the launch geometry, shared by the host (plan
// creation) and by the kernels compiled for a fixed M.
struct GeomCore {
    int rows, row_threads, row_ept;
    int cols, col_threads, col_ept;
    int ocols, ocol_threads, ocol_ept;
    int pcols, pcol_threads, pcol_ept;
    int tw_full, tw_full_col;
};

// Row-blocked layout of one slice of the paired half spectrum (the inverse
// column pass's output for the inverse row pass): rows ky come in blocks of
// kRowBlk, and within a block the columns kx < M/2 follow one another, each
// holding its kRowBlk rows contiguously:
//     element (kx, ky) at (ky / kRowBlk) (M/2) kRowBlk + kx kRowBlk + ky mod kRowBlk.
// A row-pass tile (8 rows of every column) then reads 64-byte pieces of
// consecutive 128-byte runs instead of one 64-byte piece per 16-KB column.
constexpr int kRowBlk = 16;
__host__ __device__ constexpr long row_blk_index(int kx, int ky, int H) {
    return (long)(ky / kRowBlk) * H * kRowBlk + (long)kx * kRowBlk + ky % kRowBlk;
}

__host__ __device__ constexpr void fft_threads_of(int elems, int& threads, int& ept) {
    ept = 8;
    threads = (elems + 7) / 8;
    if (threads > 1024) {
        ept = 16;
        threads = (elems + 15) / 16;
    }
}

constexpr int kRowThreadsF64 = 512;  // threads of an FP64 row-pass workgroup, at most

template <class R>
__host__ __device__ constexpr GeomCore geom_core(int M) {
    GeomCore g{};
    const int cs = (int)sizeof(R) * 2;
    const int target = sizeof(R) == 4 ? 4096 : 2048;  // complex elements per FFT workgroup
    const int H = M / 2;
#ifndef SE2N_ROW_SEG_BYTES
#define SE2N_ROW_SEG_BYTES 64
#endif
    int rows = SE2N_ROW_SEG_BYTES / cs;                // contiguous bytes per (slice, kx) segment
    while (M % rows) rows >>= 1;                       // sides with 4 | M, 8 !| M: 4-row blocks
    while (rows * 2 * H <= target && M % (rows * 2) == 0 && rows * 2 <= M) rows *= 2;
    g.rows = rows;
    fft_threads_of(rows * H, g.row_threads, g.row_ept);
#ifndef SE2N_ROW_MAX_THREADS
#define SE2N_ROW_MAX_THREADS 1024
#endif
    // FP64 row workgroups stay at 512 threads (their kernels are bounded
    // to 512 threads and get 256 registers per thread)
    const int max_threads = sizeof(R) == 8 ? kRowThreadsF64 : SE2N_ROW_MAX_THREADS;
    if (g.row_threads > max_threads && g.row_ept == 8) {  // 16 elements per thread, half the threads
        g.row_ept = 16;
        g.row_threads = (rows * H + 15) / 16;
    }
    // the row passes walk (kx, row) pairs with thread t on row t mod rows
    g.row_threads = (g.row_threads + rows - 1) / rows * rows;
    g.cols = target / M > 1 ? target / M : 1;
    fft_threads_of(g.cols * M, g.col_threads, g.col_ept);
    g.ocols = target / (2 * M) > 1 ? target / (2 * M) : 1;
    fft_threads_of(2 * g.ocols * M, g.ocol_threads, g.ocol_ept);
    g.pcols = g.cols >= 2 ? (g.cols & ~1) : 2;
    fft_threads_of(g.pcols * M, g.pcol_threads, g.pcol_ept);
    // full-period twiddle table for the row passes when it fits beside the row
    // buffer; a column workgroup transforms only a few columns, for which
    // expanding the full table would cost as much as the transform
#ifndef SE2N_ROW_LDS_BUDGET
#define SE2N_ROW_LDS_BUDGET (150 * 1024)
#endif
    g.tw_full =
        (long)tw_elems(M, true) * cs + (long)lds_padded_size(rows * (H + 2)) * cs <= SE2N_ROW_LDS_BUDGET ? 1 : 0;
    g.tw_full_col = 0;
    return g;
}

// Elements of one row-pass LDS buffer (rows x (M/2 + 2), padded), a multiple
// of 8 so that a second buffer after it stays 64-byte aligned.
__host__ __device__ constexpr int row_buf_elems(int M, int rows) {
    return (lds_padded_size(rows * (M / 2 + 2)) + 7) & ~7;
}

// Workgroups are dispatched round-robin over the chip's 8 XCDs, each with its
// own L2.  This maps dispatch index i of n to a logical index such that each
// XCD receives one contiguous range of logical indices, in order: logical
// neighbours run on the same XCD at about the same time and share the L2
// lines they both touch.  A bijection on [0, n) for any n.
__host__ __device__ constexpr int xcd_contiguous(int i, int n) {
    const int per = n / 8;
    const int rem = n % 8;
    const int xcd = i % 8;
    const int slot = i / 8;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// Propagator table: one slot per frequency class (lx, ly), lx, ly in
// [0, M/4], holding the packed upper triangles of its periodic and
// antiperiodic blocks, (N/2)(N/2 + 1) reals, padded to whole 128-byte lines
// (a negligible class that is skipped shares no line with a live one).
//
// When 4 | N the classes (lx, ly) and (ly, lx) share a slot: swapping s_kx
// and s_ky in the potential (cos e_r s_kx + sin e_r s_ky)^2 is the
// reflection e_r -> pi/2 - e_r of the orientations, r -> N/4 - r (mod N),
// under which the cyclic Laplacian is invariant, so
//     P(lx, ly)[r][c] = P(ly, lx)[N/4 - r][N/4 - c]
// (a quarter turn of the frequency, as in the rotation theorem of the
// almost-periodic view, up to the mirror s_ky -> -s_ky).  Only lx <= ly is
// stored, row lx of the upper triangle holding ly = lx .. M/4 contiguously;
// otherwise the slots are P[lx][ly], row-major.
// Reals per class: both N/2 x N/2 blocks (even N), or the whole N x N
// propagator (odd N, where the potential's period N/2 is no symmetry).
__host__ __device__ constexpr int table_class_entries(int N) {
    return (N & 1) ? N * (N + 1) / 2 : (N / 2) * (N / 2 + 1);
}
__host__ __device__ constexpr int table_class_stride(int N, int rsize) {
    const int line = 128 / rsize;
    const int E = table_class_entries(N);
    return (E + line - 1) / line * line;
}

// The negligible-class flags follow the table: one byte per class, rows of
// M/4 + 1 bytes padded to 128.
__host__ __device__ constexpr int flag_stride(int M) { return (M / 4 + 1 + 127) / 128 * 128; }

// Whether a column tile of compiled side MS with NT threads looks up the
// negligible-class flags cheaply: NT divides MS and divides or is a multiple
// of MS/2, so the rows a thread handles in one column meet one or two class
// indices (the class of row ky depends only on ky mod MS/2).
__host__ __device__ constexpr bool col_skip_shape(int MS, int NT) {
    return MS != 0 && NT <= MS && MS % NT == 0 && ((MS / 2) % NT == 0 || NT % (MS / 2) == 0);
}

// Class slots: shared by (lx, ly) and (ly, lx) when 4 | N (above).
__host__ __device__ constexpr bool table_sym(int N) { return N % 4 == 0; }
__host__ __device__ constexpr size_t table_slots(int M, int N) {
    const size_t Q = (size_t)(M / 4 + 1);
    return table_sym(N) ? Q * (Q + 1) / 2 : Q * Q;
}
// first slot of row a of the upper triangle (classes (a, b), b >= a)
__host__ __device__ constexpr size_t table_row_start(int a, int Q) { return (size_t)a * Q - (size_t)a * (a - 1) / 2; }
// slot of class (lx, ly); with 4 | N the class is read through the
// reflection exactly when lx > ly (table_transposed)
__host__ __device__ constexpr size_t table_slot(int lx, int ly, int Q, int N) {
    if (!table_sym(N)) return (size_t)lx * Q + ly;
    const int a = lx < ly ? lx : ly, b = lx < ly ? ly : lx;
    return table_row_start(a, Q) + (size_t)(b - a);
}
__host__ __device__ constexpr bool table_transposed(int lx, int ly, int N) { return table_sym(N) && lx > ly; }
// the class stored in slot s (lx <= ly when 4 | N)
__host__ __device__ inline void table_slot_class(size_t s, int Q, int N, int& lx, int& ly) {
    if (!table_sym(N)) {
        lx = (int)(s / Q);
        ly = (int)(s - (size_t)lx * Q);
        return;
    }
    // row a: table_row_start(a) <= s < table_row_start(a + 1), from the root
    // of a (2Q + 1 - a) / 2 = s, then corrected for rounding
    const double b = 2.0 * Q + 1.0;
    int a = (int)((b - sqrt(b * b - 8.0 * (double)s)) * 0.5);
    if (a < 0) a = 0;
    while (a + 1 < Q && table_row_start(a + 1, Q) <= s) ++a;
    while (a > 0 && table_row_start(a, Q) > s) --a;
    lx = a;
    ly = a + (int)(s - table_row_start(a, Q));
}

// The flags of a table at P (the bytes after its propagators): one byte per
// class, both orders of a shared slot.
__host__ __device__ inline const uint8_t* table_flags(const void* P, int M, int N, int rsize) {
    return reinterpret_cast<const uint8_t*>(P) + table_slots(M, N) * (size_t)table_class_stride(N, rsize) * (size_t)rsize;
}

// Bytes of a propagator table with its flags (and 64 bytes of slack).
__host__ __device__ constexpr size_t table_bytes(int M, int N, int rsize) {
    const size_t Q = (size_t)(M / 4 + 1);
    return table_slots(M, N) * (size_t)table_class_stride(N, rsize) * (size_t)rsize + Q * (size_t)flag_stride(M) + 64;
}

// LDS layout of the propagators a solve workgroup stages: class c at c * S,
// its periodic block at offset 0 and its antiperiodic block at the odd
// offset OQ.  A wavefront reads one entry of 32 consecutive classes from
// both blocks at once; with S = 2 (mod 4) in FP32 the even lanes' classes
// fall in distinct even banks and the odd lanes' in distinct odd banks.
__host__ __device__ constexpr int solve_q_offset(int N) { return ((N / 2) * (N / 2 + 1) / 2) | 1; }
__host__ __device__ constexpr int solve_lds_stride(int N, int rsize) {
    const int need = solve_q_offset(N) + (N / 2) * (N / 2 + 1) / 2;
    return rsize == 4 ? need + (6 - need % 4) % 4 : (need | 1);
}
// Classes per solve workgroup: the largest power of two <= 16 whose staged
// propagators fit in 72 KB of LDS.  A workgroup stages its propagators, waits
// at a barrier and then makes few passes over its modes; small workgroups let
// several of them overlap on a CU (FP32, N = 32, 2048^2: 64 classes 161 us,
// 32 classes 145 us, 16 classes 141 us, 8 classes 175 us).
__host__ __device__ constexpr int solve_classes(int N, int rsize) {
    int c = 16;
    while (c > 1 && (long)solve_lds_stride(N, rsize) * c * rsize > 72 * 1024) c >>= 1;
    return c;
}

template <class R>
hipError_t launch_row_fwd(int src, const R* f, const uint8_t* mask, const uint8_t* rmap, const R* vol,
                          C2<R>* spec, int M, int nslices, const LaunchGeom& g, const FftPlan& planH,
                          const C2<R>* tw, hipStream_t st);
// negf: the negligible-class flags of the propagators the solve applies next
// (forward pass only; those modes are then not stored), or null.
template <class R>
hipError_t launch_col_fft(bool inverse, C2<R>* spec, long ncols, int M, const LaunchGeom& g,
                          const FftPlan& planM, const C2<R>* tw, hipStream_t st, const uint8_t* negf = nullptr);
template <class R>
hipError_t launch_col_orient(C2<R>* spec, int M, const LaunchGeom& g, const FftPlan& planM,
                             const C2<R>* tw, double sigma, hipStream_t st);
template <class R>
hipError_t launch_solve(C2<R>* spec, const R* P, int M, int N, hipStream_t st, bool zfill = true);
// paired: the inverse column pass already applied the pairing step of the
// real inverse transform (launch_col_inv_paired)
// blocked: spec holds the row-blocked layout that launch_col_inv_paired writes
// into its `blk` buffer (only where row_blocked holds; paired then)
template <class R>
hipError_t launch_row_inv(int dst, const C2<R>* spec, R* out, typename Enc<R>::U* enc, uint8_t* rmap,
                          int M, int nslices, int N, R out_scale, const LaunchGeom& g,
                          int slices_per_group, const FftPlan& planH, const C2<R>* tw, hipStream_t st,
                          bool paired = false, bool blocked = false);
// Inverse column FFT of column pairs (kx, M/2-kx) of every slice, followed by
// the pairing step of the real inverse row transform.
// negf: the flags of the propagators the solve applied; their modes are then
// taken as zero and not read (pass it exactly when col_inv_masks holds, and
// run the solve without zero fill then).
// blk (only where row_blocked holds): the result goes there, in the
// row-blocked layout, instead of back into spec.
template <class R>
hipError_t launch_col_inv_paired(C2<R>* spec, int M, int N, const LaunchGeom& g, const FftPlan& planM,
                                 const C2<R>* tw, hipStream_t st, const uint8_t* negf = nullptr,
                                 C2<R>* blk = nullptr);
// Whether the inverse column pass for M can hand the inverse row pass its
// result in the row-blocked layout (the compiled sizes of both passes).
template <class R>
bool row_blocked(int M, const LaunchGeom& g);
// Whether the paired inverse column pass for M leaves out negligible modes
// cheaply (a compiled tile shape whose rows meet one or two class indices
// per column), so that the solve need not store their zeros.
template <class R>
bool col_inv_masks(int M, const LaunchGeom& g);
template <class R>
hipError_t launch_fill_enc(typename Enc<R>::U* enc, long n, hipStream_t st);
template <class R>
hipError_t launch_decode_enc(const typename Enc<R>::U* enc, R* out, long n, hipStream_t st);
template <class R>
hipError_t launch_lift(const R* f, const uint8_t* mask, const uint8_t* rmap, R* psi, int M, int N,
                       hipStream_t st);
template <class R>
hipError_t launch_project(const R* psi, R* out, int M, int N, bool mean, hipStream_t st);
// Orientation map by a separable periodic stencil (FP32 plans).  The smoothed
// central differences are g_x = d (x) g and g_y = g (x) d, where g is the
// periodic smoothing kernel and d the smoothed central difference, both the
// inverse DFT of the Fourier multipliers.  They are passed as correlation
// weights: out[y] = sum_j t[j + r] in[y + j], j in [-r, r], r the compiled
// radius (entries beyond the kernel's support are zero).
constexpr int kOrientMaxRadius = 32;
constexpr int kOrientRadii[] = {8, 12, 16, 20, 24, 32};
struct OrientTaps {
    float g[2 * kOrientMaxRadius + 1];
    float d[2 * kOrientMaxRadius + 1];
};
hipError_t launch_orient_stencil(const float* f, const uint8_t* mask, uint8_t* rmap, int M, int N, int radius,
                                 const OrientTaps& taps, hipStream_t st);

// keep_all: flag no class as negligible (every mode is then read, propagated
// and stored; used to time the passes without the skip).
template <class R>
hipError_t launch_precompute(R* Ptab, int M, int N, double beta, double T, int nsteps, int scheme,
                             hipStream_t st, bool keep_all = false);

// Per-mode Crank-Nicolson integrated step by step (se2n_solve_iter.hip):
// n_steps steps of T / n_steps on every mode of the half spectrum, in place,
// the inverse transform's 1/M^2 applied at the end.  Even N in [4, 64].
template <class R>
hipError_t launch_solve_iter(C2<R>* spec, int M, int N, double beta, double T, int nsteps, hipStream_t st);

// Restoration heuristics (se2n_restore.hip): the static mix of a real volume
// at the known pixels, and the dynamic one (set-up; then per mesh point the
// orientation maximum, the growth of the good set and the mix).
template <class R>
hipError_t launch_sr_mix(R* vol, const R* f, const uint8_t* mask, double eps, int M, int N, hipStream_t st);
template <class R>
hipError_t launch_dr_init(int16_t* join, R* href, const R* f, const uint8_t* mask, int M, hipStream_t st);
template <class R>
hipError_t launch_dr_step(R* vol, R* h, int16_t* join, R* href, double eps, int step, int M, int N, hipStream_t st);

}  // namespace se2n
