// gfx950 kernels of the semi-discrete SE(2,N) diffusion.
//
// Spectral layout.  The half spectrum of an orientation volume is stored
// "column major": spec[r][kx][ky], kx in [0, M/2], ky in [0, M) contiguous.
// Every column (r, kx) is M contiguous complex values, so the column FFTs
// and the per-mode solve read and write whole cache lines; the row passes
// move 8 (float) or 4 (double) rows at a time so that each (r, kx) segment
// they touch is 64 contiguous bytes.
//
// Pass structure of one diffusion (Theorem 2 of the paper: FFT over (Z/MZ)^2,
// M^2 decoupled N-dimensional systems, inverse FFT):
//   k_row_fwd   lift (or read the real volume) + real-to-complex FFT along x
//   k_col_fft   complex FFT along y, forward
//   k_solve     psi_hat(kx,ky) <- P(kx,ky) psi_hat(kx,ky), P the per-mode propagator
//   k_col_fft   complex FFT along y, inverse
//   k_row_inv   complex-to-real FFT along x + projection (or write the volume)
// The 1/M^2 of the inverse transform is folded into the stored propagators.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"
#include "se2n_passes.hpp"

namespace se2n {

// Workgroup -> (row block, slice group) of a row pass launched on a 1-D grid.
// The dispatcher hands consecutive workgroups to the 8 XCDs in turn.  With
// `pair` set, row blocks 2j and 2j+1 of one slice group go to two workgroups
// that the same XCD runs back to back, so both 64-byte halves of every
// 128-byte line of a (slice, kx) column run are fetched through one L2.
__device__ __forceinline__ void row_block_of(int nrb, int ngroups, bool pair, int& rb, int& g) {
    const int i = blockIdx.x;
    if (pair && (nrb & 1) == 0 && ((nrb * ngroups) & 15) == 0) {
        const int xcd = i & 7;
        const int slot = i >> 3;
        const int pr = (slot >> 1) * 8 + xcd;
        const int per_group = nrb >> 1;
        g = pr / per_group;
        rb = 2 * (pr - g * per_group) + (slot & 1);
    } else {
        g = i / nrb;
        rb = i - g * nrb;
    }
}

// ---------------------------------------------------------------------------
// Single-image kernels: one workgroup per tile; the tile bodies are shared
// with the batched kernels.
// ---------------------------------------------------------------------------
// Row passes: grid (M/rows row blocks) x (slice groups) on a 1-D grid;
// block: nthr threads; LDS: twiddles + rows x (H+2) (padded).
template <class R, int SRC, int EPT, bool TWF, int MS>
__global__ __launch_bounds__(sizeof(R) == 8 ? kRowThreadsF64 : 1024) void k_row_fwd(const R* __restrict__ f, const uint8_t* __restrict__ mask,
                          const uint8_t* __restrict__ rmap, const R* __restrict__ vol,
                          C2<R>* __restrict__ spec, int M_, int nslices, int slices_per_group,
                          int rows_, int xcd_pair, FftPlan planH, const C2<R>* __restrict__ twg) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    const int nthr = MS ? GC.row_threads : (int)blockDim.x;
    extern __shared__ unsigned char smem_raw[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, TWF);
    int rb, grp;
    row_block_of(M / rows, (nslices + slices_per_group - 1) / slices_per_group, xcd_pair != 0, rb, grp);
    const int s_begin = grp * slices_per_group;
    const int s_end = min(nslices, s_begin + slices_per_group);
    load_twiddles<R>(tw, twg, M >> 2, TWF, threadIdx.x, nthr);
    row_fwd_tile<R, SRC, EPT, TWF, MS, true>(f, mask, rmap, vol, spec, M, rows, nthr, rb, s_begin, s_end, planH, tw,
                                       buf, threadIdx.x, MS ? buf + row_buf_elems(M, rows) : nullptr);
}

// Column pass: one tile of cols_per_block contiguous columns per workgroup.
template <class R, bool INV, int EPT, bool TWF, int MS>
__global__ void k_col_fft(C2<R>* __restrict__ spec, long ncols, int M_, int cols_per_block_,
                          FftPlan planM, const C2<R>* __restrict__ twg, const uint8_t* __restrict__ negf,
                          int FS) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int cols_per_block = MS ? GC.cols : cols_per_block_;
    const int nthr = MS ? GC.col_threads : (int)blockDim.x;
    extern __shared__ unsigned char smem_raw[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, TWF);
    // tiles from the last slice to the first: the row pass before this one
    // wrote the high slices last, and the memory-side cache still holds them
    const long tile = (long)gridDim.x - 1 - (long)blockIdx.x;
    // the tile issues its own loads first and fetches the twiddles meanwhile
    col_fft_tile<R, INV, EPT, TWF, MS>(spec, ncols, M, cols_per_block, nthr, tile * cols_per_block, planM, tw, buf,
                                      threadIdx.x, negf, FS,
                                      [&] { load_twiddles<R>(tw, twg, M >> 2, TWF, threadIdx.x, nthr); });
}

template <class R, int EPT, bool TWF>
__global__ void k_col_orient(C2<R>* __restrict__ spec, int M, int cols_per_block, FftPlan planM,
                             const C2<R>* __restrict__ twg, R neg_two_pi2_sigma2_over_M2, R scale) {
    extern __shared__ unsigned char smem_raw[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, TWF);
    const int nthr = blockDim.x;
    load_twiddles<R>(tw, twg, M >> 2, TWF, threadIdx.x, nthr);
    col_orient_tile<R, EPT, TWF>(spec, M, cols_per_block, nthr, blockIdx.x * cols_per_block, planM, tw, buf,
                                 neg_two_pi2_sigma2_over_M2, scale, threadIdx.x);
}

template <class R, int DST, int EPT, bool TWF, int MS, bool PAIRED, bool BLK = false>
__global__ __launch_bounds__(sizeof(R) == 8 ? kRowThreadsF64 : 1024) void k_row_inv(const C2<R>* __restrict__ spec, R* __restrict__ out,
                          typename Enc<R>::U* __restrict__ enc, uint8_t* __restrict__ rmap,
                          int M_, int nslices, int slices_per_group, int rows_, int xcd_pair, int N,
                          R out_scale, FftPlan planH, const C2<R>* __restrict__ twg) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    const int nthr = MS ? GC.row_threads : (int)blockDim.x;
    extern __shared__ unsigned char smem_raw[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, TWF);
    int rb, grp;
    row_block_of(M / rows, (nslices + slices_per_group - 1) / slices_per_group, xcd_pair != 0, rb, grp);
    const int s_begin = grp * slices_per_group;
    const int s_end = min(nslices, s_begin + slices_per_group);
    load_twiddles<R>(tw, twg, M >> 2, TWF, threadIdx.x, nthr);
    row_inv_tile<R, DST, EPT, TWF, MS, PAIRED, BLK, true>(spec, out, enc, rmap, M, rows, nthr, rb, s_begin, s_end, N,
                                               out_scale, planH, tw, buf, threadIdx.x,
                                               MS ? buf + row_buf_elems(M, rows) : nullptr);
}

// Paired inverse column pass: one tile of column pairs per workgroup.
// TWO: each workgroup transforms slices 2s and 2s + 1 of its pair block (grid
// N/2 x pair blocks), loading the flags and twiddles once for both.
// BLK: the result goes to blk in the row-blocked layout.
template <class R, int EPT, int MS, bool TWO = false, bool BLK = false>
__global__ __launch_bounds__(1024) void k_col_inv_paired(C2<R>* __restrict__ spec, int M_, int pcols_, FftPlan planM,
                                                         const C2<R>* __restrict__ twg,
                                                         const uint8_t* __restrict__ negf, int FS,
                                                         C2<R>* __restrict__ blk) {
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int nthr = MS ? GC.pcol_threads : (int)blockDim.x;
    extern __shared__ unsigned char smem_raw[];
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, false);
    const int P = (MS ? GC.pcols : pcols_) / 2;
    const int tps = (M / 4 + 1 + P - 1) / P;
    const int nslices = (TWO ? 2 : 1) * (int)gridDim.x / tps;  // grid: slices (or slice pairs) x pair blocks
    int tile = blockIdx.x, tile2 = -1;
    if (TWO) {
        const int s2 = blockIdx.x / tps;
        tile = 2 * s2 * tps + (blockIdx.x - s2 * tps);
        tile2 = tile + tps;
    }
    // the tile fetches the twiddles while its flag loads are in flight
    auto pre = [&] { load_twiddles<R>(tw, twg, M >> 2, false, threadIdx.x, nthr); };
    col_inv_paired_tile<R, EPT, MS, true, decltype(pre), BLK>(spec, M, pcols_, nthr, tile, planM, tw, buf, threadIdx.x,
                                                              nslices, negf, FS, pre, tile2, blk);
}

// ---------------------------------------------------------------------------
// Small elementwise kernels.
// ---------------------------------------------------------------------------
template <class R>
__global__ void k_fill_enc(typename Enc<R>::U* __restrict__ enc, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) enc[i] = 0;
}

template <class R>
__global__ void k_decode_enc(const typename Enc<R>::U* __restrict__ enc, R* __restrict__ out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = Enc<R>::decode(enc[i]);
}

template <class R>
__global__ void k_lift(const R* __restrict__ f, const uint8_t* __restrict__ mask,
                       const uint8_t* __restrict__ rmap, R* __restrict__ psi, long MM, int N) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MM) return;
    const R v = mask[i] ? R(0) : f[i];
    const int r = rmap[i];
    for (int s = 0; s < N; ++s) psi[(size_t)s * MM + i] = (s == r) ? v : R(0);
}

template <class R, bool MEAN>
__global__ void k_project(const R* __restrict__ psi, R* __restrict__ out, long MM, int N) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MM) return;
    R a = psi[i];
    for (int s = 1; s < N; ++s) {
        const R v = psi[(size_t)s * MM + i];
        a = MEAN ? a + v : fmax(a, v);
    }
    out[i] = MEAN ? a / (R)N : a;
}

// ---------------------------------------------------------------------------
// Propagator precompute, FP64: one 64-thread workgroup per frequency class.
// ---------------------------------------------------------------------------
// For class (lx, ly) and each block (periodic +, antiperiodic -) of size
// h = N/2:  A = beta L_h^{+-} - diag(pot_j), pot_j = M (cos e_j s_x + sin e_j s_y)^2.
// Odd N: one periodic block of size h = N, the whole propagator.
//   CN:    C = (I - tau A/2)^{-1} (I + tau A/2) by Gauss-Jordan (the left
//          matrix is symmetric, diagonally dominant: no pivoting), P = C^n by
//          binary powering.
//   EXACT: P = e^{T A} by scaling and squaring of a degree-16 Taylor sum.
__device__ void lds_matmul(const double* A, const double* B, double* Cm, int h, int tid) {
    for (int idx = tid; idx < h * h; idx += 64) {
        const int i = idx / h;
        const int j = idx - i * h;
        double s = 0.0;
        for (int k = 0; k < h; ++k) s += A[i * h + k] * B[k * h + j];
        Cm[idx] = s;
    }
    __syncthreads();
}

__device__ void lds_copy(const double* A, double* B, int n, int tid) {
    for (int idx = tid; idx < n; idx += 64) B[idx] = A[idx];
    __syncthreads();
}

// Negligible-class flag of a slot's class, under both orders when the slot
// is shared (the column passes look flags up by (lx, ly) as they come), and
// the padding of the flag rows the slot ends (by the thread group of one
// workgroup; tid < 64).
template <class R>
__device__ void store_class_flags(R* Ptab, int M, int N, int Q, int FS, int lx, int ly, bool negligible, int tid) {
    uint8_t* flags = reinterpret_cast<uint8_t*>(Ptab + table_slots(M, N) * (size_t)table_class_stride(N, (int)sizeof(R)));
    if (tid == 0) {
        flags[(size_t)lx * FS + ly] = negligible ? 1 : 0;
        if (table_sym(N)) flags[(size_t)ly * FS + lx] = negligible ? 1 : 0;
    }
    if (ly == Q - 1)  // row padding (every row lx has the slot (lx, Q - 1))
        for (int j = Q + tid; j < FS; j += 64) flags[(size_t)lx * FS + j] = 0;
}

template <class R>
__global__ __launch_bounds__(64) void k_precompute(R* __restrict__ Ptab, int M, int N, int Q, int FS,
                                                   double beta, double T, int nsteps, int scheme,
                                                   double scale, int keep_all) {
    extern __shared__ double sm[];
    const bool odd = (N & 1) != 0;
    const int h = odd ? N : N / 2;
    const int nblk = odd ? 1 : 2;
    const int hh = h * h;
    // LDS: W (2hh) | Rs (hh) | Ts (hh) | pot (h).  CN builds the generator A
    // in Ts, fills the augmented matrix W from it, eliminates (Ts then holds
    // the pivot column), and compacts the right half of W (the one-step
    // propagator) into W's first hh entries, Bs.  EXACT keeps A in W.
    double* W = sm;          // h x 2h augmented matrix
    double* Bs = W;          // base of the powering (CN)
    double* Rs = W + 2 * hh; // running product
    double* Ts = Rs + hh;    // temporary
    double* pot = Ts + hh;
    double* A = scheme == 0 ? Ts : W;  // generator block
    const int tid = threadIdx.x;
    int lx, ly;  // the class of this workgroup's slot
    table_slot_class(blockIdx.x, Q, N, lx, ly);
    const double two_pi = 6.283185307179586476925;
    const double sx = sin(two_pi * lx / M);
    const double sy = sin(two_pi * ly / M);
    for (int j = tid; j < h; j += 64) {
        const double e = two_pi * j / N;
        const double a = cos(e) * sx + sin(e) * sy;
        pot[j] = (double)M * a * a;
    }
    __syncthreads();
    const int Eh = h * (h + 1) / 2;
    const int E = nblk * Eh;
    const int CS = table_class_stride(N, (int)sizeof(R));
    double pmax = 0.0;  // largest entry of the unscaled propagator, this thread's share
    for (int blk = 0; blk < nblk; ++blk) {
        const double wrap = blk == 0 ? 1.0 : -1.0;
        for (int idx = tid; idx < hh; idx += 64) {
            const int i = idx / h;
            const int j = idx - i * h;
            double v = (i == j) ? (-2.0 * beta - pot[i]) : 0.0;
            // neighbours i+1 and i-1 with wrap-around sign
            if (j == (i + 1) % h) v += (i + 1 < h) ? beta : wrap * beta;
            if (j == (i + h - 1) % h) v += (i >= 1) ? beta : wrap * beta;
            A[idx] = v;
        }
        __syncthreads();
        if (scheme == 0) {
            const double tau = T / nsteps;
            for (int idx = tid; idx < 2 * hh; idx += 64) {
                const int i = idx / (2 * h);
                const int j = idx - i * 2 * h;
                const double a = A[i * h + (j % h)];
                const double id = (i == (j % h)) ? 1.0 : 0.0;
                W[idx] = (j < h) ? (id - 0.5 * tau * a) : (id + 0.5 * tau * a);
            }
            __syncthreads();
            for (int piv = 0; piv < h; ++piv) {
                const double inv = 1.0 / W[piv * 2 * h + piv];
                __syncthreads();  // every thread has read the pivot
                for (int j = tid; j < 2 * h; j += 64) W[piv * 2 * h + j] *= inv;
                for (int i = tid; i < h; i += 64) Ts[i] = W[i * 2 * h + piv];
                __syncthreads();
                for (int idx = tid; idx < 2 * hh; idx += 64) {
                    const int i = idx / (2 * h);
                    const int j = idx - i * 2 * h;
                    if (i != piv) W[idx] -= Ts[i] * W[piv * 2 * h + j];
                }
                __syncthreads();
            }
            // compact the right half of W into its first hh entries, row by
            // row: row i's destination [i h, i h + h) holds only entries of
            // rows already copied (and left halves, no longer needed)
            for (int i = 0; i < h; ++i) {
                double v = 0.0;
                if (tid < h) v = W[i * 2 * h + h + tid];
                __syncthreads();
                if (tid < h) Bs[i * h + tid] = v;
                __syncthreads();
            }
            for (int idx = tid; idx < hh; idx += 64) {
                const int i = idx / h;
                const int j = idx - i * h;
                Rs[idx] = (i == j) ? 1.0 : 0.0;
            }
            __syncthreads();
            int n = nsteps;
            while (n > 0) {
                if (n & 1) {
                    lds_matmul(Rs, Bs, Ts, h, tid);
                    lds_copy(Ts, Rs, hh, tid);
                }
                n >>= 1;
                if (n) {
                    lds_matmul(Bs, Bs, Ts, h, tid);
                    lds_copy(Ts, Bs, hh, tid);
                }
            }
        } else {
            // X = T A / 2^s with ||X||_inf <= 1/2
            double nrm = 0.0;
            for (int i = 0; i < h; ++i) {
                double rs = 0.0;
                for (int j = 0; j < h; ++j) rs += fabs(A[i * h + j]);
                nrm = fmax(nrm, rs);
            }
            nrm *= T;
            __syncthreads();  // all norms read before A is scaled in place
            int sq = 0;
            while (nrm > 0.5) {
                nrm *= 0.5;
                ++sq;
            }
            const double xs = T * ldexp(1.0, -sq);
            for (int idx = tid; idx < hh; idx += 64) {
                A[idx] *= xs;
                const int i = idx / h;
                const int j = idx - i * h;
                Rs[idx] = (i == j) ? 1.0 : 0.0;
            }
            __syncthreads();
            // Horner: E = I + X (I + X/2 (I + X/3 (... (I + X/16))))
            for (int k = 16; k >= 1; --k) {
                lds_matmul(A, Rs, Ts, h, tid);
                for (int idx = tid; idx < hh; idx += 64) {
                    const int i = idx / h;
                    const int j = idx - i * h;
                    Rs[idx] = ((i == j) ? 1.0 : 0.0) + Ts[idx] / k;
                }
                __syncthreads();
            }
            for (int s = 0; s < sq; ++s) {
                lds_matmul(Rs, Rs, Ts, h, tid);
                lds_copy(Ts, Rs, hh, tid);
            }
        }
        // packed upper triangle, symmetrised, scaled, stored as R
        R* dst = Ptab + (size_t)blockIdx.x * CS;
        for (int idx = tid; idx < hh; idx += 64) {
            const int i = idx / h;
            const int j = idx - i * h;
            if (j >= i) {
                const int e = blk * Eh + i * h - i * (i - 1) / 2 + (j - i);
                const double u = 0.5 * (Rs[i * h + j] + Rs[j * h + i]);
                pmax = fmax(pmax, fabs(u));
                dst[e] = (R)(u * scale);
            }
        }
        __syncthreads();
    }
    // negligible-class flag (the workgroup is one wavefront): set when every
    // entry of both blocks is below 2^-30 (FP32) or 2^-60 (FP64); the solve
    // then writes zeros for the class's modes without reading them
    for (int off = 32; off >= 1; off >>= 1) pmax = fmax(pmax, __shfl_xor(pmax, off, 64));
    store_class_flags<R>(Ptab, M, N, Q, FS, lx, ly, !keep_all && pmax < (sizeof(R) == 4 ? 0x1p-30 : 0x1p-60), tid);
    // the class's line padding
    for (int e = E + tid; e < CS; e += 64) Ptab[(size_t)blockIdx.x * CS + e] = R(0);
}

// ---------------------------------------------------------------------------
// Propagator precompute on the FP64 matrix cores, for blocks of at most
// 16 x 16 (even N <= 32): one wavefront per frequency class, both blocks.
// ---------------------------------------------------------------------------
// Each block is embedded in a 16 x 16 matrix (the padding is the identity,
// which every step below keeps, and is never stored).  Matrices live in LDS
// row-major with a row stride of 17 doubles, so that the 16 lanes reading a
// column touch 16 distinct bank pairs.
//   CN:    the left matrix I - tau A / 2 is cyclic tridiagonal; lane c of
//          block b solves it for the unit vector e_c (Thomas elimination with
//          a Sherman-Morrison correction for the corners, as the paper's
//          remark 2 suggests for the time steps themselves), and the
//          one-step propagator is C = (I - tau A/2)^{-1} (I + tau A/2)
//          = 2 (I - tau A/2)^{-1} - I.  P = C^n by binary powering.
//   EXACT: P = e^{T A} by scaling and squaring of a degree-16 Taylor sum.
// A 16 x 16 x 16 product is four v_mfma_f64_16x16x4 (A[i][k] from lane
// i + 16 k, B[k][j] from lane j + 16 k; D[i][j] comes back in lane
// j + 16 (i mod 4), element i div 4); the two blocks' products are issued
// interleaved.
typedef double mf64x4 __attribute__((ext_vector_type(4)));
constexpr int kMS = 17;            // LDS row stride of a 16 x 16 matrix
constexpr int kMM = 16 * kMS;      // doubles per matrix

// D_b = X_b Y_b for b = 0, nb - 1 (X, Y, D: per-block matrix pointers).
__device__ __forceinline__ void mm16_pair(const double* X0, const double* Y0, double* D0, const double* X1,
                                          const double* Y1, double* D1, int nb, int l) {
    const int i = l & 15, q = l >> 4;
    mf64x4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + q;
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(X0[i * kMS + k], Y0[k * kMS + i], c0, 0, 0, 0);
        if (nb > 1) c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(X1[i * kMS + k], Y1[k * kMS + i], c1, 0, 0, 0);
    }
    __syncthreads();  // every operand read before any result is written (D may be an operand)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        D0[(4 * v + q) * kMS + i] = c0[v];
        if (nb > 1) D1[(4 * v + q) * kMS + i] = c1[v];
    }
    __syncthreads();
}

template <class R>
__global__ __launch_bounds__(64) void k_precompute_mfma(R* __restrict__ Ptab, int M, int N, int Q, int FS,
                                                        double beta, double T, int nsteps, int scheme, double scale,
                                                        int keep_all) {
    __shared__ double sm[6 * kMM];
    __shared__ double spot[16];
    const int l = threadIdx.x;
    const int h = N / 2;
    int lx, ly;  // the class of this workgroup's slot
    table_slot_class(blockIdx.x, Q, N, lx, ly);
    const double two_pi = 6.283185307179586476925;
    const double sx = sin(two_pi * lx / M);
    const double sy = sin(two_pi * ly / M);
    // per block b: base / product / scratch matrices, as offsets into sm
    // (matrix b of a kind at sm + off + b * kMM)
    int Bo = 0, Ro = 2 * kMM, To = 4 * kMM;
    // the potential pot_j = M (cos e_j s_x + sin e_j s_y)^2, j < h, once per class
    if (l < h) {
        const double e = two_pi * l / N;
        const double a = cos(e) * sx + sin(e) * sy;
        spot[l] = (double)M * a * a;
    }
    __syncthreads();
    auto pot = [&](int j) { return spot[j]; };
    if (scheme == 0) {
        const double tau = T / nsteps;
        const double o = -0.5 * tau * beta;  // off-diagonal of I - tau A / 2
        // lane l < 32: column c = l mod 16 of block b = l / 16
        if (l < 32) {
            const int b = l >> 4, c = l & 15;
            double* Bb = sm + Bo + b * kMM;
            if (c < h) {
                const double cr = b == 0 ? o : -o;  // corners: periodic (p) / antiperiodic (q)
                double d[16], cp[16], w[16], z[16];
                for (int j = 0; j < h; ++j) d[j] = 1.0 + tau * beta + 0.5 * tau * pot(j);
                const double g = -d[0];
                // Thomas factorisation of Tm (d with d_0 - g, d_{h-1} - cr^2/g), solving
                // Tm w = e_c and Tm z = u, u = (g, 0, .., 0, cr)
                double prev_cp = 0.0, pw = 0.0, pz = 0.0;
                for (int j = 0; j < h; ++j) {
                    double tj = d[j];
                    if (j == 0) tj -= g;
                    if (j == h - 1) tj -= cr * cr / g;
                    const double iden = 1.0 / (tj - (j ? o * prev_cp : 0.0));
                    cp[j] = o * iden;
                    w[j] = ((j == c ? 1.0 : 0.0) - (j ? o * pw : 0.0)) * iden;
                    z[j] = ((j == 0 ? g : 0.0) + (j == h - 1 ? cr : 0.0) - (j ? o * pz : 0.0)) * iden;
                    prev_cp = cp[j];
                    pw = w[j];
                    pz = z[j];
                }
                for (int j = h - 2; j >= 0; --j) {
                    w[j] -= cp[j] * w[j + 1];
                    z[j] -= cp[j] * z[j + 1];
                }
                const double f = (w[0] + (cr / g) * w[h - 1]) / (1.0 + z[0] + (cr / g) * z[h - 1]);
                for (int i = 0; i < 16; ++i) {
                    const double inv = i < h ? w[i] - f * z[i] : 0.0;
                    Bb[i * kMS + c] = i < h ? 2.0 * inv - (i == c ? 1.0 : 0.0) : 0.0;
                }
            } else {
                for (int i = 0; i < 16; ++i) Bb[i * kMS + c] = i == c ? 1.0 : 0.0;
            }
        }
        for (int e = l; e < 2 * 256; e += 64) {
            const int b = e >> 8, i = (e >> 4) & 15, j = e & 15;
            sm[Ro + b * kMM + i * kMS + j] = i == j ? 1.0 : 0.0;
        }
        __syncthreads();
        // binary powering: R = C^n (the roles of the three matrices rotate)
        int n = nsteps;
        while (n > 0) {
            if (n & 1) {
                mm16_pair(sm + Ro, sm + Bo, sm + To, sm + Ro + kMM, sm + Bo + kMM, sm + To + kMM, 2, l);
                const int t = Ro;
                Ro = To;
                To = t;
            }
            n >>= 1;
            if (n) {
                mm16_pair(sm + Bo, sm + Bo, sm + To, sm + Bo + kMM, sm + Bo + kMM, sm + To + kMM, 2, l);
                const int t = Bo;
                Bo = To;
                To = t;
            }
        }
    } else {
        // X = T A / 2^s with ||T A||_inf / 2^s <= 1/2 (the larger of the two blocks' norms)
        double nrm = 0.0;
        for (int i = 0; i < h; ++i)  // row sums: |diagonal| plus at most 2 beta off the diagonal
            nrm = fmax(nrm, fabs(-2.0 * beta - pot(i)) + 2.0 * beta);
        nrm *= T;
        int sq = 0;
        while (nrm > 0.5) {
            nrm *= 0.5;
            ++sq;
        }
        const double xs = T * ldexp(1.0, -sq);
        for (int e = l; e < 2 * 256; e += 64) {
            const int b = e >> 8, i = (e >> 4) & 15, j = e & 15;
            double v = 0.0;
            if (i < h && j < h) {
                const double wrap = b == 0 ? 1.0 : -1.0;
                if (i == j) v = -2.0 * beta - pot(i);
                if (j == (i + 1) % h) v += (i + 1 < h) ? beta : wrap * beta;
                if (j == (i + h - 1) % h) v += (i >= 1) ? beta : wrap * beta;
            }
            sm[Bo + b * kMM + i * kMS + j] = v * xs;
            sm[Ro + b * kMM + i * kMS + j] = i == j ? 1.0 : 0.0;
        }
        __syncthreads();
        // Horner: E = I + X (I + X/2 (I + X/3 (... (I + X/16))))
        for (int k = 16; k >= 1; --k) {
            mm16_pair(sm + Bo, sm + Ro, sm + To, sm + Bo + kMM, sm + Ro + kMM, sm + To + kMM, 2, l);
            for (int e = l; e < 2 * 256; e += 64) {
                const int b = e >> 8, i = (e >> 4) & 15, j = e & 15;
                sm[Ro + b * kMM + i * kMS + j] = (i == j ? 1.0 : 0.0) + sm[To + b * kMM + i * kMS + j] / k;
            }
            __syncthreads();
        }
        for (int s2 = 0; s2 < sq; ++s2) {
            mm16_pair(sm + Ro, sm + Ro, sm + To, sm + Ro + kMM, sm + Ro + kMM, sm + To + kMM, 2, l);
            const int t = Ro;
            Ro = To;
            To = t;
        }
    }
    // packed upper triangles of both blocks, symmetrised, scaled, stored as R
    const int Eh = h * (h + 1) / 2;
    const int CS = table_class_stride(N, (int)sizeof(R));
    R* dst = Ptab + (size_t)blockIdx.x * CS;
    double pmax = 0.0;
    for (int e = l; e < 2 * h * h; e += 64) {
        const int b = e / (h * h), r = e - b * h * h, i = r / h, j = r - (r / h) * h;
        if (j >= i) {
            const double* Rb = sm + Ro + b * kMM;
            const double u = 0.5 * (Rb[i * kMS + j] + Rb[j * kMS + i]);
            pmax = fmax(pmax, fabs(u));
            dst[b * Eh + i * h - i * (i - 1) / 2 + (j - i)] = (R)(u * scale);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) pmax = fmax(pmax, __shfl_xor(pmax, off, 64));
    store_class_flags<R>(Ptab, M, N, Q, FS, lx, ly, !keep_all && pmax < (sizeof(R) == 4 ? 0x1p-30 : 0x1p-60), l);
    for (int e = 2 * Eh + l; e < CS; e += 64) dst[e] = R(0);
}

// ---------------------------------------------------------------------------
// Launchers (host side, called by the runtime with validated arguments).
// ---------------------------------------------------------------------------
template <class R>
constexpr bool kStatic = sizeof(R) == 4;  // fixed-size kernels exist for FP32 only

// M of the kernels compiled for a fixed size that this plan can use (0: none):
// FP32, M in {512, 1024, 2048}, with the default geometry.
template <class R>
static int static_size(int M, const LaunchGeom& g) {
    if (sizeof(R) != 4 || !g.static_ok) return 0;
    if (M != 512 && M != 1024 && M != 2048) return 0;
    const GeomCore c = geom_core<R>(M);
    const bool same = g.rows == c.rows && g.row_threads == c.row_threads && g.row_ept == c.row_ept &&
                      g.cols == c.cols && g.col_threads == c.col_threads && g.col_ept == 8 && c.col_ept == 8 &&
                      g.tw_full == c.tw_full && g.tw_full_col == 0;
    return same ? M : 0;
}

// Elements per thread and twiddle table of the row kernels compiled for a fixed M.
template <int M>
constexpr int kRowEpt = geom_core<float>(M).row_ept;
template <int M>
constexpr bool kRowTwf = geom_core<float>(M).tw_full != 0;

template <class R>
static size_t tw_bytes(int M, bool full) {
    return (size_t)tw_elems(M, full) * sizeof(C2<R>);
}

template <class R>
hipError_t launch_row_fwd(int src, const R* f, const uint8_t* mask, const uint8_t* rmap, const R* vol,
                          C2<R>* spec, int M, int nslices, const LaunchGeom& g, const FftPlan& planH,
                          const C2<R>* tw, hipStream_t st) {
    const int groups = (nslices + g.row_slices - 1) / g.row_slices;
    dim3 grid((M / g.rows) * groups);
    // the kernels compiled for a fixed M run their stages between two row buffers
    const size_t lds = tw_bytes<R>(M, g.tw_full != 0) +
                       (size_t)row_buf_elems(M, g.rows) * sizeof(C2<R>) * (kStatic<R> && static_size<R>(M, g) ? 2 : 1);
#define SE2N_ROWFWD(S, E, W, MSV)                                                                          \
    hipLaunchKernelGGL((k_row_fwd<R, S, E, W, MSV>), grid, dim3(g.row_threads), lds, st, f, mask, rmap, vol,    \
                       spec, M, nslices, g.row_slices, g.rows, g.xcd_pair, planH, tw)
#define SE2N_ROWFWD_E(S)                                                    \
    if (static_size<R>(M, g) == 2048) SE2N_ROWFWD(S, kRowEpt<2048>, kRowTwf<2048>, kStatic<R> ? 2048 : 0);        \
    else if (static_size<R>(M, g) == 1024) SE2N_ROWFWD(S, kRowEpt<1024>, kRowTwf<1024>, kStatic<R> ? 1024 : 0);   \
    else if (static_size<R>(M, g) == 512) SE2N_ROWFWD(S, kRowEpt<512>, kRowTwf<512>, kStatic<R> ? 512 : 0);     \
    else if (g.tw_full) {                                                   \
        if (g.row_ept == 8) SE2N_ROWFWD(S, 8, true, 0);                     \
        else SE2N_ROWFWD(S, 16, true, 0);                                   \
    } else {                                                                \
        if (g.row_ept == 8) SE2N_ROWFWD(S, 8, false, 0);                    \
        else SE2N_ROWFWD(S, 16, false, 0);                                  \
    }
    if (src == SRC_LIFT) { SE2N_ROWFWD_E(SRC_LIFT) }
    else if (src == SRC_VOLUME) { SE2N_ROWFWD_E(SRC_VOLUME) }
    else { SE2N_ROWFWD_E(SRC_IMAGE) }
#undef SE2N_ROWFWD_E
#undef SE2N_ROWFWD
    return hipGetLastError();
}

template <class R>
hipError_t launch_col_fft(bool inverse, C2<R>* spec, long ncols, int M, const LaunchGeom& g,
                          const FftPlan& planM, const C2<R>* tw, hipStream_t st, const uint8_t* negf) {
    dim3 grid((unsigned)((ncols + g.cols - 1) / g.cols));
    const size_t lds = tw_bytes<R>(M, g.tw_full_col != 0) + (size_t)lds_padded_size(g.cols * M) * sizeof(C2<R>);
#define SE2N_COL(I, E, W, MSV)                                                                                 \
    hipLaunchKernelGGL((k_col_fft<R, I, E, W, MSV>), grid, dim3(g.col_threads), lds, st, spec, ncols, M, g.cols, planM, \
                       tw, negf, flag_stride(M))
#define SE2N_COL_E(I)                                                   \
    if (static_size<R>(M, g) == 2048) SE2N_COL(I, 8, false, kStatic<R> ? 2048 : 0);      \
    else if (static_size<R>(M, g) == 1024) SE2N_COL(I, 8, false, kStatic<R> ? 1024 : 0); \
    else if (static_size<R>(M, g) == 512) SE2N_COL(I, 8, false, kStatic<R> ? 512 : 0);   \
    else if (g.tw_full_col) {                                           \
        if (g.col_ept == 8) SE2N_COL(I, 8, true, 0);                    \
        else SE2N_COL(I, 16, true, 0);                                  \
    } else {                                                            \
        if (g.col_ept == 8) SE2N_COL(I, 8, false, 0);                   \
        else SE2N_COL(I, 16, false, 0);                                 \
    }
    if (inverse) { SE2N_COL_E(true) }
    else { SE2N_COL_E(false) }
#undef SE2N_COL_E
#undef SE2N_COL
    return hipGetLastError();
}

template <class R>
hipError_t launch_col_orient(C2<R>* spec, int M, const LaunchGeom& g, const FftPlan& planM,
                             const C2<R>* tw, double sigma, hipStream_t st) {
    const int K = M / 2 + 1;
    dim3 grid((K + g.ocols - 1) / g.ocols);
    const size_t lds = tw_bytes<R>(M, g.tw_full_col != 0) + (size_t)lds_padded_size(2 * g.ocols * M) * sizeof(C2<R>);
    const double c = -2.0 * 9.869604401089358619 * sigma * sigma / ((double)M * M);
    const double scale = sqrt((double)M) / ((double)M * M);
    if (g.ocol_ept == 8)
        hipLaunchKernelGGL((k_col_orient<R, 8, false>), grid, dim3(g.ocol_threads), lds, st, spec, M, g.ocols,
                           planM, tw, (R)c, (R)scale);
    else
        hipLaunchKernelGGL((k_col_orient<R, 16, false>), grid, dim3(g.ocol_threads), lds, st, spec, M, g.ocols,
                           planM, tw, (R)c, (R)scale);
    return hipGetLastError();
}

// The compiled size of the paired inverse kernel for M (0: the generic one).
template <class R>
static int col_inv_static(int M, const LaunchGeom& g) {
    const GeomCore c = geom_core<R>(M);
    const bool fixed = static_size<R>(M, g) != 0 && g.pcols == c.pcols && g.pcol_threads == c.pcol_threads &&
                       c.pcol_ept == 8;
    return kStatic<R> && fixed && (M == 2048 || M == 1024 || M == 512) ? M : 0;
}

template <class R>
bool col_inv_masks(int M, const LaunchGeom& g) {
    const int ms = col_inv_static<R>(M, g);
    return ms != 0 && col_skip_shape(ms, geom_core<R>(ms).pcol_threads);
}

template <class R>
bool row_blocked(int M, const LaunchGeom& g) {
    return kStatic<R> && col_inv_static<R>(M, g) != 0 && static_size<R>(M, g) == M && M % kRowBlk == 0;
}

template <class R>
hipError_t launch_col_inv_paired(C2<R>* spec, int M, int N, const LaunchGeom& g, const FftPlan& planM,
                                 const C2<R>* tw, hipStream_t st, const uint8_t* negf, C2<R>* blk) {
    if (blk != nullptr && !row_blocked<R>(M, g)) return hipErrorInvalidValue;
    const int P = g.pcols / 2;
    const int npair = M / 4 + 1;
    const size_t lds = tw_bytes<R>(M, false) + (size_t)lds_padded_size(g.pcols * M) * sizeof(C2<R>);
    const int ms = col_inv_static<R>(M, g);
    // two slices per workgroup where every tile takes the flag-reading fast
    // path (full tiles of a compiled size whose rows meet few class indices)
    // (compiled for M = 2048, whose tiles are single pairs)
    const bool two = negf != nullptr && ms == 2048 && col_inv_masks<R>(M, g) && npair % P == 0 && N % 2 == 0;
    const dim3 grid((unsigned)((two ? N / 2 : N) * ((npair + P - 1) / P)));
#define SE2N_PCOL(E, MSV, TWOV, BLKV)                                                                      \
    hipLaunchKernelGGL((k_col_inv_paired<R, E, MSV, TWOV, BLKV>), grid, dim3(g.pcol_threads), lds, st, spec, M, \
                       g.pcols, planM, tw, negf, flag_stride(M), blk)
    if constexpr (kStatic<R>) {
        if (blk != nullptr) {
            if (two) SE2N_PCOL(8, 2048, true, true);
            else if (ms == 2048) SE2N_PCOL(8, 2048, false, true);
            else if (ms == 1024) SE2N_PCOL(8, 1024, false, true);
            else SE2N_PCOL(8, 512, false, true);
            return hipGetLastError();
        }
    }
    if (two && ms == 2048) SE2N_PCOL(8, kStatic<R> ? 2048 : 0, true, false);
    else if (ms == 2048) SE2N_PCOL(8, kStatic<R> ? 2048 : 0, false, false);
    else if (ms == 1024) SE2N_PCOL(8, kStatic<R> ? 1024 : 0, false, false);
    else if (ms == 512) SE2N_PCOL(8, kStatic<R> ? 512 : 0, false, false);
    else if (g.pcol_ept == 8) SE2N_PCOL(8, 0, false, false);
    else SE2N_PCOL(16, 0, false, false);
#undef SE2N_PCOL
    return hipGetLastError();
}

template <class R>
hipError_t launch_row_inv(int dst, const C2<R>* spec, R* out, typename Enc<R>::U* enc, uint8_t* rmap,
                          int M, int nslices, int N, R out_scale, const LaunchGeom& g,
                          int slices_per_group, const FftPlan& planH, const C2<R>* tw, hipStream_t st,
                          bool paired, bool blocked) {
    if (blocked && !(paired && dst != DST_ORIENT && row_blocked<R>(M, g))) return hipErrorInvalidValue;
    const int groups = (nslices + slices_per_group - 1) / slices_per_group;
    dim3 grid((M / g.rows) * groups);
    // the kernels compiled for a fixed M run their stages between two row buffers
    const size_t lds = tw_bytes<R>(M, g.tw_full != 0) +
                       (size_t)row_buf_elems(M, g.rows) * sizeof(C2<R>) * (kStatic<R> && static_size<R>(M, g) ? 2 : 1);
#define SE2N_ROWINV(D, E, W, MSV)                                                                              \
    do {                                                                                                       \
        if (paired)                                                                                            \
            hipLaunchKernelGGL((k_row_inv<R, D, E, W, MSV, true>), grid, dim3(g.row_threads), lds, st, spec, out, \
                               enc, rmap, M, nslices, slices_per_group, g.rows, g.xcd_pair, N, out_scale, planH,  \
                               tw);                                                                            \
        else                                                                                                   \
            hipLaunchKernelGGL((k_row_inv<R, D, E, W, MSV, false>), grid, dim3(g.row_threads), lds, st, spec, out, \
                               enc, rmap, M, nslices, slices_per_group, g.rows, g.xcd_pair, N, out_scale, planH,  \
                               tw);                                                                            \
    } while (0)
#define SE2N_ROWINV_BLK(D, MSV)                                                                                 \
    hipLaunchKernelGGL((k_row_inv<R, D, kRowEpt<MSV>, kRowTwf<MSV>, MSV, true, true>), grid, dim3(g.row_threads), lds, \
                       st, spec, out, enc, rmap, M, nslices, slices_per_group, g.rows, g.xcd_pair, N, out_scale,       \
                       planH, tw)
    if constexpr (kStatic<R>) {
        if (blocked) {
            if (dst == DST_MAX) {
                if (M == 2048) SE2N_ROWINV_BLK(DST_MAX, 2048);
                else if (M == 1024) SE2N_ROWINV_BLK(DST_MAX, 1024);
                else SE2N_ROWINV_BLK(DST_MAX, 512);
            } else if (dst == DST_SUM) {
                if (M == 2048) SE2N_ROWINV_BLK(DST_SUM, 2048);
                else if (M == 1024) SE2N_ROWINV_BLK(DST_SUM, 1024);
                else SE2N_ROWINV_BLK(DST_SUM, 512);
            } else {
                if (M == 2048) SE2N_ROWINV_BLK(DST_VOLUME, 2048);
                else if (M == 1024) SE2N_ROWINV_BLK(DST_VOLUME, 1024);
                else SE2N_ROWINV_BLK(DST_VOLUME, 512);
            }
            return hipGetLastError();
        }
    }
#undef SE2N_ROWINV_BLK
#define SE2N_ROWINV_E(D)                                                    \
    if (static_size<R>(M, g) == 2048) SE2N_ROWINV(D, kRowEpt<2048>, kRowTwf<2048>, kStatic<R> ? 2048 : 0);        \
    else if (static_size<R>(M, g) == 1024) SE2N_ROWINV(D, kRowEpt<1024>, kRowTwf<1024>, kStatic<R> ? 1024 : 0);   \
    else if (static_size<R>(M, g) == 512) SE2N_ROWINV(D, kRowEpt<512>, kRowTwf<512>, kStatic<R> ? 512 : 0);     \
    else if (g.tw_full) {                                                   \
        if (g.row_ept == 8) SE2N_ROWINV(D, 8, true, 0);                     \
        else SE2N_ROWINV(D, 16, true, 0);                                   \
    } else {                                                                \
        if (g.row_ept == 8) SE2N_ROWINV(D, 8, false, 0);                    \
        else SE2N_ROWINV(D, 16, false, 0);                                  \
    }
    if (dst == DST_MAX) { SE2N_ROWINV_E(DST_MAX) }
    else if (dst == DST_SUM) { SE2N_ROWINV_E(DST_SUM) }
    else if (dst == DST_VOLUME) { SE2N_ROWINV_E(DST_VOLUME) }
    else { SE2N_ROWINV_E(DST_ORIENT) }
#undef SE2N_ROWINV_E
#undef SE2N_ROWINV
    return hipGetLastError();
}

template <class R>
hipError_t launch_fill_enc(typename Enc<R>::U* enc, long n, hipStream_t st) {
    hipLaunchKernelGGL((k_fill_enc<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, enc, n);
    return hipGetLastError();
}

template <class R>
hipError_t launch_decode_enc(const typename Enc<R>::U* enc, R* out, long n, hipStream_t st) {
    hipLaunchKernelGGL((k_decode_enc<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, enc, out, n);
    return hipGetLastError();
}

template <class R>
hipError_t launch_lift(const R* f, const uint8_t* mask, const uint8_t* rmap, R* psi, int M, int N,
                       hipStream_t st) {
    const long MM = (long)M * M;
    hipLaunchKernelGGL((k_lift<R>), dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, f, mask, rmap,
                       psi, MM, N);
    return hipGetLastError();
}

template <class R>
hipError_t launch_project(const R* psi, R* out, int M, int N, bool mean, hipStream_t st) {
    const long MM = (long)M * M;
    dim3 grid((unsigned)((MM + 255) / 256));
    if (mean) hipLaunchKernelGGL((k_project<R, true>), grid, dim3(256), 0, st, psi, out, MM, N);
    else hipLaunchKernelGGL((k_project<R, false>), grid, dim3(256), 0, st, psi, out, MM, N);
    return hipGetLastError();
}

template <class R>
hipError_t launch_precompute(R* Ptab, int M, int N, double beta, double T, int nsteps, int scheme,
                             hipStream_t st, bool keep_all) {
    const int Q = M / 4 + 1;
    const size_t slots = table_slots(M, N);  // one workgroup per stored class
    const int h = (N & 1) ? N : N / 2;
    const size_t lds = (size_t)(4 * h * h + h) * sizeof(double);
    // the inverse FFT's 1/M^2, and for even N the 1/2 of the p/q recombination
    const double scale = ((N & 1) ? 1.0 : 0.5) / ((double)M * (double)M);
    // matrix cores for blocks of 9..16 (N = 18..32, the padded 16 x 16 products
    // pay off there: N = 32 at 2048^2, 400 steps: 8.6 -> 2 ms; N = 16 is
    // faster on the scalar path); SE2N_SCALAR_PRECOMPUTE forces the scalar one
    if (!(N & 1) && h > 8 && h <= 16 && std::getenv("SE2N_SCALAR_PRECOMPUTE") == nullptr) {
        hipLaunchKernelGGL((k_precompute_mfma<R>), dim3((unsigned)slots), dim3(64), 0, st, Ptab, M, N, Q,
                           flag_stride(M), beta, T, nsteps, scheme, scale, keep_all ? 1 : 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_precompute<R>), dim3((unsigned)slots), dim3(64), lds, st, Ptab, M, N, Q,
                       flag_stride(M), beta,
                       T, nsteps, scheme, scale, keep_all ? 1 : 0);
    return hipGetLastError();
}

#define SE2N_INSTANTIATE(R)                                                                             \
    template hipError_t launch_row_fwd<R>(int, const R*, const uint8_t*, const uint8_t*, const R*,     \
                                          C2<R>*, int, int, const LaunchGeom&, const FftPlan&,         \
                                          const C2<R>*, hipStream_t);                                  \
    template hipError_t launch_col_fft<R>(bool, C2<R>*, long, int, const LaunchGeom&, const FftPlan&,  \
                                          const C2<R>*, hipStream_t, const uint8_t*);                  \
    template hipError_t launch_col_orient<R>(C2<R>*, int, const LaunchGeom&, const FftPlan&,           \
                                             const C2<R>*, double, hipStream_t);                       \
    template hipError_t launch_row_inv<R>(int, const C2<R>*, R*, typename Enc<R>::U*, uint8_t*, int,   \
                                          int, int, R, const LaunchGeom&, int, const FftPlan&,         \
                                          const C2<R>*, hipStream_t, bool, bool);                            \
    template hipError_t launch_col_inv_paired<R>(C2<R>*, int, int, const LaunchGeom&, const FftPlan&,  \
                                                 const C2<R>*, hipStream_t, const uint8_t*, C2<R>*);   \
    template bool row_blocked<R>(int, const LaunchGeom&);                                              \
    template bool col_inv_masks<R>(int, const LaunchGeom&);                                            \
    template hipError_t launch_fill_enc<R>(typename Enc<R>::U*, long, hipStream_t);                    \
    template hipError_t launch_decode_enc<R>(const typename Enc<R>::U*, R*, long, hipStream_t);        \
    template hipError_t launch_lift<R>(const R*, const uint8_t*, const uint8_t*, R*, int, int,         \
                                       hipStream_t);                                                   \
    template hipError_t launch_project<R>(const R*, R*, int, int, bool, hipStream_t);                  \
    template hipError_t launch_precompute<R>(R*, int, int, double, double, int, int, hipStream_t, bool);

SE2N_INSTANTIATE(float)
SE2N_INSTANTIATE(double)

}  // namespace se2n
