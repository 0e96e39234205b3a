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

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"

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

// (q, r) = divmod(tid + i*nthr, d) without a per-element division when nthr
// is a multiple of d or d of nthr (uniform branches); inv_d = 1/d in float.
__device__ __forceinline__ void split_index(int tid, int i, int nthr, int d, float inv_d, int& q, int& r) {
    if (nthr % d == 0) {
        const int qt = tid / d;
        q = qt + i * (nthr / d);
        r = tid - qt * d;
    } else if (d % nthr == 0) {
        const int c = d / nthr;
        q = i / c;
        r = tid + (i - q * c) * nthr;
    } else {
        const int b = tid + i * nthr;
        q = fdiv(b, inv_d);
        r = b - q * d;
    }
}

// ---------------------------------------------------------------------------
// Row pass, forward: lift + R2C along x, written transposed.
// ---------------------------------------------------------------------------
// A real row x[0..M) is transformed as the half-length complex sequence
// z[n] = x[2n] + i x[2n+1]:  with Z = FFT_H(z), H = M/2,
//   X[k] = (Z[k] + conj Z[H-k])/2 + w_M^k (Z[k] - conj Z[H-k])/(2i),  k = 0..H.
// grid: (M/ROWS row blocks, slice groups); block: nthr threads; LDS ROWS*H.
template <class R, int SRC, int EPT, bool TWF, int MS>
__global__ __launch_bounds__(1024) void k_row_fwd(const R* __restrict__ f, const uint8_t* __restrict__ mask,
                          const uint8_t* __restrict__ rmap, const R* __restrict__ vol,
                          C2<R>* __restrict__ spec, int M_, int nslices, int slices_per_group,
                          int rows_, int xcd_pair, FftPlan planH, const C2<R>* __restrict__ twg) {
    constexpr bool twfull = TWF;
    // MS != 0: compiled for M = MS with the geometry geom_core<R>(MS)
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    extern __shared__ unsigned char smem_raw[];
    const int M4 = M >> 2;
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, twfull);
    const int H = M >> 1;
    const int K = H + 1;
    const int S = H + 2;  // LDS row stride: 8 rows of the transposed phase fall in distinct banks
    const int tid = threadIdx.x;
    const int nthr = MS ? GC.row_threads : (int)blockDim.x;
    int rb, grp;
    row_block_of(M / rows, (nslices + slices_per_group - 1) / slices_per_group, xcd_pair != 0, rb, grp);
    const int y0 = rb * rows;
    const int s_begin = grp * slices_per_group;
    const int s_end = min(nslices, s_begin + slices_per_group);
    const int nel = rows * H;
    const float inv_H = 1.0f / (float)H;

    load_twiddles<R>(tw, twg, M4, twfull, tid, nthr);
    // Lift sources are read once per block and kept in registers.
    R fc0[EPT], fc1[EPT];
    uint8_t rm0[EPT], rm1[EPT];
    if (SRC != SRC_VOLUME) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * nthr;
            fc0[i] = R(0);
            fc1[i] = R(0);
            rm0[i] = 0xff;
            rm1[i] = 0xff;
            if (e < nel) {
                int row, n;
                split_index(tid, i, nthr, H, inv_H, row, n);
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

    for (int s = s_begin; s < s_end; ++s) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * nthr;
            if (e < nel) {
                C2<R> z;
                if (SRC == SRC_VOLUME) {
                    int row, n;
                    split_index(tid, i, nthr, H, inv_H, row, n);
                    z = *reinterpret_cast<const C2<R>*>(vol + ((size_t)s * M + y0 + row) * M + 2 * n);
                } else if (SRC == SRC_LIFT) {
                    z.x = (rm0[i] == s) ? fc0[i] : R(0);
                    z.y = (rm1[i] == s) ? fc1[i] : R(0);
                } else {
                    z.x = fc0[i];
                    z.y = fc1[i];
                }
                int row, n;
                split_index(tid, i, nthr, H, inv_H, row, n);
                buf[lds_pad(row * S + n)] = z;
            }
        }
        __syncthreads();
        if constexpr (MS != 0)
            fft_static<R, false, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(buf, tw, tid);
        else
            fft_lds<R, false, EPT, TWF>(buf, planH, rows, S, tw, M4, tid, nthr);
        // unpack the real transform and write (r, kx, y0..y0+rows) segments
        const int nout = rows * K;
        C2<R>* out = spec + (size_t)s * K * M + y0;
        const int rshift = __ffs(rows) - 1;  // rows is a power of two
        for (int e = tid; e < nout; e += nthr) {
            const int kx = e >> rshift;
            const int row = e & (rows - 1);
            const C2<R> z1 = buf[lds_pad(row * S + (kx == H ? 0 : kx))];
            const C2<R> z2 = buf[lds_pad(row * S + (kx == 0 ? 0 : H - kx))];
            const C2<R> ev = cmk<R>(R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y));
            // (z1 - conj z2)/(2i)
            const C2<R> d = cmk<R>(z1.x - z2.x, z1.y + z2.y);
            const C2<R> od = cmk<R>(R(0.5) * d.y, -R(0.5) * d.x);
            out[(size_t)kx * M + row] = cadd<R>(ev, cmul<R>(tw_get<R, TWF>(tw, kx, M4), od));
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Column pass: FFT along y of `cols_per_block` contiguous columns of length M.
// ---------------------------------------------------------------------------
template <class R, bool INV, int EPT, bool TWF, int MS>
__global__ void k_col_fft(C2<R>* __restrict__ spec, long ncols, int M_, int cols_per_block_,
                          FftPlan planM, const C2<R>* __restrict__ twg) {
    constexpr bool twfull = TWF;
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int cols_per_block = MS ? GC.cols : cols_per_block_;
    extern __shared__ unsigned char smem_raw[];
    const int M4 = M >> 2;
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, twfull);
    const int tid = threadIdx.x;
    const int nthr = MS ? GC.col_threads : (int)blockDim.x;
    load_twiddles<R>(tw, twg, M4, twfull, tid, nthr);
    const long c0 = (long)blockIdx.x * cols_per_block;
    const int ncb = (int)min((long)cols_per_block, ncols - c0);
    const int nel = ncb * M;
    C2<R>* base = spec + c0 * M;
    for (int e = tid; e < nel; e += nthr) buf[lds_pad(e)] = base[e];
    __syncthreads();
    if constexpr (MS != 0) {
        if (ncb == GC.cols) fft_static<R, INV, TWF, MS, GC.cols, MS, GC.col_threads, MS>(buf, tw, tid);
        else fft_lds<R, INV, EPT, TWF>(buf, planM, ncb, M, tw, M4, tid, nthr);
    } else {
        fft_lds<R, INV, EPT, TWF>(buf, planM, ncb, M, tw, M4, tid, nthr);
    }
    for (int e = tid; e < nel; e += nthr) base[e] = buf[lds_pad(e)];
}

// ---------------------------------------------------------------------------
// Orientation: column FFT of the corrupted image's row spectrum F[kx][ky]
// (slice 0), multiplication by the smoothed central-difference symbols and
// inverse column FFTs.  Writes G_x into slice 0 and G_y into slice 1.
//   G_x = F * i sqrt(M) s_kx g(kx) g(ky) / M^2,  G_y likewise with s_ky,
//   s_k = sin(2 pi k/M), g(k) = exp(-2 pi^2 sigma^2 kbar^2 / M^2).
// (The 1/M^2 only keeps magnitudes moderate; the angle ignores it.)
// ---------------------------------------------------------------------------
template <class R, int EPT, bool TWF>
__global__ void k_col_orient(C2<R>* __restrict__ spec, int M, int cols_per_block, FftPlan planM,
                             const C2<R>* __restrict__ twg, R neg_two_pi2_sigma2_over_M2, R scale) {
    constexpr bool twfull = TWF;
    extern __shared__ unsigned char smem_raw[];
    const int M4 = M >> 2;
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, twfull);
    const int H = M >> 1;
    const int K = H + 1;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    load_twiddles<R>(tw, twg, M4, twfull, tid, nthr);
    const int c0 = blockIdx.x * cols_per_block;
    const int ncb = min(cols_per_block, K - c0);
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
        const R kxb = (R)kx;                            // kx <= M/2; (M/2)^2 = (-M/2)^2
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
// Row pass, inverse: C2R along x from the transposed half spectrum, then
// projection over the block's slices (max / sum), the real volume, or the
// orientation binning (slices 0, 1 = g_x, g_y).
// With Z[k] = (X[k] + conj X[H-k]) + i w_M^{-k} (X[k] - conj X[H-k]), k < H,
// the unnormalised inverse FFT_H of Z is M (x[2n] + i x[2n+1]).
// ---------------------------------------------------------------------------
template <class R, int DST, int EPT, bool TWF, int MS>
__global__ __launch_bounds__(1024) void k_row_inv(const C2<R>* __restrict__ spec, R* __restrict__ out,
                          typename Enc<R>::U* __restrict__ enc, uint8_t* __restrict__ rmap,
                          int M_, int nslices, int slices_per_group, int rows_, int xcd_pair, int N,
                          R out_scale, FftPlan planH, const C2<R>* __restrict__ twg) {
    constexpr bool twfull = TWF;
    constexpr GeomCore GC = geom_core<R>(MS ? MS : 16);
    const int M = MS ? MS : M_;
    const int rows = MS ? GC.rows : rows_;
    extern __shared__ unsigned char smem_raw[];
    const int M4 = M >> 2;
    C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
    C2<R>* buf = tw + tw_elems(M, twfull);
    const int H = M >> 1;
    const int K = H + 1;
    const int S = H + 2;  // LDS row stride: 8 rows of the transposed phase fall in distinct banks
    const int tid = threadIdx.x;
    const int nthr = MS ? GC.row_threads : (int)blockDim.x;
    int rb, grp;
    row_block_of(M / rows, (nslices + slices_per_group - 1) / slices_per_group, xcd_pair != 0, rb, grp);
    const int y0 = rb * rows;
    const int s_begin = grp * slices_per_group;
    const int s_end = min(nslices, s_begin + slices_per_group);
    const int nel = rows * H;
    const float inv_H = 1.0f / (float)H;

    load_twiddles<R>(tw, twg, M4, twfull, tid, nthr);
    C2<R> acc[EPT], acc2[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
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
    C2<R> pre[MAXL];
#define SE2N_FETCH(SL)                                                                      \
    do {                                                                                   \
        const C2<R>* in_ = spec + (size_t)(SL) * K * M + (size_t)kx_t * M + y0 + row_t;    \
        _Pragma("unroll") for (int i = 0; i < MAXL; ++i) if (kx_t + i * kstep < K) pre[i] = \
            in_[(size_t)(i * kstep) * M];                                                   \
    } while (0)
    SE2N_FETCH(s_begin);
    for (int s = s_begin; s < s_end; ++s) {
#pragma unroll
        for (int i = 0; i < MAXL; ++i) {
            const int kx = kx_t + i * kstep;
            if (kx < K) buf[lds_pad(row_t * S + kx)] = pre[i];
        }
        __syncthreads();
        if (s + 1 < s_end) SE2N_FETCH(s + 1);
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
            const C2<R> sa = cmk<R>(a.x + b.x, a.y - b.y);      // a + conj b
            const C2<R> da = cmk<R>(a.x - b.x, a.y + b.y);      // a - conj b
            const C2<R> ta = cmul<R>(cconj<R>(tw_get<R, TWF>(tw, k, M4)), da);
            const C2<R> sb = cmk<R>(b.x + a.x, b.y - a.y);
            const C2<R> db = cmk<R>(b.x - a.x, b.y + a.y);
            const C2<R> tb = cmul<R>(cconj<R>(tw_get<R, TWF>(tw, kk, M4)), db);
            buf[lds_pad(row * S + k)] = cmk<R>(sa.x - ta.y, sa.y + ta.x);  // sa + i ta
            if (kk != k) buf[lds_pad(row * S + kk)] = cmk<R>(sb.x - tb.y, sb.y + tb.x);
        }
        __syncthreads();
        if constexpr (MS != 0)
            fft_static<R, true, TWF, MS / 2, GC.rows, MS / 2 + 2, GC.row_threads, MS>(buf, tw, tid);
        else
            fft_lds<R, true, EPT, TWF>(buf, planH, rows, S, tw, M4, tid, nthr);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * nthr;
            if (e < nel) {
                int row, n;
                split_index(tid, i, nthr, H, inv_H, row, n);
                const C2<R> z = buf[lds_pad(row * S + n)];
                if (DST == DST_VOLUME) {
                    *reinterpret_cast<C2<R>*>(out + ((size_t)s * M + y0 + row) * M + 2 * n) =
                        cmk<R>(z.x * out_scale, z.y * out_scale);
                } else if (DST == DST_MAX) {
                    acc[i].x = fmax(acc[i].x, z.x);
                    acc[i].y = fmax(acc[i].y, z.y);
                } else if (DST == DST_SUM) {
                    acc[i].x += z.x;
                    acc[i].y += z.y;
                } else {  // DST_ORIENT
                    if (s == 0) acc[i] = z;
                    else acc2[i] = z;
                }
            }
        }
        __syncthreads();
    }

    if (DST == DST_VOLUME) return;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < nel) {
            int row, n;
            split_index(tid, i, nthr, H, inv_H, row, n);
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
                int b0 = (int)floor(t0) % N;
                int b1 = (int)floor(t1) % N;
                if (b0 < 0) b0 += N;
                if (b1 < 0) b1 += N;
                const uint16_t packed = (uint16_t)((unsigned)b0 | ((unsigned)b1 << 8));
                *reinterpret_cast<uint16_t*>(rmap + p) = packed;
            }
        }
    }
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

template <class R>
__global__ __launch_bounds__(64) void k_precompute(R* __restrict__ Ptab, int M, int N, int Q, int Qs,
                                                   double beta, double T, int nsteps, int scheme,
                                                   double scale) {
    extern __shared__ double sm[];
    const int h = N / 2;
    const int hh = h * h;
    double* A = sm;          // generator block
    double* Bs = A + hh;     // base / result of the solve
    double* Rs = Bs + hh;    // running product
    double* Ts = Rs + hh;    // temporary
    double* W = Ts + hh;     // h x 2h augmented matrix
    double* pot = W + 2 * hh;
    const int tid = threadIdx.x;
    const int lx = blockIdx.x / Q;
    const int ly = blockIdx.x - lx * Q;
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
    const int E = 2 * Eh;
    for (int blk = 0; blk < 2; ++blk) {
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
            for (int idx = tid; idx < hh; idx += 64) {
                const int i = idx / h;
                const int j = idx - i * h;
                Bs[idx] = W[i * 2 * h + h + j];
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
        R* dst = Ptab + (size_t)lx * E * Qs + ly;
        for (int idx = tid; idx < hh; idx += 64) {
            const int i = idx / h;
            const int j = idx - i * h;
            if (j >= i) {
                const int e = blk * Eh + i * h - i * (i - 1) / 2 + (j - i);
                const double v = 0.5 * (Rs[i * h + j] + Rs[j * h + i]) * scale;
                dst[(size_t)e * Qs] = (R)v;
            }
        }
        __syncthreads();
    }
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
    const bool same = g.rows == c.rows && g.row_threads == c.row_threads && g.row_ept == 8 && c.row_ept == 8 &&
                      g.cols == c.cols && g.col_threads == c.col_threads && g.col_ept == 8 && c.col_ept == 8 &&
                      g.tw_full == 1 && c.tw_full == 1 && g.tw_full_col == 0;
    return same ? M : 0;
}

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
    const size_t lds = tw_bytes<R>(M, g.tw_full != 0) + (size_t)lds_padded_size(g.rows * (M / 2 + 2)) * sizeof(C2<R>);
#define SE2N_ROWFWD(S, E, W, MSV)                                                                          \
    hipLaunchKernelGGL((k_row_fwd<R, S, E, W, MSV>), grid, dim3(g.row_threads), lds, st, f, mask, rmap, vol,    \
                       spec, M, nslices, g.row_slices, g.rows, g.xcd_pair, planH, tw)
#define SE2N_ROWFWD_E(S)                                                    \
    if (static_size<R>(M, g) == 2048) SE2N_ROWFWD(S, 8, true, kStatic<R> ? 2048 : 0);        \
    else if (static_size<R>(M, g) == 1024) SE2N_ROWFWD(S, 8, true, kStatic<R> ? 1024 : 0);   \
    else if (static_size<R>(M, g) == 512) SE2N_ROWFWD(S, 8, true, kStatic<R> ? 512 : 0);     \
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
                          const FftPlan& planM, const C2<R>* tw, hipStream_t st) {
    dim3 grid((unsigned)((ncols + g.cols - 1) / g.cols));
    const size_t lds = tw_bytes<R>(M, g.tw_full_col != 0) + (size_t)lds_padded_size(g.cols * M) * sizeof(C2<R>);
#define SE2N_COL(I, E, W, MSV)                                                                                 \
    hipLaunchKernelGGL((k_col_fft<R, I, E, W, MSV>), grid, dim3(g.col_threads), lds, st, spec, ncols, M, g.cols, planM, \
                       tw)
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

template <class R>
hipError_t launch_row_inv(int dst, const C2<R>* spec, R* out, typename Enc<R>::U* enc, uint8_t* rmap,
                          int M, int nslices, int N, R out_scale, const LaunchGeom& g,
                          int slices_per_group, const FftPlan& planH, const C2<R>* tw, hipStream_t st) {
    const int groups = (nslices + slices_per_group - 1) / slices_per_group;
    dim3 grid((M / g.rows) * groups);
    const size_t lds = tw_bytes<R>(M, g.tw_full != 0) + (size_t)lds_padded_size(g.rows * (M / 2 + 2)) * sizeof(C2<R>);
#define SE2N_ROWINV(D, E, W, MSV)                                                                            \
    hipLaunchKernelGGL((k_row_inv<R, D, E, W, MSV>), grid, dim3(g.row_threads), lds, st, spec, out, enc, rmap,   \
                       M, nslices, slices_per_group, g.rows, g.xcd_pair, N, out_scale, planH, tw)
#define SE2N_ROWINV_E(D)                                                    \
    if (static_size<R>(M, g) == 2048) SE2N_ROWINV(D, 8, true, kStatic<R> ? 2048 : 0);        \
    else if (static_size<R>(M, g) == 1024) SE2N_ROWINV(D, 8, true, kStatic<R> ? 1024 : 0);   \
    else if (static_size<R>(M, g) == 512) SE2N_ROWINV(D, 8, true, kStatic<R> ? 512 : 0);     \
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
                             hipStream_t st) {
    const int Q = M / 4 + 1;
    const int h = N / 2;
    const size_t lds = (size_t)(6 * h * h + h) * sizeof(double);
    const double scale = 1.0 / (2.0 * (double)M * (double)M);
    hipLaunchKernelGGL((k_precompute<R>), dim3((unsigned)(Q * Q)), dim3(64), lds, st, Ptab, M, N, Q,
                       table_stride<R>(M), beta,
                       T, nsteps, scheme, scale);
    return hipGetLastError();
}

#define SE2N_INSTANTIATE(R)                                                                             \
    template hipError_t launch_row_fwd<R>(int, const R*, const uint8_t*, const uint8_t*, const R*,     \
                                          C2<R>*, int, int, const LaunchGeom&, const FftPlan&,         \
                                          const C2<R>*, hipStream_t);                                  \
    template hipError_t launch_col_fft<R>(bool, C2<R>*, long, int, const LaunchGeom&, const FftPlan&,  \
                                          const C2<R>*, hipStream_t);                                  \
    template hipError_t launch_col_orient<R>(C2<R>*, int, const LaunchGeom&, const FftPlan&,           \
                                             const C2<R>*, double, hipStream_t);                       \
    template hipError_t launch_row_inv<R>(int, const C2<R>*, R*, typename Enc<R>::U*, uint8_t*, int,   \
                                          int, int, R, const LaunchGeom&, int, const FftPlan&,         \
                                          const C2<R>*, hipStream_t);                                  \
    template hipError_t launch_fill_enc<R>(typename Enc<R>::U*, long, hipStream_t);                    \
    template hipError_t launch_decode_enc<R>(const typename Enc<R>::U*, R*, long, hipStream_t);        \
    template hipError_t launch_lift<R>(const R*, const uint8_t*, const uint8_t*, R*, int, int,         \
                                       hipStream_t);                                                   \
    template hipError_t launch_project<R>(const R*, R*, int, int, bool, hipStream_t);                  \
    template hipError_t launch_precompute<R>(R*, int, int, double, double, int, int, hipStream_t);

SE2N_INSTANTIATE(float)
SE2N_INSTANTIATE(double)

}  // namespace se2n
