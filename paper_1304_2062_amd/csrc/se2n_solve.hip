// Per-mode propagation kernel of the semi-discrete SE(2,N) diffusion: one
// template instance per even orientation count N in [4, 64].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"

namespace se2n {

// ---------------------------------------------------------------------------
// Per-mode solve: psi_hat(kx,ky) <- P(kx,ky) psi_hat(kx,ky).
// ---------------------------------------------------------------------------
// The potential M (cos e_r s_kx + sin e_r s_ky)^2 has period N/2 in r, so in
// the basis p_j = x_j + x_{j+N/2}, q_j = x_j - x_{j+N/2} (j < N/2) the N x N
// propagator is two symmetric N/2 x N/2 blocks (periodic and antiperiodic
// coupling).  The table holds, per frequency class (lx, ly) with
// |s_kx| = sin(2 pi lx/M), |s_ky| = sin(2 pi ly/M), lx, ly in [0, M/4], the
// packed upper triangles of both blocks, scaled by 1/(2 M^2), laid out as
// P[lx][element][ly].
//
// The members of class (lx, ly) in the half spectrum are kx in {lx, M/2-lx}
// and ky in {ly, M/2-ly, M/2+ly, M-ly}.  Where s_kx s_ky < 0 (ky > M/2) the
// potential is the class potential with r -> -r, so the propagator is the
// class one conjugated by that permutation: the kernel loads and stores
// through the mirrored orientation index.
//
// A workgroup takes one lx and CLS consecutive ly, stages their propagators
// in LDS once (a contiguous row of CLS values per element), and applies them
// to all 8 members of each class.  A wavefront handles one member for 64
// consecutive classes, i.e. 64 consecutive (or reversed) ky of one column, so
// every orientation plane is read and written in whole 512-byte runs.
template <class R, int N, int CLS>
__global__ __launch_bounds__(256) void k_solve(C2<R>* __restrict__ spec, const R* __restrict__ P, int M,
                                               int Q) {
    constexpr int h = N / 2;
    constexpr int Eh = h * (h + 1) / 2;
    constexpr int E = 2 * Eh;
    extern __shared__ unsigned char smem_raw[];
    R* Ps = reinterpret_cast<R*>(smem_raw);
    const int H = M >> 1;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lx = blockIdx.y;
    const int ly0 = blockIdx.x * CLS;
    const int ncls = min(CLS, Q - ly0);
    const R* __restrict__ src = P + (size_t)lx * E * Q + ly0;
    for (int i = tid; i < E * CLS; i += nthr) {
        const int e = i / CLS;
        const int c = i - e * CLS;
        Ps[i] = c < ncls ? src[(size_t)e * Q + c] : R(0);
    }
    __syncthreads();
    const size_t plane = (size_t)(H + 1) * M;
    for (int item = tid; item < 8 * CLS; item += nthr) {
        const int m = item / CLS;
        const int c = item - m * CLS;
        if (c >= ncls) continue;
        const int ly = ly0 + c;
        const int a = m >> 2;
        const int b = m & 3;
        if (a == 1 && 2 * lx == H) continue;              // kx = M/4 is its own mirror
        if (ly == 0 && b >= 2) continue;                  // ky in {0, M/2} only
        if (2 * ly == H && (b & 1)) continue;             // ky in {M/4, 3M/4} only
        const int kx = a ? H - lx : lx;
        int ky = b == 0 ? ly : (b == 1 ? H - ly : (b == 2 ? H + ly : M - ly));
        if (ky == M) ky = 0;
        const bool perm = ky > H;
        C2<R>* base = spec + (size_t)kx * M + ky;
        const R* Pc = Ps + c;

        C2<R> p[h], q[h];
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int a0 = perm ? (j == 0 ? 0 : N - j) : j;
            const int a1 = perm ? (N - j - h) % N : j + h;
            const C2<R> x0 = base[a0 * plane];
            const C2<R> x1 = base[a1 * plane];
            p[j] = cadd<R>(x0, x1);
            q[j] = csub<R>(x0, x1);
        }
        C2<R> yp[h], yq[h];
#pragma unroll
        for (int j = 0; j < h; ++j) {
            yp[j] = cmk<R>(R(0), R(0));
            yq[j] = cmk<R>(R(0), R(0));
        }
        {
            int e = 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
#pragma unroll
                for (int j = i; j < h; ++j) {
                    const R w = Pc[e * CLS];
                    yp[i].x += w * p[j].x;
                    yp[i].y += w * p[j].y;
                    if (j != i) {
                        yp[j].x += w * p[i].x;
                        yp[j].y += w * p[i].y;
                    }
                    ++e;
                }
            }
#pragma unroll
            for (int i = 0; i < h; ++i) {
#pragma unroll
                for (int j = i; j < h; ++j) {
                    const R w = Pc[e * CLS];
                    yq[i].x += w * q[j].x;
                    yq[i].y += w * q[j].y;
                    if (j != i) {
                        yq[j].x += w * q[i].x;
                        yq[j].y += w * q[i].y;
                    }
                    ++e;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int a0 = perm ? (j == 0 ? 0 : N - j) : j;
            const int a1 = perm ? (N - j - h) % N : j + h;
            base[a0 * plane] = cadd<R>(yp[j], yq[j]);
            base[a1 * plane] = csub<R>(yp[j], yq[j]);
        }
    }
}

// Classes per workgroup: the largest power of two <= 64 whose propagators fit
// in 72 KB of LDS.
template <class R, int N>
constexpr int solve_cls() {
    constexpr int h = N / 2;
    constexpr int E = h * (h + 1);
    int c = 64;
    while (c > 1 && (long)E * c * (long)sizeof(R) > 72 * 1024) c >>= 1;
    return c;
}

template <class R, int N>
static hipError_t launch_solve_n(C2<R>* spec, const R* P, int M, hipStream_t st) {
    constexpr int CLS = solve_cls<R, N>();
    constexpr int h = N / 2;
    constexpr int E = h * (h + 1);
    const int Q = M / 4 + 1;
    dim3 grid((Q + CLS - 1) / CLS, Q);
    const int threads = 8 * CLS < 256 ? 8 * CLS : 256;
    const size_t lds = (size_t)E * CLS * sizeof(R);
    hipLaunchKernelGGL((k_solve<R, N, CLS>), grid, dim3(threads), lds, st, spec, P, M, Q);
    return hipGetLastError();
}

template <class R>
hipError_t launch_solve(C2<R>* spec, const R* P, int M, int N, hipStream_t st) {
    switch (N) {
#define SE2N_CASE(n) \
    case n: return launch_solve_n<R, n>(spec, P, M, st);
        SE2N_CASE(4) SE2N_CASE(6) SE2N_CASE(8) SE2N_CASE(10) SE2N_CASE(12) SE2N_CASE(14)
        SE2N_CASE(16) SE2N_CASE(18) SE2N_CASE(20) SE2N_CASE(22) SE2N_CASE(24) SE2N_CASE(26)
        SE2N_CASE(28) SE2N_CASE(30) SE2N_CASE(32) SE2N_CASE(34) SE2N_CASE(36) SE2N_CASE(38)
        SE2N_CASE(40) SE2N_CASE(42) SE2N_CASE(44) SE2N_CASE(46) SE2N_CASE(48) SE2N_CASE(50)
        SE2N_CASE(52) SE2N_CASE(54) SE2N_CASE(56) SE2N_CASE(58) SE2N_CASE(60) SE2N_CASE(62)
        SE2N_CASE(64)
#undef SE2N_CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_solve<float>(C2<float>*, const float*, int, int, hipStream_t);
template hipError_t launch_solve<double>(C2<double>*, const double*, int, int, hipStream_t);

}  // namespace se2n
