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
// P[lx][element][ly] so that neighbouring ky read neighbouring addresses.
// Where s_kx s_ky < 0 the mode's potential is the class potential with
// r -> -r, so the propagator is the class one conjugated by that permutation:
// the kernel loads and stores through the mirrored orientation index.
template <class R, int N>
__global__ __launch_bounds__(256) void k_solve(C2<R>* __restrict__ spec, const R* __restrict__ P,
                                               int M, int Q) {
    constexpr int h = N / 2;
    constexpr int Eh = h * (h + 1) / 2;
    constexpr int E = 2 * Eh;
    const int H = M >> 1;
    const int K = H + 1;
    const int M4 = M >> 2;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)K * M) return;
    const int kx = (int)(idx / M);
    const int ky = (int)(idx - (long)kx * M);
    const int lx = kx <= M4 ? kx : H - kx;
    const int kp = ky < H ? ky : ky - H;
    const int ly = kp <= M4 ? kp : H - kp;
    const bool perm = ky > H;
    const R* __restrict__ Pc = P + (size_t)lx * E * Q + ly;
    const size_t plane = (size_t)K * M;
    C2<R>* base = spec + (size_t)kx * M + ky;

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
                const R w = Pc[(size_t)e * Q];
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
                const R w = Pc[(size_t)e * Q];
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

template <class R, int N>
static hipError_t launch_solve_n(C2<R>* spec, const R* P, int M, hipStream_t st) {
    const long modes = (long)(M / 2 + 1) * M;
    dim3 grid((unsigned)((modes + 255) / 256));
    hipLaunchKernelGGL((k_solve<R, N>), grid, dim3(256), 0, st, spec, P, M, M / 4 + 1);
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
