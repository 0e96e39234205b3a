// Per-mode propagation kernel of the semi-discrete SE(2,N) diffusion: one
// template instance per even orientation count N in [4, 64].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"
#include "se2n_passes.hpp"

namespace se2n {

template <class R, int N, int CLS, int WAVES>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_solve(
    C2<R>* __restrict__ spec, const R* __restrict__ P, int M, int Q, int FS, int zfill) {
    extern __shared__ unsigned char smem_raw[];
    // Workgroups go to the eight XCDs round-robin.  All class blocks of one lx
    // run on XCD lx mod 8, one after another: adjacent blocks share the cache
    // lines at the ends of their mirrored (descending) ky runs, which then
    // come from that XCD's L2 once.  Interleaving lx over the XCDs, rather
    // than giving each a band of lx, keeps their work even: the negligible
    // classes, whose modes are not read, gather at large lx.  The grid is
    // 8 * ceil(Q/8) * nb; workgroups past the last lx return at once.
    const int nb = (Q + CLS - 1) / CLS;
    const int s = blockIdx.x >> 3;
    const int row = s / nb;
    const int lx = (int)(blockIdx.x & 7) + 8 * row;
    if (lx >= Q) return;
    solve_tile<R, N, CLS>(spec, P, M, Q, FS, lx, (s - row * nb) * CLS, reinterpret_cast<R*>(smem_raw),
                          threadIdx.x, zfill != 0);
}

template <class R, int N>
static hipError_t launch_solve_n(C2<R>* spec, const R* P, int M, hipStream_t st, bool zfill) {
    constexpr int CLS = solve_cls<R, N>();
    // occupancy target: 4 waves/SIMD (<= 128 VGPRs) while a lane's half
    // vector and accumulator fit, else 2 (<= 256 VGPRs) rather than spill
    constexpr int WAVES = (N * (int)sizeof(R)) <= 160 ? 4 : 2;
    const int Q = M / 4 + 1;
    const dim3 grid((unsigned)(8 * ((Q + 7) / 8) * ((Q + CLS - 1) / CLS)));
    const int threads = 16 * CLS < 512 ? 16 * CLS : 512;  // the kernel's NT
    const size_t lds = (size_t)solve_lds_stride(N, (int)sizeof(R)) * CLS * sizeof(R);
    hipLaunchKernelGGL((k_solve<R, N, CLS, WAVES>), grid, dim3(threads), lds, st, spec, P, M, Q,
                       flag_stride(M), zfill ? 1 : 0);
    return hipGetLastError();
}

// Odd N: the propagator of class (lx, ly) is one symmetric N x N matrix,
// stored as its packed upper triangle (scaled by the inverse FFT's 1/M^2).
// One workgroup per class; thread (member m, orientation r) of its up to 8
// members (kx in {lx, M/2 - lx}, ky in {ly, M/2 - ly, M/2 + ly, M - ly})
// stages x_r of its member in LDS and forms y_r = sum_c P[r][c] x_c.  The
// members with ky > M/2 (s_ky < 0) see the class potential with r -> -r:
// for them y_r = sum_c P[-r][-c] x_c.  Negligible classes: zeros (zfill) or
// nothing.  Odd N is a correctness path (no p/q split exists), not a tuned one.
template <class R>
__global__ __launch_bounds__(512) void k_solve_odd(C2<R>* __restrict__ spec, const R* __restrict__ P, int M, int N,
                                                   int Q, int FS, int zfill) {
    extern __shared__ unsigned char smem_raw[];
    C2<R>* xs = reinterpret_cast<C2<R>*>(smem_raw);  // [8][N]
    const int lx = blockIdx.x / Q;
    const int ly = blockIdx.x - lx * Q;
    const int H = M / 2;
    const int t = threadIdx.x;
    const int m = t / N;
    const int r = t - m * N;
    const int a = m >> 2, b = m & 3;
    bool live = m < 8;
    live = live && !(a == 1 && 2 * lx == H);
    live = live && !(ly == 0 && b >= 2);
    live = live && !(2 * ly == H && (b & 1));
    const int kx = a ? H - lx : lx;
    const int ky = b == 0 ? ly : (b == 1 ? H - ly : (b == 2 ? H + ly : M - ly));
    const size_t plane = (size_t)(H + 1) * M;
    C2<R>* col = spec + (size_t)kx * M + (live ? ky : 0);
    // (odd N: no shared slots, slot lx Q + ly)
    const uint8_t* flags = reinterpret_cast<const uint8_t*>(P + table_slots(M, N) * table_class_stride(N, sizeof(R)));
    if (flags[(size_t)lx * FS + ly]) {
        if (live && zfill) col[(size_t)r * plane] = cmk<R>(R(0), R(0));
        return;
    }
    if (live) xs[m * N + r] = col[(size_t)r * plane];
    __syncthreads();
    if (!live) return;
    const R* Pc = P + table_slot(lx, ly, Q, N) * table_class_stride(N, sizeof(R));
    const bool perm = b >= 2;
    const int rr = perm ? (N - r) % N : r;
    C2<R> acc = cmk<R>(R(0), R(0));
    for (int c = 0; c < N; ++c) {
        const int cc = perm ? (N - c) % N : c;
        const int i = rr < cc ? rr : cc, j = rr < cc ? cc : rr;
        const R p = Pc[i * N - i * (i - 1) / 2 + (j - i)];
        const C2<R> x = xs[m * N + c];
        acc.x += p * x.x;
        acc.y += p * x.y;
    }
    col[(size_t)r * plane] = acc;
}

template <class R>
static hipError_t launch_solve_odd(C2<R>* spec, const R* P, int M, int N, hipStream_t st, bool zfill) {
    const int Q = M / 4 + 1;
    const int threads = (8 * N + 63) / 64 * 64;
    hipLaunchKernelGGL((k_solve_odd<R>), dim3((unsigned)(Q * Q)), dim3(threads), 8 * N * sizeof(C2<R>), st, spec, P,
                       M, N, Q, flag_stride(M), zfill ? 1 : 0);
    return hipGetLastError();
}

template <class R>
hipError_t launch_solve(C2<R>* spec, const R* P, int M, int N, hipStream_t st, bool zfill) {
    if (N & 1) return launch_solve_odd<R>(spec, P, M, N, st, zfill);
    switch (N) {
#define SE2N_CASE(n) \
    case n: return launch_solve_n<R, n>(spec, P, M, st, zfill);
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

template hipError_t launch_solve<float>(C2<float>*, const float*, int, int, hipStream_t, bool);
template hipError_t launch_solve<double>(C2<double>*, const double*, int, int, hipStream_t, bool);

}  // namespace se2n
