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

template <class R>
hipError_t launch_solve(C2<R>* spec, const R* P, int M, int N, hipStream_t st, bool zfill) {
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
