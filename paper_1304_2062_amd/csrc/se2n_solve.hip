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
// P[lx][element][ly] with a line-aligned ly stride.
//
// The members of class (lx, ly) in the half spectrum are kx in {lx, M/2-lx}
// and ky in {ly, M/2-ly, M/2+ly, M-ly}.  Where s_kx s_ky < 0 (ky > M/2) the
// potential is the class potential with r -> -r, so the propagator is the
// class one conjugated by that permutation: the kernel loads and stores
// through the mirrored orientation index.
//
// A workgroup takes one lx and CLS consecutive ly, stages their propagators
// in LDS once (a contiguous row of CLS values per element), and applies them
// to all 8 members of each class.  Each mode is handled by a pair of adjacent
// lanes: the even lane loads x_j and the odd lane x_{j+N/2} (j < N/2); one
// DPP swap gives the even lane p = x_j + x_{j+N/2} and the odd lane
// q = x_j - x_{j+N/2}; each applies its block (periodic / antiperiodic) and a
// second swap forms x'_j = y_p + y_q (even) and x'_{j+N/2} = y_p - y_q (odd).
// A wavefront covers one member for 32 consecutive classes, i.e. 32
// consecutive (or reversed) ky of one column per orientation plane.
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

template <class R, int N, int CLS, int WAVES>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_solve(C2<R>* __restrict__ spec, const R* __restrict__ P, int M,
                                               int Q, int Qs) {
    constexpr int h = N / 2;
    constexpr int Eh = h * (h + 1) / 2;
    constexpr int E = 2 * Eh;
    extern __shared__ unsigned char smem_raw[];
    R* Ps = reinterpret_cast<R*>(smem_raw);
    const int H = M >> 1;
    constexpr int NT = 16 * CLS < 512 ? 16 * CLS : 512;  // blockDim.x: two lanes per mode
    const int tid = threadIdx.x;
    const int nthr = NT;
    // adjacent class blocks of one lx share the cache lines at the ends of
    // their mirrored (reversed) ky runs: keep them on one XCD
    const int nb = (Q + CLS - 1) / CLS;
    const int blk = xcd_contiguous(blockIdx.x, gridDim.x);
    const int lx = blk / nb;
    const int ly0 = (blk - lx * nb) * CLS;
    const int ncls = min(CLS, Q - ly0);
    // Stage the block's propagators: 16-byte chunks, every load of a thread
    // issued before the first is waited on.  A chunk that starts inside the
    // block's classes lies inside the line-padded row; classes past the last
    // one are zeroed.
    {
        constexpr int VEC = 16 / (int)sizeof(R);
        typedef R vec_t __attribute__((ext_vector_type(VEC)));
        constexpr int CH = E * CLS / VEC;  // CLS >= 8 is a multiple of VEC
        constexpr int NST = (CH + NT - 1) / NT;
        constexpr int BATCH = NST < 8 ? NST : 8;  // loads in flight per thread
        const R* __restrict__ src = P + (size_t)lx * E * Qs + ly0;
        for (int k0 = 0; k0 < NST; k0 += BATCH) {
        vec_t v[BATCH];
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int i = tid + (k0 + k) * NT;
            const int e = i / (CLS / VEC);
            const int c0 = (i - e * (CLS / VEC)) * VEC;
            v[k] = vec_t(0);
            if (i < CH && c0 < ncls) v[k] = *reinterpret_cast<const vec_t*>(src + (size_t)e * Qs + c0);
#pragma unroll
            for (int q = 0; q < VEC; ++q)
                if (c0 + q >= ncls) v[k][q] = R(0);
        }
#pragma unroll
        for (int k = 0; k < BATCH; ++k) {
            const int i = tid + (k0 + k) * NT;
            if (i < CH) reinterpret_cast<vec_t*>(Ps)[i] = v[k];
        }
        }
    }
    __syncthreads();
    const size_t plane = (size_t)(H + 1) * M;
    const int odd = tid & 1;
    // A wavefront holds 32 pairs; with CLS >= 32 they all belong to one member,
    // so the member, its column kx and its orientation mirroring are uniform
    // across the wavefront and the plane addresses live in scalar registers.
    constexpr bool UNIFORM = CLS >= 32;
    // every lane of a pair runs the same iterations, so the swaps always meet
#pragma unroll 1
    for (int pair = tid >> 1; pair < 8 * CLS; pair += nthr >> 1) {
        int m = pair / CLS;
        if (UNIFORM) m = __builtin_amdgcn_readfirstlane(m);
        const int c = pair - m * CLS;
        const int ly = ly0 + c;
        const int a = m >> 2;
        const int b = m & 3;
        bool live = c < ncls;
        live = live && !(a == 1 && 2 * lx == H);           // kx = M/4 is its own mirror
        live = live && !(ly == 0 && b >= 2);               // ky in {0, M/2} only
        live = live && !(2 * ly == H && (b & 1));          // ky in {M/4, 3M/4} only
        const int kx = a ? H - lx : lx;
        int ky = b == 0 ? ly : (b == 1 ? H - ly : (b == 2 ? H + ly : M - ly));
        if (!live) ky = 0;  // harmless in-range address; nothing is stored
        // s_ky < 0 exactly for the live members b = 2, 3 (ky in (M/2, M))
        const bool perm = b >= 2;
        C2<R>* colbase = spec + (size_t)kx * M;
        const R* Pc = Ps + (size_t)odd * Eh * CLS + c;

        // this lane's half of the orientation vector (every address is valid;
        // dead lanes read row 0 and discard it)
        C2<R> x[h];
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const int r0 = j, r1 = j + h;
            const int a0 = perm ? (r0 == 0 ? 0 : N - r0) : r0;
            const int a1 = perm ? N - r1 : r1;
            const C2<R>* pl0 = colbase + (size_t)a0 * plane;  // wave-uniform
            const C2<R>* pl1 = colbase + (size_t)a1 * plane;
            const C2<R> v = odd ? pl1[ky] : pl0[ky];
            x[j].x = live ? v.x : R(0);
            x[j].y = live ? v.y : R(0);
        }
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
                    const R w = Pc[e * CLS];
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
        if (live) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const int r0 = j, r1 = j + h;
                const int a0 = perm ? (r0 == 0 ? 0 : N - r0) : r0;
                const int a1 = perm ? N - r1 : r1;
                C2<R>* pl = colbase + (size_t)(odd ? a1 : a0) * plane;
                pl[ky] = y[j];
            }
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
    // occupancy target: 4 waves/SIMD (<= 128 VGPRs) while a lane's half
    // vector and accumulator fit, else 2 (<= 256 VGPRs) rather than spill
    constexpr int WAVES = (N * (int)sizeof(R)) <= 160 ? 4 : 2;
    constexpr int h = N / 2;
    constexpr int E = h * (h + 1);
    const int Q = M / 4 + 1;
    const dim3 grid((unsigned)(((Q + CLS - 1) / CLS) * Q));
    const int threads = 16 * CLS < 512 ? 16 * CLS : 512;  // the kernel's NT
    const size_t lds = (size_t)E * CLS * sizeof(R);
    hipLaunchKernelGGL((k_solve<R, N, CLS, WAVES>), grid, dim3(threads), lds, st, spec, P, M, Q,
                       table_stride<R>(M));
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
