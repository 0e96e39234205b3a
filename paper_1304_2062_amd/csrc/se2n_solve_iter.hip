// Per-mode Crank-Nicolson integration, step by step (remark 2 after
// Theorem 2: Crank-Nicolson with a solver for the cyclic tridiagonal
// systems), as an alternative to applying the collapsed propagator.
//
// Every mode (kx, ky) of the half spectrum carries an N-vector x that obeys
// dx/dt = A x, A = beta L - diag(pot), pot_r = M (cos e_r s_kx + sin e_r s_ky)^2,
// s_k = sin(2 pi k / M).  The potential has period N/2 in r, so in the basis
// p_j = x_j + x_{j+N/2}, q_j = x_j - x_{j+N/2} (j < h = N/2) the system splits
// into two independent h-dimensional ones: periodic coupling for p,
// antiperiodic coupling (x_{-1} = -x_{h-1}) for q.  A pair of adjacent lanes
// holds one mode: the even lane integrates p, the odd lane q; they exchange
// halves (one DPP swap) only before the first and after the last step.
//
// One step with tau = T / n:  (I - tau A / 2) x' = (I + tau A / 2) x.  The
// left matrix is tridiagonal with diagonal d_j = 1 + tau beta + tau pot_j / 2,
// off-diagonal o = -tau beta / 2 and corners c = +-o.  It is solved as
//     B = Tm + u v^T,   u = (g, 0, .., 0, c),  v = (1, 0, .., 0, c / g),  g = -d_0,
// Tm being B without its corners and with Tm_00 = d_0 - g, Tm_{h-1,h-1} =
// d_{h-1} - c^2 / g: x' = y - ((y_0 + (c/g) y_{h-1}) / (1 + v.z)) z with
// Tm y = b, Tm z = u (Sherman-Morrison).  The factorisation of Tm, z and
// 1/(1 + v.z) depend only on the mode: they are formed once, in FP64, and the
// steps run in the plan's precision.  Real and imaginary parts are two
// right-hand sides.  The 1/(2 M^2) of the p/q recombination and the inverse
// FFT is applied with the last recombination, as the propagator table does.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_fft.hpp"
#include "se2n_internal.hpp"

namespace se2n {

namespace {

__device__ __forceinline__ float swap_lanes(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_lanes(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffff), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Modes per workgroup: 128 (256 threads, two per mode).
constexpr int kIterThreads = 256;

template <class R, int H>
__global__ __launch_bounds__(kIterThreads) void k_solve_iter(C2<R>* __restrict__ spec, int M, double beta, double tau,
                                                             int nsteps, double out_scale) {
    constexpr int N = 2 * H;
    const int tid = threadIdx.x;
    const int odd = tid & 1;
    const long nmodes = (long)(M / 2 + 1) * M;
    const long mode = (long)blockIdx.x * (kIterThreads / 2) + (tid >> 1);
    // both lanes of a pair take part in the swaps, so a pair past the last
    // mode works on mode 0 and stores nothing
    const bool live = mode < nmodes;
    const long md = live ? mode : 0;
    const int kx = (int)(md / M);
    const int ky = (int)(md - (long)kx * M);
    const size_t plane = (size_t)(M / 2 + 1) * M;
    C2<R>* base = spec + (size_t)kx * M + ky + (odd ? (size_t)H * plane : 0);

    // this lane's half of the orientation vector: x_j (even) or x_{j+H} (odd)
    R xr[H], xi[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const C2<R> v = base[(size_t)j * plane];
        xr[j] = v.x;
        xi[j] = v.y;
    }
    // p on the even lane, q on the odd one
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const R orr = swap_lanes(xr[j]);
        const R oi = swap_lanes(xi[j]);
        xr[j] = odd ? orr - xr[j] : xr[j] + orr;
        xi[j] = odd ? oi - xi[j] : xi[j] + oi;
    }

    // the mode's factors, in FP64
    const double two_pi = 6.283185307179586476925;
    const double sx = sin(two_pi * kx / M);
    const double sy = sin(two_pi * ky / M);
    const double o = -0.5 * tau * beta;       // off-diagonal of the left matrix
    const double c = odd ? -o : o;            // its corners (antiperiodic for q)
    double d[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const double e = two_pi * j / N;
        const double a = cos(e) * sx + sin(e) * sy;
        d[j] = 1.0 + tau * beta + 0.5 * tau * ((double)M * a * a);
    }
    const double g = -d[0];
    R cb[H], idn[H], cp[H], z[H];
    {
        double cpd[H], idd[H], zd[H];
        double prev_cp = 0.0, prev_w = 0.0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            double tj = d[j];
            if (j == 0) tj -= g;
            if (j == H - 1) tj -= c * c / g;
            const double den = tj - (j ? o * prev_cp : 0.0);
            idd[j] = 1.0 / den;
            cpd[j] = o * idd[j];
            // forward sweep of Tm z = u, u = (g, 0, .., 0, c)
            const double uj = (j == 0 ? g : 0.0) + (j == H - 1 ? c : 0.0);
            zd[j] = (uj - (j ? o * prev_w : 0.0)) * idd[j];
            prev_cp = cpd[j];
            prev_w = zd[j];
        }
#pragma unroll
        for (int j = H - 2; j >= 0; --j) zd[j] -= cpd[j] * zd[j + 1];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            cb[j] = (R)(2.0 - d[j]);  // diagonal of the right matrix: 1 - tau beta - tau pot / 2
            idn[j] = (R)idd[j];
            cp[j] = (R)cpd[j];
            z[j] = (R)zd[j];
        }
        const double vz = zd[0] + (c / g) * zd[H - 1];
        // stash the step's scalars in the last slot's neighbours below
        prev_cp = 1.0 / (1.0 + vz);
        prev_w = c / g;
        // (kappa, nu) kept in registers of the step loop
        const R kap = (R)prev_cp;
        const R nu = (R)prev_w;
        const R ro = (R)o;
        const R rq = (R)(-o);  // tau beta / 2, coefficient of the neighbours on the right
        const R rs = odd ? R(-1) : R(1);
        for (int s = 0; s < nsteps; ++s) {
            // b = (I + tau A / 2) x, then the forward sweep in place
            R br[H], bi[H];
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const R lr = j == 0 ? rs * xr[H - 1] : xr[j - 1];
                const R li = j == 0 ? rs * xi[H - 1] : xi[j - 1];
                const R ur = j == H - 1 ? rs * xr[0] : xr[j + 1];
                const R ui = j == H - 1 ? rs * xi[0] : xi[j + 1];
                br[j] = cb[j] * xr[j] + rq * (lr + ur);
                bi[j] = cb[j] * xi[j] + rq * (li + ui);
            }
#pragma unroll
            for (int j = 0; j < H; ++j) {
                if (j) {
                    br[j] -= ro * br[j - 1];
                    bi[j] -= ro * bi[j - 1];
                }
                br[j] *= idn[j];
                bi[j] *= idn[j];
            }
#pragma unroll
            for (int j = H - 2; j >= 0; --j) {
                br[j] -= cp[j] * br[j + 1];
                bi[j] -= cp[j] * bi[j + 1];
            }
            const R fr = (br[0] + nu * br[H - 1]) * kap;
            const R fi = (bi[0] + nu * bi[H - 1]) * kap;
#pragma unroll
            for (int j = 0; j < H; ++j) {
                xr[j] = br[j] - fr * z[j];
                xi[j] = bi[j] - fi * z[j];
            }
        }
    }

    // back to x: x_j = (p + q) / 2 (even lane), x_{j+H} = (p - q) / 2 (odd),
    // with the inverse FFT's 1/M^2
    const R sc = (R)out_scale;
#pragma unroll
    for (int j = 0; j < H; ++j) {
        const R orr = swap_lanes(xr[j]);
        const R oi = swap_lanes(xi[j]);
        const R vr = odd ? orr - xr[j] : xr[j] + orr;
        const R vi = odd ? oi - xi[j] : xi[j] + oi;
        if (live) base[(size_t)j * plane] = cmk<R>(vr * sc, vi * sc);
    }
}

template <class R, int H>
hipError_t launch_iter_h(C2<R>* spec, int M, double beta, double tau, int nsteps, hipStream_t st) {
    const long nmodes = (long)(M / 2 + 1) * M;
    const long per = kIterThreads / 2;
    const dim3 grid((unsigned)((nmodes + per - 1) / per));
    const double scale = 1.0 / (2.0 * (double)M * (double)M);
    hipLaunchKernelGGL((k_solve_iter<R, H>), grid, dim3(kIterThreads), 0, st, spec, M, beta, tau, nsteps, scale);
    return hipGetLastError();
}

}  // namespace

template <class R>
hipError_t launch_solve_iter(C2<R>* spec, int M, int N, double beta, double T, int nsteps, hipStream_t st) {
    const double tau = T / nsteps;
    switch (N / 2) {
#define SE2N_CASE(h) \
    case h: return launch_iter_h<R, h>(spec, M, beta, tau, nsteps, st);
        SE2N_CASE(2) SE2N_CASE(3) SE2N_CASE(4) SE2N_CASE(5) SE2N_CASE(6) SE2N_CASE(7) SE2N_CASE(8)
        SE2N_CASE(9) SE2N_CASE(10) SE2N_CASE(11) SE2N_CASE(12) SE2N_CASE(13) SE2N_CASE(14) SE2N_CASE(15)
        SE2N_CASE(16) SE2N_CASE(17) SE2N_CASE(18) SE2N_CASE(19) SE2N_CASE(20) SE2N_CASE(21) SE2N_CASE(22)
        SE2N_CASE(23) SE2N_CASE(24) SE2N_CASE(25) SE2N_CASE(26) SE2N_CASE(27) SE2N_CASE(28) SE2N_CASE(29)
        SE2N_CASE(30) SE2N_CASE(31) SE2N_CASE(32)
#undef SE2N_CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_solve_iter<float>(C2<float>*, int, int, double, double, int, hipStream_t);
template hipError_t launch_solve_iter<double>(C2<double>*, int, int, double, double, int, hipStream_t);

}  // namespace se2n
