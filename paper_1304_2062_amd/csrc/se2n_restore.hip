// Kernels of the restoration heuristics (Sec. "Heuristic complements",
// subsections "Static restoration (SR)" and "Dynamic restoration (DR)").
//
// Between two integration intervals the state is brought to real space as a
// volume vol[r][y][x]; at every pixel of the good set G its orientations are
// multiplied by one factor
//     sigma = (eps h_ref + (1 - eps) h) / h,   h = max_r vol[r][y][x],
// where h_ref is h(x, y, 0) (SR; DR for the initially good pixels) or the
// value h had when the pixel joined G (DR).  Pixels with h <= 0 are left
// unchanged (sigma is undefined there).  DR first grows G: a bad pixel with a
// good 8-neighbour joins when h is larger than the mean of h over the bad
// pixels of its 3x3 neighbourhood (itself included; periodic grid).
//
// All kernels are one thread per pixel; the volume is read and written with
// the pixel index fastest, so every slice access of a wavefront is one
// contiguous run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_internal.hpp"

namespace se2n {

namespace {

// h_ref of an initially good pixel: the maximum over orientations of the
// lifted image, which holds f(1 - mask) in one slice and zero elsewhere.
template <class R>
__device__ __forceinline__ R lift_max(R f) {
    return f > R(0) ? f : R(0);
}

// A pixel's N orientations, loaded into registers with every load issued
// before the first is used (N <= 64; the slices are MM apart, and
// consecutive threads read consecutive pixels of each slice).
template <class R>
struct PixelVec {
    R v[64];
    __device__ __forceinline__ void load(const R* __restrict__ vol, long i, long MM, int N) {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < N) v[r] = vol[(size_t)r * MM + i];
    }
    __device__ __forceinline__ R max(int N) const {
        R h = v[0];
#pragma unroll
        for (int r = 1; r < 64; ++r)
            if (r < N) h = fmax(h, v[r]);
        return h;
    }
    __device__ __forceinline__ void store_scaled(R* __restrict__ vol, long i, long MM, int N, R s) const {
#pragma unroll
        for (int r = 0; r < 64; ++r)
            if (r < N) vol[(size_t)r * MM + i] = v[r] * s;
    }
};

// SR: G is the set of known pixels, h_ref = max(f, 0) there.
template <class R>
__global__ __launch_bounds__(256) void k_sr_mix(R* __restrict__ vol, const R* __restrict__ f,
                                                const uint8_t* __restrict__ mask, R eps, long MM, int N) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MM || mask[i]) return;
    PixelVec<R> p;
    p.load(vol, i, MM, N);
    const R h = p.max(N);
    if (!(h > R(0))) return;
    const R s = (eps * lift_max(f[i]) + (R(1) - eps) * h) / h;
    p.store_scaled(vol, i, MM, N, s);
}

// DR, set-up: join = 0 on known pixels (good from the start), -1 on missing
// ones; h_ref = max(f, 0) on known pixels.
template <class R>
__global__ void k_dr_init(int16_t* __restrict__ join, R* __restrict__ href, const R* __restrict__ f,
                          const uint8_t* __restrict__ mask, long MM) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MM) return;
    const bool bad = mask[i] != 0;
    join[i] = bad ? int16_t(-1) : int16_t(0);
    href[i] = bad ? R(0) : lift_max(f[i]);
}

// DR: h = max over orientations at every pixel (the growth rule needs the
// neighbours' values before any pixel is mixed).
template <class R>
__global__ __launch_bounds__(256) void k_dr_max(const R* __restrict__ vol, R* __restrict__ h, long MM, int N) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MM) return;
    PixelVec<R> p;
    p.load(vol, i, MM, N);
    h[i] = p.max(N);
}

// DR at mesh point `step`: grow G, then mix.  A pixel q was good before this
// step iff 0 <= join[q] < step; pixels that join now write join = step, so a
// neighbour reading the map concurrently still sees them as bad, as the rule
// (simultaneous update from G_{i-1}) requires.  The mean is summed in the
// order (dy, dx) = (-1, -1), (-1, 0), ..., (1, 1).
template <class R>
__global__ __launch_bounds__(256) void k_dr_grow_mix(R* __restrict__ vol, const R* __restrict__ h, int16_t* __restrict__ join,
                              R* __restrict__ href, R eps, int step, int M, int N) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= M) return;
    const long MM = (long)M * M;
    const long i = (long)y * M + x;
    const int jp = join[i];
    bool good = jp >= 0 && jp < step;
    const R hp = h[i];
    if (!good) {
        bool near_good = false;
        R s = R(0);
        int c = 0;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy < 0 ? M - 1 : (y + dy >= M ? 0 : y + dy);
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx < 0 ? M - 1 : (x + dx >= M ? 0 : x + dx);
                const long q = (long)yy * M + xx;
                const int jq = join[q];
                const bool gq = jq >= 0 && jq < step;
                if (gq) {
                    near_good = true;
                } else {
                    s += h[q];
                    ++c;
                }
            }
        }
        if (near_good && hp > s / (R)c) {
            join[i] = (int16_t)step;
            href[i] = hp;
            good = true;
        }
    }
    if (!good || !(hp > R(0))) return;
    const R sg = (eps * href[i] + (R(1) - eps) * hp) / hp;
    PixelVec<R> p;
    p.load(vol, i, MM, N);
    p.store_scaled(vol, i, MM, N, sg);
}

}  // namespace

template <class R>
hipError_t launch_sr_mix(R* vol, const R* f, const uint8_t* mask, double eps, int M, int N, hipStream_t st) {
    const long MM = (long)M * M;
    hipLaunchKernelGGL((k_sr_mix<R>), dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, vol, f, mask, (R)eps, MM,
                       N);
    return hipGetLastError();
}

template <class R>
hipError_t launch_dr_init(int16_t* join, R* href, const R* f, const uint8_t* mask, int M, hipStream_t st) {
    const long MM = (long)M * M;
    hipLaunchKernelGGL((k_dr_init<R>), dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, join, href, f, mask, MM);
    return hipGetLastError();
}

template <class R>
hipError_t launch_dr_step(R* vol, R* h, int16_t* join, R* href, double eps, int step, int M, int N, hipStream_t st) {
    const long MM = (long)M * M;
    hipLaunchKernelGGL((k_dr_max<R>), dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, vol, h, MM, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bx = M < 256 ? M : 256;
    hipLaunchKernelGGL((k_dr_grow_mix<R>), dim3((unsigned)((M + bx - 1) / bx), (unsigned)M), dim3(bx), 0, st, vol, h,
                       join, href, (R)eps, step, M, N);
    return hipGetLastError();
}

#define SE2N_RESTORE_INSTANTIATE(R)                                                                          \
    template hipError_t launch_sr_mix<R>(R*, const R*, const uint8_t*, double, int, int, hipStream_t);      \
    template hipError_t launch_dr_init<R>(int16_t*, R*, const R*, const uint8_t*, int, hipStream_t);       \
    template hipError_t launch_dr_step<R>(R*, R*, int16_t*, R*, double, int, int, int, hipStream_t);
SE2N_RESTORE_INSTANTIATE(float)
SE2N_RESTORE_INSTANTIATE(double)
#undef SE2N_RESTORE_INSTANTIATE

}  // namespace se2n
