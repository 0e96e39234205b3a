// Orientation map of the corrupted image by a separable periodic stencil:
// the tile body shared by the single-image and the batched kernels.
//
// The orientation step smooths f_c = f (1 - mask) with a Gaussian and takes
// central differences, both as Fourier multipliers on the periodic grid
// (Sec. "A final inpainting algorithm ...").  A Fourier multiplier is a
// circular convolution with its inverse DFT, and both multipliers here are
// products of an x factor and a y factor, so
//     g_x = d (*)_x g (*)_y f_c,     g_y = g (*)_x d (*)_y f_c
// with g the inverse DFT of the 1-D Gaussian factor and d that of the
// Gaussian times the central-difference symbol.  For widths where both
// kernels fall below the FP32 rounding level within a few dozen pixels the
// convolutions are short stencils; the host truncates them there (or keeps
// the whole circle for small M) and passes the taps as kernel arguments.
//
// One workgroup makes a 128 x 32 tile of bins: a vertical pass (both kernels,
// 8 rows per thread from a register window over global memory) writes the
// two partial results for the tile's columns plus the horizontal halo to
// LDS; a horizontal pass (16 columns per thread) finishes g_x and g_y and
// bins the level-line angle atan2(g_y, g_x) + pi/2 into N orientations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "se2n_internal.hpp"

namespace se2n {

constexpr int kOrientTX = 128;  // tile columns
constexpr int kOrientTY = 32;   // tile rows
constexpr int kOrientNT = 256;  // threads
constexpr int kOrientCV = 8;    // rows per vertical item
constexpr int kOrientCH = 16;   // columns per horizontal item
static_assert(kOrientTY * kOrientTX / kOrientCH == kOrientNT, "one horizontal item per thread");

// LDS row stride (floats) of the two partial results of radius RAD.
template <int RAD>
constexpr int orient_lds_stride() { return kOrientTX + 2 * RAD + 4; }
template <int RAD>
constexpr int orient_lds_floats() { return kOrientTY * orient_lds_stride<RAD>(); }

inline int orient_tiles(int M) {
    return ((M + kOrientTX - 1) / kOrientTX) * ((M + kOrientTY - 1) / kOrientTY);
}

__device__ __forceinline__ int orient_wrap(int i, int M) {
    i %= M;
    return i < 0 ? i + M : i;
}

// Bins of tile `tile` (row-major over the tiles of the image); sa and sb hold
// orient_lds_floats<RAD>() floats each.
template <int RAD>
__device__ __forceinline__ void orient_stencil_tile(const float* __restrict__ f, const uint8_t* __restrict__ mask,
                                                    uint8_t* __restrict__ rmap, int M, int N, int tile,
                                                    const OrientTaps& taps, float* sa, float* sb, int tid) {
    constexpr int NTAP = 2 * RAD + 1;
    constexpr int W = kOrientTX + 2 * RAD;  // columns of the vertical pass
    constexpr int WS = orient_lds_stride<RAD>();
    constexpr int NV = kOrientCV + 2 * RAD;
    constexpr int NH = kOrientCH + 2 * RAD;
    static_assert(W % 4 == 0 && NH % 4 == 0, "float4 rows");
    const int tiles_x = (M + kOrientTX - 1) / kOrientTX;
    const int x0 = (tile % tiles_x) * kOrientTX;
    const int y0 = (tile / tiles_x) * kOrientTY;

    for (int it = tid; it < W * (kOrientTY / kOrientCV); it += kOrientNT) {
        const int c = it % W, q = it / W;
        const int xx = orient_wrap(x0 - RAD + c, M);
        int yy = orient_wrap(y0 + q * kOrientCV - RAD, M);
        float v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const size_t o = (size_t)yy * M + xx;
            const float fv = f[o];
            v[k] = mask[o] ? 0.f : fv;
            yy = (yy + 1 == M) ? 0 : yy + 1;
        }
#pragma unroll
        for (int i = 0; i < kOrientCV; ++i) {
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int j = 0; j < NTAP; ++j) {
                a = fmaf(taps.g[j], v[i + j], a);
                if (j != RAD) b = fmaf(taps.d[j], v[i + j], b);  // d is odd: no centre tap
            }
            sa[(q * kOrientCV + i) * WS + c] = a;
            sb[(q * kOrientCV + i) * WS + c] = b;
        }
    }
    __syncthreads();

    const int y = tid / (kOrientTX / kOrientCH), cq = tid % (kOrientTX / kOrientCH);
    float gx[kOrientCH], gy[kOrientCH];
    {
        float u[NH];
        const float* row = sa + y * WS + cq * kOrientCH;
#pragma unroll
        for (int k = 0; k < NH; k += 4) {
            const float4 t = *reinterpret_cast<const float4*>(row + k);
            u[k] = t.x;
            u[k + 1] = t.y;
            u[k + 2] = t.z;
            u[k + 3] = t.w;
        }
#pragma unroll
        for (int i = 0; i < kOrientCH; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < NTAP; ++j)
                if (j != RAD) s = fmaf(taps.d[j], u[i + j], s);
            gx[i] = s;
        }
    }
    {
        float u[NH];
        const float* row = sb + y * WS + cq * kOrientCH;
#pragma unroll
        for (int k = 0; k < NH; k += 4) {
            const float4 t = *reinterpret_cast<const float4*>(row + k);
            u[k] = t.x;
            u[k + 1] = t.y;
            u[k + 2] = t.z;
            u[k + 3] = t.w;
        }
#pragma unroll
        for (int i = 0; i < kOrientCH; ++i) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < NTAP; ++j) s = fmaf(taps.g[j], u[i + j], s);
            gy[i] = s;
        }
    }

    const int py = y0 + y, px = x0 + cq * kOrientCH;
    if (py >= M || px >= M) return;
    const float two_pi = 6.283185307179586476925f;
    const float half_pi = 1.570796326794896619231f;
    uint32_t w[kOrientCH / 4];
#pragma unroll
    for (int i = 0; i < kOrientCH / 4; ++i) w[i] = 0;
#pragma unroll
    for (int i = 0; i < kOrientCH; ++i) {
        const float t = (atan2f(gy[i], gx[i]) + half_pi) * (float)N / two_pi + 0.5f;
        // atan2 lies in [-pi, pi], so floor(t) lies in [-N/4, 3N/4]: one
        // wrap of the negative values is the remainder mod N
        int b = (int)floorf(t);
        if (b < 0) b += N;
        w[i / 4] |= (uint32_t)b << (8 * (i % 4));
    }
    uint8_t* dst = rmap + (size_t)py * M + px;
    if (px + kOrientCH <= M && (M & 7) == 0) {
        // M is a multiple of 8, so each half of the run is 8-byte aligned
        reinterpret_cast<uint2*>(dst)[0] = make_uint2(w[0], w[1]);
        reinterpret_cast<uint2*>(dst)[1] = make_uint2(w[2], w[3]);
    } else {
#pragma unroll
        for (int i = 0; i < kOrientCH; ++i)
            if (px + i < M) dst[i] = (uint8_t)(w[i / 4] >> (8 * (i % 4)));
    }
}

}  // namespace se2n
