// BF16 MFMA kernels of the learned corrector: 3x3 circular convolutions as
// implicit GEMMs on v_mfma_f32_16x16x32_bf16 (bfloat16 operands, FP32
// accumulation), their input and weight gradients, the loss and Adam.
//
// Product shape of one MFMA: D[16 x 16] += A[16 x 32] B[32 x 16] with
//   A[row][k]: lane l holds row l%16, k = 8*(l/16) .. 8*(l/16)+7
//   B[k][col]: lane l holds col l%16, the same 8 k
//   D[row][col]: lane l holds col l%16, rows 4*(l/16) .. 4*(l/16)+3
// For a conv, rows are output channels, columns pixels and k input
// channels (one tap at a time); for the weight gradient rows are output
// channels, columns input channels and k pixels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "se2n_cnn.hpp"

namespace se2n {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int C = kCnnC;
constexpr int T = kCnnTile;    // 16 x 16 output pixels per workgroup
constexpr int HT = T + 2;      // with a one-pixel halo
// LDS strides in bf16 elements, each an odd multiple of 16 bytes so that the
// 8 lanes served together by a 128-byte LDS cycle hit distinct banks.
constexpr int PS = 40;         // conv: per halo pixel (32 channels + 8)
constexpr int WS = 40;         // conv: per weight row (32 k + 8)
constexpr int GS = T * T + 8;  // weight gradient: per channel of the gradient tile
constexpr int AS = HT * T + 8; // weight gradient: per channel of one shifted input copy

__device__ __forceinline__ int wrap(int i, int M) { return i < 0 ? i + M : (i >= M ? i - M : i); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Per-image root mean square of the input volume: partial sums of squares
// over kScaleBlocks contiguous chunks, then their sum in a fixed order.
constexpr int kScaleBlocks = kCnnScaleBlocks;

__global__ __launch_bounds__(256) void k_cnn_sumsq(const float* __restrict__ psi, long n, float* __restrict__ parts);
__global__ __launch_bounds__(256) void k_cnn_scale(const float* __restrict__ parts, long n, float* __restrict__ scale);

__global__ __launch_bounds__(256) void k_cnn_pack(const float* __restrict__ psi, const float* __restrict__ scale,
                                                  bf16* __restrict__ act, int N, int M, int B) {
    const long MM = (long)M * M;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)B * 4 * MM) return;
    const long p = t % MM;
    const long q = t / MM;
    const int cb = (int)(q & 3);
    const long b = q >> 2;
    const float inv = 1.0f / scale[b];
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int c = cb * 8 + j;
        v[j] = (bf16)(c < N ? psi[(b * N + c) * MM + p] * inv : 0.0f);
    }
    *reinterpret_cast<bf16x8*>(act + (b * MM + p) * C + cb * 8) = v;
}

// One workgroup: a 16 x 16 pixel tile of one image, 4 waves of 4 rows each.
template <int EPI>
__global__ __launch_bounds__(256) void k_cnn_conv(const bf16* __restrict__ in, const bf16* __restrict__ wA,
                                                  const float* __restrict__ bias, bf16* __restrict__ act_out,
                                                  const bf16* __restrict__ mask, const float* coarse, float* out,
                                                  const float* __restrict__ scale, int N, int M) {
    __shared__ __attribute__((aligned(16))) bf16 s_in[HT * HT * PS];
    __shared__ __attribute__((aligned(16))) bf16 s_w[9 * C * WS];
    const int tid = threadIdx.x;
    const int tiles = M / T;
    const int tx = blockIdx.x % tiles;
    const int ty = (blockIdx.x / tiles) % tiles;
    const long b = blockIdx.x / (tiles * tiles);
    const int x0 = tx * T, y0 = ty * T;
    const long MM = (long)M * M;
    const bf16* inb = in + b * MM * C;

    for (int i = tid; i < 9 * C * 4; i += 256) {
        const int row = i >> 2, q = i & 3;
        *reinterpret_cast<bf16x8*>(s_w + row * WS + q * 8) = *reinterpret_cast<const bf16x8*>(wA + row * C + q * 8);
    }
    for (int i = tid; i < HT * HT * 4; i += 256) {
        const int pix = i >> 2, q = i & 3;
        const int hy = pix / HT, hx = pix - hy * HT;
        const int gy = wrap(y0 + hy - 1, M), gx = wrap(x0 + hx - 1, M);
        *reinterpret_cast<bf16x8*>(s_in + pix * PS + q * 8) =
            *reinterpret_cast<const bf16x8*>(inb + ((long)gy * M + gx) * C + q * 8);
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int col = lane & 15, kg = lane >> 4;
    // LAST: the coarse values this lane adds to, loaded while the products run
    float pre[EPI == CNN_LAST ? 4 : 1][2][4];
    if (EPI == CNN_LAST) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long p = (long)(y0 + 4 * w + r) * M + (x0 + col);
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 16 * mb + 4 * kg + i;
                    pre[r][mb][i] = c < N ? coarse[(b * N + c) * MM + p] : 0.0f;
                }
        }
    }
    f32x4 acc[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r][0] = acc[r][1] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(s_w + (tap * C + col) * WS + kg * 8);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(s_w + (tap * C + 16 + col) * WS + kg * 8);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int hy = 4 * w + r + dy + 1, hx = col + dx + 1;
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(s_in + (hy * HT + hx) * PS + kg * 8);
            acc[r][0] = mfma(a0, bv, acc[r][0]);
            acc[r][1] = mfma(a1, bv, acc[r][1]);
        }
    }

#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long p = (long)(y0 + 4 * w + r) * M + (x0 + col);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int c0 = 16 * mb + 4 * kg;
            const f32x4 v = acc[r][mb];
            if (EPI == CNN_LAST) {
                const float sc = scale[b];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = c0 + i;
                    if (c < N) {
                        const long o = (b * N + c) * MM + p;
                        out[o] = pre[r][mb][i] + sc * (v[i] + bias[c]);
                    }
                }
            } else {
                bf16x4 s;
                if (EPI == CNN_HIDDEN) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) s[i] = (bf16)fmaxf(v[i] + bias[c0 + i], 0.0f);
                } else {
                    const bf16x4 mk = *reinterpret_cast<const bf16x4*>(mask + (b * MM + p) * C + c0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) s[i] = (bf16)((float)mk[i] > 0.0f ? v[i] : 0.0f);
                }
                *reinterpret_cast<bf16x4*>(act_out + (b * MM + p) * C + c0) = s;
            }
        }
    }
}

// Weight and bias gradient partials: each workgroup sums `tpw` consecutive
// 16 x 16 tiles.  LDS holds the gradient tile transposed (channel-major) and
// three copies of the input tile with its halo, channel-major, shifted by
// dx = -1, 0, 1, so every MFMA operand is 8 consecutive pixels.  Wave w owns
// taps w, w+4 (and 8 for wave 0).
__global__ __launch_bounds__(256) void k_cnn_wgrad(const bf16* __restrict__ g, const bf16* __restrict__ a,
                                                   float* __restrict__ parts, int M, int ntiles, int tpw) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    bf16* s_g = reinterpret_cast<bf16*>(smem_raw);  // [C][GS]
    bf16* s_a = s_g + C * GS;                       // [3][C][AS]
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int col = lane & 15, kg = lane >> 4;
    const int tiles = M / T;
    const long MM = (long)M * M;
    const int nslot = w == 0 ? 3 : 2;

    f32x4 acc[3][2][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) acc[s][mb][0] = acc[s][mb][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.0f;

    for (int k = 0; k < tpw; ++k) {
        const int tile = blockIdx.x * tpw + k;
        if (tile >= ntiles) break;  // uniform across the workgroup
        const int tx = tile % tiles;
        const int ty = (tile / tiles) % tiles;
        const long b = tile / (tiles * tiles);
        const int x0 = tx * T, y0 = ty * T;
        __syncthreads();  // the previous tile's operands are no longer read
        for (int i = tid; i < T * T * 4; i += 256) {
            const int pix = i >> 2, q = i & 3;
            const int py = pix >> 4, px = pix & 15;
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(g + (b * MM + (long)(y0 + py) * M + x0 + px) * C + q * 8);
#pragma unroll
            for (int j = 0; j < 8; ++j) s_g[(q * 8 + j) * GS + pix] = v[j];
        }
        for (int i = tid; i < HT * HT * 4; i += 256) {
            const int pix = i >> 2, q = i & 3;
            const int hy = pix / HT, hx = pix - hy * HT;
            const int gy = wrap(y0 + hy - 1, M), gx = wrap(x0 + hx - 1, M);
            const bf16x8 v = *reinterpret_cast<const bf16x8*>(a + (b * MM + (long)gy * M + gx) * C + q * 8);
#pragma unroll
            for (int d = 0; d < 3; ++d) {  // copy d holds x' = hx - d in [0, 16)
                const int xs = hx - d;
                if (xs >= 0 && xs < T) {
#pragma unroll
                    for (int j = 0; j < 8; ++j) s_a[(d * C + q * 8 + j) * AS + hy * T + xs] = v[j];
                }
            }
        }
        __syncthreads();
        if (tid < C) {
            float s = 0.0f;
            for (int p = 0; p < T * T; ++p) s += (float)s_g[tid * GS + p];
            db += s;
        }
#pragma unroll 1
        for (int kc = 0; kc < T * T / 32; ++kc) {
            const int p0 = kc * 32 + kg * 8;   // this lane's 8 pixels: tile row p0/16, columns p0%16 ..
            const int ry = p0 >> 4, rx = p0 & 15;
            const bf16x8 A0 = *reinterpret_cast<const bf16x8*>(s_g + col * GS + p0);
            const bf16x8 A1 = *reinterpret_cast<const bf16x8*>(s_g + (16 + col) * GS + p0);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                if (s < nslot) {
                    const int tap = w + 4 * s;
                    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                    const bf16* src = s_a + ((dx + 1) * C) * AS + (ry + dy + 1) * T + rx;
                    const bf16x8 B0 = *reinterpret_cast<const bf16x8*>(src + col * AS);
                    const bf16x8 B1 = *reinterpret_cast<const bf16x8*>(src + (16 + col) * AS);
                    acc[s][0][0] = mfma(A0, B0, acc[s][0][0]);
                    acc[s][1][0] = mfma(A1, B0, acc[s][1][0]);
                    acc[s][0][1] = mfma(A0, B1, acc[s][0][1]);
                    acc[s][1][1] = mfma(A1, B1, acc[s][1][1]);
                }
            }
        }
    }

    float* part = parts + (long)blockIdx.x * kCnnPart;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        if (s < nslot) {
            const int tap = w + 4 * s;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = 16 * mb + 4 * kg + i, c = 16 * nb + col;
                        part[(tap * C + o) * C + c] = acc[s][mb][nb][i];
                    }
        }
    }
    if (tid < C) part[kCnnW + tid] = db;
}

// dst[s][e] = sum over rows r in slice s of src[r][e]  (rows split into S slices)
__global__ __launch_bounds__(256) void k_cnn_colsum(const float* __restrict__ src, int rows, int cols, int S,
                                                    float* __restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= cols) return;
    const int per = (rows + S - 1) / S;
    const int r0 = s * per, r1 = min(rows, r0 + per);
    float acc = 0.0f;
    for (int r = r0; r < r1; ++r) acc += src[(long)r * cols + e];
    dst[(long)s * cols + e] = acc;
}

// Final sum over S slice sums, written in the parameter order W[o][c][tap], b[o].
__global__ __launch_bounds__(256) void k_cnn_grad_final(const float* __restrict__ src, int S,
                                                        float* __restrict__ grad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kCnnPart) return;
    float acc = 0.0f;
    for (int s = 0; s < S; ++s) acc += src[(long)s * kCnnPart + e];
    if (e < kCnnW) {
        const int tap = e / (C * C), o = (e / C) % C, c = e % C;
        grad[(o * C + c) * 9 + tap] = acc;
    } else {
        grad[e] = acc;  // biases follow the weights in both layouts
    }
}

__device__ __forceinline__ float block_sum256(float v, float* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
    return s;
}

__global__ __launch_bounds__(256) void k_cnn_sumsq(const float* __restrict__ psi, long n, float* __restrict__ parts) {
    __shared__ float red[4];
    const long b = blockIdx.y;
    const long chunk = (n + kScaleBlocks - 1) / kScaleBlocks;
    const long e0 = blockIdx.x * chunk, e1 = min(n, e0 + chunk);
    const float* x = psi + b * n;
    float s = 0.0f;
#pragma unroll 4
    for (long e = e0 + threadIdx.x; e < e1; e += 256) s += x[e] * x[e];
    const float tot = block_sum256(s, red);
    if (threadIdx.x == 0) parts[b * kScaleBlocks + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_cnn_scale(const float* __restrict__ parts, long n, float* __restrict__ scale) {
    __shared__ float red[4];
    const int b = blockIdx.x;
    float s = 0.0f;
    for (int i = threadIdx.x; i < kScaleBlocks; i += 256) s += parts[b * kScaleBlocks + i];
    const float tot = block_sum256(s, red);
    if (threadIdx.x == 0) {
        const float r = sqrtf(tot / (float)n);
        scale[b] = r > 0.0f ? r : 1.0f;
    }
}

__global__ __launch_bounds__(256) void k_cnn_loss(const float* __restrict__ out, const float* __restrict__ target,
                                                  const float* __restrict__ rms, bf16* __restrict__ g,
                                                  float* __restrict__ parts, int N, int M, int B, float scale) {
    __shared__ float red[4];
    const long MM = (long)M * M;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.0f;
    if (t < (long)B * 4 * MM) {
        const long p = t % MM;
        const long q = t / MM;
        const int cb = (int)(q & 3);
        const long b = q >> 2;
        const float inv = 1.0f / rms[b];
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = cb * 8 + j;
            float d = 0.0f;
            if (c < N) {
                const long o = (b * N + c) * MM + p;
                d = (out[o] - target[o]) * inv;
            }
            s += d * d;
            v[j] = (bf16)(scale * d);
        }
        *reinterpret_cast<bf16x8*>(g + (b * MM + p) * C + cb * 8) = v;
    }
    const float tot = block_sum256(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_cnn_loss_reduce(const float* __restrict__ parts, int n, float inv_numel,
                                                         float* __restrict__ loss) {
    __shared__ float red[4];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += parts[i];
    const float tot = block_sum256(s, red);
    if (threadIdx.x == 0) loss[0] = tot * inv_numel;
}

__global__ __launch_bounds__(256) void k_cnn_adam(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                                  float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// MFMA weights of the three layers: forward A[l][tap][o][c] = W_l[o][c][tap];
// input gradient A[l][tap][c][o] = W_l[o][c][8 - tap] (the mirrored offset).
__global__ __launch_bounds__(256) void k_cnn_prep(const float* __restrict__ params, bf16* __restrict__ wf,
                                                  bf16* __restrict__ wd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * kCnnW) return;
    const int l = i / kCnnW;
    const int e = i - l * kCnnW;
    const int tap = e / (C * C), r = (e / C) % C, k = e % C;  // A[l][tap][r][k]
    const float* W = params + (long)l * kCnnL;
    wf[i] = (bf16)W[(r * C + k) * 9 + tap];
    wd[i] = (bf16)W[(k * C + r) * 9 + (8 - tap)];
}

}  // namespace

hipError_t cnn_rms(const float* psi, float* parts, float* scale, int N, int M, int B, hipStream_t st) {
    const long n = (long)N * M * M;
    hipLaunchKernelGGL(k_cnn_sumsq, dim3(kScaleBlocks, (unsigned)B), dim3(256), 0, st, psi, n, parts);
    hipLaunchKernelGGL(k_cnn_scale, dim3((unsigned)B), dim3(256), 0, st, parts, n, scale);
    return hipGetLastError();
}

hipError_t cnn_pack(const float* psi, const float* scale, bf16* act, int N, int M, int B, hipStream_t st) {
    const long n = (long)B * 4 * M * M;
    hipLaunchKernelGGL(k_cnn_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, psi, scale, act, N, M, B);
    return hipGetLastError();
}

hipError_t cnn_conv(int epi, const bf16* in, const bf16* wA, const float* bias, bf16* act_out, const bf16* mask,
                    const float* coarse, float* out, const float* scale, int N, int M, int B, hipStream_t st) {
    const dim3 grid((unsigned)((M / T) * (M / T) * B));
    if (epi == CNN_HIDDEN)
        hipLaunchKernelGGL(k_cnn_conv<CNN_HIDDEN>, grid, dim3(256), 0, st, in, wA, bias, act_out, mask, coarse, out,
                           scale, N, M);
    else if (epi == CNN_LAST)
        hipLaunchKernelGGL(k_cnn_conv<CNN_LAST>, grid, dim3(256), 0, st, in, wA, bias, act_out, mask, coarse, out,
                           scale, N, M);
    else
        hipLaunchKernelGGL(k_cnn_conv<CNN_DGRAD>, grid, dim3(256), 0, st, in, wA, bias, act_out, mask, coarse, out,
                           scale, N, M);
    return hipGetLastError();
}

int cnn_wgrad_parts(int M, int B, int tiles_per_wg) {
    const int ntiles = (M / T) * (M / T) * B;
    return (ntiles + tiles_per_wg - 1) / tiles_per_wg;
}

hipError_t cnn_wgrad(const bf16* g, const bf16* a, float* parts, int M, int B, int tiles_per_wg, hipStream_t st) {
    const int ntiles = (M / T) * (M / T) * B;
    const size_t lds = (size_t)(C * GS + 3 * C * AS) * sizeof(bf16);
    hipLaunchKernelGGL(k_cnn_wgrad, dim3((unsigned)cnn_wgrad_parts(M, B, tiles_per_wg)), dim3(256), lds, st, g, a,
                       parts, M, ntiles, tiles_per_wg);
    return hipGetLastError();
}

hipError_t cnn_wgrad_reduce(const float* parts, int nparts, float* slices, float* grad_layer, hipStream_t st) {
    const int S = nparts < kCnnSlices ? nparts : kCnnSlices;
    hipLaunchKernelGGL(k_cnn_colsum, dim3((unsigned)((kCnnPart + 255) / 256), (unsigned)S), dim3(256), 0, st, parts,
                       nparts, kCnnPart, S, slices);
    hipLaunchKernelGGL(k_cnn_grad_final, dim3((unsigned)((kCnnPart + 255) / 256)), dim3(256), 0, st, slices, S,
                       grad_layer);
    return hipGetLastError();
}

int cnn_loss_blocks(int N, int M, int B) {
    (void)N;
    const long n = (long)B * 4 * M * M;
    return (int)((n + 255) / 256);
}

hipError_t cnn_loss(const float* out, const float* target, const float* rms, bf16* g, float* loss_parts, int N,
                    int M, int B, float scale, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_loss, dim3((unsigned)cnn_loss_blocks(N, M, B)), dim3(256), 0, st, out, target, rms, g,
                       loss_parts, N, M, B, scale);
    return hipGetLastError();
}

hipError_t cnn_loss_reduce(const float* parts, int nparts, float inv_numel, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_loss_reduce, dim3(1), dim3(256), 0, st, parts, nparts, inv_numel, loss);
    return hipGetLastError();
}

hipError_t cnn_adam(float* params, const float* grads, float* m, float* v, int t, float lr, float beta1, float beta2,
                    float eps, hipStream_t st) {
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)t));
    hipLaunchKernelGGL(k_cnn_adam, dim3((kCnnP + 255) / 256), dim3(256), 0, st, params, grads, m, v, kCnnP, lr, beta1,
                       beta2, eps, (float)c1, (float)c2);
    return hipGetLastError();
}

hipError_t cnn_prep(const float* params, bf16* wfwd, bf16* wdgrad, hipStream_t st) {
    hipLaunchKernelGGL(k_cnn_prep, dim3((3 * kCnnW + 255) / 256), dim3(256), 0, st, params, wfwd, wdgrad);
    return hipGetLastError();
}

}  // namespace se2n
