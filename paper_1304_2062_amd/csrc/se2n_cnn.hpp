// Learned corrector network (BF16 MFMA kernels): shared definitions and the
// launch interface used by the host runtime.
//
// The network maps a real-space orientation volume psi[N][H][W] (FP32,
// planar) to psi + r, r = conv3(relu(conv2(relu(conv1(psi))))), each conv a
// 3x3 cross-correlation with circular padding.  Channels are padded to 32:
// the input's channels N..31 are zero and so are the weights that read them
// (layer 1) or write output channels N..31 (layer 3).
//
// Layouts
//   activations, gradients between layers: bfloat16, channels last
//       act[b][y][x][32]  (64 bytes per pixel)
//   parameters (FP32 master copy, the order of the public parameter vector):
//       for l = 0, 1, 2:  W_l[o][c][tap] (32 x 32 x 9), then b_l[o] (32),
//       tap = (dy+1)*3 + (dx+1) for the input offset (dy, dx)
//   MFMA weights (bfloat16): A[l][tap][row][k] with row the output channel of
//       the product and k the reduced channel: forward A = W[o][c] (row o,
//       k c); input gradient A = W[o][c] of the mirrored tap (row c, k o).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace se2n {

constexpr int kCnnC = 32;                       // padded channels
constexpr int kCnnW = kCnnC * kCnnC * 9;        // weights per layer
constexpr int kCnnL = kCnnW + kCnnC;            // parameters per layer
constexpr int kCnnP = 3 * kCnnL;                // parameter vector length
constexpr int kCnnTile = 16;                    // pixel tile side of the conv kernels
constexpr int kCnnPart = kCnnW + kCnnC;         // one workgroup's weight + bias gradient partial
constexpr int kCnnSlices = 64;                  // first-level sums of the partials
constexpr int kCnnScaleBlocks = 512;            // partial sums of squares per image

enum CnnEpi { CNN_HIDDEN = 0, CNN_LAST = 1, CNN_DGRAD = 2 };

using bf16 = __bf16;

// scale[b] = root mean square of psi[b] (1 if zero); parts: B*kCnnScaleBlocks floats of scratch
hipError_t cnn_rms(const float* psi, float* parts, float* scale, int N, int M, int B, hipStream_t st);
// psi planar FP32 [B][N][M][M] / scale[b] -> act bf16 channels-last [B][M][M][32] (zero channels >= N)
hipError_t cnn_pack(const float* psi, const float* scale, bf16* act, int N, int M, int B, hipStream_t st);
// One 3x3 conv 32 -> 32 over B images of side M (M % 16 == 0):
//   HIDDEN: act_out = relu(conv(in) + bias)                        (bf16, channels last)
//   LAST:   out[b][c] = coarse[b][c] + scale[b] (conv(in)[c] + bias[c]), c < N
//           (FP32 planar; out may be coarse)
//   DGRAD:  act_out = conv(in) * [mask > 0]                         (bf16, channels last; no bias)
hipError_t cnn_conv(int epi, const bf16* in, const bf16* wA, const float* bias, bf16* act_out,
                    const bf16* mask, const float* coarse, float* out, const float* scale, int N, int M, int B,
                    hipStream_t st);
// Weight + bias gradient partials of one layer: g (bf16 CL, the layer's output
// gradient), a (bf16 CL, the layer's input); one partial of kCnnPart floats per
// workgroup, each workgroup summing `tiles_per_wg` pixel tiles.
int cnn_wgrad_parts(int M, int B, int tiles_per_wg);
hipError_t cnn_wgrad(const bf16* g, const bf16* a, float* parts, int M, int B, int tiles_per_wg, hipStream_t st);
// Sum the partials into the layer's slice of the gradient vector (W[o][c][tap], b[o]),
// in a fixed order: kCnnSlices slice sums (scratch `slices`, kCnnSlices*kCnnPart
// floats), then their sum.
hipError_t cnn_wgrad_reduce(const float* parts, int nparts, float* slices, float* grad_layer, hipStream_t st);
// Loss: out, target FP32 planar [B][N][M][M], each image in units of rms[b]:
// d = (out - target)/rms[b]; g = scale*d to bf16 channels last (zero channels
// >= N); per-block partial sums of d^2.
int cnn_loss_blocks(int N, int M, int B);
hipError_t cnn_loss(const float* out, const float* target, const float* rms, bf16* g, float* loss_parts, int N,
                    int M, int B, float scale, hipStream_t st);
// loss = sum(parts) * inv_numel (one value, deterministic order)
hipError_t cnn_loss_reduce(const float* parts, int nparts, float inv_numel, float* loss, hipStream_t st);
// Adam on the FP32 parameters (step t >= 1, bias-corrected), then refresh the MFMA weights.
hipError_t cnn_adam(float* params, const float* grads, float* m, float* v, int t, float lr, float beta1,
                    float beta2, float eps, hipStream_t st);
hipError_t cnn_prep(const float* params, bf16* wfwd, bf16* wdgrad, hipStream_t st);

}  // namespace se2n
