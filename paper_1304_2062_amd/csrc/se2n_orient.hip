// Orientation map of one image by the separable periodic stencil: one
// workgroup per 128 x 32 tile of bins (the tile body and the reasoning behind
// it are in se2n_orient.hpp).
#include "se2n_orient.hpp"

namespace se2n {
namespace {

template <int RAD>
__global__ __launch_bounds__(kOrientNT) void k_orient_stencil(const float* __restrict__ f,
                                                              const uint8_t* __restrict__ mask,
                                                              uint8_t* __restrict__ rmap, int M, int N,
                                                              OrientTaps taps) {
    __shared__ float sa[orient_lds_floats<RAD>()];  // g (*)_y f_c
    __shared__ float sb[orient_lds_floats<RAD>()];  // d (*)_y f_c
    // each XCD takes one contiguous band of tiles: the halo rows two tiles
    // share are fetched through one L2
    const int tile = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    orient_stencil_tile<RAD>(f, mask, rmap, M, N, tile, taps, sa, sb, (int)threadIdx.x);
}

}  // namespace

hipError_t launch_orient_stencil(const float* f, const uint8_t* mask, uint8_t* rmap, int M, int N, int radius,
                                 const OrientTaps& taps, hipStream_t st) {
    const dim3 grid((unsigned)orient_tiles(M)), block(kOrientNT);
    switch (radius) {
#define SE2N_ORIENT_CASE(RV)                                                                             \
    case RV:                                                                                             \
        hipLaunchKernelGGL((k_orient_stencil<RV>), grid, block, 0, st, f, mask, rmap, M, N, taps);       \
        break;
        SE2N_ORIENT_CASE(8)
        SE2N_ORIENT_CASE(12)
        SE2N_ORIENT_CASE(16)
        SE2N_ORIENT_CASE(20)
        SE2N_ORIENT_CASE(24)
        SE2N_ORIENT_CASE(32)
#undef SE2N_ORIENT_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace se2n
