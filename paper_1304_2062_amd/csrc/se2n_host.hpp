// Host helpers shared by the runtime files of libse2n: error reporting,
// size checks, FFT plans and twiddle tables.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "se2n_fft.hpp"

namespace se2n {

// Record a message for se2n_last_error() on this thread and return `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what);
void clear_error();

bool is_2a3b(int M, int* twos, int* threes);
FftPlan make_fft_plan(int L, int M);

template <class R>
std::vector<C2<R>> quarter_twiddles(int M);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Every device (and pinned host) allocation of the library goes through
// these, so that se2n_debug_fail_allocations can make the k-th one fail.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t pinned_malloc(void** p, size_t bytes);

struct OrientTaps;
// Taps of the orientation stencil for side M and Gaussian width sigma: the
// radius it needs (kernel tails below 2^-26 of each kernel's absolute sum,
// or the whole circle), rounded up to a compiled radius.  Returns that
// radius, or 0 when no compiled radius covers it (the FFT route is used).
int orient_stencil_taps(int M, double sigma, OrientTaps* taps);
// The same, remembered per (M, sigma) for the process (thread-safe); taps may be NULL.
int orient_stencil_taps_cached(int M, double sigma, OrientTaps* taps);

}  // namespace se2n

#define SE2N_HIP(call, what)                                       \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::se2n::hip_fail(e_, what);   \
    } while (0)
