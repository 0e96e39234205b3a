// Device-side building blocks: complex arithmetic and an in-LDS mixed-radix
// (2, 3, 4, 8) Stockham FFT that many threads of a workgroup run together on
// a batch of equal-length transforms.
//
// Each stage reads every butterfly's inputs into registers, synchronises,
// and writes the outputs back to the same LDS buffer, so a transform needs
// no second buffer.  Twiddles come from one table of w_M^m = exp(-2 pi i m/M)
// for the plan's side M; a transform of length L | M reads it with stride M/L.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace se2n {

template <class R>
using C2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;

template <class R>
__device__ __forceinline__ C2<R> cmk(R x, R y) {
    C2<R> c;
    c.x = x;
    c.y = y;
    return c;
}
template <class R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return cmk<R>(a.x + b.x, a.y + b.y); }
template <class R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return cmk<R>(a.x - b.x, a.y - b.y); }
template <class R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
    return cmk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class R>
__device__ __forceinline__ C2<R> cconj(C2<R> a) { return cmk<R>(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <class R, bool INV>
__device__ __forceinline__ C2<R> mul_mi(C2<R> a) {
    return INV ? cmk<R>(-a.y, a.x) : cmk<R>(a.y, -a.x);
}

// Radix kernels: y_k = sum_j x_j w_R^{jk}, w_R = exp(-+ 2 pi i / R).
template <class R, bool INV>
__device__ __forceinline__ void dft2(C2<R>* v) {
    C2<R> a = v[0], b = v[1];
    v[0] = cadd<R>(a, b);
    v[1] = csub<R>(a, b);
}

template <class R, bool INV>
__device__ __forceinline__ void dft3(C2<R>* v) {
    const R h = R(0.86602540378443864676);  // sqrt(3)/2
    C2<R> a = v[0], b = v[1], c = v[2];
    C2<R> t1 = cadd<R>(b, c);
    C2<R> t2 = cmk<R>(a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y);
    C2<R> d = csub<R>(b, c);
    // forward: y1 = t2 - i h d, y2 = t2 + i h d
    C2<R> ihd = cmk<R>(-h * d.y, h * d.x);  // i*h*d
    v[0] = cadd<R>(a, t1);
    if (INV) {
        v[1] = cadd<R>(t2, ihd);
        v[2] = csub<R>(t2, ihd);
    } else {
        v[1] = csub<R>(t2, ihd);
        v[2] = cadd<R>(t2, ihd);
    }
}

template <class R, bool INV>
__device__ __forceinline__ void dft4(C2<R>* v) {
    C2<R> s02 = cadd<R>(v[0], v[2]), d02 = csub<R>(v[0], v[2]);
    C2<R> s13 = cadd<R>(v[1], v[3]), d13 = csub<R>(v[1], v[3]);
    C2<R> t = mul_mi<R, INV>(d13);  // -i d13 forward
    v[0] = cadd<R>(s02, s13);
    v[2] = csub<R>(s02, s13);
    v[1] = cadd<R>(d02, t);
    v[3] = csub<R>(d02, t);
}

template <class R, bool INV>
__device__ __forceinline__ void dft8(C2<R>* v) {
    const R q = R(0.70710678118654752440);
    C2<R> e[4] = {v[0], v[2], v[4], v[6]};
    C2<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<R, INV>(e);
    dft4<R, INV>(o);
    // twiddles w_8^k, k = 0..3 (conjugated for the inverse)
    C2<R> o1 = INV ? cmk<R>(q * (o[1].x - o[1].y), q * (o[1].x + o[1].y))
                   : cmk<R>(q * (o[1].x + o[1].y), q * (o[1].y - o[1].x));
    C2<R> o2 = mul_mi<R, INV>(o[2]);
    C2<R> o3 = INV ? cmk<R>(-q * (o[3].x + o[3].y), q * (o[3].x - o[3].y))
                   : cmk<R>(q * (o[3].y - o[3].x), -q * (o[3].x + o[3].y));
    v[0] = cadd<R>(e[0], o[0]);
    v[4] = csub<R>(e[0], o[0]);
    v[1] = cadd<R>(e[1], o1);
    v[5] = csub<R>(e[1], o1);
    v[2] = cadd<R>(e[2], o2);
    v[6] = csub<R>(e[2], o2);
    v[3] = cadd<R>(e[3], o3);
    v[7] = csub<R>(e[3], o3);
}

template <class R, int RADIX, bool INV>
__device__ __forceinline__ void dft(C2<R>* v) {
    if constexpr (RADIX == 2) dft2<R, INV>(v);
    else if constexpr (RADIX == 3) dft3<R, INV>(v);
    else if constexpr (RADIX == 4) dft4<R, INV>(v);
    else dft8<R, INV>(v);
}

// Radix sequence of one transform length (host fills it, kernels read it by value).
struct FftPlan {
    int L;          // transform length
    int nstages;    // number of stages
    int radix[16];  // radix of each stage, 2/3/4/8
};

// One Stockham stage, in place.  `nbatch` transforms of length L start at
// buf + t*bstride.  Ns is the product of the radices of the earlier stages.
// Butterfly j of a transform reads x[j + r L/RADIX], multiplies input r by
// w_{Ns RADIX}^{r (j mod Ns)}, and writes output r to
// (j / Ns) Ns RADIX + (j mod Ns) + r Ns.
// The caller guarantees nbatch*L <= EPT*nthr.
template <class R, int RADIX, bool INV, int EPT>
__device__ __forceinline__ void fft_stage(C2<R>* buf, int L, int Ns, int nbatch, int bstride,
                                          const C2<R>* __restrict__ tw, int M, int tid, int nthr) {
    constexpr int MAXB = (EPT + RADIX - 1) / RADIX;
    const int nb = L / RADIX;
    const int total = nb * nbatch;
    const int twstep = M / (Ns * RADIX);
    C2<R> v[MAXB][RADIX];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthr;
        if (b < total) {
            const int t = b / nb;
            const int j = b - t * nb;
            const C2<R>* s = buf + t * bstride + j;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[i][r] = s[r * nb];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthr;
        if (b < total) {
            const int t = b / nb;
            const int j = b - t * nb;
            const int k = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RADIX; ++r) {
                    C2<R> w = tw[r * k * twstep];
                    if (INV) w.y = -w.y;
                    v[i][r] = cmul<R>(v[i][r], w);
                }
            }
            dft<R, RADIX, INV>(v[i]);
            C2<R>* d = buf + t * bstride + (j - k) * RADIX + k;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) d[r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Unnormalised transforms of `nbatch` sequences of length plan.L held in LDS.
// Forward: X_k = sum_n x_n w_L^{nk}; inverse: the same with w_L^{-nk}.
// Must be called by all nthr threads of the workgroup (it synchronises).
template <class R, bool INV, int EPT>
__device__ void fft_lds(C2<R>* buf, const FftPlan& plan, int nbatch, int bstride,
                        const C2<R>* __restrict__ tw, int M, int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        const int rad = plan.radix[s];
        if (rad == 8) fft_stage<R, 8, INV, EPT>(buf, plan.L, Ns, nbatch, bstride, tw, M, tid, nthr);
        else if (rad == 4) fft_stage<R, 4, INV, EPT>(buf, plan.L, Ns, nbatch, bstride, tw, M, tid, nthr);
        else if (rad == 3) fft_stage<R, 3, INV, EPT>(buf, plan.L, Ns, nbatch, bstride, tw, M, tid, nthr);
        else fft_stage<R, 2, INV, EPT>(buf, plan.L, Ns, nbatch, bstride, tw, M, tid, nthr);
        Ns *= rad;
    }
}

}  // namespace se2n
