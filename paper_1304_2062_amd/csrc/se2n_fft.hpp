// Device-side building blocks: complex arithmetic and an in-LDS mixed-radix
// (2, 3, 4, 8) Stockham FFT that many threads of a workgroup run together on
// a batch of equal-length transforms.
//
// Each stage reads every butterfly's inputs into registers, synchronises,
// and writes the outputs back to the same LDS buffer, so a transform needs
// no second buffer.  Twiddles come from a full-period LDS table w_M^m of the
// plan's side M (expanded from a quarter-wave table in global memory); a
// transform of length L | M reads it with stride M/L.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace se2n {

template <class R>
using C2 = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;

// f(0), f(1), ..., f(N - 1) with compile-time indices, so that a register
// array indexed by them never needs memory (an unroll pragma leaves that to
// the optimiser).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

// LDS position of logical element i of a transform buffer: one complex of
// padding after every 32 spreads the strided writes of the early Stockham
// stages over the banks (every 16 and every 8 measured slower on gfx950).
#ifndef SE2N_LDS_PAD_SHIFT
#define SE2N_LDS_PAD_SHIFT 5
#endif
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> SE2N_LDS_PAD_SHIFT); }
__host__ __device__ constexpr int lds_padded_size(int n) { return n + (n >> SE2N_LDS_PAD_SHIFT) + 1; }

// A fixed-size stage touches the RADIX positions base + r * STRIDE of each
// butterfly.  Where the padding of those positions is base's padding plus a
// constant, one padded base and compile-time offsets replace RADIX separate
// index computations (each an add, a shift, an add and a byte scaling):
//  * reads at ib + r NB: exact when NB is a multiple of the padding period P;
//  * writes at ob + r NS, ob = t BSTRIDE + q NS RADIX + k with k < NS:
//    exact when NS is a multiple of P, or when NS divides P, NS RADIX
//    divides or is a multiple of P and BSTRIDE is a multiple of P (the
//    butterfly's outputs then cross a period boundary only at fixed r).
// The offset of element r is then r STRIDE + (r STRIDE) / P.
constexpr int kLdsPadPeriod = 1 << SE2N_LDS_PAD_SHIFT;
__host__ __device__ constexpr bool pad_linear_read(int NB) { return NB % kLdsPadPeriod == 0; }
__host__ __device__ constexpr bool pad_linear_write(int NS, int RADIX, int BSTRIDE) {
    return NS % kLdsPadPeriod == 0 ||
           (kLdsPadPeriod % NS == 0 &&
            ((NS * RADIX) % kLdsPadPeriod == 0 || kLdsPadPeriod % (NS * RADIX) == 0) &&
            BSTRIDE % kLdsPadPeriod == 0);
}
__host__ __device__ constexpr int pad_offset(int r, int stride) { return r * stride + (r * stride) / kLdsPadPeriod; }

// Exact quotient n / d for 0 <= n < 2^22 from a float reciprocal (inv = 1/d
// rounded to float): (n + 1/2) inv lies at least 1/(2d) away from an integer,
// far more than the float rounding of the product.
__device__ __forceinline__ int fdiv(int n, float inv) { return (int)(((float)n + 0.5f) * inv); }

// One stage of a Stockham transform (filled on the host).
struct FftStage {
    int radix;      // 2, 3, 4 or 8
    int nb;         // butterflies per transform = L / radix
    int Ns;         // product of the radices of the earlier stages
    int twstep;     // M / (Ns * radix): twiddle w_{Ns radix}^e = w_M^{e twstep}
    float inv_nb;   // 1/nb
    float inv_Ns;   // 1/Ns
    int lg_Ns;      // log2(Ns) when Ns is a power of two, else -1
};

// Radix sequence of one transform length.
struct FftPlan {
    int L;
    int nstages;
    FftStage st[12];
};

// LDS position of twiddle m: one complex of padding after every 2^SHIFT.  The
// middle Stockham stages read w^{r k twstep} with twstep a power of two, so
// without padding every lane of a wave falls in the same few banks.
#ifndef SE2N_TW_PAD_SHIFT
#define SE2N_TW_PAD_SHIFT 3
#endif
__host__ __device__ constexpr int tw_pos(int m) { return m + (m >> SE2N_TW_PAD_SHIFT); }

// Twiddle w_M^m = exp(-2 pi i m / M), m in [0, M), from the LDS table: the
// full period (FULL) or the quarter r in [0, M/4] with
// w_M^{a M/4 + r} = (-i)^a w_M^r.
template <class R, bool FULL>
__device__ __forceinline__ C2<R> tw_get(const C2<R>* tw, int m, int M4) {
    if (FULL) return tw[tw_pos(m)];
    const int a = (m >= M4) + (m >= 2 * M4) + (m >= 3 * M4);
    const C2<R> w = tw[tw_pos(m - __mul24(a, M4))];
    if (a == 0) return w;
    if (a == 1) return cmk<R>(w.y, -w.x);
    if (a == 2) return cmk<R>(-w.x, -w.y);
    return cmk<R>(-w.y, w.x);
}

// tw_get for an exponent known to lie below (AMAX + 1) M/4: only the
// quadrants up to AMAX are tested (AMAX = 0: a plain read).
template <class R, bool FULL, int AMAX>
__device__ __forceinline__ C2<R> tw_get_upto(const C2<R>* tw, int m, int M4) {
    if (FULL || AMAX == 0) return tw[tw_pos(m)];
    int a = m >= M4;
    if constexpr (AMAX >= 2) a += m >= 2 * M4;
    if constexpr (AMAX >= 3) a += m >= 3 * M4;
    const C2<R> w = tw[tw_pos(m - __mul24(a, M4))];
    if (a == 0) return w;
    if (AMAX == 1 || a == 1) return cmk<R>(w.y, -w.x);
    if (AMAX == 2 || a == 2) return cmk<R>(-w.x, -w.y);
    return cmk<R>(-w.y, w.x);
}

// Copy the twiddles into LDS from the quarter table q[r] = w_M^r,
// r in [0, M/4], in global memory: the full period if `full`, else the
// quarter table itself (callers synchronise afterwards).
template <class R>
__device__ __forceinline__ void load_twiddles(C2<R>* dst, const C2<R>* __restrict__ q, int M4, bool full,
                                              int tid, int nthr) {
    if (!full) {
        for (int i = tid; i <= M4; i += nthr) dst[tw_pos(i)] = q[i];
        return;
    }
    for (int m = tid; m < 4 * M4; m += nthr) {
        const int a = (m >= M4) + (m >= 2 * M4) + (m >= 3 * M4);
        const C2<R> w = q[m - a * M4];
        C2<R> v;
        if (a == 0) v = w;
        else if (a == 1) v = cmk<R>(w.y, -w.x);
        else if (a == 2) v = cmk<R>(-w.x, -w.y);
        else v = cmk<R>(-w.y, w.x);
        dst[tw_pos(m)] = v;
    }
}

// Elements the LDS twiddle table occupies (a multiple of 8: what follows
// stays 64-byte aligned).
__host__ __device__ constexpr int tw_elems(int M, bool full) {
    return (tw_pos(full ? M - 1 : M / 4) + 1 + 7) & ~7;
}

// Multiply inputs r = 1 .. RADIX-1 of a butterfly by w^{r e} (conjugated for
// the inverse).  Only w^e, w^{2e} (and w^{4e} for radix 8) are read from the
// LDS table; the other powers are products of those, which saves LDS reads
// at an error of a few ulps.
template <class R, int RADIX, bool INV, bool TWFULL>
__device__ __forceinline__ void apply_twiddles(C2<R>* v, const C2<R>* twq, int e, int M4) {
    // In a stage of radix RADIX the exponent e = k M / (Ns RADIX), k < Ns,
    // lies below M / RADIX, which bounds the quadrant of each power read.
    auto rd = [&](auto amax, int m) {
        C2<R> w = tw_get_upto<R, TWFULL, decltype(amax)::value>(twq, m, M4);
        if (INV) w.y = -w.y;
        return w;
    };
    using Q0 = std::integral_constant<int, 0>;
    using Q1 = std::integral_constant<int, 1>;
    using Q2 = std::integral_constant<int, 2>;
    if constexpr (RADIX == 2) {
        v[1] = cmul<R>(v[1], rd(Q1{}, e));  // e < M/2
    } else if constexpr (RADIX == 3) {
        v[1] = cmul<R>(v[1], rd(Q1{}, e));      // e < M/3
        v[2] = cmul<R>(v[2], rd(Q2{}, 2 * e));  // 2e < 2M/3
    } else if constexpr (RADIX == 4) {
        const C2<R> w1 = rd(Q0{}, e), w2 = rd(Q1{}, 2 * e);  // e < M/4, 2e < M/2
        v[1] = cmul<R>(v[1], w1);
        v[2] = cmul<R>(v[2], w2);
        v[3] = cmul<R>(v[3], cmul<R>(w1, w2));
    } else {
        static_assert(RADIX == 8, "radix 2, 3, 4 or 8");
        const C2<R> w1 = rd(Q0{}, e), w2 = rd(Q0{}, 2 * e), w4 = rd(Q1{}, 4 * e);  // e < M/8
        const C2<R> w3 = cmul<R>(w1, w2);
        v[1] = cmul<R>(v[1], w1);
        v[2] = cmul<R>(v[2], w2);
        v[3] = cmul<R>(v[3], w3);
        v[4] = cmul<R>(v[4], w4);
        v[5] = cmul<R>(v[5], cmul<R>(w1, w4));
        v[6] = cmul<R>(v[6], cmul<R>(w2, w4));
        v[7] = cmul<R>(v[7], cmul<R>(w3, w4));
    }
}

// One Stockham stage, in place.  `nbatch` transforms of length L start at
// buf + t*bstride.  Butterfly j of a transform reads x[j + r L/RADIX],
// multiplies input r by w_{Ns RADIX}^{r (j mod Ns)}, and writes output r to
// (j / Ns) Ns RADIX + (j mod Ns) + r Ns.  Every thread first reads all its
// butterflies, the block synchronises, then every thread writes.
// Thread tid owns butterflies b = tid + i*nthr, i.e. transform t = b / nb and
// butterfly j = b mod nb.  The caller guarantees nbatch*L <= EPT*nthr.
template <class R, int RADIX, bool INV, int EPT, bool TWFULL>
__device__ __forceinline__ void fft_stage(C2<R>* buf, const FftStage& s, int nbatch, int bstride,
                                          const C2<R>* twq, int M4, int tid, int nthr) {
    constexpr int MAXB = (EPT + RADIX - 1) / RADIX;
    // the stage parameters are uniform: keep them in scalar registers even
    // when the plan lives in memory the compiler cannot prove read-only
    const int nb = __builtin_amdgcn_readfirstlane(s.nb);
    const int Ns = __builtin_amdgcn_readfirstlane(s.Ns);
    const float inv_nb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.inv_nb)));
    const float inv_Ns = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.inv_Ns)));
    const int twstep = __builtin_amdgcn_readfirstlane(s.twstep);
    const int total = nb * nbatch;
    C2<R> v[MAXB][RADIX];
    int obase[MAXB], kk[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthr;
        if (b < total) {
            const int t = fdiv(b, inv_nb);
            const int j = b - __mul24(t, nb);
            const int q = fdiv(j, inv_Ns);
            const int k = j - __mul24(q, Ns);
            const int ib = __mul24(t, bstride) + j;
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[i][r] = buf[lds_pad(ib + r * nb)];
            obase[i] = __mul24(t, bstride) + __mul24(q, Ns * RADIX) + k;
            kk[i] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * nthr;
        if (b < total) {
            if (Ns > 1) apply_twiddles<R, RADIX, INV, TWFULL>(v[i], twq, __mul24(kk[i], twstep), M4);
            dft<R, RADIX, INV>(v[i]);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) buf[lds_pad(obase[i] + r * Ns)] = v[i][r];
        }
    }
    __syncthreads();
}

// Unnormalised transforms of `nbatch` sequences of length plan.L held in LDS
// (logical element i of the buffer at buf[lds_pad(i)]).
// Forward: X_k = sum_n x_n w_L^{nk}; inverse: the same with w_L^{-nk}.
// twq is the LDS twiddle table of the plan's side M (full period or quarter).
// All nthr threads of the workgroup call it; it synchronises the workgroup.
template <class R, bool INV, int EPT, bool TWFULL>
__device__ void fft_lds(C2<R>* buf, const FftPlan& plan, int nbatch, int bstride, const C2<R>* twq, int M4,
                        int tid, int nthr) {
    const int nst = __builtin_amdgcn_readfirstlane(plan.nstages);
    for (int s = 0; s < nst; ++s) {
        const FftStage& st = plan.st[s];
        const int radix = __builtin_amdgcn_readfirstlane(st.radix);
        if (radix == 8) fft_stage<R, 8, INV, EPT, TWFULL>(buf, st, nbatch, bstride, twq, M4, tid, nthr);
        else if (radix == 4) fft_stage<R, 4, INV, EPT, TWFULL>(buf, st, nbatch, bstride, twq, M4, tid, nthr);
        else if (radix == 3) fft_stage<R, 3, INV, EPT, TWFULL>(buf, st, nbatch, bstride, twq, M4, tid, nthr);
        else fft_stage<R, 2, INV, EPT, TWFULL>(buf, st, nbatch, bstride, twq, M4, tid, nthr);
    }
}

// ---------------------------------------------------------------------------
// Compile-time specialisation for the hot sizes: the same Stockham stages
// with the length, batch, stride, thread count and radix sequence known to
// the compiler, so every index is a shift or a constant multiply.
// ---------------------------------------------------------------------------

// Radix of stage s of a length-L transform (0 past the last stage); the same
// sequence the host builds: radix 8 where possible, then 4 (or 4,4 in place
// of 8,2), then radix 3.
__host__ __device__ constexpr int static_radix(int L, int s) {
    int a = 0, b = 0, m = L;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    int rad[16] = {};
    int n = 0;
    const int q = a / 3, r = a % 3;
    if (r == 1 && q >= 1) {
        for (int i = 0; i < q - 1; ++i) rad[n++] = 8;
        rad[n++] = 4;
        rad[n++] = 4;
    } else {
        for (int i = 0; i < q; ++i) rad[n++] = 8;
        if (r == 1) rad[n++] = 2;
        if (r == 2) rad[n++] = 4;
    }
    for (int i = 0; i < b; ++i) rad[n++] = 3;
    return s < n ? rad[s] : 0;
}

template <class R, int RADIX, bool INV, bool TWFULL, int L, int NS, int NBATCH, int BSTRIDE, int NTHR, int M>
__device__ __forceinline__ void fft_stage_static(C2<R>* buf, const C2<R>* twq, int tid) {
    constexpr int NB = L / RADIX;
    constexpr int TOTAL = NB * NBATCH;
    constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
    constexpr int TWSTEP = M / (NS * RADIX);
    constexpr int M4 = M / 4;
    C2<R> v[MAXB][RADIX];
    int obase[MAXB], kk[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || b < TOTAL) {
            const int t = b / NB;
            const int j = b - t * NB;
            const int q = j / NS;
            const int k = j - q * NS;
            const int ib = t * BSTRIDE + j;
            if constexpr (pad_linear_read(NB)) {
                const C2<R>* pa = buf + lds_pad(ib);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[i][r] = pa[pad_offset(r, NB)];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[i][r] = buf[lds_pad(ib + r * NB)];
            }
            obase[i] = t * BSTRIDE + q * NS * RADIX + k;
            kk[i] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || b < TOTAL) {
            if (NS > 1) apply_twiddles<R, RADIX, INV, TWFULL>(v[i], twq, kk[i] * TWSTEP, M4);
            dft<R, RADIX, INV>(v[i]);
            if constexpr (pad_linear_write(NS, RADIX, BSTRIDE)) {
                C2<R>* pb = buf + lds_pad(obase[i]);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) pb[pad_offset(r, NS)] = v[i][r];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) buf[lds_pad(obase[i] + r * NS)] = v[i][r];
            }
        }
    }
    __syncthreads();
}

template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, int S = 0, int NS = 1>
__device__ __forceinline__ void fft_static(C2<R>* buf, const C2<R>* twq, int tid) {
    constexpr int RADIX = static_radix(L, S);
    if constexpr (RADIX != 0) {
        fft_stage_static<R, RADIX, INV, TWFULL, L, NS, NBATCH, BSTRIDE, NTHR, M>(buf, twq, tid);
        fft_static<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, S + 1, NS * RADIX>(buf, twq, tid);
    }
}

// Input slots of the first stage: thread tid's butterfly i reads positions
// n = j + r*NB (r < RADIX) of transform t; slot = i*RADIX + r.
__host__ __device__ constexpr int static_in_slots(int L, int NBATCH, int NTHR) {
    return (L / static_radix(L, 0) * NBATCH + NTHR - 1) / NTHR * static_radix(L, 0);
}

// Butterfly b of the first stage is (transform t, butterfly j): t = b / NB
// (ROWFAST false: consecutive threads walk one transform) or t = b % NBATCH
// (ROWFAST true: consecutive threads walk the transforms, which makes the
// slots of 8 consecutive lanes one contiguous run of a transposed layout).
template <int L, int NBATCH, int NTHR, bool ROWFAST = false>
__device__ __forceinline__ bool static_in_pos(int tid, int slot, int& t, int& n) {
    constexpr int RADIX = static_radix(L, 0);
    constexpr int NB = L / RADIX;
    const int i = slot / RADIX, r = slot - (slot / RADIX) * RADIX;
    const int b = tid + i * NTHR;
    const int j = ROWFAST ? b / NBATCH : b - (b / NB) * NB;
    t = ROWFAST ? b - j * NBATCH : b / NB;
    n = j + r * NB;
    return b < NB * NBATCH;
}

// First stage of fft_static with its inputs taken from g(slot) (see
// static_in_pos) instead of LDS, followed by a barrier.  The caller
// guarantees that no thread still reads the buffer.
template <class R, bool INV, int L, int NBATCH, int BSTRIDE, int NTHR, bool ROWFAST, class G>
__device__ __forceinline__ void fft_static_first(C2<R>* buf, int tid, G&& g) {
    constexpr int RADIX = static_radix(L, 0);
    constexpr int NB = L / RADIX;
    constexpr int TOTAL = NB * NBATCH;
    constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || b < TOTAL) {
            const int j = ROWFAST ? b / NBATCH : b - (b / NB) * NB;
            const int t = ROWFAST ? b - j * NBATCH : b / NB;
            C2<R> v[RADIX];
#pragma unroll
            for (int r = 0; r < RADIX; ++r) v[r] = g(i * RADIX + r);
            dft<R, RADIX, INV>(v);  // first stage: no twiddles (Ns = 1)
            if constexpr (pad_linear_write(1, RADIX, BSTRIDE)) {
                C2<R>* pb = buf + lds_pad(t * BSTRIDE + j * RADIX);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) pb[pad_offset(r, 1)] = v[r];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) buf[lds_pad(t * BSTRIDE + j * RADIX + r)] = v[r];
            }
        }
    }
    __syncthreads();
}

// fft_static with the first stage's inputs from g(slot).
template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, class G>
__device__ __forceinline__ void fft_static_in(C2<R>* buf, const C2<R>* twq, int tid, G&& g) {
    fft_static_first<R, INV, L, NBATCH, BSTRIDE, NTHR, false>(buf, tid, g);
    fft_static<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, 1, static_radix(L, 0)>(buf, twq, tid);
}

// Radix of the last stage of a length-L transform, and the outputs each of
// NTHR threads produces in it (the thread's output slots).
__host__ __device__ constexpr int static_last_radix(int L) {
    int s = 0;
    while (static_radix(L, s + 1) != 0) ++s;
    return static_radix(L, s);
}
__host__ __device__ constexpr int static_out_slots(int L, int NBATCH, int NTHR) {
    return (L / static_last_radix(L) * NBATCH + NTHR - 1) / NTHR * static_last_radix(L);
}

// Transform t and position n of output slot `slot` of thread tid in the last
// stage; false if the slot is unused.
template <int L, int NBATCH, int NTHR>
__device__ __forceinline__ bool static_out_pos(int tid, int slot, int& t, int& n) {
    constexpr int RADIX = static_last_radix(L);
    constexpr int NB = L / RADIX;  // = NS of the last stage
    const int i = slot / RADIX, r = slot - (slot / RADIX) * RADIX;
    const int b = tid + i * NTHR;
    t = b / NB;
    n = (b - t * NB) + r * NB;
    return b < NB * NBATCH;
}

// The transforms of fft_static, except that the last stage hands each output
// to f(slot, t, n, value) (slot = i*RADIX + r of the thread's butterfly i,
// output r; transform t, position n) instead of writing it to LDS.  No
// barrier follows the last stage: every thread has read its inputs before
// the stage's own barrier, so the caller may refill the buffer at once.
template <class R, int RADIX, bool INV, bool TWFULL, int L, int NS, int NBATCH, int BSTRIDE, int NTHR, int M, class F>
__device__ __forceinline__ void fft_stage_static_out(C2<R>* buf, const C2<R>* twq, int tid, F&& f) {
    constexpr int NB = L / RADIX;
    constexpr int TOTAL = NB * NBATCH;
    constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
    constexpr int TWSTEP = M / (NS * RADIX);
    constexpr int M4 = M / 4;
    static_assert(NS * RADIX == L, "the output stage is the last one");
    C2<R> v[MAXB][RADIX];
    int tt[MAXB], kk[MAXB];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || b < TOTAL) {
            const int t = b / NB;
            const int j = b - t * NB;
            const int ib = t * BSTRIDE + j;
            if constexpr (pad_linear_read(NB)) {
                const C2<R>* pa = buf + lds_pad(ib);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[i][r] = pa[pad_offset(r, NB)];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[i][r] = buf[lds_pad(ib + r * NB)];
            }
            tt[i] = t;
            kk[i] = j;  // q = 0 in the last stage: k = j
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || b < TOTAL) {
            if (NS > 1) apply_twiddles<R, RADIX, INV, TWFULL>(v[i], twq, kk[i] * TWSTEP, M4);
            dft<R, RADIX, INV>(v[i]);
#pragma unroll
            for (int r = 0; r < RADIX; ++r) f(i * RADIX + r, tt[i], kk[i] + r * NS, v[i][r]);
        }
    }
}

// ---------------------------------------------------------------------------
// Twiddles kept in registers.  In a fixed-size transform a thread runs the
// same butterflies, hence needs the same twiddles, for every batch it
// transforms; a pass that walks many batches with fixed threads (the row
// passes walk the orientation slices) reads the base powers w^e, w^{2e}
// (and w^{4e} for radix 8) of stages 1 .. SLIM - 1 from the LDS table once
// and forms the other powers as apply_twiddles does, with the same values
// and products (bit-identical results).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int static_nstages(int L) {
    int s = 0;
    while (static_radix(L, s) != 0) ++s;
    return s;
}
__host__ __device__ constexpr int static_ns(int L, int S) {
    int ns = 1;
    for (int s = 0; s < S; ++s) ns *= static_radix(L, s);
    return ns;
}

struct NoTw {
    static constexpr int SLIM = 0;
};

template <class R, bool INV, bool TWFULL, int L, int NBATCH, int NTHR, int M, int SLIM_>
struct StageTw {
    static constexpr int SLIM = SLIM_;
    static constexpr int MB = 4;  // butterflies of a thread in one stage, at most
    C2<R> w[SLIM > 1 ? SLIM : 1][MB][3];
    template <int S>
    __device__ __forceinline__ void load_from(const C2<R>* twq, int tid) {
        if constexpr (S < SLIM && static_radix(L, S) != 0) {
            constexpr int RADIX = static_radix(L, S);
            constexpr int NS = static_ns(L, S);
            constexpr int NB = L / RADIX;
            constexpr int TOTAL = NB * NBATCH;
            constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
            static_assert(MAXB <= MB, "butterflies per thread and stage");
            constexpr int TWSTEP = M / (NS * RADIX);
            auto rd = [&](int m) {
                C2<R> v = tw_get<R, TWFULL>(twq, m, M / 4);
                if (INV) v.y = -v.y;
                return v;
            };
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                const int bf = tid + i * NTHR;
                const int j = bf - (bf / NB) * NB;
                const int e = (j - (j / NS) * NS) * TWSTEP;  // k TWSTEP, k = j mod NS
                w[S][i][0] = rd(e);
                if constexpr (RADIX >= 3) w[S][i][1] = rd(2 * e);
                if constexpr (RADIX == 8) w[S][i][2] = rd(4 * e);
            }
            load_from<S + 1>(twq, tid);
        }
    }
    // every thread of the workgroup, after the table is in LDS
    __device__ __forceinline__ void load(const C2<R>* twq, int tid) { load_from<1>(twq, tid); }
};

// apply_twiddles with the base powers wb (already conjugated for the inverse)
template <class R, int RADIX>
__device__ __forceinline__ void apply_twiddles_base(C2<R>* v, const C2<R>* wb) {
    if constexpr (RADIX == 2) {
        v[1] = cmul<R>(v[1], wb[0]);
    } else if constexpr (RADIX == 3) {
        v[1] = cmul<R>(v[1], wb[0]);
        v[2] = cmul<R>(v[2], wb[1]);
    } else if constexpr (RADIX == 4) {
        const C2<R> w1 = wb[0], w2 = wb[1];
        v[1] = cmul<R>(v[1], w1);
        v[2] = cmul<R>(v[2], w2);
        v[3] = cmul<R>(v[3], cmul<R>(w1, w2));
    } else {
        const C2<R> w1 = wb[0], w2 = wb[1], w4 = wb[2];
        const C2<R> w3 = cmul<R>(w1, w2);
        v[1] = cmul<R>(v[1], w1);
        v[2] = cmul<R>(v[2], w2);
        v[3] = cmul<R>(v[3], w3);
        v[4] = cmul<R>(v[4], w4);
        v[5] = cmul<R>(v[5], cmul<R>(w1, w4));
        v[6] = cmul<R>(v[6], cmul<R>(w2, w4));
        v[7] = cmul<R>(v[7], cmul<R>(w3, w4));
    }
}

// ---------------------------------------------------------------------------
// The same fixed-size stages between two LDS buffers.  A stage reads `a` and
// writes `b`, so no thread can overwrite what another still has to read:
// one barrier per stage instead of two, and each thread computes a butterfly
// as soon as its own loads arrive.
// ---------------------------------------------------------------------------
// Stage S (twiddles from tc for S < TC::SLIM, else from the LDS table).
template <class R, int RADIX, bool INV, bool TWFULL, int L, int NS, int NBATCH, int BSTRIDE, int NTHR, int M, int S,
          class TC>
__device__ __forceinline__ void fft_stage_pp(const C2<R>* a, C2<R>* b, const C2<R>* twq, int tid, const TC& tc) {
    constexpr int NB = L / RADIX;
    constexpr int TOTAL = NB * NBATCH;
    constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
    constexpr int TWSTEP = M / (NS * RADIX);
    constexpr int M4 = M / 4;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int bf = tid + i * NTHR;
        if (TOTAL % NTHR == 0 || bf < TOTAL) {
            const int t = bf / NB;
            const int j = bf - t * NB;
            const int q = j / NS;
            const int k = j - q * NS;
            const int ib = t * BSTRIDE + j;
            C2<R> v[RADIX];
            if constexpr (pad_linear_read(NB)) {
                const C2<R>* pa = a + lds_pad(ib);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[r] = pa[pad_offset(r, NB)];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) v[r] = a[lds_pad(ib + r * NB)];
            }
            if constexpr (S < TC::SLIM) {
                if (NS > 1) apply_twiddles_base<R, RADIX>(v, tc.w[S][i]);
            } else {
                if (NS > 1) apply_twiddles<R, RADIX, INV, TWFULL>(v, twq, k * TWSTEP, M4);
            }
            dft<R, RADIX, INV>(v);
            const int ob = t * BSTRIDE + q * NS * RADIX + k;
            if constexpr (pad_linear_write(NS, RADIX, BSTRIDE)) {
                C2<R>* pb = b + lds_pad(ob);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) pb[pad_offset(r, NS)] = v[r];
            } else {
#pragma unroll
                for (int r = 0; r < RADIX; ++r) b[lds_pad(ob + r * NS)] = v[r];
            }
        }
    }
    __syncthreads();
}

// Stages S.. of the transform, the first reading `a`; returns the buffer
// that holds the result.
template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, int S, int NS,
          class TC = NoTw>
__device__ __forceinline__ C2<R>* fft_static_pp(C2<R>* a, C2<R>* b, const C2<R>* twq, int tid, const TC& tc = TC{}) {
    constexpr int RADIX = static_radix(L, S);
    if constexpr (RADIX == 0) {
        return a;
    } else {
        fft_stage_pp<R, RADIX, INV, TWFULL, L, NS, NBATCH, BSTRIDE, NTHR, M, S>(a, b, twq, tid, tc);
        return fft_static_pp<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, S + 1, NS * RADIX>(b, a, twq, tid, tc);
    }
}

// fft_static_in on two buffers: the first stage's inputs come from g(slot)
// and go to `a`; returns the buffer holding the result.  The caller
// guarantees that no thread still reads `a`.
template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, class G, class TC = NoTw>
__device__ __forceinline__ C2<R>* fft_static_in_pp(C2<R>* a, C2<R>* b, const C2<R>* twq, int tid, G&& g,
                                                   const TC& tc = TC{}) {
    fft_static_first<R, INV, L, NBATCH, BSTRIDE, NTHR, false>(a, tid, g);
    return fft_static_pp<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, 1, static_radix(L, 0)>(a, b, twq, tid, tc);
}

// fft_static_out on two buffers, from stage S reading `a`: the last stage
// hands its outputs to f and is followed by no barrier.  Returns the buffer
// the last stage read, which threads may still be reading on return; the
// other one is free.
template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, int S, int NS, class F,
          class TC = NoTw>
__device__ __forceinline__ C2<R>* fft_static_out_pp(C2<R>* a, C2<R>* b, const C2<R>* twq, int tid, F&& f,
                                                    const TC& tc = TC{}) {
    constexpr int RADIX = static_radix(L, S);
    if constexpr (static_radix(L, S + 1) == 0) {
        constexpr int NB = L / RADIX;
        constexpr int TOTAL = NB * NBATCH;
        constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
        constexpr int TWSTEP = M / (NS * RADIX);
        constexpr int M4 = M / 4;
        static_assert(NS * RADIX == L, "the output stage is the last one");
#pragma unroll
        for (int i = 0; i < MAXB; ++i) {
            const int bf = tid + i * NTHR;
            if (TOTAL % NTHR == 0 || bf < TOTAL) {
                const int t = bf / NB;
                const int j = bf - t * NB;  // q = 0 in the last stage: k = j
                const int ib = t * BSTRIDE + j;
                C2<R> v[RADIX];
                if constexpr (pad_linear_read(NB)) {
                    const C2<R>* pa = a + lds_pad(ib);
#pragma unroll
                    for (int r = 0; r < RADIX; ++r) v[r] = pa[pad_offset(r, NB)];
                } else {
#pragma unroll
                    for (int r = 0; r < RADIX; ++r) v[r] = a[lds_pad(ib + r * NB)];
                }
                if constexpr (S < TC::SLIM) {
                    if (NS > 1) apply_twiddles_base<R, RADIX>(v, tc.w[S][i]);
                } else {
                    if (NS > 1) apply_twiddles<R, RADIX, INV, TWFULL>(v, twq, j * TWSTEP, M4);
                }
                dft<R, RADIX, INV>(v);
#pragma unroll
                for (int r = 0; r < RADIX; ++r) f(i * RADIX + r, t, j + r * NS, v[r]);
            }
        }
        return a;
    } else {
        fft_stage_pp<R, RADIX, INV, TWFULL, L, NS, NBATCH, BSTRIDE, NTHR, M, S>(a, b, twq, tid, tc);
        return fft_static_out_pp<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, S + 1, NS * RADIX>(b, a, twq, tid, f, tc);
    }
}

template <class R, bool INV, bool TWFULL, int L, int NBATCH, int BSTRIDE, int NTHR, int M, int S = 0, int NS = 1,
          class F>
__device__ __forceinline__ void fft_static_out(C2<R>* buf, const C2<R>* twq, int tid, F&& f) {
    constexpr int RADIX = static_radix(L, S);
    if constexpr (static_radix(L, S + 1) == 0) {
        fft_stage_static_out<R, RADIX, INV, TWFULL, L, NS, NBATCH, BSTRIDE, NTHR, M>(buf, twq, tid, f);
    } else {
        fft_stage_static<R, RADIX, INV, TWFULL, L, NS, NBATCH, BSTRIDE, NTHR, M>(buf, twq, tid);
        fft_static_out<R, INV, TWFULL, L, NBATCH, BSTRIDE, NTHR, M, S + 1, NS * RADIX>(buf, twq, tid, f);
    }
}

}  // namespace se2n
