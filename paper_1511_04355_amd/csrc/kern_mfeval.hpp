// Complex arithmetic and the radial functions of the fundamental solutions
// in the evaluation precision R (float for the FP32 products of the mixed
// path, double otherwise), shared by the matrix-free and hierarchical
// far-field kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fastmath64.hpp"

namespace afsbem {

template <class R>
struct cx {
    R r, i;
};
template <class R>
__device__ __forceinline__ cx<R> cxadd(cx<R> a, cx<R> b) {
    return {a.r + b.r, a.i + b.i};
}
template <class R>
__device__ __forceinline__ cx<R> cxsub(cx<R> a, cx<R> b) {
    return {a.r - b.r, a.i - b.i};
}
template <class R>
__device__ __forceinline__ cx<R> cxmul(cx<R> a, cx<R> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class R>
__device__ __forceinline__ cx<R> cxs(cx<R> a, R s) {
    return {a.r * s, a.i * s};
}

// e^a, sin b, cos b: the hardware's FP32 approximations, or the FP64 table
// functions on tab (the kFmTabLen entries after the series coefficients)
__device__ __forceinline__ void exp_sincos(float a, float b, float &e, float &sn, float &cs,
                                           const float * /*tab*/) {
    e = __expf(a);
    __sincosf(b, &sn, &cs);
}
__device__ __forceinline__ void exp_sincos(double a, double b, double &e, double &sn, double &cs,
                                           const double *__restrict__ tab) {
    e = exp_tab(a, tab);
    sincos_tab(b, tab, &sn, &cs);
}
__device__ __forceinline__ float inv_sqrt(float a) { return rsqrtf(a); }
__device__ __forceinline__ double inv_sqrt(double a) { return rsqrt_nr(a); }

// Series about 0 below |x|^2 < thr2, closed form above.  FP32: |x| < 1/2 with
// 9 terms (truncation ~1e-9; the closed form loses eps32/|x|^2 <= 5e-7 above);
// FP64: |x| < 1/4 with 13 terms (the remaining stored terms sum to below 7e-17
// of the leading ones there).
template <class R>
struct MfTraits;
template <>
struct MfTraits<float> {
    static constexpr float thr2 = 0.25f;
    static constexpr int nser = 9;
    static constexpr int unroll = 8;  // the whole Horner loop
};
template <>
struct MfTraits<double> {
    static constexpr double thr2 = 0.0625;
    static constexpr int nser = 13;
    static constexpr int unroll = 4;  // a full unroll keeps all 48 coefficients live (192 VGPRs)
};

template <class R>
struct MfRad {
    cx<R> Psi, X, Psd, Xd;
};

// The four series p_k(x) = sum_{n < NT} c[4 n + k] x^n (real coefficients) at
// complex x = (xr, xi), ax2 = |x|^2: synthetic division of each by the real
// quadratic t^2 - 2 xr t + |x|^2, whose roots are x and its conjugate, leaves
// a remainder alpha t + beta with p_k(x) = alpha x + beta (Knuth, The Art of
// Computer Programming vol. 2, 4.6.4): two real operations per coefficient
// instead of the four of a complex Horner step, with the same rounding error
// relative to sum_n |c_n| |x|^n.
template <class R, int NT, int UNROLL>
__device__ __forceinline__ void series4(const R *__restrict__ c, R xr, R xi, R ax2, R pr[4], R pi[4]) {
    static_assert(NT >= 2, "at least a linear series");
    const R rr = R(2) * xr, ss = -ax2;
    R b1[4], b2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b1[k] = c[4 * (NT - 1) + k];
        b2[k] = R(0);
    }
#pragma unroll UNROLL
    for (int n = NT - 2; n >= 1; --n)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const R bn = c[4 * n + k] + rr * b1[k] + ss * b2[k];
            b2[k] = b1[k];
            b1[k] = bn;
        }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const R beta = c[k] + ss * b2[k];
        pr[k] = b1[k] * xr + beta;
        pi[k] = b1[k] * xi;
    }
}

// inv_ax2 = 1 / |x|^2, supplied by the caller from 1/r (no division); coef:
// the 64 series coefficients, in FP64 followed by the kFmTabLen table entries
template <class R>
__device__ __forceinline__ MfRad<R> mf_radial(cx<R> x, R beta, const R *__restrict__ coef, R inv_ax2) {
    MfRad<R> o;
    const R ax2 = x.r * x.r + x.i * x.i;
    if (ax2 < MfTraits<R>::thr2) {
        R pr[4], pi[4];
        series4<R, MfTraits<R>::nser, MfTraits<R>::unroll>(coef, x.r, x.i, ax2, pr, pi);
        o.Psi = cx<R>{pr[0], pi[0]};
        o.X = cx<R>{pr[1], pi[1]};
        o.Psd = cx<R>{pr[2], pi[2]};
        o.Xd = cx<R>{pr[3], pi[3]};
        return o;
    }
    R ex, sn, cs, exq, snq, csq;
    exp_sincos(-x.r, x.i, ex, sn, cs, coef + 64);
    exp_sincos(-beta * x.r, beta * x.i, exq, snq, csq, coef + 64);
    const cx<R> e{ex * cs, -ex * sn};      // e^{-x}
    const cx<R> ep{exq * csq, -exq * snq};  // e^{-beta x}
    const R inv = inv_ax2;
    const cx<R> ix{x.r * inv, -x.i * inv};
    const cx<R> ix2 = cxmul(ix, ix);
    const R b2 = beta * beta, b3 = b2 * beta;
    const cx<R> P = cxmul(ep, cx<R>{b2 + R(3) * beta * ix.r + R(3) * ix2.r, R(3) * beta * ix.i + R(3) * ix2.i});
    o.Psi = cxsub(cxmul(e, cx<R>{R(1) + ix.r + ix2.r, ix.i + ix2.i}),
                  cxmul(ep, cx<R>{beta * ix.r + ix2.r, beta * ix.i + ix2.i}));
    o.X = cxsub(cxmul(e, cx<R>{R(1) + R(3) * ix.r + R(3) * ix2.r, R(3) * ix.i + R(3) * ix2.i}), P);
    o.Psd = cxsub(P, cxmul(e, cx<R>{x.r + R(2) + R(3) * ix.r + R(3) * ix2.r, x.i + R(3) * ix.i + R(3) * ix2.i}));
    o.Xd = cxsub(cxmul(ep, cx<R>{b3 * x.r + R(4) * b2 + R(9) * beta * ix.r + R(9) * ix2.r,
                                 b3 * x.i + R(9) * beta * ix.i + R(9) * ix2.i}),
                 cxmul(e, cx<R>{x.r + R(4) + R(9) * ix.r + R(9) * ix2.r, x.i + R(9) * ix.i + R(9) * ix2.i}));
    return o;
}

}  // namespace afsbem
