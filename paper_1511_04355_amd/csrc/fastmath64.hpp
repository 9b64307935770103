// FP64 exp, sincos and reciprocal square root for the kernel evaluation,
// written from their mathematical definitions: the argument reduction of Cody
// and Waite (Software Manual for the Elementary Functions, 1980: the reduction
// constant split into parts whose products with the integer multiple are
// exact), a table of the function at the reduction points, and Taylor
// polynomials on the remaining interval; rsqrt by the hardware estimate and
// two Newton steps.  They replace the general library routines (no
// large-argument paths, no IEEE division sequences) in the VALU-bound
// far-field loops.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace afsbem {

// Table-driven e^a and (sin y, cos y) for the FP64 kernel loops.  tab holds
// kFmTabLen doubles: tab[j] = 2^(j/64) and tab[64 + 2j], tab[65 + 2j] =
// cos, sin of j pi/32 (j = 0..63), each rounded once from extended precision,
// the zeros of the trigonometric table exact.  Reduction by multiples of
// ln 2/64 (pi/32), split into a leading part of 32 (31) significant bits and
// a remainder (two remainders for pi/32), so that the leading product with
// the multiple is exact, leaves |r| <= ln 2/128 (pi/64), where the Taylor
// polynomials of degree 5 (exp), 7 (sin) and 8 (cos) are within 5e-17; the
// table entry multiplies (exp) or rotates (sincos) the result: about 2 ulp in
// all, with 35 operations for one exp and one sincos (54 with a reduction by
// ln 2 and pi/2 alone and the longer polynomials it needs).
constexpr int kFmTabLen = 192;

__host__ __device__ __forceinline__ double exp_tab(double a, const double *__restrict__ tab) {
    a = fmin(fmax(a, -745.0), 709.0);
    const double k = rint(a * 92.33248261689366);              // a / (ln 2 / 64)
    double r = fma(-k, 0.01083042469326756, a);                // ln 2 / 64, leading 32 bits
    r = fma(-k, 2.9815858269852933e-12, r);                    // ln 2 / 64, remainder
    double p = 0.008333333333333333;                           // 1/5!
    p = fma(p, r, 0.041666666666666664);                       // 1/4!
    p = fma(p, r, 0.16666666666666666);                        // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int ki = (int)k;
    return ldexp(tab[ki & 63] * p, ki >> 6);                   // 2^(ki/64) = 2^(ki>>6) 2^((ki&63)/64)
}

// |y| < 4e5
__host__ __device__ __forceinline__ void sincos_tab(double y, const double *__restrict__ tab, double *s_out,
                                                    double *c_out) {
    const double k = rint(y * 10.185916357881302);             // y / (pi / 32)
    double r = fma(-k, 0.09817477042088285, y);                // pi / 32 in three parts
    r = fma(-k, 3.798187816439979e-12, r);
    r = fma(-k, 1.2639164054974691e-22, r);
    const double r2 = r * r;
    double ps = -0.0001984126984126984;                        // -1/7!
    ps = fma(ps, r2, 0.008333333333333333);                    // 1/5!
    ps = fma(ps, r2, -0.16666666666666666);                    // -1/3!
    const double sn = fma(ps * r2, r, r);
    double pc = 2.48015873015873e-05;                          // 1/8!
    pc = fma(pc, r2, -0.001388888888888889);                   // -1/6!
    pc = fma(pc, r2, 0.041666666666666664);                    // 1/4!
    pc = fma(pc, r2, -0.5);
    const double cs = fma(pc, r2, 1.0);
    const double *e = tab + 64 + 2 * ((int)k & 63);            // cos, sin of (k mod 64) pi / 32
    *s_out = fma(e[1], cs, e[0] * sn);
    *c_out = fma(e[0], cs, -(e[1] * sn));
}

// 1 / sqrt(a), a > 0 finite: hardware estimate refined by two Newton steps
// y <- y (3/2 - a y^2 / 2) (each step squares the relative error)
__device__ __forceinline__ double rsqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

}  // namespace afsbem
