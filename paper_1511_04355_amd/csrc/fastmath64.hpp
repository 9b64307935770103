// FP64 exp, sincos and reciprocal square root for the kernel evaluation,
// written from their mathematical definitions: the argument reduction of Cody
// and Waite (Software Manual for the Elementary Functions, 1980: ln 2 and pi/2
// split into parts whose products with the integer multiple are exact) and
// Taylor polynomials on the reduced interval, truncated below 1e-17 relative;
// rsqrt by the hardware estimate and two Newton steps.  Measured against
// long-double references: ~1 ulp.  They replace the general library routines
// (no large-argument paths, no IEEE division sequences) in the VALU-bound
// far-field loops.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace afsbem {

// e^a for a in [-745, 709]; clamped outside
__host__ __device__ __forceinline__ double exp_cw(double a) {
    a = fmin(fmax(a, -745.0), 709.0);
    const double k = rint(a * 1.4426950408889634);            // a / ln 2
    double r = fma(-k, 0.6931471803691238, a);                 // ln 2, leading 32 bits
    r = fma(-k, 1.9082149292705877e-10, r);                    // ln 2, remainder
    // |r| <= 0.347: Taylor to r^13 (next term < 2e-17)
    double p = 1.6059043836821613e-10;                         // 1/13!
    p = fma(p, r, 2.08767569878681e-09);                       // 1/12!
    p = fma(p, r, 2.505210838544172e-08);                      // 1/11!
    p = fma(p, r, 2.755731922398589e-07);                      // 1/10!
    p = fma(p, r, 2.7557319223985893e-06);                     // 1/9!
    p = fma(p, r, 2.48015873015873e-05);                       // 1/8!
    p = fma(p, r, 0.0001984126984126984);                      // 1/7!
    p = fma(p, r, 0.001388888888888889);                       // 1/6!
    p = fma(p, r, 0.008333333333333333);                       // 1/5!
    p = fma(p, r, 0.041666666666666664);                       // 1/4!
    p = fma(p, r, 0.16666666666666666);                        // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// sin y, cos y for |y| < 1e5 (reduction by multiples of pi/2 in three parts)
__host__ __device__ __forceinline__ void sincos_cw(double y, double *s_out, double *c_out) {
    const double k = rint(y * 0.6366197723675814);             // y / (pi/2)
    double r = fma(-k, 1.5707963267341256, y);
    r = fma(-k, 6.077100506303966e-11, r);
    r = fma(-k, 2.0222662487959506e-21, r);
    const double r2 = r * r;
    // |r| <= pi/4: sin to r^17, cos to r^16 (next terms < 1e-18 relative)
    double ps = 2.8114572543455206e-15;                        // 1/17!
    ps = fma(ps, r2, -7.647163731819816e-13);                  // -1/15!
    ps = fma(ps, r2, 1.6059043836821613e-10);                  // 1/13!
    ps = fma(ps, r2, -2.505210838544172e-08);                  // -1/11!
    ps = fma(ps, r2, 2.7557319223985893e-06);                  // 1/9!
    ps = fma(ps, r2, -0.0001984126984126984);                  // -1/7!
    ps = fma(ps, r2, 0.008333333333333333);                    // 1/5!
    ps = fma(ps, r2, -0.16666666666666666);                    // -1/3!
    const double sn = fma(ps * r2, r, r);
    double pc = 4.779477332387385e-14;                         // 1/16!
    pc = fma(pc, r2, -1.1470745597729725e-11);                 // -1/14!
    pc = fma(pc, r2, 2.08767569878681e-09);                    // 1/12!
    pc = fma(pc, r2, -2.755731922398589e-07);                  // -1/10!
    pc = fma(pc, r2, 2.48015873015873e-05);                    // 1/8!
    pc = fma(pc, r2, -0.001388888888888889);                   // -1/6!
    pc = fma(pc, r2, 0.041666666666666664);                    // 1/4!
    pc = fma(pc, r2, -0.5);
    const double cs = fma(pc, r2, 1.0);
    const int q = (int)((long long)k & 3);
    const double s_ = (q & 1) ? cs : sn, c_ = (q & 1) ? sn : cs;
    *s_out = (q & 2) ? -s_ : s_;
    *c_out = ((q + 1) & 2) ? -c_ : c_;
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
