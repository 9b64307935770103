// Minimal complex<double> arithmetic for device code (interleaved re, im).
#pragma once
#include <hip/hip_runtime.h>

namespace afsbem {

struct cd {
    double r, i;
};

__host__ __device__ __forceinline__ cd cadd(cd a, cd b) { return cd{a.r + b.r, a.i + b.i}; }
__host__ __device__ __forceinline__ cd csub(cd a, cd b) { return cd{a.r - b.r, a.i - b.i}; }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b) { return cd{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__host__ __device__ __forceinline__ cd cscale(cd a, double s) { return cd{a.r * s, a.i * s}; }
__host__ __device__ __forceinline__ cd cconj(cd a) { return cd{a.r, -a.i}; }
// p * x + c with c real
__host__ __device__ __forceinline__ cd cfma_real(cd p, cd x, double c) {
    return cd{p.r * x.r - p.i * x.i + c, p.r * x.i + p.i * x.r};
}
__host__ __device__ __forceinline__ cd cinv(cd a) {
    const double d = 1.0 / (a.r * a.r + a.i * a.i);
    return cd{a.r * d, -a.i * d};
}

}  // namespace afsbem
