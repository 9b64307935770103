// Multilayer perceptron forward / backward / Adam for the learned warm start,
// on gfx950 matrix cores.
//
//   Z1 = X W1 + b1, H1 = silu(Z1), Z2 = H1 W2 + b2, H2 = silu(Z2), Y = H2 W3 + b3
//   loss = mean (Y - T)^2
// Flat FP32 parameter layout: W1 [d_in, H] row-major, b1 [H], W2 [H, H], b2 [H],
// W3 [H, d_out], b3 [d_out].
//
// Every product is C[M, N] = op(A)[M, K] op(B)[K, N] with op = optional
// transpose through strides.  One wavefront computes one 16 x 16 tile of C.
// Mode 1 (production): v_mfma_f32_16x16x16_bf16 -- FP32 activations and
// weights are rounded to bfloat16 (nearest-even) when the fragments are
// loaded, products accumulate in FP32.  Mode 0 (reference arithmetic): FP32
// fused multiply-adds in the same tiling.  Lane layout of the 16x16x16 MFMA:
// lane l holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16] (j = 0..3) and
// receives D[4(l/16)+j][l%16].
#include "internal.hpp"
#include "mlp.hpp"

namespace afsbem {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (short)(u >> 16);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float sg = 1.0f / (1.0f + __expf(-z));
    return sg * (1.0f + z * (1.0f - sg));
}

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_DSILU = 3 };

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t sa_m, sa_k;  // element (m, k) of op(A) at A[m*sa_m + k*sa_k]
    const float *B;
    int64_t sb_k, sb_n;  // element (k, n) of op(B) at B[k*sb_k + n*sb_n]
    float *C;
    int64_t ldc;         // C row-major
    const float *bias;   // [N]
    float *Zout;         // EPI_BIAS_SILU: pre-activation copy (row-major, ldc)
    const float *Zin;    // EPI_DSILU: pre-activation to differentiate (row-major, ldc)
};

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tiles_n = (g.N + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    const int64_t tiles = (int64_t)((g.M + 15) / 16) * tiles_n;
    if (tile >= tiles)
        return;
    const int tm = (int)(tile / tiles_n) * 16, tn = (int)(tile % tiles_n) * 16;
    const int i = lane & 15, grp = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (MODE == 1) {
        for (int k0 = 0; k0 < g.K; k0 += 16) {
            bf16x4 a, b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = k0 + 4 * grp + j;
                const int m = tm + i, n = tn + i;
                const float av = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sa_m + (int64_t)k * g.sa_k] : 0.f;
                const float bv = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.sb_k + (int64_t)n * g.sb_n] : 0.f;
                a[j] = to_bf16(av);
                b[j] = to_bf16(bv);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
    } else {
        // the same output ownership as the MFMA layout: D[4*grp + j][i]
        const int n = tn + i;
        for (int k = 0; k < g.K; ++k) {
            const float bv = (n < g.N) ? g.B[(int64_t)k * g.sb_k + (int64_t)n * g.sb_n] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = tm + 4 * grp + j;
                const float av = (m < g.M) ? g.A[(int64_t)m * g.sa_m + (int64_t)k * g.sa_k] : 0.f;
                acc[j] = fmaf(av, bv, acc[j]);
            }
        }
    }
    const int n = tn + i;
    if (n >= g.N)
        return;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = tm + 4 * grp + j;
        if (m >= g.M)
            continue;
        const int64_t o = (int64_t)m * g.ldc + n;
        float v = acc[j];
        if (EPI == EPI_BIAS || EPI == EPI_BIAS_SILU)
            v += g.bias[n];
        if (EPI == EPI_BIAS_SILU) {
            g.Zout[o] = v;
            v = silu_f(v);
        }
        if (EPI == EPI_DSILU)
            v *= dsilu_f(g.Zin[o]);
        g.C[o] = v;
    }
}

template <int EPI>
static void gemm(int mode, const GemmArgs &g, hipStream_t st) {
    const int64_t tiles = (int64_t)((g.M + 15) / 16) * ((g.N + 15) / 16);
    const unsigned blocks = (unsigned)((tiles + 3) / 4);
    if (blocks == 0)
        return;
    if (mode == 1)
        gemm_kernel<1, EPI><<<blocks, 256, 0, st>>>(g);
    else
        gemm_kernel<0, EPI><<<blocks, 256, 0, st>>>(g);
    AFS_HIP(hipGetLastError());
}

// column sums of a row-major [M, N] matrix into out[N] (bias gradients)
__global__ __launch_bounds__(256) void colsum_kernel(int M, int N, const float *__restrict__ D, float *__restrict__ out) {
    const int n = blockIdx.x;
    __shared__ float sm[256];
    float acc = 0.f;
    for (int m = threadIdx.x; m < M; m += 256)
        acc += D[(int64_t)m * N + n];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sm[threadIdx.x] += sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[n] = sm[0];
}

// dY = 2 (Y - T) / (M N); per-block partial sums of (Y - T)^2
__global__ __launch_bounds__(256) void mse_grad_kernel(int64_t count, const float *__restrict__ Y,
                                                       const float *__restrict__ T, float inv_count,
                                                       float *__restrict__ dY, float *__restrict__ partial) {
    __shared__ float sm[256];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float r2 = 0.f;
    if (k < count) {
        const float r = Y[k] - T[k];
        dY[k] = 2.f * r * inv_count;
        r2 = r * r;
    }
    sm[threadIdx.x] = r2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sm[threadIdx.x] += sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void sum_kernel(int n, const float *__restrict__ x, float scale,
                                                  float *__restrict__ out) {
    __shared__ float sm[256];
    float acc = 0.f;
    for (int k = threadIdx.x; k < n; k += 256)
        acc += x[k];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            sm[threadIdx.x] += sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = sm[0] * scale;
}

__global__ __launch_bounds__(256) void adam_kernel(int64_t n, float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// --------------------------------------------------------------- host side --
MlpShape::MlpShape(int di, int h, int dout) : d_in(di), hidden(h), d_out(dout) {
    oW1 = 0;
    ob1 = oW1 + (int64_t)d_in * hidden;
    oW2 = ob1 + hidden;
    ob2 = oW2 + (int64_t)hidden * hidden;
    oW3 = ob2 + hidden;
    ob3 = oW3 + (int64_t)hidden * d_out;
    n_params = ob3 + d_out;
}

size_t mlp_work_floats(const MlpShape &s, int n) {
    // Z1, H1, Z2, H2 (n x H each), Y, dY (n x d_out), dZ2, dZ1 (n x H), loss partials
    return (size_t)n * (6 * (size_t)s.hidden + 2 * (size_t)s.d_out) + (size_t)((int64_t)n * s.d_out / 256 + 2) + 64;
}

void mlp_forward(const MlpShape &s, int mode, int n, const float *P, const float *X, float *Y, float *work,
                 hipStream_t st) {
    const int H = s.hidden;
    float *Z1 = work, *H1 = Z1 + (size_t)n * H, *Z2 = H1 + (size_t)n * H, *H2 = Z2 + (size_t)n * H;
    GemmArgs g{};
    g = GemmArgs{n, H, s.d_in, X, s.d_in, 1, P + s.oW1, H, 1, H1, H, P + s.ob1, Z1, nullptr};
    gemm<EPI_BIAS_SILU>(mode, g, st);
    g = GemmArgs{n, H, H, H1, H, 1, P + s.oW2, H, 1, H2, H, P + s.ob2, Z2, nullptr};
    gemm<EPI_BIAS_SILU>(mode, g, st);
    g = GemmArgs{n, s.d_out, H, H2, H, 1, P + s.oW3, s.d_out, 1, Y, s.d_out, P + s.ob3, nullptr, nullptr};
    gemm<EPI_BIAS>(mode, g, st);
}

void mlp_loss_grad(const MlpShape &s, int mode, int n, const float *P, const float *X, const float *T, float *G,
                   float *loss, float *work, hipStream_t st) {
    const int H = s.hidden, D = s.d_out;
    float *Z1 = work, *H1 = Z1 + (size_t)n * H, *Z2 = H1 + (size_t)n * H, *H2 = Z2 + (size_t)n * H;
    float *dZ2 = H2 + (size_t)n * H, *dZ1 = dZ2 + (size_t)n * H;
    float *Y = dZ1 + (size_t)n * H, *dY = Y + (size_t)n * D, *part = dY + (size_t)n * D;
    mlp_forward(s, mode, n, P, X, Y, work, st);
    const int64_t cnt = (int64_t)n * D;
    const unsigned nb = (unsigned)((cnt + 255) / 256);
    mse_grad_kernel<<<nb, 256, 0, st>>>(cnt, Y, T, 1.f / (float)cnt, dY, part);
    if (loss)
        sum_kernel<<<1, 256, 0, st>>>((int)nb, part, 1.f / (float)cnt, loss);
    AFS_HIP(hipGetLastError());
    GemmArgs g{};
    // gW3 = H2^T dY  [H, D]
    g = GemmArgs{H, D, n, H2, 1, H, dY, D, 1, G + s.oW3, D, nullptr, nullptr, nullptr};
    gemm<EPI_STORE>(mode, g, st);
    colsum_kernel<<<D, 256, 0, st>>>(n, D, dY, G + s.ob3);
    // dZ2 = (dY W3^T) * silu'(Z2)  [n, H]
    g = GemmArgs{n, H, D, dY, D, 1, P + s.oW3, 1, D, dZ2, H, nullptr, nullptr, Z2};
    gemm<EPI_DSILU>(mode, g, st);
    // gW2 = H1^T dZ2
    g = GemmArgs{H, H, n, H1, 1, H, dZ2, H, 1, G + s.oW2, H, nullptr, nullptr, nullptr};
    gemm<EPI_STORE>(mode, g, st);
    colsum_kernel<<<H, 256, 0, st>>>(n, H, dZ2, G + s.ob2);
    // dZ1 = (dZ2 W2^T) * silu'(Z1)
    g = GemmArgs{n, H, H, dZ2, H, 1, P + s.oW2, 1, H, dZ1, H, nullptr, nullptr, Z1};
    gemm<EPI_DSILU>(mode, g, st);
    // gW1 = X^T dZ1  [d_in, H]
    g = GemmArgs{s.d_in, H, n, X, 1, s.d_in, dZ1, H, 1, G + s.oW1, H, nullptr, nullptr, nullptr};
    gemm<EPI_STORE>(mode, g, st);
    colsum_kernel<<<H, 256, 0, st>>>(n, H, dZ1, G + s.ob1);
    AFS_HIP(hipGetLastError());
}

void mlp_adam(int64_t n, float *P, const float *G, float *m, float *v, int t, float lr, float b1, float b2, float eps,
              hipStream_t st) {
    const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
    adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, P, G, m, v, lr, b1, b2, eps, c1, c2);
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem

namespace afsbem {

// ------------------------------------------------ learned warm start glue --
// Element features at one frequency: centroid scaled to [-1, 1] by the mesh
// box (3), unit normal (3), s / s_scale (2), sin and cos of pi k c_d for
// k = 1..4 and the three scaled coordinates (24): kLearnFeatures = 32.
__global__ __launch_bounds__(256) void learn_features_kernel(int64_t nt, const double *__restrict__ colx,
                                                             const double *__restrict__ coly,
                                                             const double *__restrict__ colz,
                                                             const double *__restrict__ nrm, double cx, double cy,
                                                             double cz, double half, float sr, float si,
                                                             float *__restrict__ X) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= nt)
        return;
    float *x = X + m * kLearnFeatures;
    const float c[3] = {(float)((colx[m] - cx) / half), (float)((coly[m] - cy) / half), (float)((colz[m] - cz) / half)};
    x[0] = c[0];
    x[1] = c[1];
    x[2] = c[2];
    x[3] = (float)nrm[3 * m];
    x[4] = (float)nrm[3 * m + 1];
    x[5] = (float)nrm[3 * m + 2];
    x[6] = sr;
    x[7] = si;
    int o = 8;
    for (int d = 0; d < 3; ++d)
        for (int k = 1; k <= 4; ++k) {
            float sn, cs;
            __sincosf(3.14159265f * k * c[d], &sn, &cs);
            x[o++] = sn;
            x[o++] = cs;
        }
}

// targets: solution components divided by the complex scale c, as (re, im) x 3
__global__ __launch_bounds__(256) void learn_targets_kernel(int64_t nt, const double *__restrict__ a, double cr,
                                                            double ci, float *__restrict__ T) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;  // complex entry
    if (k >= 3 * nt)
        return;
    const double ar = a[2 * k], ai = a[2 * k + 1];
    const double d = cr * cr + ci * ci;
    T[2 * k] = (float)((ar * cr + ai * ci) / d);
    T[2 * k + 1] = (float)((ai * cr - ar * ci) / d);
}

__global__ __launch_bounds__(256) void learn_unpack_kernel(int64_t nt, const float *__restrict__ Y,
                                                           double *__restrict__ x0) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= 6 * nt)
        return;
    x0[k] = (double)Y[k];
}

// rows idx[0..B) of src [*, d] into dst [B, d]
__global__ __launch_bounds__(256) void gather_rows_kernel(int B, int d, const int32_t *__restrict__ idx,
                                                          const float *__restrict__ src, float *__restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)B * d)
        return;
    const int r = (int)(k / d), c = (int)(k % d);
    dst[k] = src[(int64_t)idx[r] * d + c];
}

void learn_features(int64_t nt, const DevicePlan &d, const double box[4], float sr, float si, float *X,
                    hipStream_t st) {
    learn_features_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(nt, d.colx, d.coly, d.colz, d.nrm, box[0],
                                                                        box[1], box[2], box[3], sr, si, X);
    AFS_HIP(hipGetLastError());
}

void learn_targets(int64_t nt, const double *a, double cr, double ci, float *T, hipStream_t st) {
    learn_targets_kernel<<<(unsigned)((3 * nt + 255) / 256), 256, 0, st>>>(nt, a, cr, ci, T);
    AFS_HIP(hipGetLastError());
}

void learn_unpack(int64_t nt, const float *Y, double *x0, hipStream_t st) {
    learn_unpack_kernel<<<(unsigned)((6 * nt + 255) / 256), 256, 0, st>>>(nt, Y, x0);
    AFS_HIP(hipGetLastError());
}

void gather_rows(int B, int d, const int32_t *idx, const float *src, float *dst, hipStream_t st) {
    gather_rows_kernel<<<(unsigned)(((int64_t)B * d + 255) / 256), 256, 0, st>>>(B, d, idx, src, dst);
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
