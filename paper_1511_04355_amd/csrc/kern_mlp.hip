// Multilayer perceptron forward / backward / Adam for the learned warm start,
// on gfx950 matrix cores.
//
//   Z1 = X W1 + b1, H1 = silu(Z1), Z2 = H1 W2 + b2, H2 = silu(Z2), Y = H2 W3 + b3
//   loss = mean (Y - T)^2
// Flat FP32 parameter layout: W1 [d_in, H] row-major, b1 [H], W2 [H, H], b2 [H],
// W3 [H, d_out], b3 [d_out].
//
// Every product is C[M, N] = op(A)[M, K] op(B)[K, N], op an optional
// transpose.  A work-group of four wavefronts computes a 64 x 64 tile of C,
// each wavefront a 32 x 32 quarter as 2 x 2 tiles of 16 x 16.  The K loop
// stages 64 x 32 slices of op(A) and op(B) in LDS: every thread fetches eight
// consecutive FP32 values of its operand's contiguous dimension (two 16-byte
// loads when the leading dimension allows), rounds them once (mode 1) and
// stores them k-contiguous per row of op(A) and per column of op(B), so that
// each fragment is one 8-byte LDS read; the next slice's global loads are in
// flight while the current one is contracted.  Weight gradients (K = batch
// rows) split K over grid.z into planes of partial sums that a second pass
// adds in a fixed order (and, in training, feeds straight into Adam); their
// bias gradients ride along as an extra row of ones in op(A), which the flat
// parameter layout places right after each weight matrix.
// Mode 1 (production): v_mfma_f32_16x16x16_bf16 -- FP32 activations and
// weights are rounded to bfloat16 (nearest-even) when staged, products
// accumulate in FP32.  Mode 0 (reference arithmetic): FP32 fused
// multiply-adds on the same tiles.  Lane layout of the 16x16x16 MFMA: lane l
// holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16] (j = 0..3) and receives
// D[4(l/16)+j][l%16].
#include <algorithm>

#include "internal.hpp"
#include "mlp.hpp"

namespace afsbem {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
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

constexpr int kBM = 64, kBN = 64, kBK = 32;
constexpr int kLdk = 40;  // LDS row stride in elements (16-byte aligned rows for both element types)

struct GemmArgs {
    int M, N, K;
    const float *A;
    int64_t lda;         // TA = 0: op(A)(m, k) = A[m lda + k]; TA = 1: A[k lda + m]
    const float *B;
    int64_t ldb;         // TB = 0: op(B)(k, n) = B[k ldb + n]; TB = 1: B[n ldb + k]
    float *C;
    int64_t ldc;         // C row-major
    const float *bias;   // [N]
    float *Zout;         // EPI_BIAS_SILU: pre-activation copy (row-major, ldc)
    const float *Zin;    // EPI_DSILU: pre-activation to differentiate (row-major, ldc)
    int ones_row;        // TA = 1: row M-1 of op(A) is all ones (the bias-gradient row)
    int kc;              // K per split (multiple of kBK); split z covers [z kc, min(K, (z+1) kc))
    int64_t c_split;     // elements between the output planes of consecutive splits
};

template <int MODE>
struct Lds {
    typedef typename std::conditional<MODE == 1, short, float>::type E;
};

__device__ __forceinline__ void ld8(const float *p, float (&r)[8]) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    const float4 b = *reinterpret_cast<const float4 *>(p + 4);
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w;
    r[4] = b.x; r[5] = b.y; r[6] = b.z; r[7] = b.w;
}

// eight values of op(A) for this thread's slot of the slice at k0
template <int TA>
__device__ __forceinline__ void fetch_a(const GemmArgs &g, int m0, int k0, int kend, bool vec, float (&r)[8]) {
    const int t = threadIdx.x;
    if (TA == 0) {
        const int m = m0 + (t >> 2), k = k0 + (t & 3) * 8;
        const float *p = g.A + (int64_t)m * g.lda + k;
        if (m < g.M && vec && k + 8 <= kend) {
            ld8(p, r);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                r[j] = (m < g.M && k + j < kend) ? p[j] : 0.f;
        }
    } else {
        const int k = k0 + (t >> 3), m = m0 + (t & 7) * 8;
        const int mreal = g.M - g.ones_row;
        const float *p = g.A + (int64_t)k * g.lda + m;
        if (k < kend && vec && m + 8 <= mreal) {
            ld8(p, r);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int mj = m + j;
                r[j] = (k < kend && mj < mreal) ? p[j] : ((k < kend && g.ones_row && mj == mreal) ? 1.f : 0.f);
            }
        }
    }
}

template <int TB>
__device__ __forceinline__ void fetch_b(const GemmArgs &g, int n0, int k0, int kend, bool vec, float (&r)[8]) {
    const int t = threadIdx.x;
    if (TB == 1) {
        const int n = n0 + (t >> 2), k = k0 + (t & 3) * 8;
        const float *p = g.B + (int64_t)n * g.ldb + k;
        if (n < g.N && vec && k + 8 <= kend) {
            ld8(p, r);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                r[j] = (n < g.N && k + j < kend) ? p[j] : 0.f;
        }
    } else {
        const int k = k0 + (t >> 3), n = n0 + (t & 7) * 8;
        const float *p = g.B + (int64_t)k * g.ldb + n;
        if (k < kend && vec && n + 8 <= g.N) {
            ld8(p, r);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                r[j] = (k < kend && n + j < g.N) ? p[j] : 0.f;
        }
    }
}

// slot layout: "row-contiguous" slots (TA = 0 / TB = 1) hold 8 consecutive k
// of one row; the others hold one k of 8 consecutive rows
template <int MODE, bool KCONTIG>
__device__ __forceinline__ void stage(typename Lds<MODE>::E *S, const float (&r)[8]) {
    typedef typename Lds<MODE>::E E;
    const int t = threadIdx.x;
    if (KCONTIG) {
        E *d = S + (t >> 2) * kLdk + (t & 3) * 8;
        if (MODE == 1) {
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                v[j] = to_bf16(r[j]);
            *reinterpret_cast<bf16x8 *>(d) = v;
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                d[j] = (E)r[j];
        }
    } else {
        E *d = S + (t & 7) * 8 * kLdk + (t >> 3);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (MODE == 1)
                d[j * kLdk] = to_bf16(r[j]);
            else
                d[j * kLdk] = (E)r[j];
        }
    }
}

template <int MODE, int EPI, int TA, int TB>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    typedef typename Lds<MODE>::E E;
    __shared__ __align__(16) E As[kBM * kLdk];
    __shared__ __align__(16) E Bs[kBN * kLdk];
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int kbeg = blockIdx.z * g.kc;
    const int kend = min(g.K, kbeg + g.kc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, grp = lane >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const bool va = (g.lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
    const bool vb = (g.ldb % 4 == 0) && ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0);
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    float ra[8], rb[8];
    if (kbeg < kend) {
        fetch_a<TA>(g, m0, kbeg, kend, va, ra);
        fetch_b<TB>(g, n0, kbeg, kend, vb, rb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += kBK) {
        __syncthreads();  // the previous slice has been contracted
        stage<MODE, TA == 0>(As, ra);
        stage<MODE, TB == 1>(Bs, rb);
        __syncthreads();
        if (k0 + kBK < kend) {
            fetch_a<TA>(g, m0, k0 + kBK, kend, va, ra);
            fetch_b<TB>(g, n0, k0 + kBK, kend, vb, rb);
        }
        if (MODE == 1) {
#pragma unroll
            for (int ks = 0; ks < kBK; ks += 16) {
                bf16x4 fa[2], fb[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    fa[q] = *reinterpret_cast<const bf16x4 *>(As + (wm + 16 * q + i) * kLdk + ks + 4 * grp);
                    fb[q] = *reinterpret_cast<const bf16x4 *>(Bs + (wn + 16 * q + i) * kLdk + ks + 4 * grp);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
        } else {
            // the same output ownership as the MFMA layout: D[4 grp + j][i] of each 16 x 16 tile
            for (int k = 0; k < kBK; ++k) {
                float bv[2];
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    bv[b] = (float)Bs[(wn + 16 * b + i) * kLdk + k];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float av = (float)As[(wm + 16 * a + 4 * grp + j) * kLdk + k];
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[a][b][j] = fmaf(av, bv[b], acc[a][b][j]);
                    }
            }
        }
    }
    float *C = g.C + (int64_t)blockIdx.z * g.c_split;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int n = n0 + wn + 16 * b + i;
        if (n >= g.N)
            continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = m0 + wm + 16 * a + 4 * grp + j;
                if (m >= g.M)
                    continue;
                const int64_t o = (int64_t)m * g.ldc + n;
                float v = acc[a][b][j];
                if (EPI == EPI_BIAS || EPI == EPI_BIAS_SILU)
                    v += g.bias[n];
                if (EPI == EPI_BIAS_SILU) {
                    g.Zout[o] = v;
                    v = silu_f(v);
                }
                if (EPI == EPI_DSILU)
                    v *= dsilu_f(g.Zin[o]);
                C[o] = v;
            }
    }
}

template <int EPI, int TA, int TB>
static void gemm(int mode, GemmArgs g, int splits, hipStream_t st) {
    if (g.M <= 0 || g.N <= 0)
        return;
    if (splits <= 1) {
        g.kc = (g.K + kBK - 1) / kBK * kBK;
        splits = 1;
    }
    const dim3 grid((unsigned)((g.N + kBN - 1) / kBN), (unsigned)((g.M + kBM - 1) / kBM), (unsigned)splits);
    if (mode == 1)
        gemm_kernel<1, EPI, TA, TB><<<grid, 256, 0, st>>>(g);
    else
        gemm_kernel<0, EPI, TA, TB><<<grid, 256, 0, st>>>(g);
    AFS_HIP(hipGetLastError());
}

// Split of the batch dimension of the weight-gradient products: chunks of at
// least 256 rows (whole K slices), at most 64 planes.
static int grad_chunk(int n) {
    const int per = (n + 63) / 64;
    return std::max(256, (per + kBK - 1) / kBK * kBK);
}
static int grad_splits(int n) { return std::max(1, (n + grad_chunk(n) - 1) / grad_chunk(n)); }

// G[k] = sum over the planes of partial (fixed order)
__global__ __launch_bounds__(256) void grad_reduce_kernel(int64_t n, int S, const float *__restrict__ partial,
                                                          float *__restrict__ G) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    float acc = 0.f;
    for (int z = 0; z < S; ++z)
        acc += partial[(int64_t)z * n + k];
    G[k] = acc;
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

__device__ __forceinline__ void adam_update(int64_t k, float gk, float *__restrict__ p, float *__restrict__ m,
                                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                                            float c2) {
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ __launch_bounds__(256) void adam_kernel(int64_t n, float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    adam_update(k, g[k], p, m, v, lr, b1, b2, eps, c1, c2);
}

// the gradient from its planes of partial sums (fixed order), then the Adam step
__global__ __launch_bounds__(256) void grad_reduce_adam_kernel(int64_t n, int S, const float *__restrict__ partial,
                                                               float *__restrict__ p, float *__restrict__ m,
                                                               float *__restrict__ v, float lr, float b1, float b2,
                                                               float eps, float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    float acc = 0.f;
    for (int z = 0; z < S; ++z)
        acc += partial[(int64_t)z * n + k];
    adam_update(k, acc, p, m, v, lr, b1, b2, eps, c1, c2);
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

// offsets (floats) of the regions of the work buffer for n rows
static size_t work_loss_partials(const MlpShape &s, int n) {
    return (size_t)n * (6 * (size_t)s.hidden + 2 * (size_t)s.d_out);
}
static size_t work_planes(const MlpShape &s, int n) {
    // after the loss partials, rounded up to 4 floats (16-byte aligned planes)
    return (work_loss_partials(s, n) + (size_t)((int64_t)n * s.d_out / 256 + 2) + 64 + 3) / 4 * 4;
}

size_t mlp_work_floats(const MlpShape &s, int n) {
    // Z1, H1, Z2, H2, dZ2, dZ1 (n x H each), Y, dY (n x d_out), loss partials,
    // then the gradient planes (splits x n_params)
    return work_planes(s, n) + (size_t)grad_splits(n) * (size_t)s.n_params;
}

void mlp_forward(const MlpShape &s, int mode, int n, const float *P, const float *X, float *Y, float *work,
                 hipStream_t st) {
    const int H = s.hidden;
    float *Z1 = work, *H1 = Z1 + (size_t)n * H, *Z2 = H1 + (size_t)n * H, *H2 = Z2 + (size_t)n * H;
    GemmArgs g{};
    g = GemmArgs{n, H, s.d_in, X, s.d_in, P + s.oW1, H, H1, H, P + s.ob1, Z1, nullptr, 0, 0, 0};
    gemm<EPI_BIAS_SILU, 0, 0>(mode, g, 1, st);
    g = GemmArgs{n, H, H, H1, H, P + s.oW2, H, H2, H, P + s.ob2, Z2, nullptr, 0, 0, 0};
    gemm<EPI_BIAS_SILU, 0, 0>(mode, g, 1, st);
    g = GemmArgs{n, s.d_out, H, H2, H, P + s.oW3, s.d_out, Y, s.d_out, P + s.ob3, nullptr, nullptr, 0, 0, 0};
    gemm<EPI_BIAS, 0, 0>(mode, g, 1, st);
}

// Forward, loss and the gradient planes: plane z (n_params floats) holds the
// partial gradient of rows [z kc, (z+1) kc).  Returns the number of planes.
static int loss_grad_planes(const MlpShape &s, int mode, int n, const float *P, const float *X, const float *T,
                            float *loss, float *work, float **gplanes, hipStream_t st) {
    const int H = s.hidden, D = s.d_out;
    float *Z1 = work, *H1 = Z1 + (size_t)n * H, *Z2 = H1 + (size_t)n * H, *H2 = Z2 + (size_t)n * H;
    float *dZ2 = H2 + (size_t)n * H, *dZ1 = dZ2 + (size_t)n * H;
    float *Y = dZ1 + (size_t)n * H, *dY = Y + (size_t)n * D, *part = work + work_loss_partials(s, n);
    float *GP = work + work_planes(s, n);
    *gplanes = GP;
    mlp_forward(s, mode, n, P, X, Y, work, st);
    const int64_t cnt = (int64_t)n * D;
    const unsigned nb = (unsigned)((cnt + 255) / 256);
    mse_grad_kernel<<<nb, 256, 0, st>>>(cnt, Y, T, 1.f / (float)cnt, dY, part);
    if (loss)
        sum_kernel<<<1, 256, 0, st>>>((int)nb, part, 1.f / (float)cnt, loss);
    AFS_HIP(hipGetLastError());
    const int S = grad_splits(n), kc = grad_chunk(n);
    const int64_t np = s.n_params;
    GemmArgs g{};
    // [gW3; gb3] = [H2 1]^T dY  [H + 1, D]
    g = GemmArgs{H + 1, D, n, H2, H, dY, D, GP + s.oW3, D, nullptr, nullptr, nullptr, 1, kc, np};
    gemm<EPI_STORE, 1, 0>(mode, g, S, st);
    // dZ2 = (dY W3^T) * silu'(Z2)  [n, H]
    g = GemmArgs{n, H, D, dY, D, P + s.oW3, D, dZ2, H, nullptr, nullptr, Z2, 0, 0, 0};
    gemm<EPI_DSILU, 0, 1>(mode, g, 1, st);
    // [gW2; gb2] = [H1 1]^T dZ2
    g = GemmArgs{H + 1, H, n, H1, H, dZ2, H, GP + s.oW2, H, nullptr, nullptr, nullptr, 1, kc, np};
    gemm<EPI_STORE, 1, 0>(mode, g, S, st);
    // dZ1 = (dZ2 W2^T) * silu'(Z1)
    g = GemmArgs{n, H, H, dZ2, H, P + s.oW2, H, dZ1, H, nullptr, nullptr, Z1, 0, 0, 0};
    gemm<EPI_DSILU, 0, 1>(mode, g, 1, st);
    // [gW1; gb1] = [X 1]^T dZ1  [d_in + 1, H]
    g = GemmArgs{s.d_in + 1, H, n, X, s.d_in, dZ1, H, GP + s.oW1, H, nullptr, nullptr, nullptr, 1, kc, np};
    gemm<EPI_STORE, 1, 0>(mode, g, S, st);
    return S;
}

void mlp_loss_grad(const MlpShape &s, int mode, int n, const float *P, const float *X, const float *T, float *G,
                   float *loss, float *work, hipStream_t st) {
    float *GP = nullptr;
    const int S = loss_grad_planes(s, mode, n, P, X, T, loss, work, &GP, st);
    grad_reduce_kernel<<<(unsigned)((s.n_params + 255) / 256), 256, 0, st>>>(s.n_params, S, GP, G);
    AFS_HIP(hipGetLastError());
}

void mlp_train_step(const MlpShape &s, int n, float *P, const float *X, const float *T, float *m, float *v, int t,
                    float lr, float b1, float b2, float eps, float *loss, float *work, hipStream_t st) {
    float *GP = nullptr;
    const int S = loss_grad_planes(s, 1, n, P, X, T, loss, work, &GP, st);
    const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
    grad_reduce_adam_kernel<<<(unsigned)((s.n_params + 255) / 256), 256, 0, st>>>(s.n_params, S, GP, P, m, v, lr, b1,
                                                                                   b2, eps, c1, c2);
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
