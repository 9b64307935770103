// All-DOF time synthesis (Sections 2.3 and 3: residue identification for every
// unknown with the model's common poles, then the time response of Eq. 6) as
// one real contraction on the FP64 matrix cores:
//   h[n][t] = sum_i B[n][i] K[i][t],  B[n][i] = Re X[i][n] (i < J), Im X[i-J][n] (i >= J),
// X [J][N] the sampled solutions, K [2J][Nt] built on the host from the
// pseudo-inverse of the real-coefficient basis and the basis functions' time
// responses.  v_mfma_f64_16x16x4f64: per lane, A supplies A[l%16][l/16], B
// supplies B[l/16][l%16], the 16x16 result holds D[4v + l/16][l%16], v < 4
// (rows interleaved across the four lane groups; measured on gfx950).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace afsbem {

typedef double d4_t __attribute__((ext_vector_type(4)));

// The lane's A-operand value B[n][k] (k = 4 kk + l/16 at k-step kk)
__device__ __forceinline__ double synth_a(const double *__restrict__ X, int64_t N, int J, int64_t n, int k) {
    if (n >= N || k >= 2 * J)
        return 0.0;
    const int j = k < J ? k : k - J;
    return X[2 * ((int64_t)j * N + n) + (k < J ? 0 : 1)];
}

// Rows [16 bx, +16): the four waves take time tiles w, w+4, ...; the lane's
// A fragments (one per k-step) are loaded once into registers and reused for
// every time tile (Kpad <= 4 * kMaxSteps).
constexpr int kSynthMaxSteps = 32;

__global__ __launch_bounds__(256) void synth_kernel(int64_t N, int J, int Kpad, int Nt,
                                                    const double *__restrict__ X, const double *__restrict__ Km,
                                                    double *__restrict__ h) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t n0 = (int64_t)blockIdx.x * 16;
    const int64_t n = n0 + (lane & 15);
    const int kl = lane >> 4;
    const int steps = Kpad / 4;
    double af[kSynthMaxSteps];
#pragma unroll
    for (int kk = 0; kk < kSynthMaxSteps; ++kk)
        af[kk] = kk < steps ? synth_a(X, N, J, n, 4 * kk + kl) : 0.0;
    const int tiles = (Nt + 15) / 16;
    for (int tt = w; tt < tiles; tt += 4) {
        const int t = 16 * tt + (lane & 15);
        d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < kSynthMaxSteps; ++kk) {
            if (kk < steps) {  // wave-uniform; keeps af[] indices constant (registers)
                const double b = t < Nt ? Km[(int64_t)(4 * kk + kl) * Nt + t] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[kk], b, acc, 0, 0, 0);
            }
        }
        if (t < Nt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = n0 + 4 * v + kl;
                if (row < N)
                    __builtin_nontemporal_store(acc[v], h + row * Nt + t);
            }
        }
    }
}

// Any Kpad: one time tile per wave, fragments loaded per k-step.
__global__ __launch_bounds__(256) void synth_kernel_any(int64_t N, int J, int Kpad, int Nt,
                                                        const double *__restrict__ X, const double *__restrict__ Km,
                                                        double *__restrict__ h) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t n0 = (int64_t)blockIdx.x * 16;
    const int t = blockIdx.y * 64 + 16 * w + (lane & 15);
    const int64_t n = n0 + (lane & 15);
    const int kl = lane >> 4;
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Kpad; k0 += 4) {
        const double a = synth_a(X, N, J, n, k0 + kl);
        const double b = t < Nt ? Km[(int64_t)(k0 + kl) * Nt + t] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (t >= Nt)
        return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = n0 + 4 * v + kl;
        if (row < N)
            h[row * Nt + t] = acc[v];
    }
}

void launch_synthesis(int64_t N, int J, int Kpad, int Nt, const double *X, const double *Km, double *h,
                      hipStream_t st) {
    if (Kpad <= 4 * kSynthMaxSteps) {
        synth_kernel<<<(unsigned)((N + 15) / 16), 256, 0, st>>>(N, J, Kpad, Nt, X, Km, h);
    } else {
        const dim3 g((unsigned)((N + 15) / 16), (unsigned)((Nt + 63) / 64));
        synth_kernel_any<<<g, 256, 0, st>>>(N, J, Kpad, Nt, X, Km, h);
    }
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
