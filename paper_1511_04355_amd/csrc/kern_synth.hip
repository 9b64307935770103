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

#include <utility>

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

// Main kernel.  The contraction index runs in pairs: at pair q the lane group
// l/16 takes j = 4q + l/16 and feeds Re X[j][n] and Im X[j][n] (one 16-byte
// load) to two successive matrix-core steps, whose K operands are rows j and
// J + j.  A block owns kSynthRowTiles row tiles of 16 unknowns and 64 TT times;
// wave w keeps the K fragments of its TT groups of 16 times (t = 64 TT tb +
// 64 u + 16 w + l%16) in registers for all of the block's row tiles and loads
// the next row tile's X while the current one is on the matrix cores.  The loop
// has no divergent branch: loads go to clamped addresses and are zeroed by a
// select; stores go through a buffer descriptor that spans exactly the block's
// rows, and a lane whose time is past Nt gets an offset beyond that span, so
// the hardware drops it (as it drops the rows past N).  Blocks are renumbered
// so that each XCD walks consecutive logical blocks with the time blocks
// fastest: the blocks of one row range share that XCD's L2 for X.
constexpr int kSynthRowTiles = 16;
constexpr int kSynthTT = 2;
constexpr int kSynthMaxPairs = 16;  // J <= 64
constexpr int kSynthBadOffset = 0x40000000;  // the descriptor span stays below this

typedef unsigned v2u_t __attribute__((ext_vector_type(2)));

template <int P>
__device__ __forceinline__ void synth_load_x(const double2 *__restrict__ X, int64_t N, int J, int64_t tile, int lane,
                                             double2 (&a)[P]) {
    const int64_t n = tile * 16 + (lane & 15);
    const int64_t nc = n < N ? n : N - 1;
    const int g = lane >> 4;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int j = 4 * q + g;
        const int jc = j < J ? j : J - 1;
        const double2 v = X[(int64_t)jc * N + nc];
        const bool ok = n < N && j < J;
        a[q].x = ok ? v.x : 0.0;
        a[q].y = ok ? v.y : 0.0;
    }
}

template <int P>
__global__ __launch_bounds__(256) void synth_kernel(int64_t N, int J, int Nt, int nTB, int64_t nB,
                                                   const double2 *__restrict__ X, const double *__restrict__ K,
                                                   double *__restrict__ h) {
    constexpr int TT = kSynthTT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4;
    const int64_t per = (nB + 7) / 8;
    const int64_t lb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (lb >= nB)
        return;  // the grid is rounded up to a multiple of 8
    const int tb = (int)(lb % nTB);
    const int64_t rb = lb / nTB;
    const int tbase = tb * 64 * TT + 16 * w + (lane & 15);
    double bre[TT][P], bim[TT][P];
    int tbad[TT];
#pragma unroll
    for (int u = 0; u < TT; ++u) {
        const int t = tbase + 64 * u;
        const int tc = t < Nt ? t : Nt - 1;
        tbad[u] = t < Nt ? 0 : kSynthBadOffset;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int j = 4 * q + g;
            const int jc = j < J ? j : J - 1;
            const double re = K[(int64_t)jc * Nt + tc], im = K[(int64_t)(J + jc) * Nt + tc];
            const bool ok = j < J && t < Nt;
            bre[u][q] = ok ? re : 0.0;
            bim[u][q] = ok ? im : 0.0;
        }
    }
    const int64_t ntiles = (N + 15) / 16;
    const int64_t tile0 = rb * kSynthRowTiles;
    const int rend = (int)(ntiles - tile0 < kSynthRowTiles ? ntiles - tile0 : kSynthRowTiles);
    const int64_t row0 = tile0 * 16;
    const int64_t rows = N - row0 < 16 * kSynthRowTiles ? N - row0 : 16 * kSynthRowTiles;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(h + row0 * Nt, 0, (int)(rows * Nt * 8), 0x00020000);
    double2 a[P], an[P];
    synth_load_x<P>(X, N, J, tile0, lane, a);
    for (int r = 0; r < rend; ++r) {
        // the last iteration reloads its own tile: no branch around the loads
        synth_load_x<P>(X, N, J, tile0 + (r + 1 < rend ? r + 1 : r), lane, an);
        d4_t acc[TT];
#pragma unroll
        for (int u = 0; u < TT; ++u)
            acc[u] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < P; ++q) {
#pragma unroll
            for (int u = 0; u < TT; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].x, bre[u][q], acc[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < TT; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q].y, bim[u][q], acc[u], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < TT; ++u) {
            const int t = tbase + 64 * u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int off = ((r * 16 + 4 * v + g) * Nt + t) * 8 + tbad[u];
                // element copied to a scalar first: a bit cast of the vector
                // element itself loses the element index
                const double val = acc[u][v];
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_t, val), rs, off, 0, 2 /* nt */);
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q)
            a[q] = an[q];
    }
}

template <int P>
static void synth_launch_p(int64_t N, int J, int Nt, const double *X, const double *K, double *h, hipStream_t st) {
    const int nTB = (Nt + 64 * kSynthTT - 1) / (64 * kSynthTT);
    const int64_t nRB = ((N + 15) / 16 + kSynthRowTiles - 1) / kSynthRowTiles;
    const int64_t nB = nRB * nTB;
    const int64_t grid = (nB + 7) / 8 * 8;
    synth_kernel<P><<<(unsigned)grid, 256, 0, st>>>(N, J, Nt, nTB, nB, reinterpret_cast<const double2 *>(X), K, h);
}

template <int... Ps>
static void synth_dispatch(std::integer_sequence<int, Ps...>, int P, int64_t N, int J, int Nt, const double *X,
                           const double *K, double *h, hipStream_t st) {
    ((P == Ps + 1 ? (synth_launch_p<Ps + 1>(N, J, Nt, X, K, h, st), 0) : 0), ...);
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
    const int P = (J + 3) / 4;
    // byte offsets within one block's rows stay below kSynthBadOffset
    const bool fits = (int64_t)16 * kSynthRowTiles * Nt * 8 + (int64_t)64 * kSynthTT * 8 < kSynthBadOffset;
    if (P <= kSynthMaxPairs && fits) {
        synth_dispatch(std::make_integer_sequence<int, kSynthMaxPairs>{}, P, N, J, Nt, X, Km, h, st);
    } else {
        const dim3 g((unsigned)((N + 15) / 16), (unsigned)((Nt + 63) / 64));
        synth_kernel_any<<<g, 256, 0, st>>>(N, J, Kpad, Nt, X, Km, h);
    }
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
