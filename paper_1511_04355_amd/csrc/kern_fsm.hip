// All-DOF Fourier-series inversion (Section 2.2, Eq. 4 with its 1/P factor):
// for every signal q, from its samples H_q(s_k), s_k = eta + 2 pi i k / P,
// k = 0..Ns/2, the time values
//   h_q(t_n) = (e^{eta t_n} / P) Re sum_{k=0}^{Ns-1} X_k e^{+2 pi i n k / Ns},
// t_n = n P / Ns, where X_k = w_k H_q(s_k) for k < Ns/2, X_{Ns-k} = conj(X_k)
// (a real signal), and X_{Ns/2} = w Re H_q(s_{Ns/2}) (the two end points of the
// truncated integral at +-Omega with half weight each); w_k = 1, or the Hann
// weight (1 + cos(2 pi k / Ns)) / 2.
//
// One work-group of 256 threads transforms 256 / TPS signals at once in LDS,
// TPS = Ns / 8 threads per signal (at most 256), by a Stockham
// self-sorting FFT: radix-8 passes, then one radix-2 or radix-4 pass when
// log2 Ns is not a multiple of 3.  Pass with radix R after a span NS (the
// product of the earlier radices): butterfly j < Ns / R reads the R values
// j + r Ns / R, multiplies value r by W^{r (j mod NS) Ns / (NS R)} (W =
// e^{2 pi i / Ns}), takes their R-point transform and writes value r to
// (j / NS) NS R + (j mod NS) + r NS.  The data stay in one LDS array (all
// reads of a pass complete before its writes); the last pass writes the real
// parts, scaled by e^{eta t_n} / P, straight to HBM.  Twiddles and scale
// factors come from host-computed tables (read through the caches).
#include <hip/hip_runtime.h>

#include <utility>

#include "internal.hpp"

namespace afsbem {

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ double2 c_muli(double2 a) { return {-a.y, a.x}; }  // i a

// R-point transforms with the + sign, natural order, in place on v[0..R)
__device__ __forceinline__ void dft2(double2 *v) {
    const double2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
}
__device__ __forceinline__ void dft4(double2 *v) {
    const double2 a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]);
    const double2 a2 = c_add(v[1], v[3]), a3 = c_muli(c_sub(v[1], v[3]));
    v[0] = c_add(a0, a2);
    v[1] = c_add(a1, a3);
    v[2] = c_sub(a0, a2);
    v[3] = c_sub(a1, a3);
}
// 8 points: even and odd halves by dft4, combined with e^{2 pi i k / 8}
__device__ __forceinline__ void dft8(double2 *v) {
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft4(e);
    dft4(o);
    constexpr double h = 0.70710678118654752440;  // 1 / sqrt(2)
    const double2 t0 = o[0];
    const double2 t1 = {h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)};   // (1 + i) / sqrt 2
    const double2 t2 = c_muli(o[2]);                                      // i
    const double2 t3 = {-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};  // (-1 + i) / sqrt 2
    v[0] = c_add(e[0], t0);
    v[1] = c_add(e[1], t1);
    v[2] = c_add(e[2], t2);
    v[3] = c_add(e[3], t3);
    v[4] = c_sub(e[0], t0);
    v[5] = c_sub(e[1], t1);
    v[6] = c_sub(e[2], t2);
    v[7] = c_sub(e[3], t3);
}
template <int R>
__device__ __forceinline__ void dft_r(double2 *v) {
    if constexpr (R == 2)
        dft2(v);
    else if constexpr (R == 4)
        dft4(v);
    else
        dft8(v);
}

template <int N, int TPS, int R, int NS>
__device__ __forceinline__ void fsm_pass(double2 *X, const double2 *__restrict__ W, int tl, bool live, int64_t sig,
                                         const double *__restrict__ E, double *__restrict__ h) {
    constexpr int EPT = N / TPS, NB = EPT / R;
    constexpr bool LAST = NS * R == N;
    double2 v[EPT];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tl + b * TPS;
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[b * R + r] = X[j + r * (N / R)];
    }
    if constexpr (!LAST)
        __syncthreads();  // every read of this pass before any write
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tl + b * TPS;
        const int jm = j % NS;
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r)
                v[b * R + r] = c_mul(v[b * R + r], W[r * jm * (N / (NS * R))]);
        }
        dft_r<R>(&v[b * R]);
        const int d = (j / NS) * NS * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (LAST) {
                if (live)
                    __builtin_nontemporal_store(E[d + r * NS] * v[b * R + r].x, h + sig * N + d + r * NS);
            } else {
                X[d + r * NS] = v[b * R + r];
            }
        }
    }
    if constexpr (!LAST)
        __syncthreads();
}

template <int N, int TPS, int NS>
__device__ __forceinline__ void fsm_passes(double2 *X, const double2 *__restrict__ W, int tl, bool live, int64_t sig,
                                           const double *__restrict__ E, double *__restrict__ h) {
    if constexpr (NS < N) {
        constexpr int R = N / NS >= 8 ? 8 : N / NS;
        fsm_pass<N, TPS, R, NS>(X, W, tl, live, sig, E, h);
        fsm_passes<N, TPS, NS * R>(X, W, tl, live, sig, E, h);
    }
}

template <int L>
__global__ __launch_bounds__(256) void fsm_kernel(int64_t n_sig, int window, const double2 *__restrict__ H,
                                                  const double2 *__restrict__ W, const double *__restrict__ E,
                                                  double *__restrict__ h) {
    constexpr int N = 1 << L, HALF = N / 2;
    constexpr int TPS = N / 8 < 1 ? 1 : (N / 8 > 256 ? 256 : N / 8);
    constexpr int SPB = 256 / TPS;
    __shared__ double2 buf[SPB * N];
    const int sl = threadIdx.x / TPS, tl = threadIdx.x % TPS;
    const int64_t sig = (int64_t)blockIdx.x * SPB + sl;
    const bool live = sig < n_sig;  // the last block's spare signals transform zeros and store nothing
    double2 *X = buf + sl * N;
    for (int k = tl; k <= HALF; k += TPS) {
        const double2 hk = live ? H[sig * (HALF + 1) + k] : double2{0.0, 0.0};
        const double w = window ? 0.5 * (1.0 + W[k].x) : 1.0;
        if (k == HALF) {
            X[HALF] = double2{w * hk.x, 0.0};
        } else {
            X[k] = double2{w * hk.x, w * hk.y};
            if (k > 0)
                X[N - k] = double2{w * hk.x, -w * hk.y};
        }
    }
    __syncthreads();
    fsm_passes<N, TPS, 1>(X, W, tl, live, sig, E, h);
}

template <int L>
static void fsm_launch_l(int64_t n_sig, int window, const double *H, const double *W, const double *E, double *h,
                         hipStream_t st) {
    constexpr int N = 1 << L;
    constexpr int TPS = N / 8 < 1 ? 1 : (N / 8 > 256 ? 256 : N / 8);
    constexpr int SPB = 256 / TPS;
    const int64_t blocks = (n_sig + SPB - 1) / SPB;
    fsm_kernel<L><<<(unsigned)blocks, 256, 0, st>>>(n_sig, window, reinterpret_cast<const double2 *>(H),
                                                    reinterpret_cast<const double2 *>(W), E, h);
}

template <int... Ls>
static void fsm_dispatch(std::integer_sequence<int, Ls...>, int L, int64_t n_sig, int window, const double *H,
                         const double *W, const double *E, double *h, hipStream_t st) {
    ((L == Ls + 1 ? (fsm_launch_l<Ls + 1>(n_sig, window, H, W, E, h, st), 0) : 0), ...);
}

void launch_fsm(int log2_ns, int64_t n_sig, int window, const double *H, const double *W, const double *E, double *h,
                hipStream_t st) {
    AFS_REQUIRE(log2_ns >= 1 && log2_ns <= kFsmMaxLog2, AFSBEM_EINVAL, "fsm: Ns must be a power of two <= 4096");
    fsm_dispatch(std::make_integer_sequence<int, kFsmMaxLog2>{}, log2_ns, n_sig, window, H, W, E, h, st);
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
