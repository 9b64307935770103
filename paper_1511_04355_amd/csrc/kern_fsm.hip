// All-DOF Fourier-series inversion (Section 2.2, Eq. 4 with its 1/P factor):
// for every signal q, from its samples H_q(s_k), s_k = eta + 2 pi i k / P,
// k = 0..Ns/2, the time values
//   h_q(t_n) = (e^{eta t_n} / P) Re sum_{k=0}^{Ns-1} X_k e^{+2 pi i n k / Ns},
// t_n = n P / Ns, where X_k = w_k H_q(s_k) for k < Ns/2, X_{Ns-k} = conj(X_k)
// (a real signal), and X_{Ns/2} = w Re H_q(s_{Ns/2}) (the two end points of the
// truncated integral at +-Omega with half weight each); w_k = 1, or the Hann
// weight (1 + cos(2 pi k / Ns)) / 2.
//
// A work-group of 256 threads transforms a group of 256 / TPS signals at a
// time in LDS, TPS = Ns / 8 threads per signal (at most 256), by a Stockham
// self-sorting FFT: radix-8 passes, then one radix-2 or radix-4 pass when
// log2 Ns is not a multiple of 3.  Pass with radix R after a span NS (the
// product of the earlier radices): butterfly j < Ns / R reads the R values
// j + r Ns / R, multiplies value r by W^{r (j mod NS) Ns / (NS R)} (W =
// e^{2 pi i / Ns}), takes their R-point transform and writes value r to
// (j / NS) NS R + (j mod NS) + r NS.  The data stay in one LDS array (all
// reads of a pass complete before its writes), one pad slot per 8 entries
// against bank conflicts; the last pass writes the real parts, scaled by
// e^{eta t_n} / P, straight to HBM.  Twiddles and scale factors come from
// host-computed tables, staged in LDS up to Ns = 1024.  The work-groups are
// persistent (as many as fit on the device) and load the next group's
// samples into registers while the current group is transformed; the loop
// has no divergent branch (clamped loads, the Nyquist sample broadcast to
// every lane and written by the lane holding k = 0, stores through a buffer
// descriptor spanning exactly the group's signals, so the hardware drops
// those of the spare signals of the last group).
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

typedef unsigned fsm_v2u_t __attribute__((ext_vector_type(2)));

template <int N>
__device__ __forceinline__ int fsm_px(int p) { return p + (p >> 3); }  // padded LDS index

template <int N, int TPS, int R, int NS>
__device__ __forceinline__ void fsm_pass(double2 *X, const double2 *W, int tl, const double *E,
                                         __amdgpu_buffer_rsrc_t rs, int obase) {
    constexpr int EPT = N / TPS, NB = EPT / R;
    constexpr bool LAST = NS * R == N;
    double2 v[EPT];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tl + b * TPS;
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[b * R + r] = X[fsm_px<N>(j + r * (N / R))];
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
                const double val = E[d + r * NS] * v[b * R + r].x;
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(fsm_v2u_t, val), rs, (obase + d + r * NS) * 8,
                                                      0, 2 /* nt */);
            } else {
                X[fsm_px<N>(d + r * NS)] = v[b * R + r];
            }
        }
    }
    if constexpr (!LAST)
        __syncthreads();
}

template <int N, int TPS, int NS>
__device__ __forceinline__ void fsm_passes(double2 *X, const double2 *W, int tl, const double *E,
                                           __amdgpu_buffer_rsrc_t rs, int obase) {
    if constexpr (NS < N) {
        constexpr int R = N / NS >= 8 ? 8 : N / NS;
        fsm_pass<N, TPS, R, NS>(X, W, tl, E, rs, obase);
        fsm_passes<N, TPS, NS * R>(X, W, tl, E, rs, obase);
    }
}

template <int L>
struct FsmShape {
    static constexpr int N = 1 << L, HALF = N / 2;
    static constexpr int TPS = N / 8 < 1 ? 1 : (N / 8 > 256 ? 256 : N / 8);
    static constexpr int SPB = 256 / TPS;          // signals per group
    static constexpr int KPT = HALF / TPS;         // samples k < Ns/2 per thread
    static constexpr int NP = N + (N >> 3);        // padded signal length in LDS
    static constexpr bool TLDS = N <= 1024;        // tables staged in LDS
    static_assert(KPT * TPS == HALF, "Ns/2 must be a multiple of the threads per signal");
};

template <int L>
__global__ __launch_bounds__(256) void fsm_kernel(int64_t n_sig, int64_t n_groups, int window,
                                                  const double2 *__restrict__ H, const double2 *__restrict__ Wg,
                                                  const double *__restrict__ Eg, double *__restrict__ h) {
    using S = FsmShape<L>;
    constexpr int N = S::N, HALF = S::HALF, TPS = S::TPS, SPB = S::SPB, KPT = S::KPT, NP = S::NP;
    __shared__ double2 buf[SPB * NP];
    __shared__ double2 wl[S::TLDS ? N : 1];
    __shared__ double el[S::TLDS ? N : 1];
    const double2 *W = Wg;
    const double *E = Eg;
    if constexpr (S::TLDS) {
        for (int m = threadIdx.x; m < N; m += 256) {
            wl[m] = Wg[m];
            el[m] = Eg[m];
        }
        W = wl;
        E = el;
    }
    const int sl = threadIdx.x / TPS, tl = threadIdx.x % TPS;
    double2 *X = buf + sl * NP;
    double2 pre[KPT], preh;
    auto fetch = [&](int64_t grp) {  // clamped: always KPT + 1 loads
        const int64_t gc = grp < n_groups ? grp : n_groups - 1;
        const int64_t sig = gc * SPB + sl;
        const double2 *row = H + (sig < n_sig ? sig : n_sig - 1) * (HALF + 1);
#pragma unroll
        for (int i = 0; i < KPT; ++i)
            pre[i] = row[tl + i * TPS];
        preh = row[HALF];
    };
    int64_t grp = blockIdx.x;
    fetch(grp);
    __syncthreads();  // tables
    for (; grp < n_groups; grp += gridDim.x) {
        const bool live = grp * SPB + sl < n_sig;
        const double wh = window ? 0.5 * (1.0 + W[HALF].x) : 1.0;
        const double2 nyq = double2{live ? wh * preh.x : 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < KPT; ++i) {
            const int k = tl + i * TPS;
            const double2 hk = live ? pre[i] : double2{0.0, 0.0};
            const double w = window ? 0.5 * (1.0 + W[k].x) : 1.0;
            X[fsm_px<N>(k)] = double2{w * hk.x, w * hk.y};
            const bool mirror = k > 0;  // k = 0 has no mirror: that lane writes the Nyquist entry
            X[fsm_px<N>(mirror ? N - k : HALF)] = mirror ? double2{w * hk.x, -w * hk.y} : nyq;
        }
        __syncthreads();
        fetch(grp + gridDim.x);
        const int64_t s0 = grp * SPB;
        const int64_t ns = n_sig - s0 < SPB ? n_sig - s0 : SPB;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(h + s0 * N, 0, (int)(ns * N * 8), 0x00020000);
        fsm_passes<N, TPS, 1>(X, W, tl, E, rs, sl * N);
        __syncthreads();  // the last pass's reads of X before the next group's writes
    }
}

template <int L>
static void fsm_launch_l(int64_t n_sig, int window, const double *H, const double *W, const double *E, double *h,
                         hipStream_t st) {
    using S = FsmShape<L>;
    const int64_t n_groups = (n_sig + S::SPB - 1) / S::SPB;
    static int resident = 0;  // work-groups that fit on the device at once (per instantiation)
    if (resident == 0) {
        int dev = 0, per_cu = 0;
        hipDeviceProp_t prop;
        AFS_HIP(hipGetDevice(&dev));
        AFS_HIP(hipGetDeviceProperties(&prop, dev));
        AFS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fsm_kernel<L>, 256, 0));
        resident = (per_cu > 0 ? per_cu : 1) * prop.multiProcessorCount;
    }
    const int64_t grid = n_groups < resident ? n_groups : resident;
    fsm_kernel<L><<<(unsigned)grid, 256, 0, st>>>(n_sig, n_groups, window, reinterpret_cast<const double2 *>(H),
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
