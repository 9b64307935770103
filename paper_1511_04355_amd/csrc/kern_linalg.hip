// Dense complex matrix-vector products and Krylov vector kernels for gfx950.
//
// GEMV (the GMRES operator application, HBM-bound): the matrix is
// column-major, lanes own rows and a workgroup walks a chunk of columns, so
// every load instruction of a wavefront reads 1 KiB of one column contiguously
// and the vector entry x[col] is wave-uniform (scalar load).  Columns are split
// into chunks over grid.y to put enough bytes in flight; partial sums per
// chunk are combined in FP64 by a second pass in a fixed order
// (deterministic).
//   C128: one row per lane, 16-byte loads, FP64 FMA.
//   SPLIT FP32: two rows per lane (16 bytes of the hi plane), FP32 FMA and
//               FP32 accumulation within a chunk.
//   SPLIT FP64: hi + lo planes converted to FP64 per entry, FP64 FMA.
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "cplx.hpp"
#include "tune.hpp"
#include "internal.hpp"

namespace afsbem {

constexpr int kGemvUnroll = 8;

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// streaming (non-temporal) 16-byte loads: the matrix is read once per product
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

__global__ __launch_bounds__(256) void gemv_c128_kernel(int64_t N, int64_t lda, const double2 *__restrict__ A,
                                                        const double2 *__restrict__ x, int64_t chunk,
                                                        double2 *__restrict__ partial) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = (c0 + chunk < N) ? c0 + chunk : N;
    double ar = 0.0, ai = 0.0;
    if (row < N) {
        const double2 *a = A + row;
        int64_t c = c0;
        for (; c + kGemvUnroll <= c1; c += kGemvUnroll) {
            double2 v[kGemvUnroll];
#pragma unroll
            for (int u = 0; u < kGemvUnroll; ++u)
                v[u] = ld_nt(a + (c + u) * lda);
#pragma unroll
            for (int u = 0; u < kGemvUnroll; ++u) {
                const double2 xv = x[c + u];
                ar = fma(v[u].x, xv.x, ar);
                ar = fma(-v[u].y, xv.y, ar);
                ai = fma(v[u].x, xv.y, ai);
                ai = fma(v[u].y, xv.x, ai);
            }
        }
        for (; c < c1; ++c) {
            const double2 v = a[c * lda];
            const double2 xv = x[c];
            ar = fma(v.x, xv.x, ar);
            ar = fma(-v.y, xv.y, ar);
            ai = fma(v.x, xv.y, ai);
            ai = fma(v.y, xv.x, ai);
        }
        partial[(int64_t)blockIdx.y * N + row] = make_double2(ar, ai);
    }
}

// hi plane only, FP32 arithmetic; two rows per lane.
__global__ __launch_bounds__(256) void gemv_split32_kernel(int64_t N, int64_t lda, const float4 *__restrict__ A,
                                                           const double2 *__restrict__ x, int64_t chunk,
                                                           double2 *__restrict__ partial) {
    const int64_t r2 = (int64_t)blockIdx.x * 256 + threadIdx.x;  // row pair
    const int64_t row = 2 * r2;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = (c0 + chunk < N) ? c0 + chunk : N;
    if (row >= N)
        return;
    const int64_t lda2 = lda / 2;  // float4 units per column
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f;
    const float4 *a = A + r2;
    int64_t c = c0;
    for (; c + kGemvUnroll <= c1; c += kGemvUnroll) {
        float4 v[kGemvUnroll];
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u)
            v[u] = ld_nt(a + (c + u) * lda2);
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) {
            const double2 xd = x[c + u];
            const float xr = (float)xd.x, xi = (float)xd.y;
            a0r = fmaf(v[u].x, xr, a0r);
            a0r = fmaf(-v[u].y, xi, a0r);
            a0i = fmaf(v[u].x, xi, a0i);
            a0i = fmaf(v[u].y, xr, a0i);
            a1r = fmaf(v[u].z, xr, a1r);
            a1r = fmaf(-v[u].w, xi, a1r);
            a1i = fmaf(v[u].z, xi, a1i);
            a1i = fmaf(v[u].w, xr, a1i);
        }
    }
    for (; c < c1; ++c) {
        const float4 v = a[c * lda2];
        const double2 xd = x[c];
        const float xr = (float)xd.x, xi = (float)xd.y;
        a0r = fmaf(v.x, xr, a0r);
        a0r = fmaf(-v.y, xi, a0r);
        a0i = fmaf(v.x, xi, a0i);
        a0i = fmaf(v.y, xr, a0i);
        a1r = fmaf(v.z, xr, a1r);
        a1r = fmaf(-v.w, xi, a1r);
        a1i = fmaf(v.z, xi, a1i);
        a1i = fmaf(v.w, xr, a1i);
    }
    double2 *out = partial + (int64_t)blockIdx.y * N + row;
    out[0] = make_double2(a0r, a0i);
    if (row + 1 < N)
        out[1] = make_double2(a1r, a1i);
}

// hi + lo planes, FP64 arithmetic; two rows per lane.
__global__ __launch_bounds__(256) void gemv_split64_kernel(int64_t N, int64_t lda, const float4 *__restrict__ Ah,
                                                           const float4 *__restrict__ Al,
                                                           const double2 *__restrict__ x, int64_t chunk,
                                                           double2 *__restrict__ partial) {
    const int64_t r2 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = 2 * r2;
    const int64_t c0 = (int64_t)blockIdx.y * chunk;
    const int64_t c1 = (c0 + chunk < N) ? c0 + chunk : N;
    if (row >= N)
        return;
    const int64_t lda2 = lda / 2;
    double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
    const float4 *h = Ah + r2;
    const float4 *l = Al + r2;
    int64_t c = c0;
    constexpr int U = kGemvUnroll / 2;
    for (; c + U <= c1; c += U) {
        float4 vh[U], vl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vh[u] = ld_nt(h + (c + u) * lda2);
            vl[u] = ld_nt(l + (c + u) * lda2);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double2 xv = x[c + u];
            const double e0r = (double)vh[u].x + (double)vl[u].x, e0i = (double)vh[u].y + (double)vl[u].y;
            const double e1r = (double)vh[u].z + (double)vl[u].z, e1i = (double)vh[u].w + (double)vl[u].w;
            a0r = fma(e0r, xv.x, a0r);
            a0r = fma(-e0i, xv.y, a0r);
            a0i = fma(e0r, xv.y, a0i);
            a0i = fma(e0i, xv.x, a0i);
            a1r = fma(e1r, xv.x, a1r);
            a1r = fma(-e1i, xv.y, a1r);
            a1i = fma(e1r, xv.y, a1i);
            a1i = fma(e1i, xv.x, a1i);
        }
    }
    for (; c < c1; ++c) {
        const float4 vh = h[c * lda2], vl = l[c * lda2];
        const double2 xv = x[c];
        const double e0r = (double)vh.x + (double)vl.x, e0i = (double)vh.y + (double)vl.y;
        const double e1r = (double)vh.z + (double)vl.z, e1i = (double)vh.w + (double)vl.w;
        a0r = fma(e0r, xv.x, a0r);
        a0r = fma(-e0i, xv.y, a0r);
        a0i = fma(e0r, xv.y, a0i);
        a0i = fma(e0i, xv.x, a0i);
        a1r = fma(e1r, xv.x, a1r);
        a1r = fma(-e1i, xv.y, a1r);
        a1i = fma(e1r, xv.y, a1i);
        a1i = fma(e1i, xv.x, a1i);
    }
    double2 *out = partial + (int64_t)blockIdx.y * N + row;
    out[0] = make_double2(a0r, a0i);
    if (row + 1 < N)
        out[1] = make_double2(a1r, a1i);
}

__global__ __launch_bounds__(256) void sum_partials_kernel(int64_t N, int S, const double2 *__restrict__ partial,
                                                           double2 *__restrict__ y) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= N)
        return;
    // eight partial sums in flight per lane (the loop is latency-bound), then
    // combined in a fixed order
    double rr[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ii[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = partial[(int64_t)(s + u) * N + row];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            rr[u] += v[u].x;
            ii[u] += v[u].y;
        }
    }
    for (; s < S; ++s) {
        const double2 v = partial[(int64_t)s * N + row];
        rr[0] += v.x;
        ii[0] += v.y;
    }
    double r = 0, i = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        r += rr[u];
        i += ii[u];
    }
    y[row] = make_double2(r, i);
}

// Column split of the GEMV: the default gives about 2048 work-groups (enough
// to cover the chip several times over, at least 32 columns per chunk); the
// autotuner measures 1/4x .. 4x of it.
static int gemv_chunks_default(int64_t N) {
    const int64_t gx = (N + 255) / 256;
    int64_t S = (2048 + gx - 1) / gx;
    const int64_t max_s = (N + 31) / 32;
    if (S > max_s)
        S = max_s;
    if (S < 1)
        S = 1;
    return (int)S;
}

static std::vector<int> gemv_chunk_candidates(int64_t N) {
    const int s0 = gemv_chunks_default(N);
    const int64_t max_s = std::max<int64_t>(1, (N + 31) / 32);
    std::vector<int> c;
    for (int f : {-4, -2, 1, 2, 4}) {
        int64_t s = f < 0 ? (s0 + (-f) - 1) / (-f) : (int64_t)s0 * f;
        s = std::max<int64_t>(1, std::min<int64_t>(s, max_s));
        if (std::find(c.begin(), c.end(), (int)s) == c.end())
            c.push_back((int)s);
    }
    return c;
}

int gemv_chunks(int64_t N) {
    const std::vector<int> c = gemv_chunk_candidates(N);
    return *std::max_element(c.begin(), c.end());
}

static void gemv_enqueue(int64_t N, int format, int precision, const void *A, const void *A_lo, const double *x,
                         double *y, double *partial, int S, hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end) {
    const int64_t lda = (N + 63) / 64 * 64;
    const int64_t chunk = (N + S - 1) / S;
    const int Su = (int)((N + chunk - 1) / chunk);
    double2 *part = reinterpret_cast<double2 *>(partial);
    const double2 *xv = reinterpret_cast<const double2 *>(x);
    if (ev_begin)
        AFS_HIP(hipEventRecord(ev_begin, st));
    if (format == AFSBEM_FMT_C128) {
        dim3 g((unsigned)((N + 255) / 256), (unsigned)Su);
        gemv_c128_kernel<<<g, 256, 0, st>>>(N, lda, static_cast<const double2 *>(A), xv, chunk, part);
    } else if (precision == 1) {
        dim3 g((unsigned)((N / 2 + 1 + 255) / 256), (unsigned)Su);
        gemv_split32_kernel<<<g, 256, 0, st>>>(N, lda, static_cast<const float4 *>(A), xv, chunk, part);
    } else {
        dim3 g((unsigned)((N / 2 + 1 + 255) / 256), (unsigned)Su);
        gemv_split64_kernel<<<g, 256, 0, st>>>(N, lda, static_cast<const float4 *>(A),
                                               static_cast<const float4 *>(A_lo), xv, chunk, part);
    }
    AFS_HIP(hipGetLastError());
    if (ev_end)
        AFS_HIP(hipEventRecord(ev_end, st));
    sum_partials_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, Su, part, reinterpret_cast<double2 *>(y));
    AFS_HIP(hipGetLastError());
}

void launch_gemv(int64_t N, int format, int precision, const void *A, const void *A_lo, const double *x, double *y,
                 double *partial, hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end) {
    // the split is tuned once per (device, N, format/precision) on the live
    // operands (products and partial sums together); y is overwritten below
    const int variant = format == AFSBEM_FMT_C128 ? 0 : (precision == 1 ? 1 : 2);
    const int S = autotune(
        "gemv_column_split", N, variant, gemv_chunk_candidates(N), st,
        [&](int c) { gemv_enqueue(N, format, precision, A, A_lo, x, y, partial, c, st, nullptr, nullptr); },
        gemv_chunks_default(N));
    gemv_enqueue(N, format, precision, A, A_lo, x, y, partial, S, st, ev_begin, ev_end);
}

// ------------------------------------------- GEMV without allocation --
// Partial sums of the column split in a file-scope device array instead of
// caller or allocator memory.  Each device holds its own copy; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (resolved once per device and kept), never through the
// array's name.  Every call on a device shares the array: calls that overlap
// on one device race.  Nothing in it has to start at zero (the product pass
// writes every partial sum the summation pass reads).
constexpr size_t kGemvScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kGemvScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
}  // namespace

static double *gemv_scratch_for_current_device() {
    int dev = 0;
    AFS_HIP(hipGetDevice(&dev));
    AFS_REQUIRE(dev >= 0 && dev < 64, AFSBEM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        AFS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        AFS_REQUIRE(ptr != nullptr, AFSBEM_EDEVICE, "no device address for the GEMV scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return static_cast<double *>(g_scratch_ptr[dev]);
}

int64_t gemv_noalloc_max_n() { return (int64_t)(kGemvScratchBytes / 16); }

void launch_gemv_noalloc(int64_t N, int format, int precision, const void *A, const void *A_lo, const double *x,
                         double *y, hipStream_t st) {
    // the default column split, reduced until its partial sums fit the array
    const int64_t fit = (int64_t)(kGemvScratchBytes / ((size_t)N * 16));
    AFS_REQUIRE(N >= 1 && fit >= 1, AFSBEM_EINVAL,
                "N = " + std::to_string(N) + " exceeds the allocation-free GEMV's limit of " +
                    std::to_string(gemv_noalloc_max_n()) + " unknowns (" +
                    std::to_string(kGemvScratchBytes >> 20) + " MiB of partial sums per device)");
    const int S = (int)std::min<int64_t>(gemv_chunks_default(N), fit);
    gemv_enqueue(N, format, precision, A, A_lo, x, y, gemv_scratch_for_current_device(), S, st, nullptr, nullptr);
}

// ---------------------------------------------------------- vector kernels --
__global__ __launch_bounds__(256) void precond_kernel(int64_t nt, const double *__restrict__ D,
                                                      const double *__restrict__ v, double *__restrict__ z) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= nt)
        return;
    cd vin[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        vin[j] = cd{v[6 * m + 2 * j], v[6 * m + 2 * j + 1]};
    const double *d = D + 18 * m;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cd acc{0, 0};
#pragma unroll
        for (int j = 0; j < 3; ++j)
            acc = cadd(acc, cmul(cd{d[6 * i + 2 * j], d[6 * i + 2 * j + 1]}, vin[j]));
        z[6 * m + 2 * i] = acc.r;
        z[6 * m + 2 * i + 1] = acc.i;
    }
}

void vec_precond(int64_t nt, const double *D, const double *v, double *z, hipStream_t st) {
    precond_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(nt, D, v, z);
    AFS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void sub_kernel(int64_t n2, const double *a, const double *b, double *o) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n2)
        o[k] = a[k] - b[k];
}

void vec_sub(int64_t N, const double *a, const double *b, double *out, hipStream_t st) {
    sub_kernel<<<(unsigned)((2 * N + 255) / 256), 256, 0, st>>>(2 * N, a, b, out);
    AFS_HIP(hipGetLastError());
}

// Multi-dot in two launches.  mdot_kernel: block b takes rows
// [b R, (b + 1) R) and, eight vectors at a time, forms each thread's partial
// conj(V_i) . w over its rows (w read once per eight vectors, the eight
// vectors' loads in flight together), reduces the 16 sums (vector, real /
// imaginary) over each wave by a butterfly that halves the set each lane
// keeps at every step (17 exchanges), then over the four waves through LDS,
// and stores partial[i][b].  mdot_final_kernel: one wave per vector adds its
// B partials in block order.  Every V_i is read once per call.
int mdot_blocks(int64_t N) {
    int64_t b = (N + 511) / 512;
    if (b > kMdotMaxBlocks)
        b = kMdotMaxBlocks;
    if (b < 1)
        b = 1;
    return (int)b;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// one butterfly step: lanes whose bit log2(4 H) is clear keep sums 0 .. H-1
// of their set, the others sums H .. 2H-1, each added to its partner's copy
template <int H>
__device__ __forceinline__ void md_halve(double (&s)[16], int lane) {
    const bool hi = (lane & (4 * H)) != 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double send = hi ? s[k] : s[k + H];
        const double keep = hi ? s[k + H] : s[k];
        s[k] = keep + __shfl_xor(send, 4 * H, 64);
    }
}

__global__ __launch_bounds__(256) void mdot_kernel(int64_t N, int nv, const double2 *__restrict__ V, int64_t ldv,
                                                   const double2 *__restrict__ w, int64_t R,
                                                   double2 *__restrict__ partial) {
    __shared__ double red[4][16];
    const int b = blockIdx.x, B = gridDim.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)b * R, r1 = (r0 + R < N) ? r0 + R : N;
    for (int g = 0; g < nv; g += 8) {
        const int ng = (nv - g < 8) ? nv - g : 8;
        const double2 *Vg = V + (int64_t)g * ldv;
        double s[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            s[k] = 0.0;
        for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
            // vectors past the group's last read the last one again (in
            // bounds) and are not stored
            double2 a[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                a[e] = Vg[(int64_t)(e < ng ? e : ng - 1) * ldv + r];
            const double2 x = w[r];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s[2 * e] += a[e].x * x.x + a[e].y * x.y;  // conj(a) * x
                s[2 * e + 1] += a[e].x * x.y - a[e].y * x.x;
            }
        }
        md_halve<8>(s, lane);
        md_halve<4>(s, lane);
        md_halve<2>(s, lane);
        md_halve<1>(s, lane);
        s[0] += __shfl_xor(s[0], 2, 64);
        s[0] += __shfl_xor(s[0], 1, 64);
        if ((lane & 3) == 0)
            red[wv][lane >> 2] = s[0];
        __syncthreads();
        if (threadIdx.x < 16) {
            const int k = threadIdx.x, e = k >> 1;
            if (e < ng)
                reinterpret_cast<double *>(partial)[2 * ((int64_t)(g + e) * B + b) + (k & 1)] =
                    (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void mdot_final_kernel(int B, const double2 *__restrict__ partial,
                                                        double2 *__restrict__ out) {
    const int i = blockIdx.x, lane = threadIdx.x;
    double br = 0, bi = 0;
    for (int b = lane; b < B; b += 64) {
        const double2 q = partial[(int64_t)i * B + b];
        br += q.x;
        bi += q.y;
    }
    br = wave_sum64(br);
    bi = wave_sum64(bi);
    if (lane == 0)
        out[i] = make_double2(br, bi);
}

size_t mdot_scratch_bytes(int64_t N, int nv_max) {
    return (size_t)kMdotCounterBytes + (size_t)mdot_blocks(N) * std::min(nv_max, kMdotMaxVectors) * 16;
}

// more than kMdotMaxVectors vectors: consecutive launches over groups of them
// (stream-ordered, so the groups reuse the same partials)
void vec_mdot(int64_t N, int nv, const double *V, int64_t ldv, const double *w, double *partial, double *out,
              hipStream_t st) {
    const int B = mdot_blocks(N);
    const int64_t R = (N + B - 1) / B;
    AFS_REQUIRE(nv >= 1, AFSBEM_EINVAL, "multi-dot: no vectors");
    double2 *part = reinterpret_cast<double2 *>(reinterpret_cast<char *>(partial) + kMdotCounterBytes);
    for (int c0 = 0; c0 < nv; c0 += kMdotMaxVectors) {
        const int nc = std::min(kMdotMaxVectors, nv - c0);
        mdot_kernel<<<(unsigned)B, 256, 0, st>>>(N, nc, reinterpret_cast<const double2 *>(V) + (int64_t)c0 * ldv, ldv,
                                                 reinterpret_cast<const double2 *>(w), R, part);
        mdot_final_kernel<<<(unsigned)nc, 64, 0, st>>>(B, part, reinterpret_cast<double2 *>(out) + c0);
        AFS_HIP(hipGetLastError());
    }
}

// w -= sum_i h_i V_i   (sign = -1)   or   x += sum_i y_i V_i   (sign = +1)
__global__ __launch_bounds__(256) void mcombine_kernel(int64_t N, int nv, const double2 *__restrict__ V, int64_t ldv,
                                                       const double2 *__restrict__ h, double sign,
                                                       double2 *__restrict__ w) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    double ar = 0, ai = 0;
    for (int i = 0; i < nv; ++i) {
        const double2 c = h[i], v = V[(int64_t)i * ldv + r];
        ar += c.x * v.x - c.y * v.y;
        ai += c.x * v.y + c.y * v.x;
    }
    double2 o = w[r];
    o.x += sign * ar;
    o.y += sign * ai;
    w[r] = o;
}

void vec_mupdate(int64_t N, int nv, const double *V, int64_t ldv, const double *h, double *w, hipStream_t st) {
    mcombine_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, nv, reinterpret_cast<const double2 *>(V), ldv,
                                                                 reinterpret_cast<const double2 *>(h), -1.0,
                                                                 reinterpret_cast<double2 *>(w));
    AFS_HIP(hipGetLastError());
}

void vec_combine(int64_t N, int nv, const double *V, int64_t ldv, const double *y, double *x, hipStream_t st) {
    mcombine_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, nv, reinterpret_cast<const double2 *>(V), ldv,
                                                                 reinterpret_cast<const double2 *>(y), 1.0,
                                                                 reinterpret_cast<double2 *>(x));
    AFS_HIP(hipGetLastError());
}

// out = x / sqrt(nrm2[0].re)
__global__ __launch_bounds__(256) void normalize_kernel(int64_t N, const double *__restrict__ nrm2,
                                                        const double2 *__restrict__ x, double2 *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    const double inv = 1.0 / sqrt(nrm2[0]);
    const double2 v = x[r];
    out[r] = make_double2(v.x * inv, v.y * inv);
}

void vec_normalize(int64_t N, const double *nrm2, const double *x, double *out, hipStream_t st) {
    normalize_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, nrm2, reinterpret_cast<const double2 *>(x),
                                                                  reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void split_ut_kernel(int64_t nt, const int8_t *__restrict__ kind,
                                                       const double2 *__restrict__ a, const double2 *__restrict__ bc,
                                                       double2 *__restrict__ u, double2 *__restrict__ t) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= 3 * nt)
        return;
    const bool trac = kind[k / 3] == 0;
    const double2 av = a[k], bv = bc[k];
    if (u)
        u[k] = trac ? av : bv;
    if (t)
        t[k] = trac ? bv : av;
}

void vec_split_ut(int64_t nt, const int8_t *kind, const double *a, const double *bc, double *u, double *t,
                  hipStream_t st) {
    split_ut_kernel<<<(unsigned)((3 * nt + 255) / 256), 256, 0, st>>>(
        nt, kind, reinterpret_cast<const double2 *>(a), reinterpret_cast<const double2 *>(bc),
        reinterpret_cast<double2 *>(u), reinterpret_cast<double2 *>(t));
    AFS_HIP(hipGetLastError());
}

// out = alpha x + beta y  (complex scalars; out may alias x or y)
__global__ __launch_bounds__(256) void axpby_kernel(int64_t N, double ar, double ai, const double2 *x, double br,
                                                    double bi, const double2 *y, double2 *out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    const double2 a = x[r], b = y[r];
    out[r] = make_double2(ar * a.x - ai * a.y + br * b.x - bi * b.y, ar * a.y + ai * a.x + br * b.y + bi * b.x);
}

void vec_axpby(int64_t N, double ar, double ai, const double *x, double br, double bi, const double *y, double *out,
               hipStream_t st) {
    axpby_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, ar, ai, reinterpret_cast<const double2 *>(x), br, bi,
                                                              reinterpret_cast<const double2 *>(y),
                                                              reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

// out += a x + b conj(x)
__global__ __launch_bounds__(256) void axpy_conj_kernel(int64_t N, double ar, double ai, double br, double bi,
                                                        const double2 *x, double2 *out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    const double2 v = x[r];
    double2 o = out[r];
    o.x += ar * v.x - ai * v.y + br * v.x + bi * v.y;
    o.y += ar * v.y + ai * v.x - br * v.y + bi * v.x;
    out[r] = o;
}

void vec_axpy_conj(int64_t N, double ar, double ai, double br, double bi, const double *x, double *out,
                   hipStream_t st) {
    axpy_conj_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(N, ar, ai, br, bi,
                                                                  reinterpret_cast<const double2 *>(x),
                                                                  reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
