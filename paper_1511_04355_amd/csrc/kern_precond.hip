// Cluster block-Jacobi preconditioner: the diagonal blocks of A over spatial
// clusters of up to kClusterElems elements (blocks of up to kClusterDim =
// 3*kClusterElems unknowns), inverted on the device.  This is the
// block-diagonal preconditioner of Section 4 with blocks larger than one
// collocation point.
//
// Inversion: one work-group per cluster, the block (FP32 complex, padded to
// kClusterDim with the identity) held in registers: thread t owns row t mod D
// and a third of its columns, and Gauss-Jordan elimination with partial
// pivoting runs in place, the pivot row, pivot column and the argmax going
// through LDS (a block of 147 x 147 complex would not fit in LDS).  The
// inverse is stored column-major at the cluster's dimension, in a slot of
// kClusterDim^2 entries.  Application: one work-group per cluster, a thread
// per row, z_c = inv_c v_c in FP64 arithmetic, the inverse's columns read
// coalesced.
#include "cplx.hpp"
#include "internal.hpp"

namespace afsbem {

struct cf {
    float r, i;
};

template <int FMT>
__device__ __forceinline__ cf load_entry(const void *A, const void * /*A_lo*/, int64_t lda, int64_t row, int64_t col) {
    const int64_t o = col * lda + row;
    if (FMT == AFSBEM_FMT_C128) {
        const double2 v = static_cast<const double2 *>(A)[o];
        return cf{(float)v.x, (float)v.y};
    }
    const float2 v = static_cast<const float2 *>(A)[o];
    return cf{v.x, v.y};
}

constexpr int kInvCols = 3;                          // column blocks per row
constexpr int kInvW = kClusterDim / kInvCols;        // columns per thread
constexpr int kInvThreads = (kClusterDim * kInvCols + 63) / 64 * 64;
static_assert(kClusterDim % kInvCols == 0, "columns split evenly over the threads of a row");

// LDS of one inversion
struct InvShared {
    float red_v[kClusterDim];
    int red_i[kClusterDim];
    int piv_row[kClusterDim];
    int p;
    cf rowk[kClusterDim], rowp[kClusterDim], colk[kClusterDim];
    cf ip;
    int dst[kClusterDim];
};

// Gauss-Jordan step on column k = kb W + KK (KK a compile-time index, so that
// the row segment a[] stays in registers)
template <int KK>
__device__ __forceinline__ void gj_step(cf (&a)[kInvW], InvShared &s, int kb, int i, int cb, bool act, int tid) {
    constexpr int W = kInvW, D = kClusterDim;
    const int k = kb * W + KK;
    const bool owner = act && cb == kb;  // holds column k (as a[KK])
    // pivot: largest |M[r][k]| over rows r >= k (lowest row on ties)
    if (owner) {
        s.red_v[i] = (i >= k) ? a[KK].r * a[KK].r + a[KK].i * a[KK].i : -1.f;
        s.red_i[i] = i;
    }
    __syncthreads();
    if (tid < 64) {
        float best = -2.f;
        int bi = k;
        for (int r = tid; r < D; r += 64)
            if (s.red_v[r] > best) {
                best = s.red_v[r];
                bi = s.red_i[r];
            }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (tid == 0) {
            s.p = bi;
            s.piv_row[k] = bi;
        }
    }
    __syncthreads();
    const int p = s.p;
    // row interchange k <-> p through LDS
    if (p != k) {
        if (act && i == k)
#pragma unroll
            for (int j = 0; j < W; ++j)
                s.rowk[cb * W + j] = a[j];
        if (act && i == p)
#pragma unroll
            for (int j = 0; j < W; ++j)
                s.rowp[cb * W + j] = a[j];
        __syncthreads();
        if (act && i == k)
#pragma unroll
            for (int j = 0; j < W; ++j)
                a[j] = s.rowp[cb * W + j];
        if (act && i == p)
#pragma unroll
            for (int j = 0; j < W; ++j)
                a[j] = s.rowk[cb * W + j];
        __syncthreads();
    }
    if (owner && i == k) {
        const cf pv = a[KK];
        const float den = pv.r * pv.r + pv.i * pv.i;
        s.ip = den > 0.f ? cf{pv.r / den, -pv.i / den} : cf{0.f, 0.f};
    }
    // column k before the update (the factors of every other row)
    if (owner)
        s.colk[i] = a[KK];
    __syncthreads();
    const cf ip = s.ip;
    // row k scaled, with M[k][k] = 1 before scaling (Gauss-Jordan in place)
    if (act && i == k) {
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const cf v = (cb == kb && j == KK) ? cf{1.f, 0.f} : a[j];
            a[j] = cf{v.r * ip.r - v.i * ip.i, v.r * ip.i + v.i * ip.r};
            s.rowk[cb * W + j] = a[j];
        }
    }
    __syncthreads();
    if (act && i != k) {
        const cf f = s.colk[i];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const cf rk = s.rowk[cb * W + j];
            if (cb == kb && j == KK)
                a[j] = cf{-(f.r * rk.r - f.i * rk.i), -(f.r * rk.i + f.i * rk.r)};
            else
                a[j] = cf{a[j].r - (f.r * rk.r - f.i * rk.i), a[j].i - (f.r * rk.i + f.i * rk.r)};
        }
    }
    __syncthreads();
}

template <int KK>
struct GjSteps {
    __device__ static __forceinline__ void run(cf (&a)[kInvW], InvShared &s, int kb, int i, int cb, bool act, int tid) {
        gj_step<KK>(a, s, kb, i, cb, act, tid);
        GjSteps<KK + 1>::run(a, s, kb, i, cb, act, tid);
    }
};
template <>
struct GjSteps<kInvW> {
    __device__ static __forceinline__ void run(cf (&)[kInvW], InvShared &, int, int, int, bool, int) {}
};

template <int FMT>
__global__ __launch_bounds__(kInvThreads) void cluster_inverse_kernel(int64_t lda, const int64_t *__restrict__ cptr,
                                                                      const int32_t *__restrict__ celem, const void *A,
                                                                      const void *A_lo, float2 *__restrict__ inv) {
    constexpr int D = kClusterDim, W = kInvW;
    __shared__ InvShared s;
    const int c = blockIdx.x;
    const int64_t e0 = cptr[c];
    const int ne = (int)(cptr[c + 1] - e0);
    const int d = 3 * ne;
    const int tid = threadIdx.x;
    const bool act = tid < D * kInvCols;
    const int i = act ? tid % D : 0;   // row
    const int cb = act ? tid / D : 0;  // column block: columns cb W .. cb W + W - 1
    cf a[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const int col = cb * W + j;
        cf v{(i == col) ? 1.f : 0.f, 0.f};  // identity outside the cluster's d x d block
        if (act && i < d && col < d) {
            if (FMT == kFmtBlocks) {  // blocks gathered for the matrix-free operator, row-major, stride d
                const float2 g = static_cast<const float2 *>(A)[(int64_t)c * D * D + (int64_t)i * d + col];
                v = cf{g.x, g.y};
            } else {
                const int64_t er = celem[e0 + i / 3], ek = celem[e0 + col / 3];
                v = load_entry<FMT>(A, A_lo, lda, 3 * er + i % 3, 3 * ek + col % 3);
            }
        }
        a[j] = v;
    }
    for (int kb = 0; kb < kInvCols; ++kb)
        GjSteps<0>::run(a, s, kb, i, cb, act, tid);
    // the row interchanges undone as column interchanges, last first: output
    // column q holds the column src[q] of the in-place result
    if (tid == 0) {
        for (int q = 0; q < D; ++q)
            s.red_i[q] = q;
        for (int k = D - 1; k >= 0; --k) {
            const int p = s.piv_row[k], tq = s.red_i[k];
            s.red_i[k] = s.red_i[p];
            s.red_i[p] = tq;
        }
        for (int q = 0; q < D; ++q)
            s.dst[s.red_i[q]] = q;
    }
    __syncthreads();
    // column-major at stride d (the top-left d x d block)
    float2 *out = inv + (int64_t)c * D * D;
    if (act && i < d)
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int q = s.dst[cb * W + j];
            if (q < d)
                out[(int64_t)q * d + i] = make_float2(a[j].r, a[j].i);
        }
}

__global__ __launch_bounds__(256) void cluster_apply_kernel(const int64_t *__restrict__ cptr,
                                                            const int32_t *__restrict__ celem,
                                                            const float2 *__restrict__ inv,
                                                            const double2 *__restrict__ v, double2 *__restrict__ z) {
    constexpr int D = kClusterDim;
    __shared__ double2 vs[D];
    const int c = blockIdx.x;
    const int64_t e0 = cptr[c];
    const int d = 3 * (int)(cptr[c + 1] - e0);
    for (int q = threadIdx.x; q < d; q += 256)
        vs[q] = v[3 * (int64_t)celem[e0 + q / 3] + q % 3];
    __syncthreads();
    const float2 *Mi = inv + (int64_t)c * D * D;  // column-major, stride d
    for (int r = threadIdx.x; r < d; r += 256) {
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < d; ++k) {
            const float2 m = Mi[(int64_t)k * d + r];
            const double2 x = vs[k];
            ar += (double)m.x * x.x - (double)m.y * x.y;
            ai += (double)m.x * x.y + (double)m.y * x.x;
        }
        z[3 * (int64_t)celem[e0 + r / 3] + r % 3] = make_double2(ar, ai);
    }
}

void cluster_inverse(const DevicePlan &d, int format, const void *A, const void *A_lo, float *inv, hipStream_t st) {
    const int64_t N = 3 * d.n_tri, lda = (N + 63) / 64 * 64;
    if (d.n_clusters == 0)
        return;
    if (format == AFSBEM_FMT_C128)
        cluster_inverse_kernel<AFSBEM_FMT_C128><<<(unsigned)d.n_clusters, kInvThreads, 0, st>>>(
            lda, d.clus_ptr, d.clus_elem, A, A_lo, reinterpret_cast<float2 *>(inv));
    else if (format == kFmtBlocks)
        cluster_inverse_kernel<kFmtBlocks><<<(unsigned)d.n_clusters, kInvThreads, 0, st>>>(
            lda, d.clus_ptr, d.clus_elem, A, A_lo, reinterpret_cast<float2 *>(inv));
    else
        cluster_inverse_kernel<AFSBEM_FMT_SPLIT><<<(unsigned)d.n_clusters, kInvThreads, 0, st>>>(
            lda, d.clus_ptr, d.clus_elem, A, A_lo, reinterpret_cast<float2 *>(inv));
    AFS_HIP(hipGetLastError());
}

void cluster_apply(const DevicePlan &d, const float *inv, const double *v, double *z, hipStream_t st) {
    cluster_apply_kernel<<<(unsigned)d.n_clusters, 256, 0, st>>>(d.clus_ptr, d.clus_elem,
                                                                 reinterpret_cast<const float2 *>(inv),
                                                                 reinterpret_cast<const double2 *>(v),
                                                                 reinterpret_cast<double2 *>(z));
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
