// Cluster block-Jacobi preconditioner: the diagonal blocks of A over spatial
// clusters of up to kClusterElems elements (blocks of up to 3*kClusterElems
// unknowns), inverted on the device.  This is the block-diagonal
// preconditioner of Section 4 with blocks larger than one collocation point.
//
// Inversion: one workgroup per cluster gathers its block (FP32 complex) into
// LDS and runs Gauss-Jordan elimination with partial pivoting in place; the
// inverse is stored FP32 complex at a fixed stride (kClusterDim^2 entries).
// Application: one workgroup per cluster, z_c = inv_c v_c in FP64 arithmetic.
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

template <int FMT>
__global__ __launch_bounds__(256) void cluster_inverse_kernel(int64_t lda, const int64_t *__restrict__ cptr,
                                                              const int32_t *__restrict__ celem, const void *A,
                                                              const void *A_lo, float2 *__restrict__ inv) {
    constexpr int D = kClusterDim;
    __shared__ cf M[D][D + 1];
    __shared__ int piv_row[D];
    __shared__ cf fcol[D];
    __shared__ float red_v[256];
    __shared__ int red_i[256];
    const int c = blockIdx.x;
    const int64_t e0 = cptr[c];
    const int ne = (int)(cptr[c + 1] - e0);
    const int d = 3 * ne;
    const int tid = threadIdx.x;
    for (int q = tid; q < d * d; q += 256) {
        const int r = q / d, k = q % d;
        if (FMT == kFmtBlocks) {  // blocks gathered for the matrix-free operator, stride d
            const float2 g = static_cast<const float2 *>(A)[(int64_t)c * D * D + q];
            M[r][k] = cf{g.x, g.y};
        } else {
            const int64_t er = celem[e0 + r / 3], ek = celem[e0 + k / 3];
            M[r][k] = load_entry<FMT>(A, A_lo, lda, 3 * er + r % 3, 3 * ek + k % 3);
        }
    }
    __syncthreads();
    for (int k = 0; k < d; ++k) {
        // pivot: largest |M[i][k]|, i >= k
        float best = -1.f;
        int bi = k;
        for (int i = k + tid; i < d; i += 256) {
            const float a = M[i][k].r * M[i][k].r + M[i][k].i * M[i][k].i;
            if (a > best) {
                best = a;
                bi = i;
            }
        }
        red_v[tid] = best;
        red_i[tid] = bi;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (tid < off && (red_v[tid + off] > red_v[tid] ||
                              (red_v[tid + off] == red_v[tid] && red_i[tid + off] < red_i[tid]))) {
                red_v[tid] = red_v[tid + off];
                red_i[tid] = red_i[tid + off];
            }
            __syncthreads();
        }
        const int p = red_i[0];
        if (tid == 0)
            piv_row[k] = p;
        if (p != k)
            for (int j = tid; j < d; j += 256) {
                const cf t = M[k][j];
                M[k][j] = M[p][j];
                M[p][j] = t;
            }
        __syncthreads();
        const cf pv = M[k][k];
        const float den = pv.r * pv.r + pv.i * pv.i;
        const cf ip = den > 0.f ? cf{pv.r / den, -pv.i / den} : cf{0.f, 0.f};
        __syncthreads();
        // row k scaled, with M[k][k] = 1 before scaling (Gauss-Jordan in place)
        for (int j = tid; j < d; j += 256) {
            const cf v = (j == k) ? cf{1.f, 0.f} : M[k][j];
            M[k][j] = cf{v.r * ip.r - v.i * ip.i, v.r * ip.i + v.i * ip.r};
        }
        // column k is read by every update of its row: take a copy first
        for (int i = tid; i < d; i += 256)
            if (i != k)
                fcol[i] = M[i][k];
        __syncthreads();
        for (int q = tid; q < d * d; q += 256) {
            const int i = q / d, j = q % d;
            if (i == k)
                continue;
            const cf f = fcol[i];
            const cf rk = M[k][j];
            if (j == k) {
                M[i][j] = cf{-(f.r * rk.r - f.i * rk.i), -(f.r * rk.i + f.i * rk.r)};
            } else {
                M[i][j].r -= f.r * rk.r - f.i * rk.i;
                M[i][j].i -= f.r * rk.i + f.i * rk.r;
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int k = d - 1; k >= 0; --k) {
        const int p = piv_row[k];
        if (p != k)
            for (int i = tid; i < d; i += 256) {
                const cf t = M[i][k];
                M[i][k] = M[i][p];
                M[i][p] = t;
            }
        __syncthreads();
    }
    float2 *out = inv + (int64_t)c * D * D;
    for (int q = tid; q < d * d; q += 256)
        out[q] = make_float2(M[q / d][q % d].r, M[q / d][q % d].i);
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
    const float2 *Mi = inv + (int64_t)c * D * D;
    for (int r = threadIdx.x; r < d; r += 256) {
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < d; ++k) {
            const float2 m = Mi[r * d + k];
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
        cluster_inverse_kernel<AFSBEM_FMT_C128><<<(unsigned)d.n_clusters, 256, 0, st>>>(
            lda, d.clus_ptr, d.clus_elem, A, A_lo, reinterpret_cast<float2 *>(inv));
    else if (format == kFmtBlocks)
        cluster_inverse_kernel<kFmtBlocks><<<(unsigned)d.n_clusters, 256, 0, st>>>(
            lda, d.clus_ptr, d.clus_elem, A, A_lo, reinterpret_cast<float2 *>(inv));
    else
        cluster_inverse_kernel<AFSBEM_FMT_SPLIT><<<(unsigned)d.n_clusters, 256, 0, st>>>(
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
