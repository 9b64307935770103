// Batched (lockstep) Krylov kernels: many independent systems -- frequencies
// of one mesh and meshes of uneven size -- advance together, one launch per
// step for all of them.  Vectors are concatenated over the systems (system j
// owns rows [off_j, off_j + N_j)); a per-row system index maps rows back.
// Systems that have converged are skipped through a per-system flag.
#include "batched.hpp"
#include "cplx.hpp"

namespace afsbem {

typedef double d2v_b __attribute__((ext_vector_type(2)));
typedef float f4v_b __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ldnt(const double2 *p) {
    const d2v_b v = __builtin_nontemporal_load(reinterpret_cast<const d2v_b *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ldnt(const float4 *p) {
    const f4v_b v = __builtin_nontemporal_load(reinterpret_cast<const f4v_b *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// -------------------------------------------------------------- ragged GEMV
// item = (system, row block, column chunk); precision 0: C128 or hi+lo FP64,
// 1: hi plane FP32.  Row block: 256 rows (C128) or 512 rows (two per lane).
template <int KIND>  // 0: C128, 1: split FP32, 2: split FP64
__global__ __launch_bounds__(256) void bgemv_kernel(const BSys *__restrict__ sys, const int4 *__restrict__ items,
                                                    const int *__restrict__ active, const double2 *__restrict__ x,
                                                    double2 *__restrict__ partial) {
    const int4 it = items[blockIdx.x];
    const int j = it.x;
    if (!active[j])
        return;
    const BSys S = sys[j];
    const int64_t N = S.N;
    const int64_t c0 = (int64_t)it.z * S.chunk;
    const int64_t c1 = (c0 + S.chunk < N) ? c0 + S.chunk : N;
    const double2 *xs = x + S.off;
    if (KIND == 0) {
        const int64_t row = (int64_t)it.y * 256 + threadIdx.x;
        if (row >= N)
            return;
        const double2 *a = static_cast<const double2 *>(S.A) + row;
        double ar = 0, ai = 0;
        int64_t c = c0;
        for (; c + 8 <= c1; c += 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = ldnt(a + (c + u) * S.lda);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double2 xv = xs[c + u];
                ar = fma(v[u].x, xv.x, ar);
                ar = fma(-v[u].y, xv.y, ar);
                ai = fma(v[u].x, xv.y, ai);
                ai = fma(v[u].y, xv.x, ai);
            }
        }
        for (; c < c1; ++c) {
            const double2 v = a[c * S.lda], xv = xs[c];
            ar = fma(v.x, xv.x, ar);
            ar = fma(-v.y, xv.y, ar);
            ai = fma(v.x, xv.y, ai);
            ai = fma(v.y, xv.x, ai);
        }
        partial[S.part_off + (int64_t)it.z * N + row] = make_double2(ar, ai);
    } else {
        const int64_t r2 = (int64_t)it.y * 256 + threadIdx.x;
        const int64_t row = 2 * r2;
        if (row >= N)
            return;
        const int64_t lda2 = S.lda / 2;
        const float4 *h = static_cast<const float4 *>(S.A) + r2;
        const float4 *l = static_cast<const float4 *>(S.A_lo) + r2;
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0;
        float f0r = 0, f0i = 0, f1r = 0, f1i = 0;
        int64_t c = c0;
        if (KIND == 1) {
            // eight columns in flight per lane
            for (; c + 8 <= c1; c += 8) {
                float4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = ldnt(h + (c + u) * lda2);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double2 xv = xs[c + u];
                    const float xr = (float)xv.x, xi = (float)xv.y;
                    f0r = fmaf(v[u].x, xr, f0r);
                    f0r = fmaf(-v[u].y, xi, f0r);
                    f0i = fmaf(v[u].x, xi, f0i);
                    f0i = fmaf(v[u].y, xr, f0i);
                    f1r = fmaf(v[u].z, xr, f1r);
                    f1r = fmaf(-v[u].w, xi, f1r);
                    f1i = fmaf(v[u].z, xi, f1i);
                    f1i = fmaf(v[u].w, xr, f1i);
                }
            }
        } else {
            for (; c + 4 <= c1; c += 4) {
                float4 vh[4], vl[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    vh[u] = ldnt(h + (c + u) * lda2);
                    vl[u] = ldnt(l + (c + u) * lda2);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double2 xv = xs[c + u];
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
        }
        for (; c < c1; ++c) {
            const float4 vh = ldnt(h + c * lda2);
            const double2 xv = xs[c];
            if (KIND == 1) {
                const float xr = (float)xv.x, xi = (float)xv.y;
                f0r = fmaf(vh.x, xr, f0r);
                f0r = fmaf(-vh.y, xi, f0r);
                f0i = fmaf(vh.x, xi, f0i);
                f0i = fmaf(vh.y, xr, f0i);
                f1r = fmaf(vh.z, xr, f1r);
                f1r = fmaf(-vh.w, xi, f1r);
                f1i = fmaf(vh.z, xi, f1i);
                f1i = fmaf(vh.w, xr, f1i);
            } else {
                const float4 vl = ldnt(l + c * lda2);
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
        }
        if (KIND == 1) {
            a0r = f0r;
            a0i = f0i;
            a1r = f1r;
            a1i = f1i;
        }
        double2 *out = partial + S.part_off + (int64_t)it.z * N + row;
        out[0] = make_double2(a0r, a0i);
        if (row + 1 < N)
            out[1] = make_double2(a1r, a1i);
    }
}

__global__ __launch_bounds__(256) void bsum_kernel(int64_t Ntot, const BSys *__restrict__ sys,
                                                   const int32_t *__restrict__ sys_of_row,
                                                   const int *__restrict__ active,
                                                   const double2 *__restrict__ partial, double2 *__restrict__ y) {
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (R >= Ntot)
        return;
    const int j = sys_of_row[R];
    if (!active[j])
        return;
    const BSys S = sys[j];
    const int64_t row = R - S.off;
    double r = 0, i = 0;
    for (int c = 0; c < S.S; ++c) {
        const double2 v = partial[S.part_off + (int64_t)c * S.N + row];
        r += v.x;
        i += v.y;
    }
    y[R] = make_double2(r, i);
}

// ------------------------------------------------------------ multi-dots --
// chunk = (system, first row, end row) inside one system; partial[chunk][i]
__global__ __launch_bounds__(256) void bmdot_partial_kernel(const int4 *__restrict__ chunks, const int *__restrict__ active,
                                                            const double2 *__restrict__ V, int64_t ldv,
                                                            const double2 *__restrict__ w, int nvmax,
                                                            double2 *__restrict__ partial) {
    __shared__ double sr[256], si[256];
    const int4 ch = chunks[blockIdx.x];
    const int i = blockIdx.y;
    double ar = 0, ai = 0;
    if (active[ch.x]) {
        const double2 *v = V + (int64_t)i * ldv;
        for (int64_t R = (int64_t)ch.y + threadIdx.x; R < ch.z; R += 256) {
            const double2 a = v[R], b = w[R];
            ar += a.x * b.x + a.y * b.y;
            ai += a.x * b.y - a.y * b.x;
        }
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            si[threadIdx.x] += si[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[(int64_t)blockIdx.x * nvmax + i] = make_double2(sr[0], si[0]);
}

// out[j][i] = sum over the chunks of system j; grid (B, nv)
__global__ __launch_bounds__(64) void bmdot_final_kernel(const int32_t *__restrict__ chunk_ptr,
                                                         const int *__restrict__ active, int nvmax,
                                                         const double2 *__restrict__ partial, int ldo,
                                                         double2 *__restrict__ out) {
    const int j = blockIdx.x, i = blockIdx.y;
    if (!active[j])
        return;
    __shared__ double sr[64], si[64];
    double ar = 0, ai = 0;
    for (int c = chunk_ptr[j] + threadIdx.x; c < chunk_ptr[j + 1]; c += 64) {
        const double2 v = partial[(int64_t)c * nvmax + i];
        ar += v.x;
        ai += v.y;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sr[threadIdx.x] += sr[threadIdx.x + off];
            si[threadIdx.x] += si[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[(int64_t)j * ldo + i] = make_double2(sr[0], si[0]);
}

// ------------------------------------------------------- row-wise kernels --
// w[R] += sign * sum_{i < nv} h[j][i] V_i[R]   (j the row's system)
__global__ __launch_bounds__(256) void bcombine_kernel(int64_t Ntot, const int32_t *__restrict__ sys_of_row,
                                                       const int *__restrict__ active, int nv,
                                                       const int *__restrict__ nv_sys, const double2 *__restrict__ V,
                                                       int64_t ldv, const double2 *__restrict__ h, int ldh,
                                                       double sign, double2 *__restrict__ w) {
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (R >= Ntot)
        return;
    const int j = sys_of_row[R];
    if (!active[j])
        return;
    const int n = nv_sys ? nv_sys[j] : nv;
    const double2 *hj = h + (int64_t)j * ldh;
    double ar = 0, ai = 0;
    for (int i = 0; i < n; ++i) {
        const double2 c = hj[i], v = V[(int64_t)i * ldv + R];
        ar += c.x * v.x - c.y * v.y;
        ai += c.x * v.y + c.y * v.x;
    }
    double2 o = w[R];
    o.x += sign * ar;
    o.y += sign * ai;
    w[R] = o;
}

// out[R] = x[R] * scale_j, scale_j = 1 / sqrt(nrm2[j].x)   (nrm2: complex, re part)
__global__ __launch_bounds__(256) void bnormalize_kernel(int64_t Ntot, const int32_t *__restrict__ sys_of_row,
                                                         const int *__restrict__ active,
                                                         const double2 *__restrict__ nrm2, int ld,
                                                         const double2 *__restrict__ x, double2 *__restrict__ out) {
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (R >= Ntot)
        return;
    const int j = sys_of_row[R];
    if (!active[j])
        return;
    const double n2 = nrm2[(int64_t)j * ld].x;
    const double sc = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    const double2 v = x[R];
    out[R] = make_double2(v.x * sc, v.y * sc);
}

// out = a - b (rows of active systems)
__global__ __launch_bounds__(256) void bsub_kernel(int64_t Ntot, const int32_t *__restrict__ sys_of_row,
                                                   const int *__restrict__ active, const double2 *__restrict__ a,
                                                   const double2 *__restrict__ b, double2 *__restrict__ out) {
    const int64_t R = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (R >= Ntot)
        return;
    if (!active[sys_of_row[R]])
        return;
    const double2 u = a[R], v = b[R];
    out[R] = make_double2(u.x - v.x, u.y - v.y);
}

// z = M^-1 v, 3x3 complex blocks per element (all systems' elements concatenated)
__global__ __launch_bounds__(256) void bprecond_kernel(int64_t nel, const int32_t *__restrict__ sys_of_row,
                                                       const int *__restrict__ active, const double *__restrict__ D,
                                                       const double *__restrict__ v, double *__restrict__ z) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= nel)
        return;
    if (!active[sys_of_row[3 * m]])
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

// ------------------------------------------------------------- Givens --
// One thread per system.  H[j]: (m+1) x m row-major complex; g[j]: m+1;
// cs/sn[j]: m.  h1, h2: the two Gram-Schmidt passes of column k, nrm2 =
// ||w||^2 after them.  Applies the previous rotations, forms the new one,
// updates g and the residual estimate, and closes the cycle of a system whose
// estimate meets its tolerance (cyc[j] = 0).
__global__ void bgivens_kernel(int B, int m, int k, int *__restrict__ cyc, const double2 *__restrict__ h1,
                               const double2 *__restrict__ h2, int ldh, const double2 *__restrict__ nrm2,
                               double2 *__restrict__ H, double2 *__restrict__ g, double *__restrict__ cs,
                               double2 *__restrict__ sn, const double *__restrict__ tol, double *__restrict__ est,
                               int *__restrict__ kdone) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B || !cyc[j])
        return;
    double2 *Hj = H + (int64_t)j * (m + 1) * m;
    double2 *gj = g + (int64_t)j * (m + 1);
    double *csj = cs + (int64_t)j * m;
    double2 *snj = sn + (int64_t)j * m;
    for (int i = 0; i <= k; ++i) {
        const double2 a = h1[(int64_t)j * ldh + i], b = h2[(int64_t)j * ldh + i];
        Hj[i * m + k] = make_double2(a.x + b.x, a.y + b.y);
    }
    const double hn = sqrt(fmax(nrm2[j].x, 0.0));
    Hj[(k + 1) * m + k] = make_double2(hn, 0.0);
    for (int i = 0; i < k; ++i) {
        const cd a{Hj[i * m + k].x, Hj[i * m + k].y}, c{Hj[(i + 1) * m + k].x, Hj[(i + 1) * m + k].y};
        const cd s{snj[i].x, snj[i].y};
        const double cc = csj[i];
        const cd t = cadd(cscale(a, cc), cmul(s, c));
        const cd u = cadd(cscale(cmul(cconj(s), a), -1.0), cscale(c, cc));
        Hj[i * m + k] = make_double2(t.r, t.i);
        Hj[(i + 1) * m + k] = make_double2(u.r, u.i);
    }
    const cd a{Hj[k * m + k].x, Hj[k * m + k].y}, c{Hj[(k + 1) * m + k].x, Hj[(k + 1) * m + k].y};
    const double aa = sqrt(a.r * a.r + a.i * a.i);
    const double den = sqrt(a.r * a.r + a.i * a.i + c.r * c.r + c.i * c.i);
    double cc;
    cd s;
    if (aa == 0.0) {
        cc = 0.0;
        s = cd{1.0, 0.0};
    } else {
        cc = aa / den;
        s = cscale(cmul(cscale(a, 1.0 / aa), cconj(c)), 1.0 / den);
    }
    csj[k] = cc;
    snj[k] = make_double2(s.r, s.i);
    const cd nk = cadd(cscale(a, cc), cmul(s, c));
    Hj[k * m + k] = make_double2(nk.r, nk.i);
    Hj[(k + 1) * m + k] = make_double2(0.0, 0.0);
    const cd gk{gj[k].x, gj[k].y};
    const cd g1 = cscale(cmul(cconj(s), gk), -1.0);
    gj[k + 1] = make_double2(g1.r, g1.i);
    const cd g0 = cscale(gk, cc);
    gj[k] = make_double2(g0.r, g0.i);
    const double e = sqrt(g1.r * g1.r + g1.i * g1.i);
    est[j] = e;
    kdone[j] = k + 1;
    if (!(e > 0.5 * tol[j]) || hn == 0.0 || !isfinite(e))
        cyc[j] = 0;
}

// y = H(1:k,1:k) \ g(1:k), one thread per system (in place into y[j][0..k))
__global__ void bbacksolve_kernel(int B, int m, const int *__restrict__ run, const int *__restrict__ kdone,
                                  const double2 *__restrict__ H, const double2 *__restrict__ g,
                                  double2 *__restrict__ y, int ldy) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B || !run[j])
        return;
    const int k = kdone[j];
    const double2 *Hj = H + (int64_t)j * (m + 1) * m;
    const double2 *gj = g + (int64_t)j * (m + 1);
    double2 *yj = y + (int64_t)j * ldy;
    for (int i = k - 1; i >= 0; --i) {
        cd s{gj[i].x, gj[i].y};
        for (int l = i + 1; l < k; ++l)
            s = csub(s, cmul(cd{Hj[i * m + l].x, Hj[i * m + l].y}, cd{yj[l].x, yj[l].y}));
        const cd d = cinv(cd{Hj[i * m + i].x, Hj[i * m + i].y});
        const cd r = cmul(s, d);
        yj[i] = make_double2(r.r, r.i);
    }
}

// cycle start: g = (beta, 0, ...), cyc = run && beta > tol
__global__ void bcycle_init_kernel(int B, int m, const int *__restrict__ run, const double2 *__restrict__ nrm2,
                                   const double *__restrict__ tol, double2 *__restrict__ g, int *__restrict__ cyc,
                                   int *__restrict__ kdone) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B)
        return;
    const double beta = sqrt(fmax(nrm2[j].x, 0.0));
    double2 *gj = g + (int64_t)j * (m + 1);
    for (int i = 0; i <= m; ++i)
        gj[i] = make_double2(0.0, 0.0);
    gj[0] = make_double2(beta, 0.0);
    kdone[j] = 0;
    cyc[j] = (run[j] && beta > tol[j]) ? 1 : 0;
}

__global__ void bcount_kernel(int B, const int *__restrict__ flag, int *__restrict__ out) {
    __shared__ int c;
    if (threadIdx.x == 0)
        c = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < B; j += blockDim.x)
        if (flag[j])
            atomicAdd(&c, 1);
    __syncthreads();
    if (threadIdx.x == 0)
        out[0] = c;
}

// ------------------------------------------------------------ launchers --
void bgemv(const BatchDev &b, int kind, const int *active, const double *x, double *y, hipStream_t st) {
    const double2 *xv = reinterpret_cast<const double2 *>(x);
    double2 *part = reinterpret_cast<double2 *>(b.partial);
    if (kind == 0) {
        if (b.n_items128)
            bgemv_kernel<0><<<(unsigned)b.n_items128, 256, 0, st>>>(b.sys, b.items128, active, xv, part);
    } else {
        if (b.n_items64)
            (kind == 1 ? bgemv_kernel<1> : bgemv_kernel<2>)<<<(unsigned)b.n_items64, 256, 0, st>>>(
                b.sys, b.items64, active, xv, part);
    }
    AFS_HIP(hipGetLastError());
    bsum_kernel<<<(unsigned)((b.Ntot + 255) / 256), 256, 0, st>>>(b.Ntot, b.sys, b.sys_of_row, active, part,
                                                                  reinterpret_cast<double2 *>(y));
    AFS_HIP(hipGetLastError());
}

void bmdot(const BatchDev &b, const int *active, int nv, const double *V, const double *w, double *out, int ldo,
           hipStream_t st) {
    bmdot_partial_kernel<<<dim3((unsigned)b.n_chunks, (unsigned)nv), 256, 0, st>>>(
        b.chunks, active, reinterpret_cast<const double2 *>(V), b.Ntot, reinterpret_cast<const double2 *>(w),
        b.nvmax, reinterpret_cast<double2 *>(b.dot_partial));
    bmdot_final_kernel<<<dim3((unsigned)b.B, (unsigned)nv), 64, 0, st>>>(
        b.chunk_ptr, active, b.nvmax, reinterpret_cast<const double2 *>(b.dot_partial), ldo,
        reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

void bcombine(const BatchDev &b, const int *active, int nv, const int *nv_sys, const double *V, const double *h,
              int ldh, double sign, double *w, hipStream_t st) {
    bcombine_kernel<<<(unsigned)((b.Ntot + 255) / 256), 256, 0, st>>>(
        b.Ntot, b.sys_of_row, active, nv, nv_sys, reinterpret_cast<const double2 *>(V), b.Ntot,
        reinterpret_cast<const double2 *>(h), ldh, sign, reinterpret_cast<double2 *>(w));
    AFS_HIP(hipGetLastError());
}

void bnormalize(const BatchDev &b, const int *active, const double *nrm2, int ld, const double *x, double *out,
                hipStream_t st) {
    bnormalize_kernel<<<(unsigned)((b.Ntot + 255) / 256), 256, 0, st>>>(
        b.Ntot, b.sys_of_row, active, reinterpret_cast<const double2 *>(nrm2), ld, reinterpret_cast<const double2 *>(x),
        reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

void bsub(const BatchDev &b, const int *active, const double *a, const double *c, double *out, hipStream_t st) {
    bsub_kernel<<<(unsigned)((b.Ntot + 255) / 256), 256, 0, st>>>(b.Ntot, b.sys_of_row, active,
                                                                  reinterpret_cast<const double2 *>(a),
                                                                  reinterpret_cast<const double2 *>(c),
                                                                  reinterpret_cast<double2 *>(out));
    AFS_HIP(hipGetLastError());
}

void bprecond(const BatchDev &b, const int *active, const double *v, double *z, hipStream_t st) {
    const int64_t nel = b.Ntot / 3;
    bprecond_kernel<<<(unsigned)((nel + 255) / 256), 256, 0, st>>>(nel, b.sys_of_row, active, b.precond, v, z);
    AFS_HIP(hipGetLastError());
}

void bgivens(const BatchDev &b, int m, int k, int *cyc, const double *h1, const double *h2, int ldh,
             const double *nrm2, const double *tol, hipStream_t st) {
    bgivens_kernel<<<(unsigned)((b.B + 63) / 64), 64, 0, st>>>(
        b.B, m, k, cyc, reinterpret_cast<const double2 *>(h1), reinterpret_cast<const double2 *>(h2), ldh,
        reinterpret_cast<const double2 *>(nrm2), reinterpret_cast<double2 *>(b.H), reinterpret_cast<double2 *>(b.g),
        b.cs, reinterpret_cast<double2 *>(b.sn), tol, b.est, b.kdone);
    AFS_HIP(hipGetLastError());
}

void bbacksolve(const BatchDev &b, int m, const int *run, double *y, int ldy, hipStream_t st) {
    bbacksolve_kernel<<<(unsigned)((b.B + 63) / 64), 64, 0, st>>>(b.B, m, run, b.kdone,
                                                                  reinterpret_cast<const double2 *>(b.H),
                                                                  reinterpret_cast<const double2 *>(b.g),
                                                                  reinterpret_cast<double2 *>(y), ldy);
    AFS_HIP(hipGetLastError());
}

void bcycle_init(const BatchDev &b, int m, const int *run, const double *nrm2, const double *tol, int *cyc,
                 hipStream_t st) {
    bcycle_init_kernel<<<(unsigned)((b.B + 63) / 64), 64, 0, st>>>(
        b.B, m, run, reinterpret_cast<const double2 *>(nrm2), tol, reinterpret_cast<double2 *>(b.g), cyc, b.kdone);
    AFS_HIP(hipGetLastError());
}

void bcount(const BatchDev &b, const int *flag, int *out, hipStream_t st) {
    bcount_kernel<<<1, 256, 0, st>>>(b.B, flag, out);
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
