// Matrix-free application of the collocation operator (paper Section 2.1,
// Eq. 2): y = A(s) x without storing A.  The far rule (7-point, every pair
// m != n) is evaluated on the fly at every application, in FP32 (inner
// products of the mixed solve) or FP64 (true residuals, plain solves); the
// near pairs' corrections (exact minus far rule) and the self blocks are FP64
// 3x3 blocks formed once per frequency and applied from memory.
//
// Work mapping as in the dense far-field assembly: a lane per collocation
// point m, the work-group's 256 points walk a chunk of source elements n in
// lock-step, so source nodes, normal, kind and x_n are wave-uniform (scalar
// loads).  Per source the 7 node contributions are gathered as invariants of
// the contracted kernels
//   (T v)_i = t0 v_i + t1 (rh.v) n_i + [t2 (n.v) + t3 (rh.v)] rh_i   (scaled 1/(4 pi r^2))
//   (U v)_i = Psi v_i - X (rh.v) rh_i                                (scaled 1/(4 pi mu r))
// in the evaluation precision; the per-source result is added to FP64 lane
// accumulators, which then hold one partial sum per source chunk.
#include <hip/hip_runtime.h>

#include "fastmath64.hpp"
#include "internal.hpp"
#include "kern_mfeval.hpp"

namespace afsbem {

struct MfArgs {
    double sr, si;  // s / c_s
    double beta, lam_over_mu, c_u;
    double inv_ks2;  // 1 / |s / c_s|^2 (0 at s = 0)
};

// One far source chunk per blockIdx.y.  COMP = 0: y = A x (T for kind-0
// columns, -U for kind-1 columns); COMP = 1: the right-hand-side operator on
// the boundary values (U for kind 0, -T for kind 1).
template <class R, int COMP>
__global__ __launch_bounds__(256) void mf_far_kernel(int64_t nt, MfArgs a, const R *__restrict__ col,
                                                     const R *__restrict__ src, const R *__restrict__ coef_g,
                                                     const double *__restrict__ x, int64_t chunk_len,
                                                     double2 *__restrict__ partial) {
    // series coefficients (and in FP64 the exp / sincos tables after them)
    constexpr int NC = sizeof(R) == 8 ? 64 + kFmTabLen : 64;
    __shared__ R coef[NC];
    for (int q = threadIdx.x; q < NC; q += 256)
        coef[q] = coef_g[q];
    __syncthreads();
    const int64_t N = 3 * nt;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = m < nt;
    R px = 0, py = 0, pz = 0;
    if (active) {
        px = col[4 * m];
        py = col[4 * m + 1];
        pz = col[4 * m + 2];
    }
    const R sr = (R)a.sr, si = (R)a.si, beta = (R)a.beta, lam = (R)a.lam_over_mu;
    const R cT = (R)0.079577471545947667884;  // 1 / (4 pi)
    const R cU = (R)a.c_u;
    const R iks2 = (R)a.inv_ks2;
    const int64_t n0 = (int64_t)blockIdx.y * chunk_len;
    const int64_t n1 = (n0 + chunk_len < nt) ? n0 + chunk_len : nt;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t n = n0; n < n1; ++n) {
        const R *rec = src + 32 * n;
        const R nx = rec[28], ny = rec[29], nz = rec[30];
        const int kind = (int)rec[31];
        const double *xv = x + 6 * n;
        // a source whose vector is zero contributes exactly nothing (every
        // term below is linear in it): skipped, wave-uniformly (the
        // right-hand side of a block loaded on one face reads ~3 % of them)
        if (xv[0] == 0.0 && xv[1] == 0.0 && xv[2] == 0.0 && xv[3] == 0.0 && xv[4] == 0.0 && xv[5] == 0.0)
            continue;
        const cx<R> v0{(R)xv[0], (R)xv[1]}, v1{(R)xv[2], (R)xv[3]}, v2{(R)xv[4], (R)xv[5]};
        if (!active || m == n)
            continue;
        const bool useT = (kind == 0) != (COMP != 0);
        cx<R> c0{0, 0}, c1{0, 0}, c2x{0, 0}, c2y{0, 0}, c2z{0, 0};
        if (useT) {
            const cx<R> nv = cxadd(cxadd(cxs(v0, nx), cxs(v1, ny)), cxs(v2, nz));
#pragma unroll 1
            for (int q = 0; q < kFarNodes; ++q) {
                const R dx = rec[4 * q] - px, dy = rec[4 * q + 1] - py, dz = rec[4 * q + 2] - pz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ir = inv_sqrt(r2);
                const R r = r2 * ir;
                const R hx = dx * ir, hy = dy * ir, hz = dz * ir;
                const R rn = hx * nx + hy * ny + hz * nz;
                const MfRad<R> Rd = mf_radial<R>(cx<R>{sr * r, si * r}, beta, coef, ir * ir * iks2);
                const R f = rec[4 * q + 3] * cT * ir * ir;
                const cx<R> t1 = cxsub(Rd.Psd, Rd.X);
                const cx<R> t2 = cxadd(cxs(Rd.X, R(-2)), cxs(cxsub(cxsub(Rd.Psd, Rd.Xd), cxs(Rd.X, R(2))), lam));
                const cx<R> t3 = cxs(cxsub(cxs(Rd.X, R(4)), cxs(Rd.Xd, R(2))), rn);
                const cx<R> rv = cxadd(cxadd(cxs(v0, hx), cxs(v1, hy)), cxs(v2, hz));
                const cx<R> ft1 = cxs(t1, f);
                c0 = cxadd(c0, cxs(ft1, rn));
                c1 = cxadd(c1, cxmul(ft1, rv));
                const cx<R> g = cxs(cxadd(cxmul(t2, nv), cxmul(t3, rv)), f);
                c2x = cxadd(c2x, cxs(g, hx));
                c2y = cxadd(c2y, cxs(g, hy));
                c2z = cxadd(c2z, cxs(g, hz));
            }
        } else {
#pragma unroll 1
            for (int q = 0; q < kFarNodes; ++q) {
                const R dx = rec[4 * q] - px, dy = rec[4 * q + 1] - py, dz = rec[4 * q + 2] - pz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ir = inv_sqrt(r2);
                const R r = r2 * ir;
                const R hx = dx * ir, hy = dy * ir, hz = dz * ir;
                const MfRad<R> Rd = mf_radial<R>(cx<R>{sr * r, si * r}, beta, coef, ir * ir * iks2);
                const R f = rec[4 * q + 3] * cU * ir;
                const cx<R> rv = cxadd(cxadd(cxs(v0, hx), cxs(v1, hy)), cxs(v2, hz));
                c0 = cxadd(c0, cxs(Rd.Psi, f));
                const cx<R> g = cxs(cxmul(Rd.X, rv), -f);
                c2x = cxadd(c2x, cxs(g, hx));
                c2y = cxadd(c2y, cxs(g, hy));
                c2z = cxadd(c2z, cxs(g, hz));
            }
        }
        // per-source result: c0 v + c1 n + c2, signed by the column's role
        const cx<R> o0 = cxadd(cxadd(cxmul(c0, v0), cxs(c1, nx)), c2x);
        const cx<R> o1 = cxadd(cxadd(cxmul(c0, v1), cxs(c1, ny)), c2y);
        const cx<R> o2 = cxadd(cxadd(cxmul(c0, v2), cxs(c1, nz)), c2z);
        const double sg = useT ? (COMP ? -1.0 : 1.0) : (COMP ? 1.0 : -1.0);
        acc[0] += sg * (double)o0.r;
        acc[1] += sg * (double)o0.i;
        acc[2] += sg * (double)o1.r;
        acc[3] += sg * (double)o1.i;
        acc[4] += sg * (double)o2.r;
        acc[5] += sg * (double)o2.i;
    }
    if (active) {
        double2 *out = partial + (int64_t)blockIdx.y * N + 3 * m;
        out[0] = make_double2(acc[0], acc[1]);
        out[1] = make_double2(acc[2], acc[3]);
        out[2] = make_double2(acc[4], acc[5]);
    }
}

// y_m = sum of the far partials + sum_p nearblk[p] x_{col p} + selfblk[m] x_m
// (one thread per collocation element; fixed summation order).
__global__ __launch_bounds__(256) void mf_finalize_kernel(int64_t nt, int S, const double2 *__restrict__ partial,
                                                          const int64_t *__restrict__ near_ptr,
                                                          const int32_t *__restrict__ near_col,
                                                          const double *__restrict__ nearblk,
                                                          const double *__restrict__ selfblk,
                                                          const double *__restrict__ x, double *__restrict__ y) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= nt)
        return;
    const int64_t N = 3 * nt;
    double o[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < S; ++s) {
        const double2 *p = partial + (int64_t)s * N + 3 * m;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double2 v = p[i];
            o[2 * i] += v.x;
            o[2 * i + 1] += v.y;
        }
    }
    auto apply = [&](const double *blk, const double *xn) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double ar = blk[6 * i + 2 * j], ai = blk[6 * i + 2 * j + 1];
                const double br = xn[2 * j], bi = xn[2 * j + 1];
                o[2 * i] += ar * br - ai * bi;
                o[2 * i + 1] += ar * bi + ai * br;
            }
    };
    for (int64_t p = near_ptr[m]; p < near_ptr[m + 1]; ++p)
        apply(nearblk + 18 * p, x + 6 * (int64_t)near_col[p]);
    apply(selfblk + 18 * m, x + 6 * m);
#pragma unroll
    for (int e = 0; e < 6; ++e)
        y[6 * m + e] = o[e];
}

int mf_chunks(int64_t nt) {
    const int S = far_source_chunks(nt);
    const int64_t chunk = (nt + S - 1) / S;
    return (int)((nt + chunk - 1) / chunk);
}

void mf_apply(const Problem &p, const KernelParams &kp, int precision, int comp, const double *nearblk,
              const double *selfblk, const double *x, double *y, double *partial, hipStream_t st) {
    const DevicePlan &d = p.dev;
    const int64_t nt = d.n_tri;
    const int S = far_source_chunks(nt);
    const int64_t chunk = (nt + S - 1) / S;
    const int Sused = mf_chunks(nt);
    MfArgs a;
    a.sr = kp.s_re * kp.inv_cs;
    a.si = kp.s_im * kp.inv_cs;
    a.beta = kp.beta;
    a.lam_over_mu = kp.lam_over_mu;
    a.c_u = kp.c_u;
    const double ks2 = a.sr * a.sr + a.si * a.si;
    a.inv_ks2 = ks2 > 0.0 ? 1.0 / ks2 : 0.0;
    const dim3 g((unsigned)((nt + 255) / 256), (unsigned)Sused);
    double2 *part = reinterpret_cast<double2 *>(partial);
    if (precision == 1) {
        if (comp)
            mf_far_kernel<float, 1><<<g, 256, 0, st>>>(nt, a, d.col32, d.src32, d.coef32, x, chunk, part);
        else
            mf_far_kernel<float, 0><<<g, 256, 0, st>>>(nt, a, d.col32, d.src32, d.coef32, x, chunk, part);
    } else {
        if (comp)
            mf_far_kernel<double, 1><<<g, 256, 0, st>>>(nt, a, d.col64, d.src, d.coef, x, chunk, part);
        else
            mf_far_kernel<double, 0><<<g, 256, 0, st>>>(nt, a, d.col64, d.src, d.coef, x, chunk, part);
    }
    AFS_HIP(hipGetLastError());
    if (comp)
        return;  // the caller finalizes b
    mf_finalize_kernel<<<(unsigned)((nt + 255) / 256), 256, 0, st>>>(nt, Sused, part, d.near_ptr, d.near_col, nearblk,
                                                                     selfblk, x, y);
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
