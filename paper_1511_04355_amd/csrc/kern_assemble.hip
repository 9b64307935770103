// Assembly of the collocation system A(s) a = b(s) (paper Section 2.1, Eq. 1-2)
// on gfx950, FP64 kernel evaluation.
//
// Matrix layout: column-major with leading dimension lda (a multiple of 64);
// entry (row 3m+i, col 3n+j) is the (i, j) entry of the 3x3 block of
// collocation element m and source element n.
//
// Work mapping.  The far-field kernel gives every lane one collocation point
// (row block m) and walks a chunk of source elements n in lock-step, so the
// source quadrature nodes, normal and boundary kind are wave-uniform (scalar
// loads, no divergence on the boundary-condition branch) and each store of a
// 3x3 block column lands on 3 consecutive rows per lane, i.e. one contiguous
// 48/24-byte run per lane that together with the neighbouring lanes covers
// 64*3 consecutive rows of the column.  Near pairs and self elements are few
// but need many nodes each: one wavefront per pair, lanes over nodes, then a
// wavefront reduction.
#include "cplx.hpp"
#include "fastmath64.hpp"
#include "internal.hpp"
#include "kern_eval.hpp"

namespace afsbem {

// NQ nodes per source record: kFarNodes (flat elements, the record of element
// n; skips n == m, the self element) or 1 (Nystrom points, the record of
// point n; skips the six points of the target point's own element).
template <int FMT, int NQ>
__global__ __launch_bounds__(256) void far_assemble_kernel(
    int64_t nt, int64_t lda, KernelParams kp, const double *__restrict__ colx, const double *__restrict__ coly,
    const double *__restrict__ colz, const double *__restrict__ src, const double *__restrict__ bc,
    const double *__restrict__ coef, int64_t chunk_len, void *A, void *A_lo, double *__restrict__ bpart) {
    const int64_t N = 3 * nt;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = m < nt;
    double xx = 0, xy = 0, xz = 0;
    if (active) {
        xx = colx[m];
        xy = coly[m];
        xz = colz[m];
    }
    const int64_t n0 = (int64_t)blockIdx.y * chunk_len;
    const int64_t n1 = (n0 + chunk_len < nt) ? n0 + chunk_len : nt;
    cd bacc[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
    for (int64_t n = n0; n < n1; ++n) {
        const double *rec = src + kSrcStride * n;
        const double nx = rec[28], ny = rec[29], nz = rec[30];
        const int kind = (int)rec[31];
        const double *bv = bc + 6 * n;
        const cd v[3] = {cd{bv[0], bv[1]}, cd{bv[2], bv[3]}, cd{bv[4], bv[5]}};
        if (!active || (NQ == kFarNodes ? m == n : m / 6 == n / 6))
            continue;
        BlockAcc acc;
        acc.zero();
        if (kind == 0) {
#pragma unroll 1
            for (int q = 0; q < NQ; ++q) {
                PairEval E;
                eval_pair(kp, coef, xx, xy, xz, rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], nx, ny, nz, E);
                const double w = rec[4 * q + 3];
                acc_node<0>(E, kp, nx, ny, nz, w, w, v, acc, bacc);
            }
        } else {
#pragma unroll 1
            for (int q = 0; q < NQ; ++q) {
                PairEval E;
                eval_pair(kp, coef, xx, xy, xz, rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], nx, ny, nz, E);
                const double w = rec[4 * q + 3];
                acc_node<1>(E, kp, nx, ny, nz, w, w, v, acc, bacc);
            }
        }
        cd blk[9];
        expand_block(kind, acc, nx, ny, nz, blk);
        store_block<FMT>(A, A_lo, lda, m, n, blk);
    }
    if (active) {
        double *bp = bpart + 2 * ((int64_t)blockIdx.y * N + 3 * m);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            bp[2 * i] = bacc[i].r;
            bp[2 * i + 1] = bacc[i].i;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Lane-strided walk over the subdivision-leaf nodes of one near pair, plus the
// 7 far-rule nodes whose contribution to b is removed again.
template <int KIND>
__device__ __forceinline__ void near_items(int64_t first, int64_t stride, int64_t items, int64_t n_near, int64_t L0,
                                           const double *__restrict__ leaves, const Rule7Args &rule,
                                           const double *__restrict__ rec, const KernelParams &kp,
                                           const double *__restrict__ coef, double xx, double xy, double xz,
                                           double nx, double ny, double nz, const cd v[3], double far_sA,
                                           BlockAcc &acc, cd bcor[3]) {
    for (int64_t k = first; k < items; k += stride) {
        double yx, yy, yz, w, sA, sB;
        if (k < n_near) {
            const double *L = leaves + 10 * (L0 + k / 7);
            const int q = (int)(k % 7);
            yx = L[0] + rule.b1[q] * L[3] + rule.b2[q] * L[6];
            yy = L[1] + rule.b1[q] * L[4] + rule.b2[q] * L[7];
            yz = L[2] + rule.b1[q] * L[5] + rule.b2[q] * L[8];
            w = rule.w[q] * L[9];
            sA = 1.0;
            sB = 1.0;
        } else {
            const int q = (int)(k - n_near);
            yx = rec[4 * q];
            yy = rec[4 * q + 1];
            yz = rec[4 * q + 2];
            w = rec[4 * q + 3];
            sA = far_sA;
            sB = -1.0;
        }
        PairEval E;
        eval_pair(kp, coef, xx, xy, xz, yx, yy, yz, nx, ny, nz, E);
        acc_node<KIND>(E, kp, nx, ny, nz, sA * w, sB * w, v, acc, bcor);
    }
}

// ---------------------------------------------------------------- near pairs --
// kNearLanes lanes per near pair (8 pairs per wavefront): the lanes of a group
// stride over the pair's subdivision-leaf nodes (about 8 leaves, 60 nodes on
// average) and combine the 32 accumulated doubles in log2(kNearLanes) shuffle
// steps; neighbouring groups hold neighbouring pairs.
constexpr int kNearLanes = 8;

__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = kNearLanes / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <int FMT>
__global__ __launch_bounds__(256) void near_assemble_kernel(
    int64_t /*nt*/, int64_t lda, int64_t nnz, KernelParams kp, Rule7Args rule, const double *__restrict__ colx,
    const double *__restrict__ coly, const double *__restrict__ colz, const double *__restrict__ src,
    const double *__restrict__ bc, const double *__restrict__ coef, const int32_t *__restrict__ near_row,
    const int32_t *__restrict__ near_col, const int32_t *__restrict__ near_order, const int64_t *__restrict__ leaf_ptr,
    const double *__restrict__ leaves, void *A, void *A_lo, double *__restrict__ corr) {
    // FMT == kFmtBlocks: A receives the correction block (exact - far rule) of
    // pair p at [p][9] complex, row-major (the far rule stays in the operator)
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t g = gid / kNearLanes;
    const int sub = (int)(gid % kNearLanes);
    // groups are aligned inside a wavefront, so a whole group is in or out
    if (g >= nnz)
        return;
    const int64_t p = near_order[g];
    const int64_t m = near_row[p], n = near_col[p];
    const double xx = colx[m], xy = coly[m], xz = colz[m];
    const double *rec = src + kSrcStride * n;
    const double nx = rec[28], ny = rec[29], nz = rec[30];
    const int kind = (int)rec[31];
    const double *bv = bc + 6 * n;
    const cd v[3] = {cd{bv[0], bv[1]}, cd{bv[2], bv[3]}, cd{bv[4], bv[5]}};
    const int64_t L0 = leaf_ptr[p], L1 = leaf_ptr[p + 1];
    const int64_t n_near = 7 * (L1 - L0);
    const int64_t items = n_near + kFarNodes;
    BlockAcc acc;
    acc.zero();
    cd bcor[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
    const double far_sA = (FMT == kFmtBlocks) ? -1.0 : 0.0;
    if (kind == 0)
        near_items<0>(sub, kNearLanes, items, n_near, L0, leaves, rule, rec, kp, coef, xx, xy, xz, nx, ny, nz, v,
                      far_sA, acc, bcor);
    else
        near_items<1>(sub, kNearLanes, items, n_near, L0, leaves, rule, rec, kp, coef, xx, xy, xz, nx, ny, nz, v,
                      far_sA, acc, bcor);
    acc.E.r = group_sum(acc.E.r);
    acc.E.i = group_sum(acc.E.i);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        acc.Aj[e].r = group_sum(acc.Aj[e].r);
        acc.Aj[e].i = group_sum(acc.Aj[e].i);
        acc.Ci[e].r = group_sum(acc.Ci[e].r);
        acc.Ci[e].i = group_sum(acc.Ci[e].i);
        bcor[e].r = group_sum(bcor[e].r);
        bcor[e].i = group_sum(bcor[e].i);
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        acc.D[e].r = group_sum(acc.D[e].r);
        acc.D[e].i = group_sum(acc.D[e].i);
    }
    if (sub != 0)
        return;
    cd blk[9];
    expand_block(kind, acc, nx, ny, nz, blk);
    if (FMT == kFmtBlocks)
        store_blk9(static_cast<double *>(A) + 18 * p, blk);
    else
        store_block<FMT>(A, A_lo, lda, m, n, blk);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        corr[6 * p + 2 * e] = bcor[e].r;
        corr[6 * p + 2 * e + 1] = bcor[e].i;
    }
}

// ------------------------------------------------------------- self element --
// 3x3 complex inverse by the adjugate (row-major in, row-major out).
__device__ void inv3(const cd a[9], cd out[9]) {
    const cd c00 = csub(cmul(a[4], a[8]), cmul(a[5], a[7]));
    const cd c01 = csub(cmul(a[5], a[6]), cmul(a[3], a[8]));
    const cd c02 = csub(cmul(a[3], a[7]), cmul(a[4], a[6]));
    const cd det = cadd(cadd(cmul(a[0], c00), cmul(a[1], c01)), cmul(a[2], c02));
    const cd id = cinv(det);
    out[0] = cmul(c00, id);
    out[1] = cmul(csub(cmul(a[2], a[7]), cmul(a[1], a[8])), id);
    out[2] = cmul(csub(cmul(a[1], a[5]), cmul(a[2], a[4])), id);
    out[3] = cmul(c01, id);
    out[4] = cmul(csub(cmul(a[0], a[8]), cmul(a[2], a[6])), id);
    out[5] = cmul(csub(cmul(a[2], a[3]), cmul(a[0], a[5])), id);
    out[6] = cmul(c02, id);
    out[7] = cmul(csub(cmul(a[1], a[6]), cmul(a[0], a[7])), id);
    out[8] = cmul(csub(cmul(a[0], a[4]), cmul(a[1], a[3])), id);
}

template <int FMT>
__global__ __launch_bounds__(256) void self_assemble_kernel(
    int64_t nt, int64_t lda, KernelParams kp, const double *__restrict__ colx, const double *__restrict__ coly,
    const double *__restrict__ colz, const double *__restrict__ src, const double *__restrict__ bc,
    const double *__restrict__ coef, const double *__restrict__ self_ang, const double *__restrict__ self_cpv,
    const double *__restrict__ gl_rho, int n_theta, int n_rho, void *A, void *A_lo, double *__restrict__ bself,
    double *__restrict__ precond) {
    const int64_t m = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (m >= nt)
        return;
    const double xx = colx[m], xy = coly[m], xz = colz[m];
    const double *rec = src + kSrcStride * m;
    const double nx = rec[28], ny = rec[29], nz = rec[30];
    const int kind = (int)rec[31];
    const double b2 = kp.beta * kp.beta;
    const int items = 3 * n_theta * n_rho;
    const double *ang = self_ang + (int64_t)m * 3 * n_theta * 5;
    cd G[9], H[9];
#pragma unroll
    for (int e = 0; e < 9; ++e)
        G[e] = H[e] = cd{0, 0};
    for (int k = lane; k < items; k += 64) {
        const double *a = ang + 5 * (k / n_rho);
        const int q = k % n_rho;
        const double R = a[3];
        const double rho = R * gl_rho[2 * q];
        const double w = a[4] * R * gl_rho[2 * q + 1] * rho;
        PairEval E;
        eval_pair(kp, coef, xx, xy, xz, xx + rho * a[0], xy + rho * a[1], xz + rho * a[2], nx, ny, nz, E);
        acc_U(E, kp, w, G);
        // remove the static 1/r^2 part: T0 = beta^2/(4 pi r^2)(rh_i n_j - n_i rh_j)
        E.t1 = cadd(E.t1, cd{b2, 0.0});
        E.t2 = csub(E.t2, cd{b2, 0.0});
        acc_T(E, nx, ny, nz, w, H);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        G[e].r = wave_sum(G[e].r);
        G[e].i = wave_sum(G[e].i);
        H[e].r = wave_sum(H[e].r);
        H[e].i = wave_sum(H[e].i);
    }
    if (lane != 0)
        return;
    const double *cpv = self_cpv + 9 * m;
#pragma unroll
    for (int e = 0; e < 9; ++e)
        H[e].r += cpv[e];
    H[0].r += 0.5;
    H[4].r += 0.5;
    H[8].r += 0.5;
    const double *bv = bc + 6 * m;
    const cd v[3] = {cd{bv[0], bv[1]}, cd{bv[2], bv[3]}, cd{bv[4], bv[5]}};
    cd blk[9], bs[3];
    for (int i = 0; i < 3; ++i) {
        bs[i] = cd{0, 0};
        for (int j = 0; j < 3; ++j) {
            if (kind == 0) {
                blk[3 * i + j] = H[3 * i + j];
                bs[i] = cadd(bs[i], cmul(G[3 * i + j], v[j]));
            } else {
                blk[3 * i + j] = cscale(G[3 * i + j], -1.0);
                bs[i] = csub(bs[i], cmul(H[3 * i + j], v[j]));
            }
        }
    }
    if (FMT == kFmtBlocks)
        store_blk9(static_cast<double *>(A) + 18 * m, blk);
    else
        store_block<FMT>(A, A_lo, lda, m, m, blk);
    for (int i = 0; i < 3; ++i) {
        bself[6 * m + 2 * i] = bs[i].r;
        bself[6 * m + 2 * i + 1] = bs[i].i;
    }
    if (precond) {
        cd inv[9];
        inv3(blk, inv);
        for (int e = 0; e < 9; ++e) {
            precond[18 * m + 2 * e] = inv[e].r;
            precond[18 * m + 2 * e + 1] = inv[e].i;
        }
    }
}

// b = sum over far chunks + self + near corrections (fixed order: deterministic)
__global__ __launch_bounds__(256) void finalize_b_kernel(int64_t nt, int S, const double *__restrict__ bpart,
                                                         const double *__restrict__ bself,
                                                         const int64_t *__restrict__ near_ptr,
                                                         const double *__restrict__ corr, double *__restrict__ b) {
    const int64_t N = 3 * nt;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= N)
        return;
    const int64_t m = r / 3;
    const int i = (int)(r % 3);
    // eight partial sums in flight per lane, combined in a fixed order
    const double2 *bp = reinterpret_cast<const double2 *>(bpart);
    double pr[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pi[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int s = 0;
    for (; s + 8 <= S; s += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = bp[(int64_t)(s + u) * N + r];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            pr[u] += v[u].x;
            pi[u] += v[u].y;
        }
    }
    for (; s < S; ++s) {
        const double2 v = bp[(int64_t)s * N + r];
        pr[0] += v.x;
        pi[0] += v.y;
    }
    double ar = 0, ai = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        ar += pr[u];
        ai += pi[u];
    }
    ar += bself[6 * m + 2 * i];
    ai += bself[6 * m + 2 * i + 1];
    for (int64_t p = near_ptr[m]; p < near_ptr[m + 1]; ++p) {
        ar += corr[6 * p + 2 * i];
        ai += corr[6 * p + 2 * i + 1];
    }
    b[2 * r] = ar;
    b[2 * r + 1] = ai;
}

// ----------------------------------------------------------------- launch --
int far_source_chunks(int64_t nt) {
    const int64_t gx = (nt + 255) / 256;
    int64_t S = (4096 + gx - 1) / gx;
    if (S > nt)
        S = nt;
    if (S < 1)
        S = 1;
    return (int)S;
}

size_t assembly_scratch_bytes(const Problem &p) {
    const int64_t nt = p.dev.n_tri, N = 3 * nt;
    const int S = far_source_chunks(nt);
    return (size_t)S * N * 16 + (size_t)nt * 48 + (size_t)std::max<int64_t>(p.dev.nnz, 1) * 48 + 4096;
}

KernelParams kernel_params(const MaterialDerived &m, double s_re, double s_im) {
    KernelParams k;
    k.s_re = s_re;
    k.s_im = s_im;
    k.inv_cs = 1.0 / m.cs;
    k.beta = m.beta;
    k.c_u = 1.0 / (4.0 * 3.14159265358979323846 * m.mu);
    k.lam_over_mu = m.lam_over_mu;
    const double s2 = s_re * s_re + s_im * s_im;
    k.inv_ks2 = s2 > 0.0 ? m.cs * m.cs / s2 : 0.0;  // only the closed form (|x| >= 1/4) uses it
    return k;
}

static Rule7Args rule7_args() {
    Rule7Args r;
    const double q = std::sqrt(15.0);
    const double oa[2] = {(6.0 - q) / 21.0, (6.0 + q) / 21.0};
    const double ow[2] = {(155.0 - q) / 1200.0, (155.0 + q) / 1200.0};
    r.b1[0] = r.b2[0] = 1.0 / 3.0;
    r.w[0] = 0.225;
    for (int o = 0; o < 2; ++o)
        for (int k = 0; k < 3; ++k) {
            const int i = 1 + 3 * o + k;
            // barycentric (l0, l1, l2) with l_k = 1 - 2a, the others a
            r.b1[i] = (k == 1) ? 1.0 - 2.0 * oa[o] : oa[o];
            r.b2[i] = (k == 2) ? 1.0 - 2.0 * oa[o] : oa[o];
            r.w[i] = ow[o];
        }
    return r;
}

void launch_assembly(const Problem &p, const KernelParams &kp, const double *bc_val, int format, void *A,
                     void *A_lo, double *b, double *precond, void *scratch, hipStream_t st, hipEvent_t far_begin,
                     hipEvent_t far_end) {
    const DevicePlan &d = p.dev;
    const int64_t nt = d.n_tri, N = 3 * nt;
    const int64_t lda = (N + 63) / 64 * 64;
    const int S = far_source_chunks(nt);
    const int64_t chunk = (nt + S - 1) / S;
    const int Sused = (int)((nt + chunk - 1) / chunk);
    double *bpart = static_cast<double *>(scratch);
    double *bself = bpart + 2 * (size_t)S * N;
    double *corr = bself + 6 * nt;
    const double *coef = d.coef;
    dim3 gfar((unsigned)((nt + 255) / 256), (unsigned)Sused);
    const unsigned gnear = (unsigned)((d.nnz * kNearLanes + 255) / 256);
    const unsigned gself = (unsigned)((nt * 64 + 255) / 256);
    const Rule7Args rule = rule7_args();
    if (far_begin)
        AFS_HIP(hipEventRecord(far_begin, st));
    if (d.disc == 1) {
        if (format == AFSBEM_FMT_C128)
            far_assemble_kernel<AFSBEM_FMT_C128, 1><<<gfar, 256, 0, st>>>(nt, lda, kp, d.colx, d.coly, d.colz, d.src,
                                                                         bc_val, coef, chunk, A, A_lo, bpart);
        else
            far_assemble_kernel<AFSBEM_FMT_SPLIT, 1><<<gfar, 256, 0, st>>>(nt, lda, kp, d.colx, d.coly, d.colz, d.src,
                                                                          bc_val, coef, chunk, A, A_lo, bpart);
        if (far_end)
            AFS_HIP(hipEventRecord(far_end, st));
        AFS_HIP(hipGetLastError());
        launch_nystrom_near_self(p, kp, bc_val, format, A, A_lo, bself, corr, precond, st);
        finalize_b_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(nt, Sused, bpart, bself, d.near_ptr, corr, b);
        AFS_HIP(hipGetLastError());
        return;
    }
    if (format == AFSBEM_FMT_C128)
        far_assemble_kernel<AFSBEM_FMT_C128, kFarNodes><<<gfar, 256, 0, st>>>(
            nt, lda, kp, d.colx, d.coly, d.colz, d.src, bc_val, coef, chunk, A, A_lo, bpart);
    else
        far_assemble_kernel<AFSBEM_FMT_SPLIT, kFarNodes><<<gfar, 256, 0, st>>>(
            nt, lda, kp, d.colx, d.coly, d.colz, d.src, bc_val, coef, chunk, A, A_lo, bpart);
    if (far_end)
        AFS_HIP(hipEventRecord(far_end, st));
    if (format == AFSBEM_FMT_C128) {
        if (d.nnz)
            near_assemble_kernel<AFSBEM_FMT_C128><<<gnear, 256, 0, st>>>(
                nt, lda, d.nnz, kp, rule, d.colx, d.coly, d.colz, d.src, bc_val, coef, d.near_row, d.near_col, d.near_order,
                d.leaf_ptr, d.leaves, A, A_lo, corr);
        self_assemble_kernel<AFSBEM_FMT_C128><<<gself, 256, 0, st>>>(nt, lda, kp, d.colx, d.coly, d.colz, d.src,
                                                                    bc_val, coef, d.self_ang, d.self_cpv, d.gl_rho,
                                                                    d.n_theta, d.n_rho, A, A_lo, bself, precond);
    } else {
        if (d.nnz)
            near_assemble_kernel<AFSBEM_FMT_SPLIT><<<gnear, 256, 0, st>>>(
                nt, lda, d.nnz, kp, rule, d.colx, d.coly, d.colz, d.src, bc_val, coef, d.near_row, d.near_col, d.near_order,
                d.leaf_ptr, d.leaves, A, A_lo, corr);
        self_assemble_kernel<AFSBEM_FMT_SPLIT><<<gself, 256, 0, st>>>(nt, lda, kp, d.colx, d.coly, d.colz, d.src,
                                                                     bc_val, coef, d.self_ang, d.self_cpv, d.gl_rho,
                                                                     d.n_theta, d.n_rho, A, A_lo, bself, precond);
    }
    AFS_HIP(hipGetLastError());
    finalize_b_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(nt, Sused, bpart, bself, d.near_ptr, corr, b);
    AFS_HIP(hipGetLastError());
}

// Diagonal blocks of the cluster preconditioner for the matrix-free operator
// (no stored matrix to read them from): the operator's block (m, n) is the
// self block for m = n, else the far rule's block plus the pair's near
// correction (exact - far rule) when (m, n) is a near pair -- the same sum a
// matrix-free product forms.  One thread per element pair of the cluster,
// FP64 evaluation; output FP32 complex, row-major with the cluster's own
// dimension d = 3 ne as stride, at the cluster's slot of kClusterDim^2 entries.
__global__ __launch_bounds__(256) void cluster_gather_mf_kernel(
    KernelParams kp, const double *__restrict__ colx, const double *__restrict__ coly,
    const double *__restrict__ colz, const double *__restrict__ src, const double *__restrict__ coef,
    const int64_t *__restrict__ near_ptr, const int32_t *__restrict__ near_col, const double *__restrict__ nearblk,
    const double *__restrict__ selfblk, const int64_t *__restrict__ cptr, const int32_t *__restrict__ celem,
    float2 *__restrict__ out) {
    const int c = blockIdx.x;
    const int64_t e0 = cptr[c];
    const int ne = (int)(cptr[c + 1] - e0);
    const int d = 3 * ne;
    float2 *blkout = out + (int64_t)c * kClusterDim * kClusterDim;
    for (int q = threadIdx.x; q < ne * ne; q += 256) {
        const int r = q / ne, k = q % ne;
        const int64_t m = celem[e0 + r], n = celem[e0 + k];
        cd blk[9];
        if (m == n) {
            const double *sb = selfblk + 18 * m;
#pragma unroll
            for (int e = 0; e < 9; ++e)
                blk[e] = cd{sb[2 * e], sb[2 * e + 1]};
        } else {
            const double *rec = src + kSrcStride * n;
            const double nx = rec[28], ny = rec[29], nz = rec[30];
            const int kind = (int)rec[31];
            const cd v0[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
            cd bdummy[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
            BlockAcc acc;
            acc.zero();
            const double xx = colx[m], xy = coly[m], xz = colz[m];
#pragma unroll 1
            for (int qn = 0; qn < kFarNodes; ++qn) {
                PairEval E;
                eval_pair(kp, coef, xx, xy, xz, rec[4 * qn], rec[4 * qn + 1], rec[4 * qn + 2], nx, ny, nz, E);
                const double w = rec[4 * qn + 3];
                if (kind == 0)
                    acc_node<0>(E, kp, nx, ny, nz, w, 0.0, v0, acc, bdummy);
                else
                    acc_node<1>(E, kp, nx, ny, nz, w, 0.0, v0, acc, bdummy);
            }
            expand_block(kind, acc, nx, ny, nz, blk);
            for (int64_t pp = near_ptr[m]; pp < near_ptr[m + 1]; ++pp)
                if (near_col[pp] == n) {
                    const double *nb = nearblk + 18 * pp;
#pragma unroll
                    for (int e = 0; e < 9; ++e)
                        blk[e] = cadd(blk[e], cd{nb[2 * e], nb[2 * e + 1]});
                    break;
                }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                blkout[(3 * r + a) * d + 3 * k + b] = make_float2((float)blk[3 * a + b].r, (float)blk[3 * a + b].i);
    }
}

void cluster_gather_mf(const Problem &p, const KernelParams &kp, const double *nearblk, const double *selfblk,
                       float *out, hipStream_t st) {
    const DevicePlan &d = p.dev;
    if (d.n_clusters == 0)
        return;
    cluster_gather_mf_kernel<<<(unsigned)d.n_clusters, 256, 0, st>>>(
        kp, d.colx, d.coly, d.colz, d.src, d.coef, d.near_ptr, d.near_col, nearblk, selfblk, d.clus_ptr, d.clus_elem,
        reinterpret_cast<float2 *>(out));
    AFS_HIP(hipGetLastError());
}

void launch_block_setup(const Problem &p, const KernelParams &kp, const double *bc_val, double *nearblk,
                        double *selfblk, double *precond, void *scratch, hipStream_t st) {
    const DevicePlan &d = p.dev;
    const int64_t nt = d.n_tri;
    const int S = far_source_chunks(nt);
    const int64_t N = 3 * nt;
    double *bpart = static_cast<double *>(scratch);
    double *bself = bpart + 2 * (size_t)S * N;
    double *corr = bself + 6 * nt;
    const unsigned gnear = (unsigned)((d.nnz * kNearLanes + 255) / 256);
    const unsigned gself = (unsigned)((nt * 64 + 255) / 256);
    const Rule7Args rule = rule7_args();
    if (d.nnz)
        near_assemble_kernel<kFmtBlocks><<<gnear, 256, 0, st>>>(nt, 0, d.nnz, kp, rule, d.colx, d.coly, d.colz, d.src,
                                                                bc_val, d.coef, d.near_row, d.near_col, d.near_order, d.leaf_ptr,
                                                                d.leaves, nearblk, nullptr, corr);
    self_assemble_kernel<kFmtBlocks><<<gself, 256, 0, st>>>(nt, 0, kp, d.colx, d.coly, d.colz, d.src, bc_val, d.coef,
                                                            d.self_ang, d.self_cpv, d.gl_rho, d.n_theta, d.n_rho,
                                                            selfblk, nullptr, bself, precond);
    AFS_HIP(hipGetLastError());
}

void launch_finalize_b(const Problem &p, int S, const double *bpart, const void *scratch, double *b,
                       hipStream_t st) {
    const DevicePlan &d = p.dev;
    const int64_t nt = d.n_tri, N = 3 * nt;
    const int Smax = far_source_chunks(nt);
    const double *bself = static_cast<const double *>(scratch) + 2 * (size_t)Smax * N;
    const double *corr = bself + 6 * nt;
    finalize_b_kernel<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(nt, S, bpart, bself, d.near_ptr, corr, b);
    AFS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Nystrom discretisation of six-node elements (paper Section 2.1): the near
// pairs (target point, element) and the self elements.  Both sum a kernel
// times the six Lagrange basis functions over many quadrature points; one
// wavefront per pair (or per target point), lanes over points, and the
// 6 x 36 weighted sums formed through LDS in chunks of 64 points (point data
// staged once, then each lane forms 3-4 of the 216 sums), so no lane carries
// 216 accumulators.
// ---------------------------------------------------------------------------
// rule table in device memory (48 doubles): [0, 12) rule points (xi, eta);
// [12, 48) the Lagrange basis, L_b = sum_k tab[12 + 6 b + k] m_k,
// m = 1, xi, eta, xi^2, xi eta, eta^2

struct QGeo {
    double y[3], n[3], J, tx[3], te[3];
};

// quadratic element map: point, unit normal, Jacobian, tangents
__device__ __forceinline__ void q6_geo(const double *P, double xi, double eta, QGeo &g) {
    const double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
    const double N[6] = {l0 * (2.0 * l0 - 1.0), l1 * (2.0 * l1 - 1.0), l2 * (2.0 * l2 - 1.0),
                         4.0 * l0 * l1,         4.0 * l1 * l2,         4.0 * l2 * l0};
    const double Nx[6] = {-(4.0 * l0 - 1.0), 4.0 * l1 - 1.0, 0.0, 4.0 * (l0 - l1), 4.0 * l2, -4.0 * l2};
    const double Ne[6] = {-(4.0 * l0 - 1.0), 0.0, 4.0 * l2 - 1.0, -4.0 * l1, 4.0 * l1, 4.0 * (l0 - l2)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double y = 0.0, tx = 0.0, te = 0.0;
#pragma unroll
        for (int a = 0; a < 6; ++a) {
            y += N[a] * P[3 * a + k];
            tx += Nx[a] * P[3 * a + k];
            te += Ne[a] * P[3 * a + k];
        }
        g.y[k] = y;
        g.tx[k] = tx;
        g.te[k] = te;
    }
    const double c0 = g.tx[1] * g.te[2] - g.tx[2] * g.te[1];
    const double c1 = g.tx[2] * g.te[0] - g.tx[0] * g.te[2];
    const double c2 = g.tx[0] * g.te[1] - g.tx[1] * g.te[0];
    g.J = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    g.n[0] = c0 / g.J;
    g.n[1] = c1 / g.J;
    g.n[2] = c2 / g.J;
}

__device__ __forceinline__ void lag6(const double *__restrict__ tab, double xi, double eta, double L[6]) {
    const double m[6] = {1.0, xi, eta, xi * xi, xi * eta, eta * eta};
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            v += tab[12 + 6 * b + k] * m[k];
        L[b] = v;
    }
}

constexpr int kNysOut = 216;    // 6 basis functions x (U, T) x 9 complex
constexpr int kNysKStride = 19; // LDS row of one point's 18 weighted values of U or T (+1 against bank conflicts)

// U and T are staged and contracted one after the other (half the LDS of
// staging both: more work-groups resident per CU)
struct NysLds {
    double K[64 * kNysKStride];
    double L[64 * 6];
    double out[kNysOut];
    double bv[6 * 6];
};

// the lane's sums: acc[0..1] for U (outputs o = lane + 64 r < 108, b = o / 18,
// c = o % 18), acc[2..3] for T; out[36 b + c] (U) and out[36 b + 18 + c] (T)
__device__ __forceinline__ void nys_contract_half(const NysLds &sh, int lane, int n_live, double acc[2]) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int o = lane + 64 * r;
        if (o < 108) {
            const int b = o / 18, c = o % 18;
            double v = acc[r];
#pragma unroll 4
            for (int p = 0; p < n_live; ++p)
                v += sh.L[p * 6 + b] * sh.K[p * kNysKStride + c];
            acc[r] = v;
        }
    }
}

// stage one point (or zeros), contract U, then T; n_live: points staged in
// this chunk (wave-uniform, <= 64).  Every lane of the work-group calls it.
__device__ __forceinline__ void nys_stage_contract(NysLds &sh, int lane, bool live, const PairEval &E,
                                                   const KernelParams &kp, const double n[3], double w,
                                                   const double L[6], int n_live, double acc[4]) {
    cd U[9], T[9];
#pragma unroll
    for (int e = 0; e < 9; ++e)
        U[e] = T[e] = cd{0, 0};
    if (live) {
        acc_U(E, kp, w, U);
        acc_T(E, n[0], n[1], n[2], w, T);
    }
    double *k = &sh.K[lane * kNysKStride];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        k[2 * e] = U[e].r;
        k[2 * e + 1] = U[e].i;
    }
#pragma unroll
    for (int b = 0; b < 6; ++b)
        sh.L[lane * 6 + b] = live ? L[b] : 0.0;
    __syncthreads();
    nys_contract_half(sh, lane, n_live, acc);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        k[2 * e] = T[e].r;
        k[2 * e + 1] = T[e].i;
    }
    __syncthreads();
    nys_contract_half(sh, lane, n_live, acc + 2);
    __syncthreads();
}

// the sums into sh.out in the (b, U 9 complex, T 9 complex) layout
__device__ __forceinline__ void nys_store_sums(NysLds &sh, int lane, const double acc[4]) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int o = lane + 64 * r;
            if (o < 108)
                sh.out[36 * (o / 18) + 18 * h + o % 18] = acc[2 * h + r];
        }
}

// near pair p = (target point i, element e): the six corrected column blocks
// of row i (overwriting the rule's blocks written by the far kernel) and b's
// correction (corrected minus the rule's blocks) times the prescribed values
template <int FMT>
__global__ __launch_bounds__(64) void nys_near_kernel(
    int64_t lda, KernelParams kp, Rule7Args rule, const double *__restrict__ ntab, const double *__restrict__ colx,
    const double *__restrict__ coly, const double *__restrict__ colz, const double *__restrict__ src,
    const double *__restrict__ bc, const double *__restrict__ coef, const int32_t *__restrict__ near_row,
    const int32_t *__restrict__ near_col, const int32_t *__restrict__ near_order, const int64_t *__restrict__ leaf_ptr,
    const double *__restrict__ leaves, const double *__restrict__ geom, void *A, void *A_lo, double *__restrict__ corr) {
    __shared__ NysLds sh;
    const int lane = threadIdx.x;
    const int64_t p = near_order[blockIdx.x];
    const int64_t i = near_row[p], e = near_col[p];
    const double xx = colx[i], xy = coly[i], xz = colz[i];
    double P[18];
#pragma unroll
    for (int k = 0; k < 18; ++k)
        P[k] = geom[18 * e + k];
    const int64_t l0 = leaf_ptr[p];
    const int64_t items = 7 * (leaf_ptr[p + 1] - l0);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c0 = 0; c0 < items; c0 += 64) {
        const int64_t it = c0 + lane;
        const bool live = it < items;
        PairEval E;
        QGeo g;
        double L[6], w = 0.0;
        if (live) {
            const double *q = leaves + 6 * (l0 + it / 7);
            const int r = (int)(it % 7);
            const double b1 = rule.b1[r], b2 = rule.b2[r], b0 = 1.0 - b1 - b2;
            const double xi = b0 * q[0] + b1 * q[2] + b2 * q[4];
            const double eta = b0 * q[1] + b1 * q[3] + b2 * q[5];
            const double area = 0.5 * fabs((q[2] - q[0]) * (q[5] - q[1]) - (q[4] - q[0]) * (q[3] - q[1]));
            q6_geo(P, xi, eta, g);
            lag6(ntab, xi, eta, L);
            eval_pair(kp, coef, xx, xy, xz, g.y[0], g.y[1], g.y[2], g.n[0], g.n[1], g.n[2], E);
            w = rule.w[r] * area * g.J;
        }
        nys_stage_contract(sh, lane, live, E, kp, g.n, w, L, (int)(items - c0 < 64 ? items - c0 : 64), acc);
    }
    nys_store_sums(sh, lane, acc);
    __syncthreads();
    if (lane < 6) {
        const int64_t j = 6 * e + lane;
        const double *rec = src + kSrcStride * j;
        const int kind = (int)rec[31];
        // the block of column j: H (u unknown) or -G (t unknown)
        const double *mat = &sh.out[36 * lane + (kind == 0 ? 18 : 0)];
        const double sg = kind == 0 ? 1.0 : -1.0;
        cd blk[9];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            blk[k] = cd{sg * mat[2 * k], sg * mat[2 * k + 1]};
        store_block<FMT>(A, A_lo, lda, i, j, blk);
        // b correction: (corrected - rule) block of the prescribed side times v
        const double *known = &sh.out[36 * lane + (kind == 0 ? 0 : 18)];
        const double *bv = bc + 6 * j;
        const cd v[3] = {cd{bv[0], bv[1]}, cd{bv[2], bv[3]}, cd{bv[4], bv[5]}};
        cd far[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
        PairEval E;
        eval_pair(kp, coef, xx, xy, xz, rec[0], rec[1], rec[2], rec[28], rec[29], rec[30], E);
        if (kind == 0)
            acc_Uv(E, kp, rec[3], v, far);
        else
            acc_Tv(E, rec[28], rec[29], rec[30], rec[3], v, far);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cd d = cscale(far[a], -1.0);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                d = cadd(d, cmul(cd{known[2 * (3 * a + c)], known[2 * (3 * a + c) + 1]}, v[c]));
            sh.bv[6 * lane + 2 * a] = sg * d.r;
            sh.bv[6 * lane + 2 * a + 1] = sg * d.i;
        }
    }
    __syncthreads();
    if (lane < 6) {
        double v = 0.0;
        for (int q = 0; q < 6; ++q)
            v += sh.bv[6 * q + lane];
        corr[6 * p + lane] = v;
    }
}

// self element of target point i (rule point b0 of element e): polar rule in
// the parameter plane about the point.  For the node's own basis function the
// leading rho^-1 term of T, J0 T0(A(theta)) / rho with A = x_xi cos + x_eta sin
// and T0(r) = beta^2/(4 pi |r|^2)(rh_i n0_j - rh_j n0_i), is subtracted point by
// point and restored as its principal value over a circular exclusion,
// int J0 T0(A) ln(R |A|) dtheta; both are antisymmetric, carried as the
// vector of (rh x n0).  Then 1/2 I, the six blocks of row i, b's self part and
// the inverse of the diagonal block (block-Jacobi).
template <int FMT>
__global__ __launch_bounds__(64) void nys_self_kernel(
    int64_t lda, KernelParams kp, const double *__restrict__ ntab, const double *__restrict__ colx, const double *__restrict__ coly,
    const double *__restrict__ colz, const double *__restrict__ src, const double *__restrict__ bc,
    const double *__restrict__ coef, const double *__restrict__ geom, const double *__restrict__ table,
    const double *__restrict__ gl_rho, int n_theta, int n_rho, void *A, void *A_lo, double *__restrict__ bself,
    double *__restrict__ precond) {
    __shared__ NysLds sh;
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int64_t e = i / 6;
    const int b0 = (int)(i % 6);
    const double xx = colx[i], xy = coly[i], xz = colz[i];
    double P[18];
#pragma unroll
    for (int k = 0; k < 18; ++k)
        P[k] = geom[18 * e + k];
    const double xi0 = ntab[2 * b0], eta0 = ntab[2 * b0 + 1];
    QGeo g0;
    q6_geo(P, xi0, eta0, g0);
    const double cT0 = g0.J * kp.beta * kp.beta * kInv4Pi;
    const double *tab = table + (size_t)b0 * 6 * n_theta * 4;
    const int64_t items = (int64_t)6 * n_theta * n_rho;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double sv[3] = {0.0, 0.0, 0.0};
    for (int64_t c0 = 0; c0 < items; c0 += 64) {
        const int64_t it = c0 + lane;
        const bool live = it < items;
        PairEval E;
        QGeo g;
        double L[6], w = 0.0;
        if (live) {
            const double *t = tab + 4 * (it / n_rho);
            const int r = (int)(it % n_rho);
            const double cs = t[0], sn = t[1], wth = t[2], R = t[3];
            const double rho = R * gl_rho[2 * r], wr = R * gl_rho[2 * r + 1];
            const double xi = xi0 + rho * cs, eta = eta0 + rho * sn;
            q6_geo(P, xi, eta, g);
            lag6(ntab, xi, eta, L);
            eval_pair(kp, coef, xx, xy, xz, g.y[0], g.y[1], g.y[2], g.n[0], g.n[1], g.n[2], E);
            w = wth * wr * rho * g.J;
            // leading term: c(theta) (rh x n0), rh = A / |A|, c = J0 beta^2 / (4 pi |A|^2)
            double Av[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                Av[k] = g0.tx[k] * cs + g0.te[k] * sn;
            const double A2 = Av[0] * Av[0] + Av[1] * Av[1] + Av[2] * Av[2];
            const double Al = sqrt(A2);
            const double cx[3] = {(Av[1] * g0.n[2] - Av[2] * g0.n[1]) / Al, (Av[2] * g0.n[0] - Av[0] * g0.n[2]) / Al,
                                  (Av[0] * g0.n[1] - Av[1] * g0.n[0]) / Al};
            double f = -wth * wr / rho * (cT0 / A2);
            if (r == 0)
                f += wth * (cT0 / A2) * log(R * Al);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                sv[k] += f * cx[k];
        }
        nys_stage_contract(sh, lane, live, E, kp, g.n, w, L, (int)(items - c0 < 64 ? items - c0 : 64), acc);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        sv[k] = wave_sum(sv[k]);
    nys_store_sums(sh, lane, acc);
    __syncthreads();
    if (lane == 0) {
        // H_b0 += (antisymmetric matrix of sv) + 1/2 I  (real parts)
        double *H = &sh.out[36 * b0 + 18];
        H[2 * 1] += sv[2];
        H[2 * 3] -= sv[2];
        H[2 * 5] += sv[0];
        H[2 * 7] -= sv[0];
        H[2 * 6] += sv[1];
        H[2 * 2] -= sv[1];
        H[0] += 0.5;
        H[2 * 4] += 0.5;
        H[2 * 8] += 0.5;
    }
    __syncthreads();
    if (lane < 6) {
        const int64_t j = 6 * e + lane;
        const int kind = (int)src[kSrcStride * j + 31];
        const double *mat = &sh.out[36 * lane + (kind == 0 ? 18 : 0)];
        const double sg = kind == 0 ? 1.0 : -1.0;
        cd blk[9];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            blk[k] = cd{sg * mat[2 * k], sg * mat[2 * k + 1]};
        store_block<FMT>(A, A_lo, lda, i, j, blk);
        const double *known = &sh.out[36 * lane + (kind == 0 ? 0 : 18)];
        const double *bv = bc + 6 * j;
        const cd v[3] = {cd{bv[0], bv[1]}, cd{bv[2], bv[3]}, cd{bv[4], bv[5]}};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cd d = cd{0, 0};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                d = cadd(d, cmul(cd{known[2 * (3 * a + c)], known[2 * (3 * a + c) + 1]}, v[c]));
            sh.bv[6 * lane + 2 * a] = sg * d.r;
            sh.bv[6 * lane + 2 * a + 1] = sg * d.i;
        }
        if (lane == b0 && precond) {
            cd inv[9];
            inv3(blk, inv);
            for (int k = 0; k < 9; ++k) {
                precond[18 * i + 2 * k] = inv[k].r;
                precond[18 * i + 2 * k + 1] = inv[k].i;
            }
        }
    }
    __syncthreads();
    if (lane < 6) {
        double v = 0.0;
        for (int q = 0; q < 6; ++q)
            v += sh.bv[6 * q + lane];
        bself[6 * i + lane] = v;
    }
}

void launch_nystrom_near_self(const Problem &p, const KernelParams &kp, const double *bc_val, int format, void *A,
                              void *A_lo, double *bself, double *corr, double *precond, hipStream_t st) {
    const DevicePlan &d = p.dev;
    const int64_t lda = (3 * d.n_tri + 63) / 64 * 64;
    const double *na = d.nys_tab;
    const Rule7Args rule = rule7_args();
    AFS_REQUIRE(d.nnz < (int64_t)1 << 31 && d.n_tri < (int64_t)1 << 31, AFSBEM_EINVAL, "Nystrom plan too large");
    if (format == AFSBEM_FMT_C128) {
        if (d.nnz)
            nys_near_kernel<AFSBEM_FMT_C128><<<(unsigned)d.nnz, 64, 0, st>>>(
                lda, kp, rule, na, d.colx, d.coly, d.colz, d.src, bc_val, d.coef, d.near_row, d.near_col,
                d.near_order, d.leaf_ptr, d.nys_leaves, d.nys_geom, A, A_lo, corr);
        nys_self_kernel<AFSBEM_FMT_C128><<<(unsigned)d.n_tri, 64, 0, st>>>(
            lda, kp, na, d.colx, d.coly, d.colz, d.src, bc_val, d.coef, d.nys_geom, d.nys_self, d.gl_rho, d.n_theta,
            d.n_rho, A, A_lo, bself, precond);
    } else {
        if (d.nnz)
            nys_near_kernel<AFSBEM_FMT_SPLIT><<<(unsigned)d.nnz, 64, 0, st>>>(
                lda, kp, rule, na, d.colx, d.coly, d.colz, d.src, bc_val, d.coef, d.near_row, d.near_col,
                d.near_order, d.leaf_ptr, d.nys_leaves, d.nys_geom, A, A_lo, corr);
        nys_self_kernel<AFSBEM_FMT_SPLIT><<<(unsigned)d.n_tri, 64, 0, st>>>(
            lda, kp, na, d.colx, d.coly, d.colz, d.src, bc_val, d.coef, d.nys_geom, d.nys_self, d.gl_rho, d.n_theta,
            d.n_rho, A, A_lo, bself, precond);
    }
    AFS_HIP(hipGetLastError());
}

}  // namespace afsbem
