// Per-frequency solve: assembly, right block-Jacobi-preconditioned GMRES(m)
// (paper Section 2.1 and Section 4: GMRES with the block diagonal
// preconditioner), and FP32-operator / FP64-residual iterative refinement.
//
// The Krylov basis, the Hessenberg columns and every residual are FP64; only
// the operator application of the inner solve of the mixed path streams the
// FP32 hi plane.  Orthogonalisation is classical Gram-Schmidt applied twice.
// The small (m+1) x m least-squares problem is reduced on the host with
// Givens rotations: one device-to-host copy of the new Hessenberg column per
// iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>

#include "internal.hpp"
#include "solver.hpp"
#include "mlp.hpp"

namespace afsbem {

using cplx = std::complex<double>;

static void *dalloc(size_t bytes) {
    void *p = nullptr;
    if (bytes == 0)
        bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        throw Error{AFSBEM_ENOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e)};
    return p;
}

Workspace::~Workspace() { release(); }

void Workspace::hm_release() {
    for (void *p : {(void *)hm_dense, (void *)hm_pool, (void *)hm_ctr, (void *)hm_offs, (void *)hm_t,
                    (void *)hm_xp, (void *)hm_yp, (void *)hm_rank, (void *)hm_status, (void *)hm_items})
        if (p)
            (void)hipFree(p);
    if (hm_host)
        (void)hipHostFree(hm_host);
    if (hm_items_host)
        (void)hipHostFree(hm_items_host);
    hm_items = hm_items_host = nullptr;
    hm_n_items = 0;
    if (hm_used_host)
        (void)hipHostFree(hm_used_host);
    hm_host = nullptr;
    hm_used_host = nullptr;
    hm_dense = hm_pool = nullptr;
    hm_ctr = nullptr;
    hm_offs = nullptr;
    hm_pool_cap = 0;
    hm_t = hm_xp = hm_yp = nullptr;
    hm_rank = hm_status = nullptr;
    hm_cap[0] = hm_cap[1] = hm_cap[2] = 0;
    hm_ok = false;
}

void Workspace::hm_alloc(const Problem &p, const HmatPlan &H) {
    const size_t nd = (size_t)H.dense_off.back(), nl = H.lowrank.size() / 4;
    // pool: 1.25 x the largest build of this problem so far (48 terms per
    // block before the first), or what a build that ran out asked for, within
    // half the free memory; a build that runs out is repeated with a larger
    // pool (hmat_finish reports it), and one that still cannot fit leaves its
    // frequency on the on-the-fly operator
    const size_t first = p.hm_need > 0.0 ? 0 : (size_t)H.lr_rows * 48;
    const size_t want = std::max({first, (size_t)(1.25 * p.hm_need), hm_want});
    // hm_cap[1] records the size asked for (the pool itself may have been capped):
    // the same request reuses the buffers instead of reallocating them per frequency
    if (hm_dense && hm_cap[0] >= nd && hm_cap[1] >= want && hm_cap[2] >= nl)
        return;
    hm_release();
    size_t free_b = 0, total_b = 0;
    AFS_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t nf =
        std::min(want, (size_t)(0.5 * (double)(free_b > (size_t)nd * 8 ? free_b - (size_t)nd * 8 : 0)) / 8);
    hm_dense = (float2 *)dalloc(std::max<size_t>(nd, 1) * 8);
    hm_pool = (float2 *)dalloc(std::max<size_t>(nf, 1) * 8);
    hm_pool_cap = nf;
    hm_ctr = (unsigned long long *)dalloc(sizeof(unsigned long long));
    hm_offs = (int64_t *)dalloc(std::max<size_t>(nl, 1) * hm_slots(H.kmax) * sizeof(int64_t));
    hm_rank = (int *)dalloc(std::max<size_t>(nl, 1) * 4);
    hm_status = (int *)dalloc(std::max<size_t>(nl, 1) * 4);
    hm_t = (double2 *)dalloc(std::max<size_t>(nl, 1) * H.kmax * 16);
    hm_xp = (double2 *)dalloc((size_t)std::max<int64_t>(H.n, 1) * 3 * 16);
    hm_yp = (double2 *)dalloc((size_t)std::max<int64_t>(H.n, 1) * 3 * 16 * kHmatApplyParts);
    hm_items = (int32_t *)dalloc(std::max<size_t>(nl, 1) * hm_slots(H.kmax) * sizeof(int32_t));
    AFS_HIP(hipHostMalloc((void **)&hm_host, std::max<size_t>(nl, 1) * 2 * sizeof(int), hipHostMallocDefault));
    AFS_HIP(hipHostMalloc((void **)&hm_items_host, std::max<size_t>(nl, 1) * hm_slots(H.kmax) * sizeof(int32_t),
                          hipHostMallocDefault));
    AFS_HIP(hipHostMalloc((void **)&hm_used_host, sizeof(unsigned long long), hipHostMallocDefault));
    hm_cap[0] = nd;
    hm_cap[1] = want;
    hm_cap[2] = nl;
}

void Workspace::release() {
    hm_release();
    for (void *p : {(void *)A, (void *)A_lo, (void *)nearblk, (void *)selfblk, (void *)b, (void *)precond, (void *)asm_scratch, (void *)gemv_partial,
                    (void *)V, (void *)w, (void *)z, (void *)x, (void *)r, (void *)tmp, (void *)rin, (void *)xo,
                    (void *)xstart, (void *)aug,
                    (void *)dots_partial, (void *)small, (void *)one, (void *)clinv, (void *)clgath})
        if (p)
            (void)hipFree(p);
    if (host_small)
        (void)hipHostFree(host_small);
    for (hipEvent_t e : ev)
        (void)hipEventDestroy(e);
    ev.clear();
    for (auto &e : ev_far)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    far_timed = false;
    ev_prec.clear();
    ev_used = 0;
    // reset every field in place (no temporary Workspace: its destructor would
    // call release() again)
    N = 0;
    format = -1;
    m = 0;
    A = A_lo = asm_scratch = nullptr;
    nearblk = selfblk = nullptr;
    b = precond = gemv_partial = V = w = z = x = r = tmp = rin = xo = xstart = aug = nullptr;
    dots_partial = small = one = host_small = nullptr;
    clinv = clgath = nullptr;
    prec_kind = 0;
    plan = nullptr;
}

void Workspace::apply_precond(const double *v, double *z, hipStream_t st) const {
    if (prec_kind == 1)
        cluster_apply(*plan, clinv, v, z, st);
    else
        vec_precond(plan->n_tri, precond, v, z, st);
}

void Workspace::ensure(const Problem &p, int format, int restart_m, int prec) {
    const int64_t nt = p.dev.n_tri, N = 3 * nt;
    const int64_t lda = (N + 63) / 64 * 64;
    plan = &p.dev;
    const size_t clbytes = (size_t)std::max<int64_t>(p.dev.n_clusters, 1) * kClusterDim * kClusterDim * 8;
    if (N == this->N && format == this->format && restart_m <= this->m && b) {
        if (prec == 1 && !clinv)
            clinv = (float *)dalloc(clbytes);
        if (prec == 1 && format == kFmtBlocks && !clgath)
            clgath = (float *)dalloc(clbytes);
        prec_kind = prec;
        return;
    }
    release();
    plan = &p.dev;
    prec_kind = prec;
    if (prec == 1)
        clinv = (float *)dalloc(clbytes);
    if (prec == 1 && format == kFmtBlocks)
        clgath = (float *)dalloc(clbytes);
    this->N = N;
    this->format = format;
    this->m = restart_m;
    if (format == kFmtBlocks) {
        nearblk = (double *)dalloc((size_t)std::max<int64_t>(p.dev.nnz, 1) * 144);
        selfblk = (double *)dalloc((size_t)nt * 144);
    } else {
        const size_t plane = (size_t)N * lda * (format == AFSBEM_FMT_C128 ? 16 : 8);
        A = dalloc(plane);
        if (format == AFSBEM_FMT_SPLIT)
            A_lo = dalloc(plane);
    }
    b = (double *)dalloc((size_t)N * 16);
    precond = (double *)dalloc((size_t)nt * 9 * 16);
    asm_scratch = dalloc(assembly_scratch_bytes(p));
    gemv_partial = (double *)dalloc((size_t)(format == kFmtBlocks ? mf_chunks(nt) : gemv_chunks(N)) * N * 16);
    V = (double *)dalloc((size_t)(restart_m + 2) * N * 16);  // [c,] v_0..v_m
    w = (double *)dalloc((size_t)N * 16);
    z = (double *)dalloc((size_t)N * 16);
    x = (double *)dalloc((size_t)N * 16);
    r = (double *)dalloc((size_t)N * 16);
    tmp = (double *)dalloc((size_t)N * 16);
    rin = (double *)dalloc((size_t)N * 16);
    xo = (double *)dalloc((size_t)N * 16);
    xstart = (double *)dalloc((size_t)N * 16);
    aug = (double *)dalloc((size_t)N * 16);
    dots_partial = (double *)dalloc(mdot_scratch_bytes(N, restart_m + 2));
    small = (double *)dalloc((size_t)(4 * (restart_m + 2)) * 16);
    AFS_HIP(hipHostMalloc((void **)&host_small, (size_t)(4 * (restart_m + 2)) * 16, hipHostMallocDefault));
    one = (double *)dalloc(16);
    const double unit[2] = {1.0, 0.0};
    AFS_HIP(hipMemcpy(one, unit, 16, hipMemcpyHostToDevice));
}

// --------------------------------------------------------------- operator --
void Operator::apply(const double *xin, double *yout, hipStream_t st) const {
    hipEvent_t eb = nullptr, ee = nullptr;
    if (prof) {
        Workspace &w = *prof;
        const int slot = w.ev_used;
        if (slot < 4096) {
            while ((int)w.ev.size() < 2 * (slot + 1)) {
                hipEvent_t e;
                AFS_HIP(hipEventCreate(&e));
                w.ev.push_back(e);
            }
            eb = w.ev[2 * slot];
            ee = w.ev[2 * slot + 1];
            w.ev_prec.push_back(format == AFSBEM_FMT_C128 ? 2 : precision);
            ++w.ev_used;
        }
    }
    if (format == kFmtBlocks) {
        if (eb)
            AFS_HIP(hipEventRecord(eb, st));
        const bool hier = precision == 1 && hm && hm->hm_ok;
        if (hier)
            hmat_apply(*prob, *hm, xin, yout, st);
        else
            mf_apply(*prob, kp, precision, 0, nearblk, selfblk, xin, yout, partial, st);
        if (ee)
            AFS_HIP(hipEventRecord(ee, st));
        ++*counter;
        // stored bytes read: the hierarchical form, or the near and self blocks
        *bytes += hier ? hm->hm_bytes : (double)(prob->dev.nnz + prob->dev.n_tri) * 144.0;
        return;
    }
    launch_gemv(N, format, precision, A, A_lo, xin, yout, partial, st, eb, ee);
    ++*counter;
    *bytes += (double)N * N * ((format == AFSBEM_FMT_C128 || precision == 0) ? 16.0 : 8.0);
}

static double norm2_dev(Workspace &ws, int64_t N, const double *v, hipStream_t st) {
    vec_mdot(N, 1, v, N, v, ws.dots_partial, ws.small, st);
    AFS_HIP(hipMemcpyAsync(ws.host_small, ws.small, 16, hipMemcpyDeviceToHost, st));
    AFS_HIP(hipStreamSynchronize(st));
    return std::sqrt(std::max(ws.host_small[0], 0.0));
}

// r = b - op(x)
static void residual(const Operator &op, Workspace &ws, const double *b, const double *x, double *r, hipStream_t st) {
    op.apply(x, ws.tmp, st);
    vec_sub(op.N, b, ws.tmp, r, st);
}

// Givens rotation (c real, s) with c a + s b = r, -conj(s) a + c b = 0,
// applied to the pair (a, b) in place
static void givens_make(cplx &a, cplx &b, cplx &c, cplx &s) {
    const double den = std::sqrt(std::norm(a) + std::norm(b));
    if (std::abs(a) == 0.0) {
        c = 0.0;
        s = 1.0;
    } else {
        c = std::abs(a) / den;
        s = (a / std::abs(a)) * std::conj(b) / den;
    }
    a = c * a + s * b;
    b = 0.0;
}
static void givens_apply(cplx c, cplx s, cplx &a, cplx &b) {
    const cplx a0 = a;
    a = c * a0 + s * b;
    b = -std::conj(s) * a0 + std::conj(c) * b;
}

GmresResult gmres(const Operator &op, Workspace &ws, int64_t /*n_tri*/, const double *rhs, double rhs_norm,
                  double *x, bool x_is_zero, double tol_abs, int restart, int max_iter, hipStream_t st,
                  bool verify, const double *r0, double r0_norm, const double *aug, int recycle,
                  const std::function<void(double)> &progress) {
    const int64_t N = op.N;
    GmresResult res;
    // Hessenberg columns packed one after another (column j holds rows 0..j+1),
    // grown as the cycle proceeds: long restarts pay only for the columns used
    std::vector<cplx> Hm, Bc, g(restart + 1), cs(restart), sn(restart);
    auto hix = [](int i, int j) { return (size_t)j * (size_t)(j + 3) / 2 + (size_t)i; };
    // basis slot 0 holds c = A aug / |A aug| in an augmented cycle; the Krylov
    // vectors v_0, v_1, ... follow it, so that one multi-dot covers [c, V]
    double *const Cv = ws.V;
    double *const Vk = ws.V + 2 * N;
    double *hbuf = ws.small;            // device: first-pass dots, then y
    double *h2 = ws.small + 2 * (restart + 2);  // second-pass dots, then ||w||^2
    double *host = ws.host_small;
    // initial residual
    double beta;
    if (x_is_zero) {
        AFS_HIP(hipMemcpyAsync(ws.r, rhs, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
        beta = rhs_norm;
    } else if (r0) {
        if (r0 != ws.r)
            AFS_HIP(hipMemcpyAsync(ws.r, r0, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
        beta = r0_norm;
    } else {
        residual(op, ws, rhs, x, ws.r, st);
        beta = norm2_dev(ws, N, ws.r, st);
    }
    res.est = beta;
    const bool use_kept = recycle == 2 && ws.rc_valid && !aug && x_is_zero && ws.rc_k >= 1 &&
                          ws.rc_k + 2 <= restart;
    if (!use_kept)
        ws.rc_valid = false;  // the cycles below overwrite the basis
    if (use_kept && beta > tol_abs && res.iters < max_iter) {
        // Recycled first cycle (GCRO with the kept subspace).  The kept cycle
        // gives A M^-1 V_K = W H_K with W = V_{K+1} (Krylov slots 0..K) and
        // rotations Q with Q H_K = [R_K; 0], so C = W Q^H[:, 0..K-1] is an
        // orthonormal basis of the image A U of U = M^-1 V_K R_K^-1.  The
        // residual's part in C is removed at once (coefficients c = C^H r);
        // the new Arnoldi vectors (slots K+1, ...) start from the rest and are
        // kept orthogonal to C (not to the last direction of W), the
        // projections B = C^H A M^-1 V_new recorded; the cycle then minimises
        // over the new vectors and the update is M^-1 (V_K R_K^-1 (c - B y)
        // + V_new y).  Projections onto C are formed through W: the W
        // coordinates rotated by Q, their last entry dropped, rotated back.
        const int K = ws.rc_k, nw = K + 1;
        double *const Vn = Vk + 2 * (int64_t)nw * N;
        std::vector<cplx> coef;
        // one classical Gram-Schmidt pass of v against C and the first nn new
        // vectors; adds the C coordinates to bacc and the new ones to hacc
        auto pass = [&](double *v, int nn, cplx *bacc, cplx *hacc) {
            const int nv = nw + nn;
            vec_mdot(N, nv, Vk, N, v, ws.dots_partial, hbuf, st);
            AFS_HIP(hipMemcpyAsync(host, hbuf, (size_t)nv * 16, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipStreamSynchronize(st));
            coef.assign(nv, cplx(0));
            for (int i = 0; i < nv; ++i)
                coef[i] = cplx(host[2 * i], host[2 * i + 1]);
            for (int i = 0; i < K; ++i)
                givens_apply(ws.rc_cs[i], ws.rc_sn[i], coef[i], coef[i + 1]);
            coef[K] = 0.0;  // the direction of W outside C stays
            for (int i = 0; i < K; ++i)
                bacc[i] += coef[i];
            for (int i = K - 1; i >= 0; --i) {  // back to W coordinates: Q^H
                const cplx a = coef[i], b = coef[i + 1], c = ws.rc_cs[i], s = ws.rc_sn[i];
                coef[i] = std::conj(c) * a - s * b;
                coef[i + 1] = std::conj(s) * a + c * b;
            }
            for (int i = 0; i < nn; ++i)
                hacc[i] += coef[nw + i];
            for (int i = 0; i < nv; ++i) {
                host[2 * i] = coef[i].real();
                host[2 * i + 1] = coef[i].imag();
            }
            AFS_HIP(hipMemcpyAsync(hbuf, host, (size_t)nv * 16, hipMemcpyHostToDevice, st));
            vec_mupdate(N, nv, Vk, N, hbuf, v, st);
        };
        auto sqnorm = [&](const double *v) {
            vec_mdot(N, 1, v, N, v, ws.dots_partial, h2, st);
            AFS_HIP(hipMemcpyAsync(host, h2, 16, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipStreamSynchronize(st));
            return std::max(host[0], 0.0);
        };
        std::vector<cplx> cc(K, cplx(0));
        pass(ws.r, 0, cc.data(), nullptr);
        pass(ws.r, 0, cc.data(), nullptr);
        const double bp2 = sqnorm(ws.r);
        const double bp = std::sqrt(bp2);
        const int mmax = std::min(restart - nw, max_iter - res.iters);
        std::vector<cplx> Bn, gq(mmax + 1, cplx(0)), c2(mmax), s2(mmax);
        gq[0] = bp;
        double est = bp;
        int kn = 0;
        if (bp > 0.0 && std::isfinite(bp) && est > 0.5 * tol_abs) {
            vec_normalize(N, h2, ws.r, Vn, st);  // h2[0] = ||r||^2 on the device
            std::vector<cplx> bcol(K), hcol;
            for (int j = 0; j < mmax; ++j) {
                ws.apply_precond(Vn + 2 * (int64_t)j * N, ws.z, st);
                op.apply(ws.z, ws.w, st);
                std::fill(bcol.begin(), bcol.end(), cplx(0));
                hcol.assign(j + 2, cplx(0));
                pass(ws.w, j + 1, bcol.data(), hcol.data());
                pass(ws.w, j + 1, bcol.data(), hcol.data());
                const double hn2 = sqnorm(ws.w);
                const double hn = std::sqrt(hn2);
                ++res.iters;
                if (!std::isfinite(hn)) {
                    res.nan = true;
                    return res;
                }
                if (hn > 0.0)
                    vec_normalize(N, h2, ws.w, Vn + 2 * (int64_t)(j + 1) * N, st);
                Bn.insert(Bn.end(), bcol.begin(), bcol.end());
                hcol[j + 1] = hn;
                if (Hm.size() < hix(0, j + 1))
                    Hm.resize(hix(0, j + 1));
                for (int i = 0; i < j; ++i)
                    givens_apply(c2[i], s2[i], hcol[i], hcol[i + 1]);
                givens_make(hcol[j], hcol[j + 1], c2[j], s2[j]);
                for (int i = 0; i <= j; ++i)
                    Hm[hix(i, j)] = hcol[i];
                givens_apply(c2[j], s2[j], gq[j], gq[j + 1]);
                kn = j + 1;
                est = std::abs(gq[j + 1]);
                if (est <= 0.5 * tol_abs || res.iters >= max_iter || hn == 0.0)
                    break;
            }
        }
        // y for the new vectors, then the kept ones: z = R_K^-1 (c - B y)
        std::vector<cplx> yn(kn), z(K);
        for (int i = kn - 1; i >= 0; --i) {
            cplx s = gq[i];
            for (int l = i + 1; l < kn; ++l)
                s -= Hm[hix(i, l)] * yn[l];
            yn[i] = s / Hm[hix(i, i)];
        }
        for (int i = K - 1; i >= 0; --i) {
            cplx s = cc[i];
            for (int l = 0; l < kn; ++l)
                s -= Bn[(size_t)l * K + i] * yn[l];
            for (int l = i + 1; l < K; ++l)
                s -= ws.rc_R[hix(i, l)] * z[l];
            z[i] = s / ws.rc_R[hix(i, i)];
        }
        // coefficients over Krylov slots 0..K+kn (slot K, outside the kept domain: 0)
        const int nc = nw + kn;
        for (int i = 0; i < nc; ++i) {
            const cplx v = i < K ? z[i] : (i == K ? cplx(0) : yn[i - nw]);
            host[2 * i] = v.real();
            host[2 * i + 1] = v.imag();
        }
        AFS_HIP(hipMemcpyAsync(hbuf, host, (size_t)nc * 16, hipMemcpyHostToDevice, st));
        AFS_HIP(hipMemsetAsync(ws.tmp, 0, (size_t)N * 16, st));
        vec_combine(N, nc, Vk, N, hbuf, ws.tmp, st);
        ws.apply_precond(ws.tmp, x, st);  // x was zero: x = M^-1 (...)
        x_is_zero = false;
        ++res.cycles;
        res.est = est;
        if (!verify && est <= 0.5 * tol_abs) {
            res.converged = true;  // the kept subspace stays valid for a further step
            return res;
        }
        ws.rc_valid = false;
        residual(op, ws, rhs, x, ws.r, st);
        beta = norm2_dev(ws, N, ws.r, st);
        res.est = beta;
    }
    // Augmentation (first cycle): u = aug / gamma with c = A u of unit norm;
    // the start takes the residual-optimal multiple of u (x += u c^H r,
    // r -= c c^H r), and the cycle's Arnoldi vectors are kept orthogonal to
    // c, the projections b_j = c^H A M^-1 v_j recorded, so that the cycle
    // minimises the residual over x + span{u} + M^-1 K (projected operator);
    // the update then subtracts u B y.
    bool augc = false;
    double gamma = 0.0;
    if (aug && beta > tol_abs && res.iters < max_iter) {
        op.apply(aug, ws.w, st);
        ++res.iters;
        vec_mdot(N, 1, ws.w, N, ws.w, ws.dots_partial, ws.small, st);
        vec_mdot(N, 1, ws.w, N, ws.r, ws.dots_partial, ws.small + 2, st);
        AFS_HIP(hipMemcpyAsync(host, ws.small, 32, hipMemcpyDeviceToHost, st));
        AFS_HIP(hipStreamSynchronize(st));
        const double g2 = host[0];
        const cplx wr(host[2], host[3]);
        // the vector joins the search space only when it explains a useful
        // part of the residual (projection lowers it by more than 5 %): a
        // direction unrelated to the solution would only perturb the
        // projected operator's Krylov space
        const double b2_new = beta * beta - std::norm(wr) / g2;
        if (g2 > 0.0 && std::isfinite(g2) && std::isfinite(wr.real()) && std::isfinite(wr.imag()) &&
            b2_new < 0.9025 * beta * beta) {
            gamma = std::sqrt(g2);
            const cplx alpha = wr / g2;  // coefficient of aug
            vec_normalize(N, ws.small, ws.w, Cv, st);  // c (device ||w||^2 at small[0])
            if (x_is_zero) {
                vec_axpby(N, alpha.real(), alpha.imag(), aug, 0.0, 0.0, aug, x, st);
                x_is_zero = false;
            } else {
                vec_axpby(N, 1.0, 0.0, x, alpha.real(), alpha.imag(), aug, x, st);
            }
            vec_axpby(N, 1.0, 0.0, ws.r, -alpha.real(), -alpha.imag(), ws.w, ws.r, st);
            const double b_new = norm2_dev(ws, N, ws.r, st);
            res.aug_gain = b_new > 0.0 ? beta / b_new : 1e30;
            beta = b_new;
            res.est = beta;
            augc = true;
        }
    }
    if (x_is_zero && (!(beta > tol_abs) || res.iters >= max_iter))
        AFS_HIP(hipMemsetAsync(x, 0, (size_t)N * 16, st));  // leave a valid (zero) iterate
    while (true) {
        if (!(beta > tol_abs) || res.iters >= max_iter) {
            res.est = beta;
            res.converged = beta <= tol_abs;
            if (!std::isfinite(beta))
                res.nan = true;
            return res;
        }
        // V_0 = r / beta
        host[0] = beta * beta;
        AFS_HIP(hipMemcpyAsync(ws.small + 4 * (restart + 2) + 2, host, 8, hipMemcpyHostToDevice, st));
        vec_normalize(N, ws.small + 4 * (restart + 2) + 2, ws.r, Vk, st);
        std::fill(g.begin(), g.end(), cplx(0));
        g[0] = beta;
        Bc.clear();
        int k = 0;
        const int e = augc ? 1 : 0;          // leading vectors of the multi-dot besides V
        double *const Vd = augc ? Cv : Vk;   // [c,] v_0, v_1, ...
        for (int j = 0; j < restart; ++j) {
            double *vj = Vk + 2 * (int64_t)j * N;
            ws.apply_precond(vj, ws.z, st);
            op.apply(ws.z, ws.w, st);
            // classical Gram-Schmidt, twice, against [c,] v_0..v_j
            const int nv = j + 1 + e;
            vec_mdot(N, nv, Vd, N, ws.w, ws.dots_partial, hbuf, st);
            vec_mupdate(N, nv, Vd, N, hbuf, ws.w, st);
            vec_mdot(N, nv, Vd, N, ws.w, ws.dots_partial, h2, st);
            vec_mupdate(N, nv, Vd, N, h2, ws.w, st);
            vec_mdot(N, 1, ws.w, N, ws.w, ws.dots_partial, h2 + 2 * nv, st);
            AFS_HIP(hipMemcpyAsync(host, hbuf, (size_t)nv * 16, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipMemcpyAsync(host + 2 * (restart + 2), h2, (size_t)(nv + 1) * 16, hipMemcpyDeviceToHost, st));
            AFS_HIP(hipStreamSynchronize(st));
            const double *hd = host + 2 * (restart + 2);
            const double hn = std::sqrt(std::max(hd[2 * nv], 0.0));
            if (Hm.size() < hix(0, j + 1))
                Hm.resize(hix(0, j + 1));
            if (augc)
                Bc.push_back(cplx(host[0] + hd[0], host[1] + hd[1]));
            for (int i = 0; i <= j; ++i)
                Hm[hix(i, j)] = cplx(host[2 * (i + e)] + hd[2 * (i + e)], host[2 * (i + e) + 1] + hd[2 * (i + e) + 1]);
            Hm[hix(j + 1, j)] = hn;
            ++res.iters;
            if (!std::isfinite(hn)) {
                res.nan = true;
                return res;
            }
            if (hn > 0.0) {
                // V_{j+1} = w / hn  (device scalar ||w||^2 after the dots)
                vec_normalize(N, h2 + 2 * nv, ws.w, Vk + 2 * (int64_t)(j + 1) * N, st);
            }
            for (int i = 0; i < j; ++i) {
                cplx a = Hm[hix(i, j)], c = Hm[hix(i + 1, j)];
                Hm[hix(i, j)] = cs[i] * a + sn[i] * c;
                Hm[hix(i + 1, j)] = -std::conj(sn[i]) * a + std::conj(cs[i]) * c;
            }
            cplx a = Hm[hix(j, j)], c = Hm[hix(j + 1, j)];
            const double den = std::sqrt(std::norm(a) + std::norm(c));
            if (std::abs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = std::abs(a) / den;
                sn[j] = (a / std::abs(a)) * std::conj(c) / den;
            }
            Hm[hix(j, j)] = cs[j] * a + sn[j] * c;
            Hm[hix(j + 1, j)] = 0.0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            res.est = std::abs(g[j + 1]);
            if (progress)
                progress(res.est);
            if (res.est <= 0.5 * tol_abs || res.iters >= max_iter || hn == 0.0)
                break;
        }
        // y = H(1:k,1:k) \ g(1:k)
        std::vector<cplx> y(k);
        for (int i = k - 1; i >= 0; --i) {
            cplx s = g[i];
            for (int l = i + 1; l < k; ++l)
                s -= Hm[hix(i, l)] * y[l];
            y[i] = s / Hm[hix(i, i)];
        }
        for (int i = 0; i < k; ++i) {
            host[2 * i] = y[i].real();
            host[2 * i + 1] = y[i].imag();
        }
        if (recycle == 1) {
            // keep this cycle for later corrections with the same operator
            ws.rc_valid = !augc && k >= 1;
            if (ws.rc_valid) {
                ws.rc_k = k;
                ws.rc_R.assign(Hm.begin(), Hm.begin() + hix(0, k));
                ws.rc_cs.assign(cs.begin(), cs.begin() + k);
                ws.rc_sn.assign(sn.begin(), sn.begin() + k);
            }
        }
        // augmented cycle: the coefficient of aug, -(B y) / gamma, after y
        cplx du(0.0);
        if (augc) {
            for (int i = 0; i < k; ++i)
                du -= Bc[i] * y[i];
            du /= gamma;
            host[2 * k] = du.real();
            host[2 * k + 1] = du.imag();
        }
        AFS_HIP(hipMemcpyAsync(hbuf, host, (size_t)(k + (augc ? 1 : 0)) * 16, hipMemcpyHostToDevice, st));
        AFS_HIP(hipMemsetAsync(ws.tmp, 0, (size_t)N * 16, st));
        // x += M^-1 sum_j y_j v_j  (- u B y in the augmented cycle)
        if (k > 0)
            vec_combine(N, k, Vk, N, hbuf, ws.tmp, st);
        ws.apply_precond(ws.tmp, ws.z, st);
        if (augc)
            vec_combine(N, 1, aug, N, hbuf + 2 * k, ws.z, st);
        if (x_is_zero) {
            AFS_HIP(hipMemcpyAsync(x, ws.z, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
            x_is_zero = false;
        } else {
            vec_combine(N, 1, ws.z, N, ws.one, x, st);  // x += z
        }
        ++res.cycles;
        augc = false;  // later cycles: plain restarts
        if (!verify && res.est <= 0.5 * tol_abs) {
            // an outer loop judges the iterate with its own residual
            res.converged = true;
            return res;
        }
        // true residual of this operator for the restart
        residual(op, ws, rhs, x, ws.r, st);
        beta = norm2_dev(ws, N, ws.r, st);
        res.est = beta;
    }
}

// Residual-optimal scaling of a warm start: y = op(x0), alpha = y^H b / y^H y,
// x = alpha x0, r = b - alpha y.  Returns ||r||.  The scaling absorbs the
// change of load amplitude and phase between neighbouring frequencies at no
// extra operator application.
static double scaled_start(const Operator &op, Workspace &ws, const double *b, const double *x0, double *x, double *r,
                           hipStream_t st) {
    const int64_t N = op.N;
    op.apply(x0, ws.tmp, st);
    vec_mdot(N, 1, ws.tmp, N, b, ws.dots_partial, ws.small, st);
    vec_mdot(N, 1, ws.tmp, N, ws.tmp, ws.dots_partial, ws.small + 2, st);
    AFS_HIP(hipMemcpyAsync(ws.host_small, ws.small, 32, hipMemcpyDeviceToHost, st));
    AFS_HIP(hipStreamSynchronize(st));
    const std::complex<double> yb(ws.host_small[0], ws.host_small[1]);
    const double yy = ws.host_small[2];
    const std::complex<double> alpha = (yy > 0.0 && std::isfinite(yy)) ? yb / yy : std::complex<double>(0.0);
    vec_axpby(N, alpha.real(), alpha.imag(), x0, 0.0, 0.0, x0, x, st);
    vec_axpby(N, 1.0, 0.0, b, -alpha.real(), -alpha.imag(), ws.tmp, r, st);
    return norm2_dev(ws, N, r, st);
}

// Two-vector residual-minimising start: x = alpha x1 + beta x2 minimising
// ||b - alpha A x1 - beta A x2||, solved in an orthogonalised basis of the
// images (y2' = y2 - mu y1, mu = y1^H y2 / |y1|^2) so that the coefficients and
// the starting residual stay accurate; x2 is dropped (x1 alone) when its image
// adds less than 10% of a new direction.  Returns ||r|| (sets *used2).
static double scaled_start2(const Operator &op, Workspace &ws, const double *b, const double *x1, const double *x2,
                            double *x, double *r, hipStream_t st, bool *used2, double *gain) {
    const int64_t N = op.N;
    double *y1 = ws.tmp, *y2 = ws.w;
    op.apply(x1, y1, st);
    op.apply(x2, y2, st);
    double *d = ws.small;
    vec_mdot(N, 1, y1, N, y1, ws.dots_partial, d, st);      // |y1|^2
    vec_mdot(N, 1, y1, N, y2, ws.dots_partial, d + 2, st);  // y1^H y2
    vec_mdot(N, 1, y2, N, y2, ws.dots_partial, d + 4, st);  // |y2|^2
    vec_mdot(N, 1, y1, N, b, ws.dots_partial, d + 6, st);   // y1^H b
    vec_mdot(N, 1, y2, N, b, ws.dots_partial, d + 8, st);   // y2^H b
    AFS_HIP(hipMemcpyAsync(ws.host_small, d, 80, hipMemcpyDeviceToHost, st));
    AFS_HIP(hipStreamSynchronize(st));
    using C = std::complex<double>;
    const double *h = ws.host_small;
    const double g11 = h[0], g22 = h[4];
    const C g12(h[2], h[3]), c1(h[6], h[7]), c2(h[8], h[9]);
    *used2 = false;
    *gain = 1.0;
    if (!(g11 > 0.0) || !std::isfinite(g11) || !(g22 > 0.0) || !std::isfinite(g22)) {
        // degenerate image: fall back to whichever vector has one
        const bool one = g11 > 0.0 && std::isfinite(g11);
        const C a = one ? c1 / g11 : (g22 > 0.0 && std::isfinite(g22) ? c2 / g22 : C(0.0));
        const double *xs = one ? x1 : x2;
        const double *ys = one ? y1 : y2;
        vec_axpby(N, a.real(), a.imag(), xs, 0.0, 0.0, xs, x, st);
        vec_axpby(N, 1.0, 0.0, b, -a.real(), -a.imag(), ys, r, st);
        return norm2_dev(ws, N, r, st);
    }
    const C mu = g12 / g11;
    const double g2p = g22 - std::norm(g12) / g11;  // |y2'|^2
    if (!(g2p > 0.01 * g22)) {
        const C a = c1 / g11;
        vec_axpby(N, a.real(), a.imag(), x1, 0.0, 0.0, x1, x, st);
        vec_axpby(N, 1.0, 0.0, b, -a.real(), -a.imag(), y1, r, st);
        return norm2_dev(ws, N, r, st);
    }
    const C a = c1 / g11;
    const C c = (c2 - std::conj(mu) * c1) / g2p;  // y2'^H b / |y2'|^2
    const C alpha = a - c * mu;
    *used2 = true;
    {
        // residual norms with x1 alone and with the pair (normal equations)
        double bb = 0.0;
        vec_mdot(N, 1, b, N, b, ws.dots_partial, ws.small, st);
        AFS_HIP(hipMemcpyAsync(ws.host_small, ws.small, 16, hipMemcpyDeviceToHost, st));
        AFS_HIP(hipStreamSynchronize(st));
        bb = ws.host_small[0];
        const double r1 = std::max(bb - std::norm(c1) / g11, 0.0);
        const double r2 = std::max(r1 - std::norm(c) * g2p, 0.0);
        *gain = r2 > 0.0 ? std::sqrt(r1 / r2) : 1e30;
    }
    vec_axpby(N, alpha.real(), alpha.imag(), x1, c.real(), c.imag(), x2, x, st);
    // r = b - a y1 - c (y2 - mu y1) = b - alpha y1 - c y2, formed from the orthogonal pieces
    vec_axpby(N, 1.0, 0.0, y2, -mu.real(), -mu.imag(), y1, y2, st);  // y2 <- y2'
    vec_axpby(N, 1.0, 0.0, b, -a.real(), -a.imag(), y1, r, st);
    vec_axpby(N, 1.0, 0.0, r, -c.real(), -c.imag(), y2, r, st);
    return norm2_dev(ws, N, r, st);
}

// Starting iterate from the available guesses (previous-frequency solution
// and/or network prediction); returns the residual norm (x_zero: b itself).
static double start_iterate(const Operator &op, Workspace &ws, const double *b, double bnorm, const double *x_prev,
                            const double *x_net, double *x, double *r, bool &x_zero, hipStream_t st,
                            bool *used_net, double *net_gain) {
    x_zero = false;
    *used_net = false;
    *net_gain = 0.0;
    if (x_prev && x_net)
        return scaled_start2(op, ws, b, x_prev, x_net, x, r, st, used_net, net_gain);
    if (x_net)
        *used_net = true;
    if (x_net)
        return scaled_start(op, ws, b, x_net, x, r, st);
    if (x_prev)
        return scaled_start(op, ws, b, x_prev, x, r, st);
    x_zero = true;
    AFS_HIP(hipMemsetAsync(x, 0, (size_t)op.N * 16, st));
    AFS_HIP(hipMemcpyAsync(r, b, (size_t)op.N * 16, hipMemcpyDeviceToDevice, st));
    return bnorm;
}

// ------------------------------------------------------------ one solve --
static double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    return (double)ms;
}

// matrix_free = 2: the inner products of the mixed path through the
// hierarchical form of the operator (built per frequency in assemble_into)
static void hm_settings(Workspace &ws, const afsbem_solve_opts &o) {
    ws.hm_enabled = o.matrix_free == 2;
    ws.hm_eps = o.hmat_eps > 0.0 ? o.hmat_eps : 1e-5;
    ws.hm_eta = o.hmat_eta > 0.0 ? o.hmat_eta : 1.0;
    ws.hm_ok = false;
}

static void assemble_into(Problem &p, Workspace &ws, int fmt, double s_re, double s_im, const double *d_bc,
                          hipStream_t st, bool profile = false) {
    KernelParams kp = kernel_params(p.mat, s_re, s_im);
    if (fmt == kFmtBlocks) {
        // near/self blocks and b (far part evaluated on the fly in FP64)
        launch_block_setup(p, kp, d_bc, ws.nearblk, ws.selfblk, ws.precond, ws.asm_scratch, st);
        double *bpart = static_cast<double *>(ws.asm_scratch);
        mf_apply(p, kp, 0, 1, nullptr, nullptr, d_bc, nullptr, bpart, st);
        launch_finalize_b(p, mf_chunks(p.dev.n_tri), bpart, ws.asm_scratch, ws.b, st);
        if (ws.prec_kind == 1) {
            cluster_gather_mf(p, kp, ws.nearblk, ws.selfblk, ws.clgath, st);
            cluster_inverse(p.dev, kFmtBlocks, ws.clgath, nullptr, ws.clinv, st);
        }
        if (ws.hm_enabled) {
            hmat_ensure(p, ws.hm_eta);
            hmat_setup(p, ws, kp, ws.hm_eps, st);
        }
        return;
    }
    if (profile)
        for (auto &e : ws.ev_far)
            if (!e)
                AFS_HIP(hipEventCreate(&e));
    ws.far_timed = profile;
    launch_assembly(p, kp, d_bc, fmt, ws.A, ws.A_lo, ws.b, ws.precond, ws.asm_scratch, st,
                    profile ? ws.ev_far[0] : nullptr, profile ? ws.ev_far[1] : nullptr);
    if (ws.prec_kind == 1)
        cluster_inverse(p.dev, fmt, ws.A, ws.A_lo, ws.clinv, st);
}

// Krylov phase of one frequency on an assembled workspace (stream st); the
// timing events bracket the assembly (ea0, ea1, possibly on another stream)
// and this phase.
// on_residual (nullable): called once, when the first inner solve of the
// mixed refinement comes within 50x of its target, else right after the first
// FP64 residual is enqueued, else at the end of the phase
static int krylov_phase(Problem &p, Workspace &ws, const afsbem_solve_opts &o, int fmt, double s_re, double s_im,
                        const double *d_bc, const double *d_x0, double *d_a, double *d_u, double *d_t,
                        afsbem_solve_stats *stats, hipStream_t st, hipEvent_t ea0, hipEvent_t ea1, hipEvent_t e2,
                        const std::function<void()> &on_residual = {}) {
    bool residual_called = false;
    auto residual_hook = [&]() {
        if (on_residual && !residual_called) {
            residual_called = true;
            on_residual();
        }
    };
    const int64_t nt = p.dev.n_tri, N = 3 * nt;
    hipEvent_t ek;  // start of this phase on st
    AFS_HIP(hipEventCreate(&ek));
    struct EvGuard {
        hipEvent_t e;
        ~EvGuard() { (void)hipEventDestroy(e); }
    } ek_guard{ek};
    AFS_HIP(hipEventRecord(ek, st));
    int matvecs = 0;
    double bytes = 0.0;
    Workspace *prof = o.profile ? &ws : nullptr;
    ws.reset_timing();
    Operator op64{N, fmt, 0, ws.A, ws.A_lo, ws.gemv_partial, &matvecs, &bytes, prof};
    const KernelParams kp = kernel_params(p.mat, s_re, s_im);
    op64.prob = &p;
    op64.kp = kp;
    op64.nearblk = ws.nearblk;
    op64.selfblk = ws.selfblk;
    op64.hm = ws.hm_enabled ? &ws : nullptr;
    const bool mixed = o.precision == AFSBEM_PREC_MIXED;
    const double bnorm = norm2_dev(ws, N, ws.b, st);
    if (ws.hm_enabled && fmt == kFmtBlocks) {
        // the frequency's assembly has completed (st waited for it, then
        // synchronised); a build that ran out of pool is repeated with more
        for (int tries = 0; !hmat_finish(p, ws, st) && ws.hm_exhausted && tries < 3; ++tries) {
            hmat_setup(p, ws, kernel_params(p.mat, s_re, s_im), ws.hm_eps, st);
            AFS_HIP(hipStreamSynchronize(st));
        }
    }
    const bool learned = o.warm_start == AFSBEM_WARM_LEARNED;
    const bool user_aug = o.warm_start == AFSBEM_WARM_USER_AUG;
    const double *x_prev = (d_x0 && o.warm_start != AFSBEM_WARM_NONE && !user_aug) ? d_x0 : nullptr;
    const double *x_net = nullptr;
    if (learned) {
        if (!p.learn) {
            p.learn = new LearnState();
            p.learn->s_scale = std::max(1.0, std::fabs(s_im));
            p.learn->init(p);
        }
        if (p.learn->rows > 0 && p.learn->query_now()) {
            // the augmentation vector must outlive the preconditioned vectors (ws.z) of GMRES
            double *dst = o.learn_aug ? ws.aug : ws.z;
            p.learn->predict(p, s_re, s_im, dst, st);
            x_net = dst;
        }
    }
    // the prediction's roles: in the starting iterate (learn_aug 0 or 2) and/or
    // as a direction of the first GMRES cycle (learn_aug 1 or 2)
    const double *x_net_start = (x_net && o.learn_aug != 1) ? x_net : nullptr;
    const double *aug_vec = user_aug ? d_x0 : ((x_net && o.learn_aug != 0) ? x_net : nullptr);
    double aug_gain = 0.0;
    bool x_zero = true, used_net = false;
    double net_gain = 0.0;
    int status = AFSBEM_OK, refine = 0, fallback = 0;
    double relres = 1.0, rel_start = 1.0;
    if (bnorm == 0.0) {
        AFS_HIP(hipMemsetAsync(ws.x, 0, (size_t)N * 16, st));
        relres = 0.0;
    } else {
        // Starting iterate.  A guess whose residual is not finite or not below
        // ||b|| is rejected for the zero start (stats.fallback = 1).  The mixed
        // path seeds its inner solve with the FP32 operator's residual.
        Operator op32 = op64;
        op32.precision = 1;
        double *xs = mixed ? ws.xo : ws.x, *rs = mixed ? ws.rin : ws.r;
        double r0n = start_iterate(mixed ? op32 : op64, ws, ws.b, bnorm, x_prev, x_net_start, xs, rs, x_zero, st,
                                   &used_net, &net_gain);
        if (!x_zero && (o.fault_inject & AFSBEM_FAULT_NAN_START)) {
            // test hook: the guess turned out non-finite
            AFS_HIP(hipMemsetAsync(xs, 0xff, (size_t)N * 16, st));
            residual(mixed ? op32 : op64, ws, ws.b, xs, rs, st);
            r0n = norm2_dev(ws, N, rs, st);
        }
        if (!x_zero && !(r0n < bnorm)) {
            AFS_HIP(hipMemsetAsync(xs, 0, (size_t)N * 16, st));
            AFS_HIP(hipMemcpyAsync(rs, ws.b, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
            r0n = bnorm;
            x_zero = true;
            used_net = false;
            fallback = 1;
        }
        rel_start = r0n / bnorm;
        bool plain = !mixed;
        if (mixed) {
            // outer residual with the FP64 operator (hi + lo planes, or FP64
            // evaluation), inner GMRES on the FP32 operator for the correction
            // d: A32 d = r.  Two outer steps that do not reduce the residual
            // to 0.9 of its value, or a non-finite residual, hand the solve
            // to FP64 GMRES from the best iterate (stats.fallback = 2).
            double rnorm = r0n;
            int stalls = 0;
            bool from_zero = false;
            while (true) {
                const double tol_in = std::max(o.inner_tol * rnorm, 0.5 * o.tol * bnorm);
                const double *av = refine == 0 ? aug_vec : nullptr;
                // later steps search the first inner solve's Krylov subspace first
                const int rcy = o.no_recycle ? 0 : (refine == 0 ? 1 : 2);
                // the caller's hook (the next frequency's build) also fires once the
                // first inner solve is within 50x of its target, its last ~20 products
                std::function<void(double)> progress;
                if (on_residual && refine == 0)
                    progress = [&, tol_in](double est) {
                        if (est <= 50.0 * tol_in)
                            residual_hook();
                    };
                GmresResult g = gmres(op32, ws, nt, ws.rin, rnorm, ws.x, true, tol_in, o.restart,
                                      std::max(1, o.max_iter - matvecs), st, false, nullptr, 0.0, av, rcy, progress);
                if (av)
                    aug_gain = g.aug_gain;
                if (!(o.fault_inject & AFSBEM_FAULT_STALL_INNER))  // test hook: the correction is lost
                    vec_combine(N, 1, ws.x, N, ws.one, ws.xo, st);  // x_outer += d
                residual(op64, ws, ws.b, ws.xo, ws.rin, st);         // FP64 judge
                residual_hook();
                const double rn = norm2_dev(ws, N, ws.rin, st);
                ++refine;
                if (!std::isfinite(rn) || g.nan) {
                    AFS_HIP(hipMemsetAsync(ws.xo, 0, (size_t)N * 16, st));
                    rnorm = bnorm;
                    plain = from_zero = true;
                    break;
                }
                stalls = rn > 0.9 * rnorm ? stalls + 1 : 0;
                rnorm = rn;
                if (rnorm <= o.tol * bnorm || matvecs >= o.max_iter)
                    break;
                if (stalls >= 2) {
                    plain = true;
                    break;
                }
            }
            relres = rnorm / bnorm;
            AFS_HIP(hipMemcpyAsync(ws.x, ws.xo, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
            if (plain) {
                fallback = 2;
                x_zero = from_zero;  // after a non-finite residual: from zero
                r0n = rnorm;
                AFS_HIP(hipMemcpyAsync(ws.r, from_zero ? ws.b : ws.rin, (size_t)N * 16, hipMemcpyDeviceToDevice,
                                       st));
            }
        }
        if (plain) {
            const double *av = mixed ? nullptr : aug_vec;  // a mixed solve handed over has used it
            GmresResult g = gmres(op64, ws, nt, ws.b, bnorm, ws.x, x_zero, o.tol * bnorm, o.restart,
                                  std::max(1, o.max_iter - matvecs), st, true, x_zero ? nullptr : ws.r, r0n, av);
            if (av)
                aug_gain = g.aug_gain;
            // final true FP64 residual (after the last restart gmres already formed r)
            relres = g.est / bnorm;
            if (g.nan)
                status = AFSBEM_ENAN;
        }
        if (!std::isfinite(relres))
            status = AFSBEM_ENAN;
    }
    residual_hook();
    AFS_HIP(hipEventRecord(e2, st));
    if (d_a)
        AFS_HIP(hipMemcpyAsync(d_a, ws.x, (size_t)N * 16, hipMemcpyDeviceToDevice, st));
    if (d_u || d_t)
        vec_split_ut(nt, p.dev.kind, ws.x, d_bc, d_u, d_t, st);
    // gate of the network: the residual reduction its prediction brought (the
    // augmentation direction alone, or the second vector of the start)
    if (learned && aug_vec && o.learn_aug == 1)
        p.learn->record_gain(aug_gain);
    else if (learned && x_net_start && x_prev)
        p.learn->record_gain(net_gain);
    if (aug_vec && !user_aug)
        used_net = true;
    if (learned && !p.learn->retired && std::isfinite(relres)) {
        p.learn->add_solution(p, s_re, s_im, ws.x, st);
        p.learn->train(o.learn_steps > 0 ? o.learn_steps : p.learn->steps_per_sample, st);
    }
    AFS_HIP(hipStreamSynchronize(st));
    if (status == AFSBEM_OK && !(relres <= o.tol))
        status = AFSBEM_ENOCONV;
    if (stats) {
        stats->iters = matvecs;
        stats->refine_steps = refine;
        stats->fallback = fallback;
        stats->status = status;
        stats->rel_res_fp64 = relres;
        stats->rel_res_start = rel_start;
        stats->used_net = used_net ? 1 : 0;
        stats->t_assemble_ms = elapsed_ms(ea0, ea1);
        stats->t_solve_ms = elapsed_ms(ek, e2);
        stats->bytes = bytes;
        stats->gemv_ms = stats->gemv64_ms = 0.0;
        stats->t_far_ms = ws.far_timed ? elapsed_ms(ws.ev_far[0], ws.ev_far[1]) : 0.0;
        stats->gemv_count = stats->gemv64_count = 0;
        for (int k = 0; k < ws.ev_used; ++k) {
            const double ms = elapsed_ms(ws.ev[2 * k], ws.ev[2 * k + 1]);
            // Krylov operator: FP32 hi plane (mixed) or C128 (plain); FP64 split = residual operator
            if (ws.ev_prec[k] == 0) {
                stats->gemv64_ms += ms;
                ++stats->gemv64_count;
            } else {
                stats->gemv_ms += ms;
                ++stats->gemv_count;
            }
        }
    }
    return status;
}


int solve_one(Problem &p, const afsbem_solve_opts &o, double s_re, double s_im, const double *d_bc,
              const double *d_x0, double *d_a, double *d_u, double *d_t, afsbem_solve_stats *stats,
              hipStream_t st) {
    AFS_REQUIRE(!(o.matrix_free && p.dev.disc == 1), AFSBEM_EINVAL,
                "matrix-free application is not available for six-node (Nystrom) problems");
    const int fmt = o.matrix_free ? kFmtBlocks
                                  : ((o.precision == AFSBEM_PREC_MIXED) ? AFSBEM_FMT_SPLIT : AFSBEM_FMT_C128);
    if (!p.ws)
        p.ws = new Workspace();
    Workspace &ws = *p.ws;
    ws.ensure(p, fmt, o.restart, o.precond);
    hm_settings(ws, o);
    hipEvent_t e0, e1, e2;
    AFS_HIP(hipEventCreate(&e0));
    AFS_HIP(hipEventCreate(&e1));
    AFS_HIP(hipEventCreate(&e2));
    AFS_HIP(hipEventRecord(e0, st));
    assemble_into(p, ws, fmt, s_re, s_im, d_bc, st, o.profile != 0);
    AFS_HIP(hipEventRecord(e1, st));
    int rc;
    try {
        rc = krylov_phase(p, ws, o, fmt, s_re, s_im, d_bc, d_x0, d_a, d_u, d_t, stats, st, e0, e1, e2);
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    return rc;
}

// Linear extrapolation in s of y(s) = s a(s) from the solutions at s0 and s1
// to s2: a(s2) ~ c1 a(s1) + c2 a(s0).  False when s0 = s1 or s2 = 0.
bool extrap_coeffs(std::complex<double> s0, std::complex<double> s1, std::complex<double> s2,
                   std::complex<double> &c1, std::complex<double> &c2) {
    const std::complex<double> d = s1 - s0;
    if (std::abs(d) == 0.0 || std::abs(s2) == 0.0)
        return false;
    const std::complex<double> al = (s2 - s1) / d;
    c1 = s1 * (1.0 + al) / s2;
    c2 = -al * s0 / s2;
    return std::isfinite(c1.real()) && std::isfinite(c1.imag()) && std::isfinite(c2.real()) &&
           std::isfinite(c2.imag());
}

// Starting guess of frequency k of a call for PREV / LEARNED / EXTRAP / USER
// (nullptr: zero start); EXTRAP forms its vector in xbuf on stream st.
const double *start_guess(const afsbem_solve_opts &o, int32_t k, int64_t N, const double *s, const double *x0_user,
                          const double *a_out, double *xbuf, hipStream_t st) {
    using C = std::complex<double>;
    if (o.warm_start == AFSBEM_WARM_USER || o.warm_start == AFSBEM_WARM_USER_AUG)
        return x0_user + 2 * (size_t)k * N;
    const bool prev_like = o.warm_start == AFSBEM_WARM_PREV || o.warm_start == AFSBEM_WARM_LEARNED ||
                           o.warm_start == AFSBEM_WARM_EXTRAP;
    if (!prev_like)
        return nullptr;
    if (k == 0)
        return x0_user;  // the caller's previous solution (nullable)
    if (!a_out)
        return nullptr;
    const double *a1 = a_out + 2 * (size_t)(k - 1) * N;
    if (o.warm_start != AFSBEM_WARM_EXTRAP) {
        // the solution of the nearest frequency solved before in this call
        // (the previous one for an ordered list; an adaptive sampling order
        // visits the band out of order)
        const C sk(s[2 * k], s[2 * k + 1]);
        int32_t best = k - 1;
        double bd = std::abs(sk - C(s[2 * best], s[2 * best + 1]));
        for (int32_t j = k - 2; j >= 0; --j) {
            const double d = std::abs(sk - C(s[2 * j], s[2 * j + 1]));
            if (d < bd) {
                bd = d;
                best = j;
            }
        }
        return a_out + 2 * (size_t)best * N;
    }
    C c1, c2;
    if (o.warm_start == AFSBEM_WARM_EXTRAP && k >= 2 && xbuf &&
        extrap_coeffs(C(s[2 * (k - 2)], s[2 * (k - 2) + 1]), C(s[2 * (k - 1)], s[2 * (k - 1) + 1]),
                      C(s[2 * k], s[2 * k + 1]), c1, c2)) {
        vec_axpby(N, c1.real(), c1.imag(), a1, c2.real(), c2.imag(), a_out + 2 * (size_t)(k - 2) * N, xbuf, st);
        return xbuf;
    }
    return a1;
}

// Two frequencies in flight: the FP64 assembly of frequency k+1 (VALU-bound)
// runs on one library stream while the Krylov phase of frequency k
// (HBM-bound GEMVs, latency-bound Arnoldi steps with host round trips) runs on
// another; two workspaces alternate.  Ordering with the caller's stream is
// kept by events at entry and exit.
int solve_pipelined(Problem &p, const afsbem_solve_opts &o, int32_t n_s, const double *s, const double *bc,
                    const double *x0_user, double *a_out, double *u_out, double *t_out,
                    afsbem_solve_stats *stats, hipStream_t caller) {
    const int64_t N = 3 * p.dev.n_tri;
    AFS_REQUIRE(!(o.matrix_free && p.dev.disc == 1), AFSBEM_EINVAL,
                "matrix-free application is not available for six-node (Nystrom) problems");
    const int fmt = o.matrix_free ? kFmtBlocks
                                  : ((o.precision == AFSBEM_PREC_MIXED) ? AFSBEM_FMT_SPLIT : AFSBEM_FMT_C128);
    if (!p.ws)
        p.ws = new Workspace();
    if (!p.ws2)
        p.ws2 = new Workspace();
    Workspace *W[2] = {p.ws, p.ws2};
    W[0]->ensure(p, fmt, o.restart, o.precond);
    W[1]->ensure(p, fmt, o.restart, o.precond);
    hm_settings(*W[0], o);
    hm_settings(*W[1], o);
    if (!p.st_asm)
        AFS_HIP(hipStreamCreateWithFlags(&p.st_asm, hipStreamNonBlocking));
    if (!p.st_sol)
        AFS_HIP(hipStreamCreateWithFlags(&p.st_sol, hipStreamNonBlocking));
    hipStream_t SA = p.st_asm, SS = p.st_sol;
    std::vector<hipEvent_t> evs;
    auto mk = [&]() {
        hipEvent_t e;
        AFS_HIP(hipEventCreate(&e));
        evs.push_back(e);
        return e;
    };
    int rc = AFSBEM_OK;
    try {
        hipEvent_t entry = mk();
        AFS_HIP(hipEventRecord(entry, caller));
        AFS_HIP(hipStreamWaitEvent(SA, entry, 0));
        AFS_HIP(hipStreamWaitEvent(SS, entry, 0));
        std::vector<hipEvent_t> a0(n_s), a1(n_s), sdone(n_s), e2(n_s);
        for (int32_t k = 0; k < n_s; ++k) {
            a0[k] = mk();
            a1[k] = mk();
            sdone[k] = mk();
            e2[k] = mk();
        }
        auto enqueue_asm = [&](int32_t k) {
            Workspace &w = *W[k % 2];
            if (k >= 2)
                AFS_HIP(hipStreamWaitEvent(SA, sdone[k - 2], 0));  // workspace free again
            AFS_HIP(hipEventRecord(a0[k], SA));
            assemble_into(p, w, fmt, s[2 * k], s[2 * k + 1], bc + 2 * (size_t)k * N, SA, o.profile != 0);
            AFS_HIP(hipEventRecord(a1[k], SA));
        };
        // batch 2: the build of frequency k+1 starts near the end of frequency
        // k's first inner solve (see krylov_phase), so that it overlaps the
        // VALU-bound FP64 residual rather than the HBM-bound inner products
        // (the hierarchical build is HBM-bound too)
        const bool at_residual = o.batch == 2;
        enqueue_asm(0);
        for (int32_t k = 0; k < n_s; ++k) {
            if (k + 1 < n_s && !at_residual)
                enqueue_asm(k + 1);
            std::function<void()> hook;
            if (k + 1 < n_s && at_residual)
                hook = [&enqueue_asm, k]() { enqueue_asm(k + 1); };
            AFS_HIP(hipStreamWaitEvent(SS, a1[k], 0));
            const double *x0 = start_guess(o, k, N, s, x0_user, a_out, W[k % 2]->xstart, SS);
            afsbem_solve_opts ok = o;
            if (ok.warm_start == AFSBEM_WARM_EXTRAP)
                ok.warm_start = AFSBEM_WARM_PREV;  // the guess is formed; the solve treats it as any other
            if (!x0 && ok.warm_start != AFSBEM_WARM_LEARNED)
                ok.warm_start = AFSBEM_WARM_NONE;
            int r = krylov_phase(p, *W[k % 2], ok, fmt, s[2 * k], s[2 * k + 1], bc + 2 * (size_t)k * N, x0,
                                 a_out ? a_out + 2 * (size_t)k * N : nullptr, u_out ? u_out + 2 * (size_t)k * N : nullptr,
                                 t_out ? t_out + 2 * (size_t)k * N : nullptr, stats ? &stats[k] : nullptr, SS, a0[k],
                                 a1[k], e2[k], hook);
            AFS_HIP(hipEventRecord(sdone[k], SS));
            if (r != AFSBEM_OK && rc == AFSBEM_OK)
                rc = r;
        }
        hipEvent_t ex_a = mk(), ex_s = mk();
        AFS_HIP(hipEventRecord(ex_a, SA));
        AFS_HIP(hipEventRecord(ex_s, SS));
        AFS_HIP(hipStreamWaitEvent(caller, ex_a, 0));
        AFS_HIP(hipStreamWaitEvent(caller, ex_s, 0));
        AFS_HIP(hipStreamSynchronize(SS));
        AFS_HIP(hipStreamSynchronize(SA));
    } catch (...) {
        (void)hipStreamSynchronize(SA);
        (void)hipStreamSynchronize(SS);
        for (hipEvent_t e : evs)
            (void)hipEventDestroy(e);
        throw;
    }
    for (hipEvent_t e : evs)
        (void)hipEventDestroy(e);
    return rc;
}

}  // namespace afsbem
