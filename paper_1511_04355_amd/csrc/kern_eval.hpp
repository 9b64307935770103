// Device-side evaluation of the fundamental solutions at point pairs and the
// 3x3 block accumulators shared by the assembly, preconditioner-gather and
// hierarchical far-field kernels (FP64).
#pragma once
#include "cplx.hpp"
#include "fastmath64.hpp"
#include "internal.hpp"
#include "kern_mfeval.hpp"

namespace afsbem {

struct Rule7Args {
    double b1[7], b2[7], w[7];  // barycentric weights of vertices 1 and 2, rule weight
};

// ---------------------------------------------------------------------------
// Kernel evaluation at one point pair.  r^k-scaled radial functions
//   Psi = r psi, X = r chi, Psd = r^2 psi', Xd = r^2 chi'
// of x = s r / c_s; series about 0 for |x| < 1/4 (the P/S cancellation makes
// the closed form lose eps/|x|^2), closed form above.
// ---------------------------------------------------------------------------
struct Radial {
    cd Psi, X, Psd, Xd;
};

constexpr int kSer64 = 13;  // FP64 series terms used (of the 16 stored)

// inv_ax2 = 1 / |x|^2, supplied by the caller (from 1/r, without a division);
// coef: the plan's 64 series coefficients, then the kFmTabLen table entries
__device__ __forceinline__ Radial radial64(cd x, double beta, const double *__restrict__ coef, double inv_ax2) {
    Radial R;
    const double ax2 = x.r * x.r + x.i * x.i;
    if (ax2 < 0.0625) {
        // coef: [16][4] = a_n, b_n, (n-1) a_n, (n-1) b_n, summed from the top.
        // Terms n <= kSer64 - 1 only: at |x| <= 1/4 the rest sum to below
        // 7e-17 of the leading ones (the coefficients fall as (n+1)^2/(n+2)!)
        double pr[4], pi[4];
        series4<double, kSer64, kSer64>(coef, x.r, x.i, ax2, pr, pi);
        R.Psi = cd{pr[0], pi[0]};
        R.X = cd{pr[1], pi[1]};
        R.Psd = cd{pr[2], pi[2]};
        R.Xd = cd{pr[3], pi[3]};
        return R;
    }
    // coef + 64: the tables of the FP64 exp and sincos
    double sn, cs;
    sincos_tab(x.i, coef + 64, &sn, &cs);
    const double ex = exp_tab(-x.r, coef + 64);
    const cd e = cd{ex * cs, -ex * sn};
    sincos_tab(beta * x.i, coef + 64, &sn, &cs);
    const double exp_ = exp_tab(-beta * x.r, coef + 64);
    const cd ep = cd{exp_ * cs, -exp_ * sn};
    const double inv = inv_ax2;
    const cd ix = cd{x.r * inv, -x.i * inv};
    const cd ix2 = cmul(ix, ix);
    const double b2 = beta * beta;
    // P = ep (beta^2 + 3 beta ix + 3 ix^2)
    const cd P = cmul(ep, cd{b2 + 3.0 * beta * ix.r + 3.0 * ix2.r, 3.0 * beta * ix.i + 3.0 * ix2.i});
    R.Psi = csub(cmul(e, cd{1.0 + ix.r + ix2.r, ix.i + ix2.i}), cmul(ep, cd{beta * ix.r + ix2.r, beta * ix.i + ix2.i}));
    R.X = csub(cmul(e, cd{1.0 + 3.0 * ix.r + 3.0 * ix2.r, 3.0 * ix.i + 3.0 * ix2.i}), P);
    R.Psd = csub(P, cmul(e, cd{x.r + 2.0 + 3.0 * ix.r + 3.0 * ix2.r, x.i + 3.0 * ix.i + 3.0 * ix2.i}));
    const double b3 = b2 * beta;
    R.Xd = csub(cmul(ep, cd{b3 * x.r + 4.0 * b2 + 9.0 * beta * ix.r + 9.0 * ix2.r, b3 * x.i + 9.0 * beta * ix.i + 9.0 * ix2.i}),
                cmul(e, cd{x.r + 4.0 + 9.0 * ix.r + 9.0 * ix2.r, x.i + 9.0 * ix.i + 9.0 * ix2.i}));
    return R;
}

// Coefficients of T_ij = (1/(4 pi r^2)) [t0 d_ij + t1 n_i rh_j + t2 rh_i n_j + t3 rh_i rh_j]
// and U_ij = (1/(4 pi mu r)) [Psi d_ij - X rh_i rh_j].
struct PairEval {
    double rh[3];
    double r, ir, rn;
    cd Psi, X;             // U coefficients (without 1/(4 pi mu r))
    cd t0, t1, t2, t3;     // T coefficients (without 1/(4 pi r^2))
};

__device__ __forceinline__ void eval_pair(const KernelParams &kp, const double *__restrict__ coef,
                                          double xx, double xy, double xz, double yx, double yy, double yz,
                                          double nx, double ny, double nz, PairEval &E) {
    const double dx = yx - xx, dy = yy - xy, dz = yz - xz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt_nr(r2);
    const double r = r2 * ir;
    E.r = r;
    E.ir = ir;
    E.rh[0] = dx * ir;
    E.rh[1] = dy * ir;
    E.rh[2] = dz * ir;
    E.rn = E.rh[0] * nx + E.rh[1] * ny + E.rh[2] * nz;
    const cd x = cd{kp.s_re * r * kp.inv_cs, kp.s_im * r * kp.inv_cs};
    const Radial R = radial64(x, kp.beta, coef, ir * ir * kp.inv_ks2);
    E.Psi = R.Psi;
    E.X = R.X;
    const cd b1 = csub(R.Psd, R.X);
    E.t1 = b1;
    E.t0 = cscale(b1, E.rn);
    // t2 = -2X + (lam/mu)(Psd - Xd - 2X)
    const cd tmp = csub(csub(R.Psd, R.Xd), cscale(R.X, 2.0));
    E.t2 = cadd(cscale(R.X, -2.0), cscale(tmp, kp.lam_over_mu));
    E.t3 = cscale(csub(cscale(R.X, 4.0), cscale(R.Xd, 2.0)), E.rn);
}

constexpr double kInv4Pi = 0.079577471545947667884;  // 1 / (4 pi)

// full 3x3 T block times weight w, accumulated into blk (row-major i*3+j)
__device__ __forceinline__ void acc_T(const PairEval &E, double nx, double ny, double nz, double w,
                                      cd blk[9]) {
    const double n[3] = {nx, ny, nz};
    const double f = w * kInv4Pi * E.ir * E.ir;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd v = cadd(cadd(cscale(E.t1, n[i] * E.rh[j]), cscale(E.t2, E.rh[i] * n[j])),
                        cscale(E.t3, E.rh[i] * E.rh[j]));
            if (i == j)
                v = cadd(v, E.t0);
            blk[3 * i + j] = cadd(blk[3 * i + j], cscale(v, f));
        }
}

__device__ __forceinline__ void acc_U(const PairEval &E, const KernelParams &kp, double w, cd blk[9]) {
    const double f = w * kp.c_u * E.ir;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd v = cscale(E.X, -E.rh[i] * E.rh[j]);
            if (i == j)
                v = cadd(v, E.Psi);
            blk[3 * i + j] = cadd(blk[3 * i + j], cscale(v, f));
        }
}

// acc += w * T . v   (v complex 3-vector)
__device__ __forceinline__ void acc_Tv(const PairEval &E, double nx, double ny, double nz, double w,
                                       const cd v[3], cd acc[3]) {
    const double n[3] = {nx, ny, nz};
    const double f = w * kInv4Pi * E.ir * E.ir;
    const cd rv = cadd(cadd(cscale(v[0], E.rh[0]), cscale(v[1], E.rh[1])), cscale(v[2], E.rh[2]));
    const cd nv = cadd(cadd(cscale(v[0], nx), cscale(v[1], ny)), cscale(v[2], nz));
    const cd a1 = cmul(E.t1, rv), a2 = cmul(E.t2, nv), a3 = cmul(E.t3, rv);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cd t = cadd(cmul(E.t0, v[i]), cadd(cscale(a1, n[i]), cscale(cadd(a2, a3), E.rh[i])));
        acc[i] = cadd(acc[i], cscale(t, f));
    }
}

// acc += w * U . v
__device__ __forceinline__ void acc_Uv(const PairEval &E, const KernelParams &kp, double w, const cd v[3],
                                       cd acc[3]) {
    const double f = w * kp.c_u * E.ir;
    const cd rv = cadd(cadd(cscale(v[0], E.rh[0]), cscale(v[1], E.rh[1])), cscale(v[2], E.rh[2]));
    const cd xr = cmul(E.X, rv);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cd t = csub(cmul(E.Psi, v[i]), cscale(xr, E.rh[i]));
        acc[i] = cadd(acc[i], cscale(t, f));
    }
}

template <int FMT>
__device__ __forceinline__ void store_block(void *A, void *A_lo, int64_t lda, int64_t m, int64_t n, const cd blk[9]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int64_t base = (3 * n + j) * lda + 3 * m;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const cd v = blk[3 * i + j];
            if (FMT == AFSBEM_FMT_C128) {
                reinterpret_cast<double2 *>(A)[base + i] = make_double2(v.r, v.i);
            } else {
                const float hr = (float)v.r, hi = (float)v.i;
                reinterpret_cast<float2 *>(A)[base + i] = make_float2(hr, hi);
                reinterpret_cast<float2 *>(A_lo)[base + i] =
                    make_float2((float)(v.r - (double)hr), (float)(v.i - (double)hi));
            }
        }
    }
}

// 3x3 complex block, row-major, to 18 consecutive doubles
__device__ __forceinline__ void store_blk9(double *out, const cd blk[9]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        out[2 * e] = blk[e].r;
        out[2 * e + 1] = blk[e].i;
    }
}

// ---------------------------------------------------------------- far field --
// Per (collocation point, source element) the 3x3 traction block is
//   sum_q f_q [t0 d_ij + t1 n_i rh_j + t2 rh_i n_j + t3 rh_i rh_j],  f_q = w_q/(4 pi r_q^2),
// and n is constant over the element, so it is accumulated as the invariants
//   E = sum f t0,  Aj = sum f t1 rh_j,  Ci = sum f t2 rh_i,  Dij = sum f t3 rh_i rh_j (symmetric)
// and expanded to T_ij = E d_ij + n_i Aj + Ci n_j + Dij once per pair.  The
// displacement block likewise from E = sum g Psi, Dij = sum g X rh_i rh_j,
// g_q = w_q / (4 pi mu r_q):  U_ij = E d_ij - Dij.
struct BlockAcc {
    cd E, Aj[3], Ci[3], D[6];  // D: xx, yy, zz, xy, xz, yz
    __device__ __forceinline__ void zero() {
        E = cd{0, 0};
#pragma unroll
        for (int k = 0; k < 3; ++k)
            Aj[k] = Ci[k] = cd{0, 0};
#pragma unroll
        for (int k = 0; k < 6; ++k)
            D[k] = cd{0, 0};
    }
};

__device__ __forceinline__ int sym_idx(int i, int j) {
    return (i == j) ? i : ((i + j == 1) ? 3 : ((i + j == 2) ? 4 : 5));
}

__device__ __forceinline__ void acc_sym(cd D[6], cd c, const double rh[3]) {
    D[0] = cadd(D[0], cscale(c, rh[0] * rh[0]));
    D[1] = cadd(D[1], cscale(c, rh[1] * rh[1]));
    D[2] = cadd(D[2], cscale(c, rh[2] * rh[2]));
    D[3] = cadd(D[3], cscale(c, rh[0] * rh[1]));
    D[4] = cadd(D[4], cscale(c, rh[0] * rh[2]));
    D[5] = cadd(D[5], cscale(c, rh[1] * rh[2]));
}

// One quadrature node.  kind 0 (traction known): the block collects T with
// weight wA and b collects U.v with weight wB; kind 1 (displacement known): the
// block collects U with weight wA (negated at expansion) and b collects -T.v.
template <int KIND>
__device__ __forceinline__ void acc_node(const PairEval &E, const KernelParams &kp, double nx, double ny,
                                         double nz, double wA, double wB, const cd v[3], BlockAcc &acc,
                                         cd bacc[3]) {
    if (KIND == 0) {
        const double f = wA * kInv4Pi * E.ir * E.ir;
        acc.E = cadd(acc.E, cscale(E.t0, f));
        const cd ft1 = cscale(E.t1, f), ft2 = cscale(E.t2, f);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc.Aj[k] = cadd(acc.Aj[k], cscale(ft1, E.rh[k]));
            acc.Ci[k] = cadd(acc.Ci[k], cscale(ft2, E.rh[k]));
        }
        acc_sym(acc.D, cscale(E.t3, f), E.rh);
        acc_Uv(E, kp, wB, v, bacc);
    } else {
        const double g = wA * kp.c_u * E.ir;
        acc.E = cadd(acc.E, cscale(E.Psi, g));
        acc_sym(acc.D, cscale(E.X, g), E.rh);
        acc_Tv(E, nx, ny, nz, -wB, v, bacc);
    }
}

// A-matrix block: T (kind 0) or -U (kind 1)
__device__ __forceinline__ void expand_block(int kind, const BlockAcc &acc, double nx, double ny, double nz,
                                             cd blk[9]) {
    const double nn[3] = {nx, ny, nz};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const cd d = acc.D[sym_idx(i, j)];
            if (kind == 0) {
                const cd e = cadd(cadd(cscale(acc.Aj[j], nn[i]), cscale(acc.Ci[i], nn[j])), d);
                blk[3 * i + j] = (i == j) ? cadd(e, acc.E) : e;
            } else {
                blk[3 * i + j] = (i == j) ? csub(d, acc.E) : d;
            }
        }
}

}  // namespace afsbem
