/*
 * FP64 CPU oracle for the Laplace-domain elastodynamic collocation BEM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the GPU library: everything here
 * (fundamental solutions, quadrature rules, Gauss-Legendre nodes, geometry,
 * subdivision, singular integration, assembly) is written out independently
 * and kept deliberately plain: double precision, C99 complex, no blocking,
 * no fusion.
 *
 * What it computes (paper Section 2.1, Eq. 1 and Eq. 2):
 *   c_ij u_j(x) + PV int T_ij(x,y;s) u_j(y) dG = int U_ij(x,y;s) t_j(y) dG,
 * discretised with flat triangles, constant u and t per element and one
 * collocation point (the centroid) per element, c = 1/2 I at the centroid.
 * For each collocation row block m and element n,
 *   G_mn = int_{G_n} U(x_m, y) dG,   H_mn = 1/2 delta_mn I + PV int_{G_n} T(x_m, y) dG,
 * and the boundary conditions move known columns to the right-hand side:
 *   A[:,n] = H[:,n] (traction prescribed, u_n unknown) or -G[:,n] (displacement
 *   prescribed, t_n unknown);  b = sum_known-t G t_bar - sum_known-u H u_bar.
 *
 * Readings of the paper used here (it omits the fundamental solutions):
 *  - c_p = sqrt((lambda + 2 mu)/rho) (the printed formula misplaces the bracket);
 *  - U_ij = (psi delta_ij - chi rh_i rh_j)/(4 pi mu), rh = (y - x)/r, with psi and
 *    chi the Laplace-domain radial functions of the damped P and S waves;
 *  - T_ij is the traction at y, on the normal n(y) pointing out of the solid, of
 *    the displacement field U_i. (force along i at x), obtained from grad U and
 *    Hooke's law;
 *  - quadrature policy (identical on both sides of any parity comparison): the
 *    7-point degree-5 rule when |x - c_n| >= far_ratio * h_n; otherwise 4-way
 *    midpoint subdivision applied recursively with the same test on each
 *    sub-triangle, up to max_subdiv levels; the self element in polar
 *    coordinates about the centroid (three sub-triangles, Gauss-Legendre
 *    n_theta x n_rho) with the static 1/r^2 part of T taken as a Cauchy
 *    principal value over a circular exclusion.
 *
 * A second discretisation, the paper's own (curved six-node triangles and
 * the locally-corrected Nystrom method), is at the end of this file.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* material                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    double mu, nu, rho;
    double lam;   /* lambda = 2 mu nu / (1 - 2 nu) */
    double cs, cp, beta; /* beta = cs / cp */
} material_t;

static material_t make_material(const double mat[3])
{
    material_t m;
    m.mu = mat[0];
    m.nu = mat[1];
    m.rho = mat[2];
    m.lam = 2.0 * m.mu * m.nu / (1.0 - 2.0 * m.nu);
    m.cs = sqrt(m.mu / m.rho);
    m.cp = sqrt((m.lam + 2.0 * m.mu) / m.rho);
    m.beta = m.cs / m.cp;
    return m;
}

/* ------------------------------------------------------------------------- */
/* radial functions                                                           */
/* With x = s r / c_s and x_p = beta x, the displacement solution is          */
/*   U = (1/(4 pi rho s^2)) [ (s/c_s)^2 delta g_s - d_i d_j (g_s - g_p) ],    */
/*   g_a = exp(-s r / c_a) / r,                                               */
/* which gives U_ij = (psi delta_ij - chi rh_i rh_j)/(4 pi mu) with           */
/*   r psi = e^{-x}(1 + 1/x + 1/x^2) - beta^2 e^{-xp}(1/xp + 1/xp^2)          */
/*   r chi = e^{-x}(1 + 3/x + 3/x^2) - beta^2 e^{-xp}(1 + 3/xp + 3/xp^2).      */
/* out[0] = r psi, out[1] = r chi, out[2] = r^2 psi', out[3] = r^2 chi'.      */
/* ------------------------------------------------------------------------- */
static void radial_closed(cplx x, double beta, cplx out[4])
{
    cplx xp = beta * x;
    cplx e = cexp(-x), ep = cexp(-xp);
    cplx ix = 1.0 / x, ixp = 1.0 / xp;
    double b2 = beta * beta;
    out[0] = e * (1.0 + ix + ix * ix) - b2 * ep * (ixp + ixp * ixp);
    out[1] = e * (1.0 + 3.0 * ix + 3.0 * ix * ix) - b2 * ep * (1.0 + 3.0 * ixp + 3.0 * ixp * ixp);
    out[2] = -e * (x + 2.0 + 3.0 * ix + 3.0 * ix * ix) + b2 * ep * (1.0 + 3.0 * ixp + 3.0 * ixp * ixp);
    out[3] = -e * (x + 4.0 + 9.0 * ix + 9.0 * ix * ix) + b2 * ep * (xp + 4.0 + 9.0 * ixp + 9.0 * ixp * ixp);
}

/* Taylor series of the same four functions about x = 0 (the 1/x and 1/x^2
 * terms of the P and S parts cancel exactly):
 *   r psi = sum a_n x^n,  a_n = (-1)^n [(n+1)^2 + (n+1) beta^(n+2)] / (n+2)!
 *   r chi = sum b_n x^n,  b_n = (-1)^n (n^2 - 1)(1 - beta^(n+2)) / (n+2)!
 *   r^2 psi' = sum (n-1) a_n x^n,  r^2 chi' = sum (n-1) b_n x^n.            */
#define ORC_NSERIES 40
static void radial_series(cplx x, double beta, cplx out[4])
{
    cplx xn = 1.0;
    double fact = 2.0;            /* (n+2)! at n = 0 */
    double bp = beta * beta;      /* beta^(n+2) */
    double sg = 1.0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (int n = 0; n < ORC_NSERIES; ++n) {
        double a = sg * ((n + 1.0) * (n + 1.0) + (n + 1.0) * bp) / fact;
        double b = sg * ((double)n * n - 1.0) * (1.0 - bp) / fact;
        out[0] += a * xn;
        out[1] += b * xn;
        out[2] += (n - 1.0) * a * xn;
        out[3] += (n - 1.0) * b * xn;
        xn *= x;
        fact *= (n + 3.0);
        bp *= beta;
        sg = -sg;
    }
}

/* mode 0: series for |x| < 1, closed form otherwise; 1: series; 2: closed */
static void radial(cplx x, double beta, int mode, cplx out[4])
{
    if (mode == 1 || (mode == 0 && cabs(x) < 1.0))
        radial_series(x, beta, out);
    else
        radial_closed(x, beta, out);
}

/* ------------------------------------------------------------------------- */
/* fundamental solutions at one point pair                                   */
/* U[i*3+j], T[i*3+j]: i = direction of the point force at x, j = component   */
/* at y.  T uses the unit normal n at y.                                      */
/* ------------------------------------------------------------------------- */
static void kernel_UT(cplx s, const material_t *m, const double x[3], const double y[3],
                      const double n[3], int mode, cplx U[9], cplx T[9])
{
    double rv[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    cplx f[4];
    radial(s * r / m->cs, m->beta, mode, f);
    cplx psi = f[0] / r, chi = f[1] / r;
    cplx dpsi = f[2] / (r * r), dchi = f[3] / (r * r);
    double c = 1.0 / (4.0 * ORC_PI * m->mu);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            U[i * 3 + j] = c * (psi * (i == j) - chi * rh[i] * rh[j]);
    if (!T)
        return;
    /* dU_ij/dy_l = c [ psi' rh_l d_ij - chi' rh_i rh_j rh_l
     *                 - (chi/r)(d_il rh_j + d_jl rh_i - 2 rh_i rh_j rh_l) ] */
    cplx dU[3][3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l)
                dU[i][j][l] = c * (dpsi * rh[l] * (i == j) - dchi * rh[i] * rh[j] * rh[l]
                                   - (chi / r) * ((i == l) * rh[j] + (j == l) * rh[i]
                                                  - 2.0 * rh[i] * rh[j] * rh[l]));
    /* stress of the field U_i.: sigma_jk = lam d_jk div + mu (d_k U_ij + d_j U_ik);
     * traction component j on normal n: T_ij = sigma_jk n_k */
    for (int i = 0; i < 3; ++i) {
        cplx div = dU[i][0][0] + dU[i][1][1] + dU[i][2][2];
        for (int j = 0; j < 3; ++j) {
            cplx t = m->lam * div * n[j];
            for (int k = 0; k < 3; ++k)
                t += m->mu * (dU[i][j][k] + dU[i][k][j]) * n[k];
            T[i * 3 + j] = t;
        }
    }
}

/* static strongly singular part of T on a flat element through x (r.n = 0):
 * T0_ij = beta^2 / (4 pi r^2) (rh_i n_j - rh_j n_i) */
static void static_T0(const material_t *m, const double x[3], const double y[3], const double n[3],
                      cplx T0[9])
{
    double rv[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double r2 = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
    double r = sqrt(r2);
    double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double c = m->beta * m->beta / (4.0 * ORC_PI * r2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T0[i * 3 + j] = c * (rh[i] * n[j] - rh[j] * n[i]);
}

/* ------------------------------------------------------------------------- */
/* geometry and quadrature rules                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
    double p[3][3];
    double n[3];
    double area;
    double c[3];
    double h;
} tri_t;

static void tri_make(tri_t *t, const double *a, const double *b, const double *cc)
{
    for (int k = 0; k < 3; ++k) {
        t->p[0][k] = a[k];
        t->p[1][k] = b[k];
        t->p[2][k] = cc[k];
    }
    double e1[3], e2[3], cr[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = cc[k] - a[k];
        t->c[k] = (a[k] + b[k] + cc[k]) / 3.0;
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    t->area = 0.5 * len;
    for (int k = 0; k < 3; ++k)
        t->n[k] = cr[k] / len;
    double h = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *u = t->p[e], *v = t->p[(e + 1) % 3];
        double d = sqrt((u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) +
                        (u[2] - v[2]) * (u[2] - v[2]));
        if (d > h)
            h = d;
    }
    t->h = h;
}

/* 7-point degree-5 rule on the triangle (barycentric coordinates, weights
 * normalised to sum 1): centroid 9/40; (a,a,1-2a) with a = (6 -+ sqrt15)/21
 * and weights (155 -+ sqrt15)/1200. */
static void radon7(double bary[7][3], double w[7])
{
    double r15 = sqrt(15.0);
    double a1 = (6.0 - r15) / 21.0, w1 = (155.0 - r15) / 1200.0;
    double a2 = (6.0 + r15) / 21.0, w2 = (155.0 + r15) / 1200.0;
    double third = 1.0 / 3.0;
    bary[0][0] = bary[0][1] = bary[0][2] = third;
    w[0] = 9.0 / 40.0;
    double as[2] = {a1, a2}, ws[2] = {w1, w2};
    int q = 1;
    for (int g = 0; g < 2; ++g)
        for (int k = 0; k < 3; ++k) {
            bary[q][0] = bary[q][1] = bary[q][2] = as[g];
            bary[q][k] = 1.0 - 2.0 * as[g];
            w[q] = ws[g];
            ++q;
        }
}

/* Gauss-Legendre nodes and weights on [-1,1] by Newton iteration on P_n. */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        /* recompute derivative at the converged node */
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

typedef struct {
    double far_ratio;
    int max_subdiv;
    int n_theta, n_rho;
} policy_t;

static policy_t make_policy(const double pol[4])
{
    policy_t p;
    p.far_ratio = pol[0];
    p.max_subdiv = (int)pol[1];
    p.n_theta = (int)pol[2];
    p.n_rho = (int)pol[3];
    return p;
}

/* ------------------------------------------------------------------------- */
/* element integrals                                                          */
/* ------------------------------------------------------------------------- */
/* regular or nearly singular element: 7-point rule, with recursive 4-way
 * midpoint subdivision while |x - centroid| < far_ratio * longest edge. */
static void integrate_regular(const tri_t *t, const double x[3], cplx s, const material_t *m,
                              const policy_t *pol, int depth, int mode, cplx G[9], cplx H[9])
{
    double dx = x[0] - t->c[0], dy = x[1] - t->c[1], dz = x[2] - t->c[2];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (d < pol->far_ratio * t->h && depth < pol->max_subdiv) {
        double m01[3], m12[3], m20[3];
        for (int k = 0; k < 3; ++k) {
            m01[k] = 0.5 * (t->p[0][k] + t->p[1][k]);
            m12[k] = 0.5 * (t->p[1][k] + t->p[2][k]);
            m20[k] = 0.5 * (t->p[2][k] + t->p[0][k]);
        }
        tri_t ch[4];
        tri_make(&ch[0], t->p[0], m01, m20);
        tri_make(&ch[1], m01, t->p[1], m12);
        tri_make(&ch[2], m20, m12, t->p[2]);
        tri_make(&ch[3], m01, m12, m20);
        for (int c = 0; c < 4; ++c) {
            /* children inherit the parent's exact normal */
            memcpy(ch[c].n, t->n, sizeof t->n);
            integrate_regular(&ch[c], x, s, m, pol, depth + 1, mode, G, H);
        }
        return;
    }
    double bary[7][3], w[7];
    radon7(bary, w);
    for (int q = 0; q < 7; ++q) {
        double y[3];
        for (int k = 0; k < 3; ++k)
            y[k] = bary[q][0] * t->p[0][k] + bary[q][1] * t->p[1][k] + bary[q][2] * t->p[2][k];
        cplx U[9], T[9];
        kernel_UT(s, m, x, y, t->n, mode, U, H ? T : NULL);
        double wq = w[q] * t->area;
        for (int e = 0; e < 9; ++e) {
            G[e] += wq * U[e];
            if (H)
                H[e] += wq * T[e];
        }
    }
}

/* self element, collocation point at its centroid: polar coordinates about x
 * over the three sub-triangles (x, P_a, P_b).  U: rho*U is bounded, direct
 * Gauss-Legendre in (theta, rho).  T: T - T0 is bounded and integrated the same
 * way; the principal value of T0 over a circular exclusion is
 *   beta^2/(4 pi) int_0^{2pi} (e_i(theta) n_j - e_j(theta) n_i) ln R(theta) dtheta,
 * the ln(epsilon) term vanishing because e(theta) integrates to zero. */
static void integrate_self(const tri_t *t, cplx s, const material_t *m, const policy_t *pol,
                           int mode, cplx G[9], cplx H[9])
{
    const double *x = t->c;
    const double *n = t->n;
    double e1[3], e2[3];
    double l0 = 0.0;
    for (int k = 0; k < 3; ++k) {
        e1[k] = t->p[0][k] - x[k];
        l0 += e1[k] * e1[k];
    }
    l0 = sqrt(l0);
    for (int k = 0; k < 3; ++k)
        e1[k] /= l0;
    e2[0] = n[1] * e1[2] - n[2] * e1[1];
    e2[1] = n[2] * e1[0] - n[0] * e1[2];
    e2[2] = n[0] * e1[1] - n[1] * e1[0];

    double *gt = malloc(sizeof(double) * 2 * pol->n_theta);
    double *gr = malloc(sizeof(double) * 2 * pol->n_rho);
    gauss_legendre(pol->n_theta, gt, gt + pol->n_theta);
    gauss_legendre(pol->n_rho, gr, gr + pol->n_rho);
    double cpv = m->beta * m->beta / (4.0 * ORC_PI);

    for (int e = 0; e < 3; ++e) {
        const double *pa = t->p[e], *pb = t->p[(e + 1) % 3];
        double va[3], vb[3];
        for (int k = 0; k < 3; ++k) {
            va[k] = pa[k] - x[k];
            vb[k] = pb[k] - x[k];
        }
        double ta = atan2(va[0] * e2[0] + va[1] * e2[1] + va[2] * e2[2],
                          va[0] * e1[0] + va[1] * e1[1] + va[2] * e1[2]);
        double tb = atan2(vb[0] * e2[0] + vb[1] * e2[1] + vb[2] * e2[2],
                          vb[0] * e1[0] + vb[1] * e1[1] + vb[2] * e1[2]);
        if (tb < ta)
            tb += 2.0 * ORC_PI;
        /* foot of the perpendicular from x to the edge line */
        double ed[3], ee = 0.0, ve = 0.0;
        for (int k = 0; k < 3; ++k) {
            ed[k] = vb[k] - va[k];
            ee += ed[k] * ed[k];
            ve += va[k] * ed[k];
        }
        double tt = -ve / ee, foot[3], pp = 0.0;
        for (int k = 0; k < 3; ++k) {
            foot[k] = va[k] + tt * ed[k];
            pp += foot[k] * foot[k];
        }
        pp = sqrt(pp);
        double phi0 = atan2(foot[0] * e2[0] + foot[1] * e2[1] + foot[2] * e2[2],
                            foot[0] * e1[0] + foot[1] * e1[1] + foot[2] * e1[2]);
        for (int it = 0; it < pol->n_theta; ++it) {
            double th = ta + 0.5 * (tb - ta) * (1.0 + gt[it]);
            double wth = 0.5 * (tb - ta) * gt[pol->n_theta + it];
            double R = pp / cos(th - phi0);
            double eh[3];
            for (int k = 0; k < 3; ++k)
                eh[k] = cos(th) * e1[k] + sin(th) * e2[k];
            for (int ir = 0; ir < pol->n_rho; ++ir) {
                double rho = 0.5 * R * (1.0 + gr[ir]);
                double wr = 0.5 * R * gr[pol->n_rho + ir];
                double y[3];
                for (int k = 0; k < 3; ++k)
                    y[k] = x[k] + rho * eh[k];
                cplx U[9], T[9], T0[9];
                kernel_UT(s, m, x, y, n, mode, U, T);
                static_T0(m, x, y, n, T0);
                double wq = wth * wr * rho;
                for (int q = 0; q < 9; ++q) {
                    G[q] += wq * U[q];
                    H[q] += wq * (T[q] - T0[q]);
                }
            }
            double lr = log(R);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    H[i * 3 + j] += wth * cpv * (eh[i] * n[j] - eh[j] * n[i]) * lr;
        }
    }
    free(gt);
    free(gr);
}

/* G_mn and H_mn (free term included when m == n) */
static void element_blocks(const tri_t *tris, int64_t m, int64_t nidx, cplx s, const material_t *mat,
                           const policy_t *pol, int mode, cplx G[9], cplx H[9])
{
    for (int e = 0; e < 9; ++e)
        G[e] = H[e] = 0.0;
    if (m == nidx) {
        integrate_self(&tris[m], s, mat, pol, mode, G, H);
        H[0] += 0.5;
        H[4] += 0.5;
        H[8] += 0.5;
    } else {
        integrate_regular(&tris[nidx], tris[m].c, s, mat, pol, 0, mode, G, H);
    }
}

static tri_t *build_tris(const double *xyz, int64_t nt, const int32_t *tri)
{
    tri_t *t = malloc(sizeof(tri_t) * (size_t)nt);
    for (int64_t e = 0; e < nt; ++e)
        tri_make(&t[e], xyz + 3 * tri[3 * e], xyz + 3 * tri[3 * e + 1], xyz + 3 * tri[3 * e + 2]);
    return t;
}

/* ========================================================================= */
/* exported entry points (ctypes)                                             */
/* complex values are interleaved (re, im) doubles.                           */
/* ========================================================================= */

int orc_radial(double xr, double xi, double beta, int mode, double out[8])
{
    cplx f[4];
    radial(xr + I * xi, beta, mode, f);
    for (int k = 0; k < 4; ++k) {
        out[2 * k] = creal(f[k]);
        out[2 * k + 1] = cimag(f[k]);
    }
    return 0;
}

int orc_kernel(double sr, double si, const double mat[3], const double x[3], const double y[3],
               const double n[3], int mode, double U_out[18], double T_out[18])
{
    material_t m = make_material(mat);
    cplx U[9], T[9];
    kernel_UT(sr + I * si, &m, x, y, n, mode, U, T);
    for (int e = 0; e < 9; ++e) {
        U_out[2 * e] = creal(U[e]);
        U_out[2 * e + 1] = cimag(U[e]);
        T_out[2 * e] = creal(T[e]);
        T_out[2 * e + 1] = cimag(T[e]);
    }
    return 0;
}

int orc_radon7(double bary[21], double w[7])
{
    double b[7][3];
    radon7(b, w);
    memcpy(bary, b, sizeof b);
    return 0;
}

int orc_gauss_legendre(int n, double *x, double *w)
{
    double *tmp = malloc(sizeof(double) * 2 * n);
    gauss_legendre(n, tmp, tmp + n);
    memcpy(x, tmp, sizeof(double) * n);
    memcpy(w, tmp + n, sizeof(double) * n);
    free(tmp);
    return 0;
}

/* geometry per element: centroid (3), normal (3), area, longest edge */
int orc_geometry(const double *xyz, int64_t nt, const int32_t *tri, double *out8)
{
    tri_t *t = build_tris(xyz, nt, tri);
    for (int64_t e = 0; e < nt; ++e) {
        double *o = out8 + 8 * e;
        for (int k = 0; k < 3; ++k) {
            o[k] = t[e].c[k];
            o[3 + k] = t[e].n[k];
        }
        o[6] = t[e].area;
        o[7] = t[e].h;
    }
    free(t);
    return 0;
}

/* blocks G_mn, H_mn for a list of (m, n) pairs */
int orc_blocks(const double *xyz, int64_t nt, const int32_t *tri, double sr, double si,
               const double mat[3], const double pol[4], int64_t npairs, const int64_t *pairs,
               double *G_out, double *H_out)
{
    tri_t *t = build_tris(xyz, nt, tri);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
    cplx s = sr + I * si;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < npairs; ++k) {
        cplx G[9], H[9];
        element_blocks(t, pairs[2 * k], pairs[2 * k + 1], s, &m, &p, 0, G, H);
        for (int e = 0; e < 9; ++e) {
            G_out[18 * k + 2 * e] = creal(G[e]);
            G_out[18 * k + 2 * e + 1] = cimag(G[e]);
            H_out[18 * k + 2 * e] = creal(H[e]);
            H_out[18 * k + 2 * e + 1] = cimag(H[e]);
        }
    }
    free(t);
    return 0;
}

/* Rows of the collocation system for the listed row elements (all elements
 * when rows == NULL): A_out is [nrows*3][3*nt] complex row-major, b_out is
 * [nrows*3] complex.  bc_val is [nt][3] complex: the prescribed traction
 * (kind 0) or displacement (kind 1) at this s. */
int orc_assemble_rows(const double *xyz, int64_t nt, const int32_t *tri, const int8_t *bc_kind,
                      const double *bc_val, double sr, double si, const double mat[3],
                      const double pol[4], int64_t nrows, const int64_t *rows, double *A_out,
                      double *b_out)
{
    tri_t *t = build_tris(xyz, nt, tri);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
    cplx s = sr + I * si;
    int64_t N = 3 * nt;
    if (!rows)
        nrows = nt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t me = rows ? rows[r] : r;
        cplx b[3] = {0, 0, 0};
        for (int64_t ne = 0; ne < nt; ++ne) {
            cplx G[9], H[9];
            element_blocks(t, me, ne, s, &m, &p, 0, G, H);
            const double *v = bc_val + 6 * ne;
            cplx val[3] = {v[0] + I * v[1], v[2] + I * v[3], v[4] + I * v[5]};
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) {
                    cplx a, rhs;
                    if (bc_kind[ne] == 0) { /* traction known: u unknown */
                        a = H[i * 3 + j];
                        rhs = G[i * 3 + j] * val[j];
                    } else {                /* displacement known: t unknown */
                        a = -G[i * 3 + j];
                        rhs = -H[i * 3 + j] * val[j];
                    }
                    b[i] += rhs;
                    double *dst = A_out + 2 * ((3 * r + i) * N + 3 * ne + j);
                    dst[0] = creal(a);
                    dst[1] = cimag(a);
                }
            }
        }
        for (int i = 0; i < 3; ++i) {
            b_out[2 * (3 * r + i)] = creal(b[i]);
            b_out[2 * (3 * r + i) + 1] = cimag(b[i]);
        }
    }
    free(t);
    return 0;
}

/* Static (s = 0) row sums of H for every collocation row block:
 * out[m][i][j] = sum_n H_mn,ij (real).  Rigid-body translation gives I for an
 * exterior (unbounded) domain and 0 for a bounded one. */
int orc_rowsum_H_static(const double *xyz, int64_t nt, const int32_t *tri, const double mat[3],
                        const double pol[4], double *out9)
{
    tri_t *t = build_tris(xyz, nt, tri);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t me = 0; me < nt; ++me) {
        double acc[9] = {0};
        for (int64_t ne = 0; ne < nt; ++ne) {
            cplx G[9], H[9];
            element_blocks(t, me, ne, 0.0, &m, &p, 0, G, H);
            for (int e = 0; e < 9; ++e)
                acc[e] += creal(H[e]);
        }
        memcpy(out9 + 9 * me, acc, sizeof acc);
    }
    free(t);
    return 0;
}

/* ========================================================================= */
/* Curved quadratic triangles, locally-corrected Nystrom discretisation      */
/* (paper Section 2.1: six-node elements; the unknowns sit at the points of  */
/* the 6-point Gauss rule, n_k = 6 n_e; nearly singular integrals by         */
/* recursive subdivision, singular ones in polar coordinates).               */
/*                                                                           */
/* Element map x(xi, eta) = sum_k N_k(xi, eta) P_k on the reference triangle */
/* {xi, eta >= 0, xi + eta <= 1}; P0, P1, P2 corners, P3 on edge 01, P4 on   */
/* edge 12, P5 on edge 20; normal (x_xi x x_eta) / J, J = |x_xi x x_eta|.    */
/* Unknown q of element e (index 6 e + q) sits at rule point q.  Block of    */
/* target node i (point x_i on element e_i) and node q of element e:         */
/*   far  (|x_i - x_e(1/3, 1/3)| >= far_ratio h_e, h_e the longest corner    */
/*         chord): w_q J_q K(x_i, y_q) (the rule itself);                    */
/*   near: int_e K(x_i, y) L_q dG, recursive 4-way subdivision of the        */
/*         parameter triangle with the same test on each piece's image, the  */
/*         7-point rule on the leaves (locally corrected weights);           */
/*   self (e = e_i): polar coordinates about the node in the parameter plane */
/*         (three sub-triangles, each split at the foot of the perpendicular */
/*         to its edge, Gauss-Legendre n_theta x n_rho per half); for T the  */
/*         leading rho^-1 term of the node's own basis function is removed   */
/*         and restored as a principal value over a circular exclusion;      */
/*         1/2 I added to the node's own block.                              */
/* L_q: the quadratic interpolant through the six rule points.               */
/* ========================================================================= */

/* 6-point degree-4 rule on the triangle, closed forms of its two orbits.
 * Point q: orbit g = q / 3 (a, then b); barycentric (l0, l1, l2) all equal to
 * the orbit's value except l_{q % 3} = 1 - 2 * value; (xi, eta) = (l1, l2);
 * weights include the reference area 1/2. */
static void gauss6(double pt[6][2], double w[6])
{
    double s10 = sqrt(10.0);
    double r = sqrt(38.0 - 44.0 * sqrt(0.4));
    double q = sqrt(213125.0 - 53320.0 * s10);
    double val[2] = {(8.0 - s10 + r) / 18.0, (8.0 - s10 - r) / 18.0};
    double wt[2] = {(620.0 + q) / 3720.0, (620.0 - q) / 3720.0};
    for (int g = 0; g < 2; ++g)
        for (int k = 0; k < 3; ++k) {
            double l[3] = {val[g], val[g], val[g]};
            l[k] = 1.0 - 2.0 * val[g];
            pt[3 * g + k][0] = l[1];
            pt[3 * g + k][1] = l[2];
            w[3 * g + k] = 0.5 * wt[g];
        }
}

static void mono6(double xi, double eta, double m[6])
{
    m[0] = 1.0;
    m[1] = xi;
    m[2] = eta;
    m[3] = xi * xi;
    m[4] = xi * eta;
    m[5] = eta * eta;
}

/* Lagrange basis on the rule points: L_b = sum_k C[b][k] m_k with
 * L_b(pt_c) = delta_bc, i.e. C = (V^-1)^T, V[c][k] = m_k(pt_c); Gauss-Jordan
 * elimination with partial pivoting. */
static void lagrange6(const double pt[6][2], double C[6][6])
{
    double M[6][12];
    for (int c = 0; c < 6; ++c) {
        mono6(pt[c][0], pt[c][1], M[c]);
        for (int k = 0; k < 6; ++k)
            M[c][6 + k] = (c == k) ? 1.0 : 0.0;
    }
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        for (int r = col + 1; r < 6; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col]))
                piv = r;
        for (int k = 0; k < 12; ++k) {
            double t = M[col][k];
            M[col][k] = M[piv][k];
            M[piv][k] = t;
        }
        double d = M[col][col];
        for (int k = 0; k < 12; ++k)
            M[col][k] /= d;
        for (int r = 0; r < 6; ++r) {
            if (r == col)
                continue;
            double f = M[r][col];
            for (int k = 0; k < 12; ++k)
                M[r][k] -= f * M[col][k];
        }
    }
    /* M[:, 6:] = V^-1 */
    for (int b = 0; b < 6; ++b)
        for (int k = 0; k < 6; ++k)
            C[b][k] = M[k][6 + b];
}

static void lag_eval(const double C[6][6], double xi, double eta, double L[6])
{
    double m[6];
    mono6(xi, eta, m);
    for (int b = 0; b < 6; ++b) {
        L[b] = 0.0;
        for (int k = 0; k < 6; ++k)
            L[b] += C[b][k] * m[k];
    }
}

/* quadratic map: point, unit normal, Jacobian, tangent vectors */
static void q6_map(const double P[6][3], double xi, double eta, double y[3], double n[3], double *J,
                   double dxi[3], double deta[3])
{
    double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
    double N[6] = {l0 * (2.0 * l0 - 1.0), l1 * (2.0 * l1 - 1.0), l2 * (2.0 * l2 - 1.0),
                   4.0 * l0 * l1, 4.0 * l1 * l2, 4.0 * l2 * l0};
    double Nx[6] = {-(4.0 * l0 - 1.0), 4.0 * l1 - 1.0, 0.0, 4.0 * (l0 - l1), 4.0 * l2, -4.0 * l2};
    double Ne[6] = {-(4.0 * l0 - 1.0), 0.0, 4.0 * l2 - 1.0, -4.0 * l1, 4.0 * l1, 4.0 * (l0 - l2)};
    for (int k = 0; k < 3; ++k) {
        y[k] = dxi[k] = deta[k] = 0.0;
        for (int a = 0; a < 6; ++a) {
            y[k] += N[a] * P[a][k];
            dxi[k] += Nx[a] * P[a][k];
            deta[k] += Ne[a] * P[a][k];
        }
    }
    double cr[3] = {dxi[1] * deta[2] - dxi[2] * deta[1], dxi[2] * deta[0] - dxi[0] * deta[2],
                    dxi[0] * deta[1] - dxi[1] * deta[0]};
    *J = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int k = 0; k < 3; ++k)
        n[k] = cr[k] / *J;
}

typedef struct {
    double P[6][3];
    double c[3];   /* x(1/3, 1/3) */
    double h;      /* longest chord between the corners */
} q6_t;

static void q6_make(q6_t *e, const double *xyz, const int32_t *t6)
{
    for (int a = 0; a < 6; ++a)
        for (int k = 0; k < 3; ++k)
            e->P[a][k] = xyz[3 * t6[a] + k];
    double n[3], J, d1[3], d2[3];
    q6_map(e->P, 1.0 / 3.0, 1.0 / 3.0, e->c, n, &J, d1, d2);
    double h = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double *u = e->P[a], *v = e->P[(a + 1) % 3];
        double d = sqrt((u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) + (u[2] - v[2]) * (u[2] - v[2]));
        if (d > h)
            h = d;
    }
    e->h = h;
}

static q6_t *build_q6(const double *xyz, int64_t nt, const int32_t *tri6)
{
    q6_t *e = malloc(sizeof(q6_t) * (size_t)nt);
    for (int64_t k = 0; k < nt; ++k)
        q6_make(&e[k], xyz, tri6 + 6 * k);
    return e;
}

static double dist3(const double a[3], const double b[3])
{
    return sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
}

/* int over the parameter sub-triangle q of K(x, y) L_b J, b = 0..5 */
static void nys_regular(const q6_t *e, const double C[6][6], const double x[3], const double q[3][2], cplx s,
                        const material_t *m, const policy_t *pol, int depth, cplx G[6][9], cplx H[6][9])
{
    double Y[3][3], yc[3], nn[3], J, d1[3], d2[3];
    for (int k = 0; k < 3; ++k)
        q6_map(e->P, q[k][0], q[k][1], Y[k], nn, &J, d1, d2);
    q6_map(e->P, (q[0][0] + q[1][0] + q[2][0]) / 3.0, (q[0][1] + q[1][1] + q[2][1]) / 3.0, yc, nn, &J, d1, d2);
    double h = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = dist3(Y[k], Y[(k + 1) % 3]);
        if (d > h)
            h = d;
    }
    if (dist3(x, yc) < pol->far_ratio * h && depth < pol->max_subdiv) {
        double m01[2] = {0.5 * (q[0][0] + q[1][0]), 0.5 * (q[0][1] + q[1][1])};
        double m12[2] = {0.5 * (q[1][0] + q[2][0]), 0.5 * (q[1][1] + q[2][1])};
        double m20[2] = {0.5 * (q[2][0] + q[0][0]), 0.5 * (q[2][1] + q[0][1])};
        double ch[4][3][2] = {{{q[0][0], q[0][1]}, {m01[0], m01[1]}, {m20[0], m20[1]}},
                              {{m01[0], m01[1]}, {q[1][0], q[1][1]}, {m12[0], m12[1]}},
                              {{m20[0], m20[1]}, {m12[0], m12[1]}, {q[2][0], q[2][1]}},
                              {{m01[0], m01[1]}, {m12[0], m12[1]}, {m20[0], m20[1]}}};
        for (int c = 0; c < 4; ++c)
            nys_regular(e, C, x, (const double(*)[2])ch[c], s, m, pol, depth + 1, G, H);
        return;
    }
    double bary[7][3], w7[7];
    radon7(bary, w7);
    double area = 0.5 * fabs((q[1][0] - q[0][0]) * (q[2][1] - q[0][1]) - (q[2][0] - q[0][0]) * (q[1][1] - q[0][1]));
    for (int p = 0; p < 7; ++p) {
        double xi = bary[p][0] * q[0][0] + bary[p][1] * q[1][0] + bary[p][2] * q[2][0];
        double eta = bary[p][0] * q[0][1] + bary[p][1] * q[1][1] + bary[p][2] * q[2][1];
        double y[3], n[3], Jy, a1[3], a2[3], L[6];
        q6_map(e->P, xi, eta, y, n, &Jy, a1, a2);
        lag_eval(C, xi, eta, L);
        cplx U[9], T[9];
        kernel_UT(s, m, x, y, n, 0, U, T);
        double w = w7[p] * area * Jy;
        for (int b = 0; b < 6; ++b)
            for (int k = 0; k < 9; ++k) {
                G[b][k] += w * L[b] * U[k];
                H[b][k] += w * L[b] * T[k];
            }
    }
}

/* self element, target at rule point b0 of the element */
static void nys_self(const q6_t *e, const double C[6][6], const double pt[6][2], int b0, cplx s, const material_t *m,
                     const policy_t *pol, cplx G[6][9], cplx H[6][9])
{
    double xi0 = pt[b0][0], eta0 = pt[b0][1];
    double x[3], n0[3], J0, a1[3], a2[3];
    q6_map(e->P, xi0, eta0, x, n0, &J0, a1, a2);
    double *gt = malloc(sizeof(double) * 2 * pol->n_theta);
    double *gr = malloc(sizeof(double) * 2 * pol->n_rho);
    gauss_legendre(pol->n_theta, gt, gt + pol->n_theta);
    gauss_legendre(pol->n_rho, gr, gr + pol->n_rho);
    const double V[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    for (int k = 0; k < 3; ++k) {
        double va[2] = {V[k][0] - xi0, V[k][1] - eta0};
        double vb[2] = {V[(k + 1) % 3][0] - xi0, V[(k + 1) % 3][1] - eta0};
        double ta = atan2(va[1], va[0]), tb = atan2(vb[1], vb[0]);
        if (tb < ta)
            tb += 2.0 * ORC_PI;
        double ed[2] = {vb[0] - va[0], vb[1] - va[1]};
        double tt = -(va[0] * ed[0] + va[1] * ed[1]) / (ed[0] * ed[0] + ed[1] * ed[1]);
        double foot[2] = {va[0] + tt * ed[0], va[1] + tt * ed[1]};
        double p = sqrt(foot[0] * foot[0] + foot[1] * foot[1]);
        double phi = atan2(foot[1], foot[0]);
        while (phi < ta)
            phi += 2.0 * ORC_PI;
        double lim[3] = {ta, phi, tb};
        for (int half = 0; half < 2; ++half) {
            double t0 = lim[half], t1 = lim[half + 1];
            for (int it = 0; it < pol->n_theta; ++it) {
                double th = t0 + 0.5 * (t1 - t0) * (1.0 + gt[it]);
                double wth = 0.5 * (t1 - t0) * gt[pol->n_theta + it];
                double R = p / cos(th - phi);
                double c = cos(th), sn = sin(th);
                double A[3], xa[3];
                for (int d = 0; d < 3; ++d) {
                    A[d] = a1[d] * c + a2[d] * sn;
                    xa[d] = x[d] + A[d];
                }
                double Alen = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
                cplx F1[9];
                static_T0(m, x, xa, n0, F1);
                for (int q = 0; q < 9; ++q)
                    F1[q] *= J0;
                for (int ir = 0; ir < pol->n_rho; ++ir) {
                    double rho = 0.5 * R * (1.0 + gr[ir]);
                    double wr = 0.5 * R * gr[pol->n_rho + ir];
                    double xi = xi0 + rho * c, eta = eta0 + rho * sn;
                    double y[3], n[3], Jy, d1[3], d2[3], L[6];
                    q6_map(e->P, xi, eta, y, n, &Jy, d1, d2);
                    lag_eval(C, xi, eta, L);
                    cplx U[9], T[9];
                    kernel_UT(s, m, x, y, n, 0, U, T);
                    double w = wth * wr * rho * Jy;
                    for (int b = 0; b < 6; ++b)
                        for (int q = 0; q < 9; ++q) {
                            G[b][q] += w * L[b] * U[q];
                            H[b][q] += w * L[b] * T[q];
                        }
                    for (int q = 0; q < 9; ++q)
                        H[b0][q] -= wth * wr / rho * F1[q];
                }
                double lr = log(R * Alen);
                for (int q = 0; q < 9; ++q)
                    H[b0][q] += wth * F1[q] * lr;
            }
        }
    }
    H[b0][0] += 0.5;
    H[b0][4] += 0.5;
    H[b0][8] += 0.5;
    free(gt);
    free(gr);
}

/* G, H blocks of target node i against the six nodes of element e */
static void nys_blocks(const q6_t *els, const double pt[6][2], const double w6[6], const double C[6][6], int64_t i,
                       int64_t e, cplx s, const material_t *m, const policy_t *pol, cplx G[6][9], cplx H[6][9])
{
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q < 9; ++q)
            G[b][q] = H[b][q] = 0.0;
    int64_t ei = i / 6;
    int bi = (int)(i % 6);
    if (e == ei) {
        nys_self(&els[e], C, pt, bi, s, m, pol, G, H);
        return;
    }
    double x[3], nx[3], Jx, d1[3], d2[3];
    q6_map(els[ei].P, pt[bi][0], pt[bi][1], x, nx, &Jx, d1, d2);
    if (dist3(x, els[e].c) < pol->far_ratio * els[e].h) {
        const double ref[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
        nys_regular(&els[e], C, x, ref, s, m, pol, 0, G, H);
        return;
    }
    for (int q = 0; q < 6; ++q) {
        double y[3], n[3], Jy;
        q6_map(els[e].P, pt[q][0], pt[q][1], y, n, &Jy, d1, d2);
        cplx U[9], T[9];
        kernel_UT(s, m, x, y, n, 0, U, T);
        for (int k = 0; k < 9; ++k) {
            G[q][k] = w6[q] * Jy * U[k];
            H[q][k] = w6[q] * Jy * T[k];
        }
    }
}

int orc_gauss6(double pt[12], double w[6])
{
    gauss6((double(*)[2])pt, w);
    return 0;
}

/* C[b][k]: coefficients of L_b on (1, xi, eta, xi^2, xi eta, eta^2) */
int orc_lagrange6(double C[36])
{
    double pt[6][2], w[6];
    gauss6(pt, w);
    lagrange6(pt, (double(*)[6])C);
    return 0;
}

/* out8 per parameter point: y(3), n(3), J, 0 */
int orc_q6_map(const double P18[18], int64_t n_pts, const double *xieta, double *out8)
{
    for (int64_t k = 0; k < n_pts; ++k) {
        double d1[3], d2[3];
        q6_map((const double(*)[3])P18, xieta[2 * k], xieta[2 * k + 1], out8 + 8 * k, out8 + 8 * k + 3,
               out8 + 8 * k + 6, d1, d2);
        out8[8 * k + 7] = 0.0;
    }
    return 0;
}

/* Nystrom nodes: out8[6 e + q] = y(3), n(3), w_q J_q, 0 */
int orc_nys_nodes(const double *xyz, int64_t nt, const int32_t *tri6, double *out8)
{
    double pt[6][2], w6[6];
    gauss6(pt, w6);
    q6_t *els = build_q6(xyz, nt, tri6);
    for (int64_t e = 0; e < nt; ++e)
        for (int q = 0; q < 6; ++q) {
            double *o = out8 + 8 * (6 * e + q), d1[3], d2[3], J;
            q6_map(els[e].P, pt[q][0], pt[q][1], o, o + 3, &J, d1, d2);
            o[6] = w6[q] * J;
            o[7] = 0.0;
        }
    free(els);
    return 0;
}

/* one element's six G, H blocks seen from an arbitrary point x: the self
 * rule about rule point b0 when b0 >= 0, else the subdivision rule (which
 * takes the 7-point rule on the whole element when x is far) */
int orc_nys_element(const double P18[18], const double x[3], int b0, double sr, double si, const double mat[3],
                    const double pol[4], double *G_out, double *H_out)
{
    q6_t e;
    memcpy(e.P, P18, sizeof e.P);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
    double pt[6][2], w6[6], C[6][6];
    gauss6(pt, w6);
    lagrange6(pt, C);
    cplx G[6][9], H[6][9];
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q < 9; ++q)
            G[b][q] = H[b][q] = 0.0;
    if (b0 >= 0) {
        nys_self(&e, C, pt, b0, sr + I * si, &m, &p, G, H);
    } else {
        const double ref[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
        nys_regular(&e, C, x, ref, sr + I * si, &m, &p, 0, G, H);
    }
    for (int b = 0; b < 6; ++b)
        for (int q = 0; q < 9; ++q) {
            G_out[18 * b + 2 * q] = creal(G[b][q]);
            G_out[18 * b + 2 * q + 1] = cimag(G[b][q]);
            H_out[18 * b + 2 * q] = creal(H[b][q]);
            H_out[18 * b + 2 * q + 1] = cimag(H[b][q]);
        }
    return 0;
}

/* Rows of the Nystrom system for the listed target nodes (all when rows is
 * NULL): A_out [3 nrows][3 n_k] complex row-major, b_out [3 nrows];
 * bc_val [n_k][3] complex, the prescribed value at each node (kind per
 * element: 0 traction prescribed, 1 displacement prescribed). */
int orc_nys_assemble_rows(const double *xyz, int64_t nt, const int32_t *tri6, const int8_t *bc_kind,
                          const double *bc_val, double sr, double si, const double mat[3], const double pol[4],
                          int64_t nrows, const int64_t *rows, double *A_out, double *b_out)
{
    q6_t *els = build_q6(xyz, nt, tri6);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
    double pt[6][2], w6[6], C[6][6];
    gauss6(pt, w6);
    lagrange6(pt, C);
    cplx s = sr + I * si;
    int64_t nk = 6 * nt, N = 3 * nk;
    if (!rows)
        nrows = nk;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        cplx b[3] = {0, 0, 0};
        for (int64_t e = 0; e < nt; ++e) {
            cplx G[6][9], H[6][9];
            nys_blocks(els, pt, w6, C, i, e, s, &m, &p, G, H);
            for (int q = 0; q < 6; ++q) {
                int64_t j = 6 * e + q;
                const double *v = bc_val + 6 * j;
                cplx val[3] = {v[0] + I * v[1], v[2] + I * v[3], v[4] + I * v[5]};
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) {
                        cplx av, rhs;
                        if (bc_kind[e] == 0) {
                            av = H[q][3 * a + c];
                            rhs = G[q][3 * a + c] * val[c];
                        } else {
                            av = -G[q][3 * a + c];
                            rhs = -H[q][3 * a + c] * val[c];
                        }
                        b[a] += rhs;
                        double *dst = A_out + 2 * ((3 * r + a) * N + 3 * j + c);
                        dst[0] = creal(av);
                        dst[1] = cimag(av);
                    }
            }
        }
        for (int a = 0; a < 3; ++a) {
            b_out[2 * (3 * r + a)] = creal(b[a]);
            b_out[2 * (3 * r + a) + 1] = cimag(b[a]);
        }
    }
    free(els);
    return 0;
}

/* static (s = 0) row sums of H over all nodes for every target node */
int orc_nys_rowsum_H_static(const double *xyz, int64_t nt, const int32_t *tri6, const double mat[3],
                            const double pol[4], double *out9)
{
    q6_t *els = build_q6(xyz, nt, tri6);
    material_t m = make_material(mat);
    policy_t p = make_policy(pol);
    double pt[6][2], w6[6], C[6][6];
    gauss6(pt, w6);
    lagrange6(pt, C);
    int64_t nk = 6 * nt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nk; ++i) {
        double acc[9] = {0};
        for (int64_t e = 0; e < nt; ++e) {
            cplx G[6][9], H[6][9];
            nys_blocks(els, pt, w6, C, i, e, 0.0, &m, &p, G, H);
            for (int q = 0; q < 6; ++q)
                for (int k = 0; k < 9; ++k)
                    acc[k] += creal(H[q][k]);
        }
        memcpy(out9 + 9 * i, acc, sizeof acc);
    }
    free(els);
    return 0;
}
