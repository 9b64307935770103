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
