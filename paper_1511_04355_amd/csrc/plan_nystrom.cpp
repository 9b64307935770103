// s-independent plan of the locally-corrected Nystrom discretisation on
// curved six-node triangles (paper Section 2.1: quadratic elements, the points
// of the 6-point Gauss rule as the unknowns, n_k = 6 n_e; nearly singular
// integrals by recursive subdivision, singular ones in polar coordinates).
//
// Element map x(xi, eta) = sum_a N_a(xi, eta) P_a over the reference triangle
// {xi, eta >= 0, xi + eta <= 1}: P0..P2 the corners, P3, P4, P5 on edges 01,
// 12, 20.  Unknown-carrying point 6 e + q is rule point q of element e.  For a
// target point x and a source element e:
//  * far (|x - x_e(1/3, 1/3)| >= far_ratio h_e, h_e the longest corner
//    chord): the rule itself, w_q J_q K(x, y_q) -- one source record per point;
//  * near: the corrected weights int_e K(x, y) L_q dG over parameter-plane
//    triangles found by 4-way midpoint subdivision, repeated while a piece's
//    image fails the same test (up to max_subdiv levels), 7-point rule on the
//    leaves;
//  * self: polar coordinates about the point in the parameter plane, the three
//    sub-triangles split at the foot of the perpendicular to their edge; table
//    per rule point of (cos, sin, w_theta, R(theta)).
// L_q is the quadratic interpolant through the six rule points.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "internal.hpp"

namespace afsbem {

namespace {

constexpr double kPi = 3.14159265358979323846;

// 6-point degree-4 rule: orbits (a, a, 1-2a) and (b, b, 1-2b) in barycentric
// coordinates (l0, l1, l2), closed forms; point q: orbit q / 3 with
// l_{q % 3} the odd coordinate; (xi, eta) = (l1, l2); weights carry the area 1/2
void rule6(double pt[12], double w[6]) {
    const double r10 = std::sqrt(10.0);
    const double disc = std::sqrt(38.0 - 44.0 * std::sqrt(0.4));
    const double wd = std::sqrt(213125.0 - 53320.0 * r10);
    const double orbit[2] = {(8.0 - r10 + disc) / 18.0, (8.0 - r10 - disc) / 18.0};
    const double weight[2] = {(620.0 + wd) / 3720.0, (620.0 - wd) / 3720.0};
    for (int q = 0; q < 6; ++q) {
        const double a = orbit[q / 3];
        double l[3] = {a, a, a};
        l[q % 3] = 1.0 - 2.0 * a;
        pt[2 * q] = l[1];
        pt[2 * q + 1] = l[2];
        w[q] = 0.5 * weight[q / 3];
    }
}

// monomials 1, xi, eta, xi^2, xi eta, eta^2
inline void monomials(double xi, double eta, double m[6]) {
    m[0] = 1.0;
    m[1] = xi;
    m[2] = eta;
    m[3] = xi * xi;
    m[4] = xi * eta;
    m[5] = eta * eta;
}

// lag[6 b + k]: coefficients of L_b = sum_k lag[6 b + k] m_k with
// L_b(pt_c) = delta_bc, i.e. lag V^T = I with V[c][k] = m_k(pt_c), so lag is
// the transpose of V^-1.  V^-1 by elimination with partial pivoting on [V | I].
void lagrange_basis(const double pt[12], double lag[36]) {
    double M[6][12];
    for (int c = 0; c < 6; ++c) {
        monomials(pt[2 * c], pt[2 * c + 1], M[c]);
        for (int b = 0; b < 6; ++b)
            M[c][6 + b] = (c == b) ? 1.0 : 0.0;
    }
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        for (int r = col + 1; r < 6; ++r)
            if (std::fabs(M[r][col]) > std::fabs(M[piv][col]))
                piv = r;
        if (piv != col)
            for (int k = 0; k < 12; ++k)
                std::swap(M[col][k], M[piv][k]);
        for (int r = col + 1; r < 6; ++r) {
            const double f = M[r][col] / M[col][col];
            for (int k = col; k < 12; ++k)
                M[r][k] -= f * M[col][k];
        }
    }
    for (int col = 5; col >= 0; --col)
        for (int k = 6; k < 12; ++k) {
            double v = M[col][k];
            for (int j = col + 1; j < 6; ++j)
                v -= M[col][j] * M[j][k];
            M[col][k] = v / M[col][col];
        }
    // M[:, 6:] = V^-1; lag[b][k] = (V^-1)[k][b]
    for (int b = 0; b < 6; ++b)
        for (int k = 0; k < 6; ++k)
            lag[6 * b + k] = M[k][6 + b];
}

struct Pt3 {
    double v[3];
};

inline double dist(const double a[3], const double b[3]) {
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

// point, normal and Jacobian of the quadratic map at (xi, eta)
void qmap(const double *P, double xi, double eta, double y[3], double n[3], double &J) {
    const double l0 = 1.0 - xi - eta, l1 = xi, l2 = eta;
    const double N[6] = {l0 * (2.0 * l0 - 1.0), l1 * (2.0 * l1 - 1.0), l2 * (2.0 * l2 - 1.0),
                         4.0 * l0 * l1,         4.0 * l1 * l2,         4.0 * l2 * l0};
    const double Nx[6] = {-(4.0 * l0 - 1.0), 4.0 * l1 - 1.0, 0.0, 4.0 * (l0 - l1), 4.0 * l2, -4.0 * l2};
    const double Ne[6] = {-(4.0 * l0 - 1.0), 0.0, 4.0 * l2 - 1.0, -4.0 * l1, 4.0 * l1, 4.0 * (l0 - l2)};
    double tx[3], te[3];
    for (int k = 0; k < 3; ++k) {
        y[k] = tx[k] = te[k] = 0.0;
        for (int a = 0; a < 6; ++a) {
            y[k] += N[a] * P[3 * a + k];
            tx[k] += Nx[a] * P[3 * a + k];
            te[k] += Ne[a] * P[3 * a + k];
        }
    }
    const double c[3] = {tx[1] * te[2] - tx[2] * te[1], tx[2] * te[0] - tx[0] * te[2], tx[0] * te[1] - tx[1] * te[0]};
    J = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    for (int k = 0; k < 3; ++k)
        n[k] = c[k] / J;
}

// recursive subdivision of the parameter triangle q (xi, eta pairs) seen
// from x; leaves appended as 6 doubles
void split_leaves(const double *P, const double x[3], const double q[6], double ratio, int depth, int max_depth,
                  std::vector<double> &leaves) {
    double Y[3][3], yc[3], n[3], J;
    for (int k = 0; k < 3; ++k)
        qmap(P, q[2 * k], q[2 * k + 1], Y[k], n, J);
    qmap(P, (q[0] + q[2] + q[4]) / 3.0, (q[1] + q[3] + q[5]) / 3.0, yc, n, J);
    double h = 0.0;
    for (int k = 0; k < 3; ++k)
        h = std::max(h, dist(Y[k], Y[(k + 1) % 3]));
    if (dist(x, yc) < ratio * h && depth < max_depth) {
        const double m01[2] = {0.5 * (q[0] + q[2]), 0.5 * (q[1] + q[3])};
        const double m12[2] = {0.5 * (q[2] + q[4]), 0.5 * (q[3] + q[5])};
        const double m20[2] = {0.5 * (q[4] + q[0]), 0.5 * (q[5] + q[1])};
        const double c0[6] = {q[0], q[1], m01[0], m01[1], m20[0], m20[1]};
        const double c1[6] = {m01[0], m01[1], q[2], q[3], m12[0], m12[1]};
        const double c2[6] = {m20[0], m20[1], m12[0], m12[1], q[4], q[5]};
        const double c3[6] = {m01[0], m01[1], m12[0], m12[1], m20[0], m20[1]};
        split_leaves(P, x, c0, ratio, depth + 1, max_depth, leaves);
        split_leaves(P, x, c1, ratio, depth + 1, max_depth, leaves);
        split_leaves(P, x, c2, ratio, depth + 1, max_depth, leaves);
        split_leaves(P, x, c3, ratio, depth + 1, max_depth, leaves);
        return;
    }
    leaves.insert(leaves.end(), q, q + 6);
}

}  // namespace

void build_plan_nystrom(const double *xyz, int64_t nv, const int32_t *tri6, int64_t n_el, const int8_t *kind,
                        const afsbem_quad_policy &pol, const MaterialDerived &mat, HostPlan &P) {
    (void)nv;
    const int64_t np = 6 * n_el;
    P.disc = 1;
    P.n_el = n_el;
    P.n_tri = np;
    P.n_theta = pol.self_n_theta;
    P.n_rho = pol.self_n_rho;
    double w6[6];
    rule6(P.nys_pt, w6);
    lagrange_basis(P.nys_pt, P.nys_lag);
    P.nys_geom.resize(18 * (size_t)n_el);
    P.cen.resize(3 * (size_t)np);
    P.nrm.resize(3 * (size_t)np);
    P.src.assign(kSrcStride * (size_t)np, 0.0);
    P.kind.resize(np);
    std::vector<Pt3> centre(n_el);
    std::vector<double> hel(n_el);
    for (int64_t e = 0; e < n_el; ++e) {
        double *G = &P.nys_geom[18 * e];
        for (int a = 0; a < 6; ++a)
            for (int k = 0; k < 3; ++k)
                G[3 * a + k] = xyz[3 * (size_t)tri6[6 * e + a] + k];
        double n[3], J;
        qmap(G, 1.0 / 3.0, 1.0 / 3.0, centre[e].v, n, J);
        double h = 0.0;
        for (int a = 0; a < 3; ++a)
            h = std::max(h, dist(&G[3 * a], &G[3 * ((a + 1) % 3)]));
        hel[e] = h;
        for (int q = 0; q < 6; ++q) {
            const int64_t i = 6 * e + q;
            double y[3];
            qmap(G, P.nys_pt[2 * q], P.nys_pt[2 * q + 1], y, n, J);
            AFS_REQUIRE(J > 0.0 && std::isfinite(J), AFSBEM_EINVAL,
                        "degenerate six-node element " + std::to_string(e));
            double *rec = &P.src[kSrcStride * i];
            for (int k = 0; k < 3; ++k) {
                P.cen[3 * i + k] = y[k];
                P.nrm[3 * i + k] = n[k];
                rec[k] = y[k];
                rec[28 + k] = n[k];
            }
            rec[3] = w6[q] * J;
            rec[31] = (double)kind[e];
            P.kind[i] = kind[e];
        }
    }

    // ---- near pairs (target point, element): grid over element centres
    double hmax = 0.0;
    double lo[3] = {1e300, 1e300, 1e300};
    for (int64_t e = 0; e < n_el; ++e) {
        hmax = std::max(hmax, hel[e]);
        for (int k = 0; k < 3; ++k)
            lo[k] = std::min(lo[k], centre[e].v[k]);
    }
    const double cell = std::max(pol.far_ratio * hmax, 1e-300);
    auto cell_of = [&](const double *c, int64_t *ijk) {
        for (int k = 0; k < 3; ++k)
            ijk[k] = (int64_t)std::floor((c[k] - lo[k]) / cell);
    };
    auto key = [](int64_t i, int64_t j, int64_t k) {
        return (uint64_t)((i & 0x1fffff) | ((j & 0x1fffff) << 21) | ((k & 0x1fffff) << 42));
    };
    std::unordered_map<uint64_t, std::vector<int32_t>> grid;
    for (int64_t e = 0; e < n_el; ++e) {
        int64_t c[3];
        cell_of(centre[e].v, c);
        grid[key(c[0], c[1], c[2])].push_back((int32_t)e);
    }
    P.near_ptr.assign(np + 1, 0);
    P.near_col.clear();
    P.near_row.clear();
    P.leaf_ptr.assign(1, 0);
    P.nys_leaves.clear();
    const double ref[6] = {0.0, 0.0, 1.0, 0.0, 0.0, 1.0};
    std::vector<int32_t> cand;
    for (int64_t i = 0; i < np; ++i) {
        const double *x = &P.cen[3 * i];
        const int64_t ei = i / 6;
        cand.clear();
        if (pol.far_ratio > 0.0) {
            int64_t c[3];
            cell_of(x, c);
            for (int64_t a = c[0] - 1; a <= c[0] + 1; ++a)
                for (int64_t b = c[1] - 1; b <= c[1] + 1; ++b)
                    for (int64_t d = c[2] - 1; d <= c[2] + 1; ++d) {
                        auto it = grid.find(key(a, b, d));
                        if (it == grid.end())
                            continue;
                        for (int32_t e : it->second)
                            if (e != ei && dist(x, centre[e].v) < pol.far_ratio * hel[e])
                                cand.push_back(e);
                    }
        }
        std::sort(cand.begin(), cand.end());
        for (int32_t e : cand) {
            P.near_row.push_back((int32_t)i);
            P.near_col.push_back(e);
            split_leaves(&P.nys_geom[18 * (size_t)e], x, ref, pol.far_ratio, 0, pol.max_subdiv, P.nys_leaves);
            P.leaf_ptr.push_back((int64_t)(P.nys_leaves.size() / 6));
        }
        P.near_ptr[i + 1] = (int64_t)P.near_col.size();
    }
    const int64_t nnz = (int64_t)P.near_col.size();
    P.near_order.resize(nnz);
    for (int64_t q = 0; q < nnz; ++q)
        P.near_order[q] = (int32_t)q;
    std::stable_sort(P.near_order.begin(), P.near_order.end(), [&](int32_t a, int32_t b) {
        return P.leaf_ptr[a + 1] - P.leaf_ptr[a] > P.leaf_ptr[b + 1] - P.leaf_ptr[b];
    });

    // ---- polar tables of the self element, per rule point
    const int nth = pol.self_n_theta, nrh = pol.self_n_rho;
    std::vector<double> gx(std::max(nth, nrh)), gw(std::max(nth, nrh));
    gauss_legendre(nrh, gx.data(), gw.data());
    P.gl_rho.resize(2 * nrh);
    for (int i = 0; i < nrh; ++i) {
        P.gl_rho[2 * i] = 0.5 * (1.0 + gx[i]);
        P.gl_rho[2 * i + 1] = 0.5 * gw[i];
    }
    gauss_legendre(nth, gx.data(), gw.data());
    P.nys_self.assign((size_t)6 * 6 * nth * 4, 0.0);
    const double corner[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    for (int b0 = 0; b0 < 6; ++b0) {
        const double x0 = P.nys_pt[2 * b0], y0 = P.nys_pt[2 * b0 + 1];
        for (int k = 0; k < 3; ++k) {
            const double ua = corner[k][0] - x0, va = corner[k][1] - y0;
            const double ub = corner[(k + 1) % 3][0] - x0, vb = corner[(k + 1) % 3][1] - y0;
            const double ta = std::atan2(va, ua);
            double tb = std::atan2(vb, ub);
            if (tb < ta)
                tb += 2.0 * kPi;
            const double du = ub - ua, dv = vb - va;
            const double t = -(ua * du + va * dv) / (du * du + dv * dv);
            const double fu = ua + t * du, fv = va + t * dv;
            const double pd = std::sqrt(fu * fu + fv * fv);
            double phi = std::atan2(fv, fu);
            while (phi < ta)
                phi += 2.0 * kPi;
            const double lim[3] = {ta, phi, tb};
            for (int half = 0; half < 2; ++half) {
                const double t0 = lim[half], t1 = lim[half + 1];
                for (int it = 0; it < nth; ++it) {
                    const double th = t0 + 0.5 * (t1 - t0) * (1.0 + gx[it]);
                    double *r = &P.nys_self[(((size_t)b0 * 6 + 2 * k + half) * nth + it) * 4];
                    r[0] = std::cos(th);
                    r[1] = std::sin(th);
                    r[2] = 0.5 * (t1 - t0) * gw[it];
                    r[3] = pd / std::cos(th - phi);
                }
            }
        }
    }
    plan_clusters(P);
    plan_series(mat, P);
}

}  // namespace afsbem
