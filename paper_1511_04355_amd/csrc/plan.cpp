// s-independent quadrature plan, built once per mesh on the host.
//
// Quadrature policy (paper Section 2.1 names Gauss rules for regular element
// integrals, recursive subdivision for nearly singular ones and a dedicated
// scheme for the singular ones; this is the scheme used here):
//  * regular pairs: the 7-point degree-5 triangle rule;
//  * nearly singular pairs (|x_m - c_n| < far_ratio * h_n): 4-way midpoint
//    subdivision, repeated on every sub-triangle that still fails the same test,
//    up to max_subdiv levels; the leaves carry the 7-point rule;
//  * the self element: polar coordinates about the collocation point over the
//    three sub-triangles it spans with the element's edges; tables of
//    (direction, edge distance R(theta), angular weight) per Gauss-Legendre
//    angle, and the principal value of the static 1/r^2 traction part,
//    beta^2/(4 pi) int (e_i n_j - e_j n_i) ln R(theta) dtheta.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "fastmath64.hpp"
#include "internal.hpp"

namespace afsbem {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 mul(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 mid(V3 a, V3 b) { return {0.5 * (a.x + b.x), 0.5 * (a.y + b.y), 0.5 * (a.z + b.z)}; }

struct Tri {
    V3 p[3];
    V3 c;      // centroid
    double h;  // longest edge
    double area;
};

Tri make_tri(V3 a, V3 b, V3 c) {
    Tri t;
    t.p[0] = a;
    t.p[1] = b;
    t.p[2] = c;
    t.c = {(a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0, (a.z + b.z + c.z) / 3.0};
    double l01 = norm(sub(b, a)), l12 = norm(sub(c, b)), l20 = norm(sub(a, c));
    t.h = std::max(l01, std::max(l12, l20));
    t.area = 0.5 * norm(cross(sub(b, a), sub(c, a)));
    return t;
}

// 7-point degree-5 rule: centroid and two orbits (a, a, 1-2a).
struct Rule7 {
    double b[7][3];
    double w[7];
    Rule7() {
        const double q = std::sqrt(15.0);
        const double orbit_a[2] = {(6.0 - q) / 21.0, (6.0 + q) / 21.0};
        const double orbit_w[2] = {(155.0 - q) / 1200.0, (155.0 + q) / 1200.0};
        b[0][0] = b[0][1] = b[0][2] = 1.0 / 3.0;
        w[0] = 0.225;
        for (int o = 0; o < 2; ++o)
            for (int k = 0; k < 3; ++k) {
                int i = 1 + 3 * o + k;
                for (int c = 0; c < 3; ++c)
                    b[i][c] = (c == k) ? 1.0 - 2.0 * orbit_a[o] : orbit_a[o];
                w[i] = orbit_w[o];
            }
    }
};

void subdivide(const Tri &t, V3 x, double ratio, int depth, int max_depth, std::vector<double> &leaves) {
    double d = norm(sub(x, t.c));
    if (d < ratio * t.h && depth < max_depth) {
        V3 m01 = mid(t.p[0], t.p[1]), m12 = mid(t.p[1], t.p[2]), m20 = mid(t.p[2], t.p[0]);
        subdivide(make_tri(t.p[0], m01, m20), x, ratio, depth + 1, max_depth, leaves);
        subdivide(make_tri(m01, t.p[1], m12), x, ratio, depth + 1, max_depth, leaves);
        subdivide(make_tri(m20, m12, t.p[2]), x, ratio, depth + 1, max_depth, leaves);
        subdivide(make_tri(m01, m12, m20), x, ratio, depth + 1, max_depth, leaves);
        return;
    }
    V3 e1 = sub(t.p[1], t.p[0]), e2 = sub(t.p[2], t.p[0]);
    const double rec[10] = {t.p[0].x, t.p[0].y, t.p[0].z, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z, t.area};
    leaves.insert(leaves.end(), rec, rec + 10);
}

}  // namespace

void gauss_legendre(int n, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        // Tricomi initial guess, then Newton on P_n
        double z = std::cos(pi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double dpn = 1.0;
        for (int it = 0; it < 100; ++it) {
            double pkm1 = 1.0, pk = z;
            for (int k = 1; k < n; ++k) {
                double pkp1 = ((2.0 * k + 1.0) * z * pk - k * pkm1) / (k + 1.0);
                pkm1 = pk;
                pk = pkp1;
            }
            dpn = n * (pkm1 - z * pk) / (1.0 - z * z);
            double step = pk / dpn;
            z -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(z) + 1e-300) {
                pkm1 = 1.0;
                pk = z;
                for (int k = 1; k < n; ++k) {
                    double pkp1 = ((2.0 * k + 1.0) * z * pk - k * pkm1) / (k + 1.0);
                    pkm1 = pk;
                    pk = pkp1;
                }
                dpn = n * (pkm1 - z * pk) / (1.0 - z * z);
                break;
            }
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
    }
}

MaterialDerived derive_material(const afsbem_material &m) {
    MaterialDerived d;
    d.mu = m.mu;
    d.nu = m.nu;
    d.rho = m.rho;
    d.lam = 2.0 * m.mu * m.nu / (1.0 - 2.0 * m.nu);
    d.cs = std::sqrt(m.mu / m.rho);
    d.cp = std::sqrt((d.lam + 2.0 * m.mu) / m.rho);
    d.beta = d.cs / d.cp;
    d.lam_over_mu = d.lam / m.mu;
    return d;
}

// Preconditioner clusters: recursive coordinate bisection of the collocation
// points P.cen (split at the median of the longest box side) until a cell holds
// at most kClusterElems points.
void plan_clusters(HostPlan &P) {
    const int64_t nt = P.n_tri;
    {
        std::vector<int32_t> ids(nt);
        for (int64_t e = 0; e < nt; ++e)
            ids[e] = (int32_t)e;
        P.clus_ptr.assign(1, 0);
        P.clus_elem.clear();
        std::vector<std::pair<int64_t, int64_t>> stack{{0, nt}};
        while (!stack.empty()) {
            auto [b, e] = stack.back();
            stack.pop_back();
            if (e - b <= kClusterElems) {
                for (int64_t q = b; q < e; ++q)
                    P.clus_elem.push_back(ids[q]);
                P.clus_ptr.push_back((int64_t)P.clus_elem.size());
                continue;
            }
            double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
            for (int64_t q = b; q < e; ++q) {
                const double *cc = &P.cen[3 * (size_t)ids[q]];
                for (int dd = 0; dd < 3; ++dd) {
                    lo3[dd] = std::min(lo3[dd], cc[dd]);
                    hi3[dd] = std::max(hi3[dd], cc[dd]);
                }
            }
            int ax = 0;
            for (int dd = 1; dd < 3; ++dd)
                if (hi3[dd] - lo3[dd] > hi3[ax] - lo3[ax])
                    ax = dd;
            const int64_t mid = b + (e - b) / 2;
            auto key = [&](int32_t id) { return P.cen[3 * (size_t)id + ax]; };
            std::nth_element(ids.begin() + b, ids.begin() + mid, ids.begin() + e,
                             [&](int32_t u, int32_t w) { return key(u) < key(w) || (key(u) == key(w) && u < w); });
            stack.push_back({mid, e});
            stack.push_back({b, mid});
        }
    }
}

// Taylor coefficients of r psi and r chi in x = s r / c_s (and of r^2 psi',
// r^2 chi', whose n-th coefficient is (n-1) times the former): expanding
// e^{-x} and e^{-beta x} in the closed forms, the negative powers cancel and
// the x^n coefficient is
//   r psi: (-1)^n [(n+1)^2 + (n+1) beta^(n+2)] / (n+2)!
//   r chi: (-1)^n (n^2 - 1)(1 - beta^(n+2)) / (n+2)!
void plan_series(const MaterialDerived &mat, HostPlan &P) {
    P.coef.assign(64 + kFmTabLen, 0.0);
    for (int n = 0; n < 16; ++n) {
        double inv_fact = 1.0;
        for (int k = 2; k <= n + 2; ++k)
            inv_fact /= k;
        const double sgn = (n % 2) ? -1.0 : 1.0;
        const double bpow = std::pow(mat.beta, n + 2);
        const double a = sgn * ((n + 1.0) * (n + 1.0) + (n + 1.0) * bpow) * inv_fact;
        const double b = sgn * ((double)n * n - 1.0) * (1.0 - bpow) * inv_fact;
        P.coef[4 * n + 0] = a;
        P.coef[4 * n + 1] = b;
        P.coef[4 * n + 2] = (n - 1.0) * a;
        P.coef[4 * n + 3] = (n - 1.0) * b;
    }
    // tables of the FP64 exp and sincos (after the series): 2^(j/64), and
    // cos, sin of j pi/32 from the first quadrant by exact quarter turns
    double *tab = P.coef.data() + 64;
    const long double pi_l = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < 64; ++j) {
        tab[j] = (double)std::exp2((long double)j / 64.0L);
        const int q = j / 16, m = j % 16;
        const long double th = pi_l * m / 32.0L;
        const double c = m ? (double)std::cos(th) : 1.0, s = m ? (double)std::sin(th) : 0.0;
        const double cq[4] = {c, -s, -c, s}, sq[4] = {s, c, -s, -c};
        tab[64 + 2 * j] = cq[q];
        tab[65 + 2 * j] = sq[q];
    }
}

void build_plan(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, const int8_t *kind,
                const afsbem_quad_policy &pol, const MaterialDerived &mat, HostPlan &P) {
    (void)nv;
    P.n_tri = nt;
    P.n_theta = pol.self_n_theta;
    P.n_rho = pol.self_n_rho;
    P.vtx.resize(9 * nt);
    P.cen.resize(3 * nt);
    P.nrm.resize(3 * nt);
    P.area.resize(nt);
    P.hmax.resize(nt);
    P.src.assign(kSrcStride * nt, 0.0);
    P.kind.assign(kind, kind + nt);
    std::vector<Tri> tris(nt);
    std::vector<V3> nrm(nt);
    static const Rule7 rule;
    for (int64_t e = 0; e < nt; ++e) {
        V3 p[3];
        for (int k = 0; k < 3; ++k) {
            const double *v = xyz + 3 * tri[3 * e + k];
            p[k] = {v[0], v[1], v[2]};
            P.vtx[9 * e + 3 * k + 0] = v[0];
            P.vtx[9 * e + 3 * k + 1] = v[1];
            P.vtx[9 * e + 3 * k + 2] = v[2];
        }
        tris[e] = make_tri(p[0], p[1], p[2]);
        V3 cr = cross(sub(p[1], p[0]), sub(p[2], p[0]));
        double len = norm(cr);
        AFS_REQUIRE(len > 0.0 && std::isfinite(len), AFSBEM_EINVAL,
                    "degenerate triangle " + std::to_string(e));
        nrm[e] = mul(1.0 / len, cr);
        const Tri &t = tris[e];
        P.cen[3 * e] = t.c.x;
        P.cen[3 * e + 1] = t.c.y;
        P.cen[3 * e + 2] = t.c.z;
        P.nrm[3 * e] = nrm[e].x;
        P.nrm[3 * e + 1] = nrm[e].y;
        P.nrm[3 * e + 2] = nrm[e].z;
        P.area[e] = t.area;
        P.hmax[e] = t.h;
        double *s = &P.src[kSrcStride * e];
        for (int q = 0; q < kFarNodes; ++q) {
            V3 y = add(add(mul(rule.b[q][0], p[0]), mul(rule.b[q][1], p[1])), mul(rule.b[q][2], p[2]));
            s[4 * q + 0] = y.x;
            s[4 * q + 1] = y.y;
            s[4 * q + 2] = y.z;
            s[4 * q + 3] = rule.w[q] * t.area;
        }
        s[28] = nrm[e].x;
        s[29] = nrm[e].y;
        s[30] = nrm[e].z;
        s[31] = (double)kind[e];
    }

    // ---- near pairs: a uniform grid over centroids, cell = far_ratio * max h
    double hmax_all = 0.0;
    V3 lo = tris.empty() ? V3{0, 0, 0} : tris[0].c, hi = lo;
    for (const Tri &t : tris) {
        hmax_all = std::max(hmax_all, t.h);
        lo = {std::min(lo.x, t.c.x), std::min(lo.y, t.c.y), std::min(lo.z, t.c.z)};
        hi = {std::max(hi.x, t.c.x), std::max(hi.y, t.c.y), std::max(hi.z, t.c.z)};
    }
    const double cell = std::max(pol.far_ratio * hmax_all, 1e-300);
    auto cell_of = [&](V3 c, int64_t *ijk) {
        ijk[0] = (int64_t)std::floor((c.x - lo.x) / cell);
        ijk[1] = (int64_t)std::floor((c.y - lo.y) / cell);
        ijk[2] = (int64_t)std::floor((c.z - lo.z) / cell);
    };
    auto key = [](int64_t i, int64_t j, int64_t k) {
        return (uint64_t)((i & 0x1fffff) | ((j & 0x1fffff) << 21) | ((k & 0x1fffff) << 42));
    };
    std::unordered_map<uint64_t, std::vector<int32_t>> grid;
    for (int64_t e = 0; e < nt; ++e) {
        int64_t c[3];
        cell_of(tris[e].c, c);
        grid[key(c[0], c[1], c[2])].push_back((int32_t)e);
    }
    std::vector<std::vector<int32_t>> near_of(nt);  // per collocation row: source elements
    if (pol.far_ratio > 0.0) {
        for (int64_t n = 0; n < nt; ++n) {
            const Tri &t = tris[n];
            const double rad = pol.far_ratio * t.h;
            int64_t c[3];
            cell_of(t.c, c);
            const int64_t reach = (int64_t)std::ceil(rad / cell);
            for (int64_t i = c[0] - reach; i <= c[0] + reach; ++i)
                for (int64_t j = c[1] - reach; j <= c[1] + reach; ++j)
                    for (int64_t k = c[2] - reach; k <= c[2] + reach; ++k) {
                        auto it = grid.find(key(i, j, k));
                        if (it == grid.end())
                            continue;
                        for (int32_t m : it->second) {
                            if (m == n)
                                continue;
                            double d = norm(sub(tris[m].c, t.c));
                            if (d < rad)
                                near_of[m].push_back((int32_t)n);
                        }
                    }
        }
    }
    P.near_ptr.assign(nt + 1, 0);
    for (int64_t m = 0; m < nt; ++m) {
        std::sort(near_of[m].begin(), near_of[m].end());
        P.near_ptr[m + 1] = P.near_ptr[m] + (int64_t)near_of[m].size();
    }
    const int64_t nnz = P.near_ptr[nt];
    P.near_col.resize(nnz);
    P.near_row.resize(nnz);
    P.leaf_ptr.assign(nnz + 1, 0);
    P.leaves.clear();
    int64_t k = 0;
    for (int64_t m = 0; m < nt; ++m) {
        for (int32_t n : near_of[m]) {
            P.near_col[k] = n;
            P.near_row[k] = (int32_t)m;
            subdivide(tris[n], tris[m].c, pol.far_ratio, 0, pol.max_subdiv, P.leaves);
            P.leaf_ptr[k + 1] = (int64_t)(P.leaves.size() / 10);
            ++k;
        }
    }
    // The near kernel gives each pair a fixed group of lanes and a wave holds
    // several pairs: taking the pairs in decreasing order of their leaf count
    // keeps the pairs of a wave alike (edge neighbours of a collocation point
    // have ~10x the median leaf count; in row order nearly every wave holds one).
    P.near_order.resize(nnz);
    for (int64_t q = 0; q < nnz; ++q)
        P.near_order[q] = (int32_t)q;
    std::stable_sort(P.near_order.begin(), P.near_order.end(), [&](int32_t a, int32_t b) {
        return P.leaf_ptr[a + 1] - P.leaf_ptr[a] > P.leaf_ptr[b + 1] - P.leaf_ptr[b];
    });

    // ---- self element polar tables
    const int nth = pol.self_n_theta, nrh = pol.self_n_rho;
    std::vector<double> gx(std::max(nth, nrh)), gw(std::max(nth, nrh));
    P.gl_rho.resize(2 * nrh);
    gauss_legendre(nrh, gx.data(), gw.data());
    for (int i = 0; i < nrh; ++i) {
        P.gl_rho[2 * i] = 0.5 * (1.0 + gx[i]);
        P.gl_rho[2 * i + 1] = 0.5 * gw[i];
    }
    gauss_legendre(nth, gx.data(), gw.data());
    P.self_ang.assign((size_t)nt * 3 * nth * 5, 0.0);
    P.self_cpv.assign((size_t)nt * 9, 0.0);
    const double cpv_scale = mat.beta * mat.beta / (4.0 * 3.14159265358979323846);
    for (int64_t e = 0; e < nt; ++e) {
        const Tri &t = tris[e];
        const V3 n = nrm[e];
        V3 f1 = sub(t.p[0], t.c);
        f1 = mul(1.0 / norm(f1), f1);
        V3 f2 = cross(n, f1);
        // vertices in the in-plane frame
        double u[3], v[3];
        for (int a = 0; a < 3; ++a) {
            V3 d = sub(t.p[a], t.c);
            u[a] = dot(d, f1);
            v[a] = dot(d, f2);
        }
        double cpv[9] = {0};
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3;
            double ta = std::atan2(v[a], u[a]), tb = std::atan2(v[b], u[b]);
            while (tb <= ta)
                tb += 2.0 * 3.14159265358979323846;
            // distance from the origin to the edge line and the angle of its normal
            const double du = u[b] - u[a], dv = v[b] - v[a];
            const double elen = std::sqrt(du * du + dv * dv);
            const double pdist = std::fabs(u[a] * v[b] - u[b] * v[a]) / elen;
            const double phi0 = std::atan2(-du, dv);  // outward normal of a CCW edge
            for (int i = 0; i < nth; ++i) {
                const double th = ta + 0.5 * (tb - ta) * (1.0 + gx[i]);
                const double wth = 0.5 * (tb - ta) * gw[i];
                const double R = pdist / std::cos(th - phi0);
                const V3 dir = add(mul(std::cos(th), f1), mul(std::sin(th), f2));
                double *rec = &P.self_ang[((size_t)e * 3 * nth + (size_t)a * nth + i) * 5];
                rec[0] = dir.x;
                rec[1] = dir.y;
                rec[2] = dir.z;
                rec[3] = R;
                rec[4] = wth;
                const double dd[3] = {dir.x, dir.y, dir.z}, nn[3] = {n.x, n.y, n.z};
                const double lr = std::log(R);
                for (int ii = 0; ii < 3; ++ii)
                    for (int jj = 0; jj < 3; ++jj)
                        cpv[3 * ii + jj] += wth * lr * (dd[ii] * nn[jj] - dd[jj] * nn[ii]);
            }
        }
        for (int q = 0; q < 9; ++q)
            P.self_cpv[9 * e + q] = cpv_scale * cpv[q];
    }

    plan_clusters(P);
    plan_series(mat, P);
}

}  // namespace afsbem
