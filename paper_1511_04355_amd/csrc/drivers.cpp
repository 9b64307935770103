// Frequency-domain drivers on top of the per-frequency solve (host code):
//  * Fourier-series-method grid and inversion by FFT (paper Section 2.2, Eq. 3-4);
//  * vector fitting with common poles (Section 2.3, Eq. 5-6);
//  * adaptive frequency sampling (Section 3, Eq. 7-14, the Algorithm of 3.4).
//
// Readings (the same ones the documentation lists): Eq. 4 carries the factor
// 1/P; the end point of the truncated Bromwich sum carries the half
// trapezoid weight; the time response of r/(s-a) is r e^{a t}; the Chebyshev
// initial frequencies are Omega [1 - cos(j pi / (2 (J0 - 1)))]; maxima over
// [0, Omega] are taken on a uniform grid; samples closer than dw/4 to an
// existing one are not chosen again; E1 at step 0 is infinite and its
// integrals use composite Simpson on 4 Ns + 1 points.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <limits>
#include <vector>

#include "internal.hpp"
#include "solver.hpp"

namespace afsbem {

using cplx = std::complex<double>;
static const double kPi = 3.14159265358979323846;

// ======================================================================= FFT
// In-place radix-2 decimation-in-time FFT, sign = +1 computes sum x_k e^{+2 pi i k n / N}.
static void fft_pow2(std::vector<cplx> &x, int sign) {
    const size_t n = x.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j)
            std::swap(x[i], x[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = sign * 2.0 * kPi / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const cplx w = std::polar(1.0, ang * (double)k);
                const cplx u = x[i + k], v = x[i + k + len / 2] * w;
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
    }
}

// y_n = sum_k x_k e^{+2 pi i k n / N} for any N (radix-2, or a direct sum)
static std::vector<cplx> dft_plus(const std::vector<cplx> &x) {
    const size_t n = x.size();
    if (n && (n & (n - 1)) == 0) {
        std::vector<cplx> y = x;
        fft_pow2(y, +1);
        return y;
    }
    std::vector<cplx> y(n);
    for (size_t m = 0; m < n; ++m) {
        cplx acc = 0.0;
        for (size_t k = 0; k < n; ++k)
            acc += x[k] * std::polar(1.0, 2.0 * kPi * (double)((k * m) % n) / (double)n);
        y[m] = acc;
    }
    return y;
}

// ============================================================ dense helpers
// Least squares min ||A x - B|| for a real m x n matrix (column-major, m >= n)
// and k right-hand sides, by Householder QR of the column-scaled matrix;
// columns whose pivot falls below 1e-13 of the largest are dropped (x = 0).
static void lstsq(int m, int n, std::vector<double> A, int k, std::vector<double> B, std::vector<double> &X) {
    std::vector<double> scale(n, 1.0);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i)
            s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        s = std::sqrt(s);
        scale[j] = s > 0 ? 1.0 / s : 1.0;
        for (int i = 0; i < m; ++i)
            A[(size_t)j * m + i] *= scale[j];
    }
    std::vector<double> v(m);
    for (int j = 0; j < n; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i)
            nrm += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0)
            continue;
        const double a0 = A[(size_t)j * m + j];
        const double alpha = a0 > 0 ? -nrm : nrm;
        for (int i = j; i < m; ++i)
            v[i] = A[(size_t)j * m + i];
        v[j] -= alpha;
        double vn = 0.0;
        for (int i = j; i < m; ++i)
            vn += v[i] * v[i];
        if (vn == 0.0)
            continue;
        for (int c = j; c < n; ++c) {
            double d = 0.0;
            for (int i = j; i < m; ++i)
                d += v[i] * A[(size_t)c * m + i];
            d *= 2.0 / vn;
            for (int i = j; i < m; ++i)
                A[(size_t)c * m + i] -= d * v[i];
        }
        for (int c = 0; c < k; ++c) {
            double d = 0.0;
            for (int i = j; i < m; ++i)
                d += v[i] * B[(size_t)c * m + i];
            d *= 2.0 / vn;
            for (int i = j; i < m; ++i)
                B[(size_t)c * m + i] -= d * v[i];
        }
    }
    double rmax = 0.0;
    for (int j = 0; j < n; ++j)
        rmax = std::max(rmax, std::fabs(A[(size_t)j * m + j]));
    X.assign((size_t)n * k, 0.0);
    for (int c = 0; c < k; ++c)
        for (int j = n - 1; j >= 0; --j) {
            const double rjj = A[(size_t)j * m + j];
            if (std::fabs(rjj) <= 1e-13 * rmax)
                continue;
            double s = B[(size_t)c * m + j];
            for (int l = j + 1; l < n; ++l)
                s -= A[(size_t)l * m + j] * X[(size_t)c * n + l];
            X[(size_t)c * n + j] = s / rjj;
        }
    for (int c = 0; c < k; ++c)
        for (int j = 0; j < n; ++j)
            X[(size_t)c * n + j] *= scale[j];
}

// Householder QR of a real m x n block (column-major), returning the n x n R
// factor and Q^T applied to nothing else: used to eliminate unknowns.
static void qr_r(int m, int n, std::vector<double> &A) {
    std::vector<double> v(m);
    for (int j = 0; j < n && j < m; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i)
            nrm += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0)
            continue;
        const double a0 = A[(size_t)j * m + j];
        const double alpha = a0 > 0 ? -nrm : nrm;
        for (int i = j; i < m; ++i)
            v[i] = A[(size_t)j * m + i];
        v[j] -= alpha;
        double vn = 0.0;
        for (int i = j; i < m; ++i)
            vn += v[i] * v[i];
        if (vn == 0.0)
            continue;
        for (int c = j; c < n; ++c) {
            double d = 0.0;
            for (int i = j; i < m; ++i)
                d += v[i] * A[(size_t)c * m + i];
            d *= 2.0 / vn;
            for (int i = j; i < m; ++i)
                A[(size_t)c * m + i] -= d * v[i];
        }
    }
}

// Eigenvalues of a real n x n matrix (row-major): Householder reduction to
// upper Hessenberg form, then the complex shifted QR iteration (Wilkinson
// shifts, Givens rotations, deflation of negligible subdiagonals).
static std::vector<cplx> eigenvalues(std::vector<double> A, int n) {
    for (int k = 0; k + 2 < n; ++k) {
        std::vector<double> v(n, 0.0);
        double nrm = 0.0;
        for (int i = k + 1; i < n; ++i)
            nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0)
            continue;
        const double x0 = A[(size_t)(k + 1) * n + k];
        const double alpha = x0 > 0 ? -nrm : nrm;
        for (int i = k + 1; i < n; ++i)
            v[i] = A[(size_t)i * n + k];
        v[k + 1] -= alpha;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i)
            vn += v[i] * v[i];
        if (vn == 0.0)
            continue;
        for (int c = 0; c < n; ++c) {  // left: (I - 2vv^T/vn) A
            double d = 0.0;
            for (int i = k + 1; i < n; ++i)
                d += v[i] * A[(size_t)i * n + c];
            d *= 2.0 / vn;
            for (int i = k + 1; i < n; ++i)
                A[(size_t)i * n + c] -= d * v[i];
        }
        for (int r = 0; r < n; ++r) {  // right: A (I - 2vv^T/vn)
            double d = 0.0;
            for (int i = k + 1; i < n; ++i)
                d += A[(size_t)r * n + i] * v[i];
            d *= 2.0 / vn;
            for (int i = k + 1; i < n; ++i)
                A[(size_t)r * n + i] -= d * v[i];
        }
    }
    std::vector<cplx> H((size_t)n * n);
    for (size_t i = 0; i < H.size(); ++i)
        H[i] = A[i];
    auto at = [&](int i, int j) -> cplx & { return H[(size_t)i * n + j]; };
    std::vector<cplx> eig;
    std::vector<double> gc(n);
    std::vector<cplx> gs(n);
    int hi = n - 1, iter = 0;
    const double eps = std::numeric_limits<double>::epsilon();
    while (hi >= 0) {
        int lo = hi;
        while (lo > 0 && std::abs(at(lo, lo - 1)) > eps * (std::abs(at(lo, lo)) + std::abs(at(lo - 1, lo - 1))))
            --lo;
        if (lo > 0)
            at(lo, lo - 1) = 0.0;
        if (lo == hi) {
            eig.push_back(at(hi, hi));
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 1000)
            throw Error{AFSBEM_EINVAL, "eigenvalue iteration did not converge"};
        const cplx a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
        const cplx half = 0.5 * (a - d);
        const cplx disc = std::sqrt(half * half + b * c);
        cplx mu1 = 0.5 * (a + d) + disc, mu2 = 0.5 * (a + d) - disc;
        cplx mu = (std::abs(mu1 - d) < std::abs(mu2 - d)) ? mu1 : mu2;
        if (iter % 11 == 10)
            mu = d + std::abs(c);  // exceptional shift
        for (int i = lo; i <= hi; ++i)
            at(i, i) -= mu;
        for (int k = lo; k < hi; ++k) {
            const cplx x = at(k, k), y = at(k + 1, k);
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            double cc;
            cplx ss;
            if (r == 0.0) {
                cc = 1.0;
                ss = 0.0;
            } else if (std::abs(x) == 0.0) {
                cc = 0.0;
                ss = std::conj(y) / std::abs(y);
            } else {
                cc = std::abs(x) / r;
                ss = (x / std::abs(x)) * std::conj(y) / r;
            }
            gc[k] = cc;
            gs[k] = ss;
            for (int j = k; j <= hi; ++j) {
                const cplx u = at(k, j), w = at(k + 1, j);
                at(k, j) = cc * u + ss * w;
                at(k + 1, j) = -std::conj(ss) * u + cc * w;
            }
        }
        for (int k = lo; k < hi; ++k) {
            const double cc = gc[k];
            const cplx ss = gs[k];
            const int rmax = std::min(k + 2, hi);
            for (int i = lo; i <= rmax; ++i) {
                const cplx u = at(i, k), w = at(i, k + 1);
                at(i, k) = cc * u + std::conj(ss) * w;
                at(i, k + 1) = -ss * u + cc * w;
            }
        }
        for (int i = lo; i <= hi; ++i)
            at(i, i) += mu;
    }
    return eig;
}

// ======================================================== vector fitting
struct PoleSet {
    std::vector<cplx> rep;    // representative: real pole, or the member with Im > 0
    std::vector<bool> pair;
    int dim() const {
        int d = 0;
        for (bool p : pair)
            d += p ? 2 : 1;
        return d;
    }
    std::vector<cplx> all() const {
        std::vector<cplx> out;
        for (size_t i = 0; i < rep.size(); ++i) {
            out.push_back(rep[i]);
            if (pair[i])
                out.push_back(std::conj(rep[i]));
        }
        return out;
    }
};

// Group poles into real ones and conjugate pairs.  Eigenvalues of a real
// matrix computed in complex arithmetic carry round-off: a real eigenvalue may
// show a tiny imaginary part and the members of a pair may differ slightly.
// Poles are visited by decreasing |Im|; each takes the nearest unused
// conjugate as partner (the pair is snapped to an exact conjugate pair); a pole
// whose imaginary part is negligible, or that finds no partner, becomes real.
// Every input pole is consumed exactly once, so the count is preserved.
static PoleSet group_poles(const std::vector<cplx> &p, double rel_tol = 1e-8) {
    PoleSet ps;
    const size_t n = p.size();
    double scale = 1.0;
    for (const cplx &a : p)
        scale = std::max(scale, std::abs(a));
    std::vector<bool> used(n, false);
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i)
        order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return std::fabs(p[a].imag()) > std::fabs(p[b].imag()); });
    for (size_t oi : order) {
        if (used[oi])
            continue;
        used[oi] = true;
        const cplx a = p[oi];
        if (std::fabs(a.imag()) > rel_tol * scale) {
            size_t best = n;
            double bd = 1e300;
            for (size_t j = 0; j < n; ++j)
                if (!used[j] && std::abs(p[j] - std::conj(a)) < bd) {
                    bd = std::abs(p[j] - std::conj(a));
                    best = j;
                }
            if (best < n && bd <= 1e-6 * scale) {
                used[best] = true;
                const double re = 0.5 * (a.real() + p[best].real());
                const double im = 0.5 * (std::fabs(a.imag()) + std::fabs(p[best].imag()));
                ps.rep.push_back(cplx(re, im));
                ps.pair.push_back(true);
                continue;
            }
        }
        ps.rep.push_back(cplx(a.real(), 0.0));
        ps.pair.push_back(false);
    }
    return ps;
}

// real-coefficient basis values phi_c(s_j), column-major [J][dim]
static std::vector<cplx> basis_values(const std::vector<cplx> &s, const PoleSet &ps) {
    const int J = (int)s.size(), M = ps.dim();
    std::vector<cplx> Phi((size_t)J * M);
    int c = 0;
    const cplx I(0.0, 1.0);
    for (size_t q = 0; q < ps.rep.size(); ++q) {
        const cplx a = ps.rep[q];
        for (int j = 0; j < J; ++j) {
            const cplx u = 1.0 / (s[j] - a);
            if (ps.pair[q]) {
                const cplx w = 1.0 / (s[j] - std::conj(a));
                Phi[(size_t)c * J + j] = u + w;
                Phi[(size_t)(c + 1) * J + j] = I * u - I * w;
            } else {
                Phi[(size_t)c * J + j] = u;
            }
        }
        c += ps.pair[q] ? 2 : 1;
    }
    return Phi;
}

std::vector<cplx> vf_initial_poles(int M, double omega_max) {
    std::vector<cplx> p;
    const int npair = M / 2;
    for (int m = 1; m <= npair; ++m) {
        const double b = omega_max * (double)m / (double)npair;
        p.push_back(cplx(-b / 100.0, b));
        p.push_back(cplx(-b / 100.0, -b));
    }
    if (M % 2)
        p.push_back(cplx(-omega_max / 100.0, 0.0));
    return p;
}

// One relaxed pole identification.  The residue unknowns of each function are
// eliminated by a QR factorisation of its block [Phi, -F_k Phi] (real form);
// the trailing rows of every R factor form the least-squares system of the
// sigma coefficients.  The new poles are the zeros of sigma.
static std::vector<cplx> vf_identify_poles(const std::vector<cplx> &s, int K, const std::vector<cplx> &F /*[K][J]*/,
                                           const std::vector<cplx> &poles) {
    const int J = (int)s.size();
    const PoleSet ps = group_poles(poles);
    const int M = ps.dim();
    const std::vector<cplx> Phi = basis_values(s, ps);
    const int rows = 2 * J, cols = 2 * M;
    std::vector<double> red((size_t)K * M * M), rhs((size_t)K * M);
    const int rr = std::min(rows, cols + 1);
    for (int k = 0; k < K; ++k) {
        // block [Phi, -F Phi | F], real/imag stacked, column-major rows x (cols+1)
        std::vector<double> B((size_t)rows * (cols + 1));
        for (int c = 0; c < M; ++c)
            for (int j = 0; j < J; ++j) {
                const cplx ph = Phi[(size_t)c * J + j];
                const cplx fp = -F[(size_t)k * J + j] * ph;
                B[(size_t)c * rows + j] = ph.real();
                B[(size_t)c * rows + J + j] = ph.imag();
                B[(size_t)(M + c) * rows + j] = fp.real();
                B[(size_t)(M + c) * rows + J + j] = fp.imag();
            }
        for (int j = 0; j < J; ++j) {
            B[(size_t)cols * rows + j] = F[(size_t)k * J + j].real();
            B[(size_t)cols * rows + J + j] = F[(size_t)k * J + j].imag();
        }
        qr_r(rows, cols + 1, B);
        // rows M..2M-1 of R: the sigma part and the transformed right-hand side
        for (int i = 0; i < M; ++i) {
            const int r = M + i;
            for (int c = 0; c < M; ++c)
                red[(size_t)c * (K * M) + (size_t)k * M + i] = (r < rr) ? B[(size_t)(M + c) * rows + r] : 0.0;
            rhs[(size_t)k * M + i] = (r < rr) ? B[(size_t)cols * rows + r] : 0.0;
        }
    }
    std::vector<double> ct;
    lstsq(K * M, M, red, 1, rhs, ct);
    // real block realisation of the poles and the zeros of sigma
    std::vector<double> Ah((size_t)M * M, 0.0);
    std::vector<double> bh(M, 0.0);
    int c = 0;
    for (size_t q = 0; q < ps.rep.size(); ++q) {
        const cplx a = ps.rep[q];
        if (ps.pair[q]) {
            Ah[(size_t)c * M + c] = a.real();
            Ah[(size_t)c * M + c + 1] = a.imag();
            Ah[(size_t)(c + 1) * M + c] = -a.imag();
            Ah[(size_t)(c + 1) * M + c + 1] = a.real();
            bh[c] = 2.0;
            c += 2;
        } else {
            Ah[(size_t)c * M + c] = a.real();
            bh[c] = 1.0;
            c += 1;
        }
    }
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j)
            Ah[(size_t)i * M + j] -= bh[i] * ct[j];
    return group_poles(eigenvalues(Ah, M)).all();
}

// residues [n_fun][M] (complex, aligned with group_poles(poles).all())
static std::vector<cplx> vf_identify_residues(const std::vector<cplx> &s, int64_t n_fun, const std::vector<cplx> &F,
                                              const std::vector<cplx> &poles, std::vector<cplx> &poles_out) {
    const int J = (int)s.size();
    const PoleSet ps = group_poles(poles);
    const int M = ps.dim();
    poles_out = ps.all();
    const std::vector<cplx> Phi = basis_values(s, ps);
    std::vector<double> A((size_t)2 * J * M), B((size_t)2 * J * n_fun);
    for (int c = 0; c < M; ++c)
        for (int j = 0; j < J; ++j) {
            A[(size_t)c * 2 * J + j] = Phi[(size_t)c * J + j].real();
            A[(size_t)c * 2 * J + J + j] = Phi[(size_t)c * J + j].imag();
        }
    for (int64_t k = 0; k < n_fun; ++k)
        for (int j = 0; j < J; ++j) {
            B[(size_t)k * 2 * J + j] = F[(size_t)k * J + j].real();
            B[(size_t)k * 2 * J + J + j] = F[(size_t)k * J + j].imag();
        }
    std::vector<double> X;
    lstsq(2 * J, M, A, (int)n_fun, B, X);
    std::vector<cplx> R((size_t)n_fun * M);
    for (int64_t k = 0; k < n_fun; ++k) {
        int c = 0;
        for (size_t q = 0; q < ps.rep.size(); ++q) {
            if (ps.pair[q]) {
                const cplx r(X[(size_t)k * M + c], X[(size_t)k * M + c + 1]);
                R[(size_t)k * M + c] = r;
                R[(size_t)k * M + c + 1] = std::conj(r);
                c += 2;
            } else {
                R[(size_t)k * M + c] = X[(size_t)k * M + c];
                c += 1;
            }
        }
    }
    return R;
}

struct VfModel {
    std::vector<cplx> poles;  // [M]
    std::vector<cplx> res;    // [n_fun][M]
};

static VfModel vf_fit_model(const std::vector<cplx> &s, int K, const std::vector<cplx> &Fo, int64_t n_fun,
                            const std::vector<cplx> &Fall, int M, std::vector<cplx> poles, int n_iter) {
    for (int it = 0; it < n_iter; ++it) {
        std::vector<cplx> nw = vf_identify_poles(s, K, Fo, poles);
        bool same = nw.size() == poles.size();
        if (same) {
            std::vector<cplx> a = nw, b = poles;
            auto key = [](const cplx &x, const cplx &y) {
                return x.real() < y.real() || (x.real() == y.real() && x.imag() < y.imag());
            };
            std::sort(a.begin(), a.end(), key);
            std::sort(b.begin(), b.end(), key);
            double mx = 0.0, sc = 1.0;
            for (size_t i = 0; i < a.size(); ++i) {
                mx = std::max(mx, std::abs(a[i] - b[i]));
                sc = std::max(sc, std::abs(b[i]));
            }
            same = mx <= 1e-10 * sc;
        }
        poles = nw;
        if (same)
            break;
    }
    VfModel m;
    m.res = vf_identify_residues(s, n_fun, Fall, poles, m.poles);
    (void)M;
    return m;
}

static cplx vf_eval1(const VfModel &m, int64_t k, cplx s) {
    const size_t M = m.poles.size();
    cplx acc = 0.0;
    for (size_t q = 0; q < M; ++q)
        acc += m.res[(size_t)k * M + q] / (s - m.poles[q]);
    return acc;
}

static double vf_time1(const VfModel &m, int64_t k, double t) {
    const size_t M = m.poles.size();
    cplx acc = 0.0;
    for (size_t q = 0; q < M; ++q)
        acc += m.res[(size_t)k * M + q] * std::exp(m.poles[q] * t);
    return acc.real();
}

// ====================================================== all-DOF synthesis
// For any function sampled as F_j at s_j (B = [Re F; Im F], 2J reals), its
// residues with the given poles are the least-squares coefficients x = A^+ B
// of the real-coefficient basis (as in residue identification, Section 2.3).
// Any linear functional of the model -- its time response at t (Eq. 6), its
// value at a complex frequency z -- is then sum_c x_c phi_c = sum_i B_i K_i
// with K_i = sum_c A^+[c][i] phi_c.  synthesis_pinv returns A^+ as X[i][c].
static std::vector<double> synthesis_pinv(const std::vector<cplx> &s, const PoleSet &ps) {
    const int J = (int)s.size();
    const int M = ps.dim();
    const std::vector<cplx> Phi = basis_values(s, ps);
    std::vector<double> A((size_t)2 * J * M), I((size_t)2 * J * 2 * J, 0.0), X;
    for (int c = 0; c < M; ++c)
        for (int j = 0; j < J; ++j) {
            A[(size_t)c * 2 * J + j] = Phi[(size_t)c * J + j].real();
            A[(size_t)c * 2 * J + J + j] = Phi[(size_t)c * J + j].imag();
        }
    for (int i = 0; i < 2 * J; ++i)
        I[(size_t)i * 2 * J + i] = 1.0;
    lstsq(2 * J, M, A, 2 * J, I, X);  // X[i][c] = A^+[c][i]
    return X;
}

// K [Kpad][ncol]: K[i][n] = sum_c X[i][c] phi[c][n] (rows 2J..Kpad-1 zero)
static std::vector<double> synthesis_contract(const std::vector<double> &X, int J, int M,
                                              const std::vector<double> &phi, int ncol, int Kpad) {
    std::vector<double> K((size_t)Kpad * ncol, 0.0);
    for (int i = 0; i < 2 * J; ++i)
        for (int cc = 0; cc < M; ++cc) {
            const double w = X[(size_t)i * M + cc];
            for (int n = 0; n < ncol; ++n)
                K[(size_t)i * ncol + n] += w * phi[(size_t)cc * ncol + n];
        }
    return K;
}

// Time responses of the basis functions (Eq. 6): 2 Re e^{a t} and -2 Im e^{a t}
// for a conjugate pair, e^{a t} for a real pole.
static std::vector<double> synthesis_matrix(const std::vector<cplx> &s, const std::vector<cplx> &poles,
                                            const double *t, int Nt, int Kpad) {
    const PoleSet ps = group_poles(poles);
    const int M = ps.dim();
    const std::vector<double> X = synthesis_pinv(s, ps);
    std::vector<double> phi((size_t)M * Nt);
    int c = 0;
    for (size_t q = 0; q < ps.rep.size(); ++q) {
        const cplx a = ps.rep[q];
        for (int n = 0; n < Nt; ++n) {
            const cplx e = std::exp(a * t[n]);
            if (ps.pair[q]) {
                phi[(size_t)c * Nt + n] = 2.0 * e.real();
                phi[(size_t)(c + 1) * Nt + n] = -2.0 * e.imag();
            } else {
                phi[(size_t)c * Nt + n] = e.real();
            }
        }
        c += ps.pair[q] ? 2 : 1;
    }
    return synthesis_contract(X, (int)s.size(), M, phi, Nt, Kpad);
}

// Values of the basis functions at complex frequencies z (Eq. 5), as
// interleaved (Re, Im) columns: K [Kpad][2 n_z].
static std::vector<double> sampling_matrix(const std::vector<cplx> &s, const std::vector<cplx> &poles,
                                           const std::vector<cplx> &z, int Kpad) {
    const PoleSet ps = group_poles(poles);
    const int M = ps.dim(), nz = (int)z.size();
    const std::vector<double> X = synthesis_pinv(s, ps);
    const std::vector<cplx> Pz = basis_values(z, ps);  // [M][nz]
    std::vector<double> phi((size_t)M * 2 * nz);
    for (int c = 0; c < M; ++c)
        for (int k = 0; k < nz; ++k) {
            phi[(size_t)c * 2 * nz + 2 * k] = Pz[(size_t)c * nz + k].real();
            phi[(size_t)c * 2 * nz + 2 * k + 1] = Pz[(size_t)c * nz + k].imag();
        }
    return synthesis_contract(X, (int)s.size(), M, phi, 2 * nz, Kpad);
}

// e^{2 pi i m / N}, angle formed and evaluated in extended precision
static cplx unit_root(int64_t m, int64_t N) {
    const long double pi_l = 3.14159265358979323846264338327950288L;
    const long double a = 2.0L * pi_l * (long double)m / (long double)N;
    return cplx((double)std::cos(a), (double)std::sin(a));
}

// =================================================================== AFS
struct AfsResult {
    std::vector<cplx> s;           // samples
    std::vector<cplx> F;           // [Nc][Kt]
    VfModel model;                 // final order-M_H model over all Kt functions
    std::vector<double> E1, E2;    // per analysis step
    std::vector<int> J, MH, ML;
    int converged = 0;
    int capped = 0;                // the sample cap ended the run (also inside the Jc validation steps)
    int Kt = 0;
    int64_t matvecs = 0;           // GPU solves (afs_run_problem): Krylov products in all
    int unconverged = 0;           // GPU solves that missed opts.tol (their iterate was still sampled)
    double worst_rel_res = 0.0;    // largest FP64 true relative residual over the GPU solves
};

// responses [n][Kt] at the frequencies asked for; model: the current order-M_H
// fit (null in the initial round)
using ResponseFn = std::function<void(const std::vector<cplx> &, std::vector<cplx> &, const VfModel *)>;

// Weights (alpha_j, beta_j) such that the model's prediction at s_new of any
// function sampled at s_j (j < J) is sum_j alpha_j F_j + beta_j conj(F_j): the
// residues of that function with the given poles are the least-squares
// solution of the real-coefficient basis (as in residue identification), which
// is real-linear in (Re F, Im F).
static void vf_prediction_weights(const std::vector<cplx> &s, const std::vector<cplx> &poles, cplx s_new,
                                  std::vector<cplx> &alpha, std::vector<cplx> &beta) {
    const int J = (int)s.size();
    const PoleSet ps = group_poles(poles);
    const int M = ps.dim();
    const std::vector<cplx> Phi = basis_values(s, ps);
    std::vector<double> A((size_t)2 * J * M), I((size_t)2 * J * 2 * J, 0.0), X;
    for (int c = 0; c < M; ++c)
        for (int j = 0; j < J; ++j) {
            A[(size_t)c * 2 * J + j] = Phi[(size_t)c * J + j].real();
            A[(size_t)c * 2 * J + J + j] = Phi[(size_t)c * J + j].imag();
        }
    for (int i = 0; i < 2 * J; ++i)
        I[(size_t)i * 2 * J + i] = 1.0;
    lstsq(2 * J, M, A, 2 * J, I, X);  // X[i][m]: column i of the pseudo-inverse
    const std::vector<cplx> phi = basis_values(std::vector<cplx>{s_new}, ps);
    alpha.assign(J, 0.0);
    beta.assign(J, 0.0);
    const cplx Im(0.0, 1.0);
    for (int j = 0; j < J; ++j) {
        cplx u = 0.0, v = 0.0;  // weights of Re F_j and Im F_j
        for (int m = 0; m < M; ++m) {
            u += phi[m] * X[(size_t)j * M + m];
            v += phi[m] * X[(size_t)(J + j) * M + m];
        }
        alpha[j] = 0.5 * (u - Im * v);
        beta[j] = 0.5 * (u + Im * v);
    }
}

// New frequencies from the discrepancy d on the uniform grid (G points on
// [0, Omega]): grid points within dw/4 of a sample are excluded; the first
// pick is the largest remaining value (Section 3.2; smallest w on ties), each
// further one (q > 1) the next largest local maximum (d[g] > d[g-1],
// d[g] >= d[g+1], one-sided at the ends; smallest w on ties) at least dw/4
// from every earlier pick.  Returns grid indices; -1 if every point is taken.
static std::vector<int> afs_select(const std::vector<double> &d0, int G, double omega, const std::vector<cplx> &S,
                                   double dw, int q) {
    std::vector<double> d(d0);
    std::vector<char> taken(G, 0);
    auto wof = [&](int g) { return (G > 1) ? omega * g / (G - 1) : 0.0; };
    for (int g = 0; g < G; ++g)
        for (const cplx &sv : S)
            if (std::fabs(wof(g) - sv.imag()) < dw / 4) {
                taken[g] = 1;
                d[g] = -1.0;
                break;
            }
    int gbest = -1;
    double best = -1.0;
    for (int g = 0; g < G; ++g)
        if (!taken[g] && d[g] > best) {
            best = d[g];
            gbest = g;
        }
    std::vector<int> picks{gbest};
    if (q > 1 && gbest >= 0) {
        std::vector<int> cand;
        for (int g = 0; g < G; ++g) {
            if (taken[g])
                continue;
            const bool left = g > 0 ? d[g] > d[g - 1] : true;
            const bool right = g < G - 1 ? d[g] >= d[g + 1] : true;
            if (left && right)
                cand.push_back(g);
        }
        std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return d[a] > d[b]; });
        for (int g : cand) {
            if ((int)picks.size() >= q)
                break;
            bool far = true;
            for (int h : picks)
                if (std::fabs(wof(g) - wof(h)) < dw / 4) {
                    far = false;
                    break;
                }
            if (far)
                picks.push_back(g);
        }
    }
    return picks;
}

static void afs_run_impl(const afsbem_afs_params &P, int K, int Kt, const ResponseFn &resp, AfsResult &R) {
    const double omega = kPi * P.Ns / P.T;
    const double dw = 2.0 * kPi / P.T;
    const int max_Nc = P.max_Nc > 0 ? P.max_Nc : P.Ns / 2 + 1;
    const int G = P.grid_pts;
    const int nt = 4 * P.Ns + 1;
    R.Kt = Kt;
    std::vector<cplx> S;
    for (int j = 0; j < P.J0; ++j)
        S.push_back(cplx(P.eta, omega * (1.0 - std::cos(j * kPi / (2.0 * (P.J0 - 1))))));
    std::vector<cplx> Fv;
    resp(S, Fv, nullptr);
    std::vector<double> prev_td;
    std::vector<cplx> s_new;

    auto analyse = [&]() -> std::pair<double, double> {
        const int J = (int)S.size();
        const int MH = (int)std::floor(J / P.alpha_H), ML = (int)std::floor(J / P.alpha_L);
        // ORF data [K][J] and all functions [Kt][J]
        std::vector<cplx> Fo((size_t)K * J), Fa((size_t)Kt * J);
        for (int j = 0; j < J; ++j)
            for (int k = 0; k < Kt; ++k) {
                Fa[(size_t)k * J + j] = Fv[(size_t)j * Kt + k];
                if (k < K)
                    Fo[(size_t)k * J + j] = Fv[(size_t)j * Kt + k];
            }
        VfModel mH = vf_fit_model(S, K, Fo, Kt, Fa, MH, vf_initial_poles(MH, omega), P.n_iter);
        VfModel mL = vf_fit_model(S, K, Fo, Kt, Fa, ML, vf_initial_poles(ML, omega), P.n_iter);
        std::vector<double> e(Kt), dmax(Kt);
        std::vector<double> diff_kmax;
        std::vector<std::vector<double>> diffs(Kt, std::vector<double>(G));
        for (int k = 0; k < Kt; ++k) {
            double dm = 0.0, fm = 0.0;
            for (int g = 0; g < G; ++g) {
                const double w = (G > 1) ? omega * g / (G - 1) : 0.0;
                const cplx sg(P.eta, w);
                const cplx fh = vf_eval1(mH, k, sg), fl = vf_eval1(mL, k, sg);
                diffs[k][g] = std::abs(fh - fl);
                dm = std::max(dm, diffs[k][g]);
                fm = std::max(fm, std::abs(fh));
            }
            e[k] = dm / fm;
        }
        double E2 = 0.0;
        for (double v : e)
            E2 = std::max(E2, v);
        // time responses of the order-M_H model on [0, T]
        std::vector<double> td((size_t)Kt * nt);
        const double h = P.T / (nt - 1);
        for (int k = 0; k < Kt; ++k)
            for (int i = 0; i < nt; ++i)
                td[(size_t)k * nt + i] = vf_time1(mH, k, h * i);
        double E1 = std::numeric_limits<double>::infinity();
        if (!prev_td.empty()) {
            E1 = 0.0;
            for (int k = 0; k < Kt; ++k) {
                double num = 0.0, den = 0.0;
                for (int i = 0; i < nt; ++i) {
                    const double wgt = (i == 0 || i == nt - 1) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
                    const double a = td[(size_t)k * nt + i], b = prev_td[(size_t)k * nt + i];
                    num += wgt * (a - b) * (a - b);
                    den += wgt * a * a;
                }
                E1 = std::max(E1, num / den);
            }
        }
        prev_td.swap(td);
        int kmax = 0;
        for (int k = 1; k < K; ++k)
            if (e[k] > e[kmax])
                kmax = k;
        s_new.clear();
        for (int g : afs_select(diffs[kmax], G, omega, S, dw, P.q))
            s_new.push_back(cplx(P.eta, g >= 0 ? omega * g / (G - 1) : omega));
        R.E1.push_back(E1);
        R.E2.push_back(E2);
        R.J.push_back(J);
        R.MH.push_back(MH);
        R.ML.push_back(ML);
        R.model = mH;
        return {E1, E2};
    };
    auto add = [&](std::vector<cplx> sn) {
        if ((int)sn.size() > max_Nc - (int)S.size())
            sn.resize(std::max(0, max_Nc - (int)S.size()));
        if (sn.empty())
            return;
        std::vector<cplx> f;
        resp(sn, f, R.model.poles.empty() ? nullptr : &R.model);
        S.insert(S.end(), sn.begin(), sn.end());
        Fv.insert(Fv.end(), f.begin(), f.end());
    };
    auto pass = [&](std::pair<double, double> e) { return e.first < P.E1_bar && e.second < P.E2_bar; };
    std::pair<double, double> err = analyse();
    bool converged = false, capped = false;
    while (true) {
        if (pass(err)) {
            // stage 3 (Eq. 14): Jc further steps, one frequency each, must all pass
            int passed = 0;
            while (passed < P.Jc && (int)S.size() < max_Nc) {
                add(std::vector<cplx>(s_new.begin(), s_new.begin() + 1));
                err = analyse();
                if (!pass(err))
                    break;
                ++passed;
            }
            if (passed == P.Jc) {
                converged = true;
                break;
            }
            if ((int)S.size() >= max_Nc) {
                capped = true;  // validation cut short by the cap: not converged
                break;
            }
            continue;
        }
        if ((int)S.size() >= max_Nc) {
            capped = true;
            break;
        }
        add(s_new);
        err = analyse();
    }
    R.s = S;
    R.F = Fv;
    R.converged = converged ? 1 : 0;
    R.capped = capped ? 1 : 0;
}

}  // namespace afsbem

using namespace afsbem;

struct afsbem_afs_result {
    AfsResult r;
};

template <class F>
static int guarded_d(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return AFSBEM_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return AFSBEM_EINVAL;
    }
}

extern "C" {

int afsbem_fsm_grid(double P, double eta, int32_t Ns, double *s_out) {
    return guarded_d([&] {
        AFS_REQUIRE(P > 0 && Ns >= 2 && Ns % 2 == 0 && s_out && std::isfinite(eta), AFSBEM_EINVAL,
                    "fsm_grid needs P > 0, even Ns >= 2 and an output array");
        for (int k = 0; k <= Ns / 2; ++k) {
            s_out[2 * k] = eta;
            s_out[2 * k + 1] = 2.0 * kPi * k / P;
        }
        return AFSBEM_OK;
    });
}

int afsbem_fsm_invert(double P, double eta, int32_t Ns, int window, int64_t n_sig, const double *H, double *h_out) {
    return guarded_d([&] {
        AFS_REQUIRE(P > 0 && Ns >= 2 && Ns % 2 == 0 && n_sig >= 0 && H && h_out, AFSBEM_EINVAL,
                    "fsm_invert needs P > 0, even Ns >= 2 and non-null arrays");
        AFS_REQUIRE(window == 0 || window == 1, AFSBEM_EINVAL, "window must be 0 (none) or 1 (Hann)");
        const int half = Ns / 2;
        for (int64_t q = 0; q < n_sig; ++q) {
            // full spectrum by conjugate symmetry, trapezoid weights, window
            std::vector<cplx> X(Ns);
            for (int k = 0; k <= half; ++k) {
                cplx hk(H[2 * ((size_t)q * (half + 1) + k)], H[2 * ((size_t)q * (half + 1) + k) + 1]);
                double w = window ? 0.5 * (1.0 + std::cos(2.0 * kPi * k / Ns)) : 1.0;
                if (k == half) {
                    // the +-Omega end points of the trapezoid, half weight each
                    X[k] = w * hk.real();
                    continue;
                }
                X[k] = w * hk;
                if (k > 0)
                    X[Ns - k] = w * std::conj(hk);
            }
            std::vector<cplx> y = dft_plus(X);
            for (int n = 0; n < Ns; ++n) {
                const double t = n * P / Ns;
                h_out[(size_t)q * Ns + n] = std::exp(eta * t) * y[n].real() / P;
            }
        }
        return AFSBEM_OK;
    });
}

int afsbem_vf_fit(int32_t J, const double *s, int32_t K, const double *F, int32_t M, const double *init_poles,
                  int32_t n_iter, double omega_max, double *poles_out, double *residues_out, double *rms_out) {
    return guarded_d([&] {
        AFS_REQUIRE(J >= 1 && K >= 1 && M >= 1 && s && F && poles_out && residues_out, AFSBEM_EINVAL,
                    "vf_fit: bad sizes or null pointers");
        AFS_REQUIRE(2 * J >= M, AFSBEM_EINVAL, "vf_fit: need at least M/2 samples");
        std::vector<cplx> sv(J), Fv((size_t)K * J);
        for (int j = 0; j < J; ++j)
            sv[j] = cplx(s[2 * j], s[2 * j + 1]);
        for (size_t i = 0; i < Fv.size(); ++i)
            Fv[i] = cplx(F[2 * i], F[2 * i + 1]);
        std::vector<cplx> p0;
        if (init_poles) {
            for (int m = 0; m < M; ++m)
                p0.push_back(cplx(init_poles[2 * m], init_poles[2 * m + 1]));
        } else {
            double om = omega_max;
            if (!(om > 0))
                for (const cplx &x : sv)
                    om = std::max(om, x.imag());
            p0 = vf_initial_poles(M, om);
        }
        VfModel mdl = vf_fit_model(sv, K, Fv, K, Fv, M, p0, n_iter);
        AFS_REQUIRE((int)mdl.poles.size() == M, AFSBEM_EINVAL, "vf_fit: pole count changed");
        for (int m = 0; m < M; ++m) {
            poles_out[2 * m] = mdl.poles[m].real();
            poles_out[2 * m + 1] = mdl.poles[m].imag();
        }
        double ss = 0.0;
        for (int k = 0; k < K; ++k) {
            for (int m = 0; m < M; ++m) {
                residues_out[2 * ((size_t)k * M + m)] = mdl.res[(size_t)k * M + m].real();
                residues_out[2 * ((size_t)k * M + m) + 1] = mdl.res[(size_t)k * M + m].imag();
            }
            for (int j = 0; j < J; ++j)
                ss += std::norm(vf_eval1(mdl, k, sv[j]) - Fv[(size_t)k * J + j]);
        }
        if (rms_out)
            *rms_out = std::sqrt(ss / ((double)K * J));
        return AFSBEM_OK;
    });
}

int afsbem_vf_residues(int32_t J, const double *s, int64_t n_fun, const double *F, int32_t M, const double *poles,
                       double *residues_out) {
    return guarded_d([&] {
        AFS_REQUIRE(J >= 1 && n_fun >= 1 && M >= 1 && s && F && poles && residues_out, AFSBEM_EINVAL,
                    "vf_residues: bad sizes or null pointers");
        std::vector<cplx> sv(J), Fv((size_t)n_fun * J), p(M);
        for (int j = 0; j < J; ++j)
            sv[j] = cplx(s[2 * j], s[2 * j + 1]);
        for (size_t i = 0; i < Fv.size(); ++i)
            Fv[i] = cplx(F[2 * i], F[2 * i + 1]);
        for (int m = 0; m < M; ++m)
            p[m] = cplx(poles[2 * m], poles[2 * m + 1]);
        std::vector<cplx> pout;
        std::vector<cplx> R = vf_identify_residues(sv, n_fun, Fv, p, pout);
        // residues are returned in the caller's pole order
        for (int m = 0; m < M; ++m) {
            int best = 0;
            for (int q = 1; q < M; ++q)
                if (std::abs(pout[q] - p[m]) < std::abs(pout[best] - p[m]))
                    best = q;
            for (int64_t k = 0; k < n_fun; ++k) {
                residues_out[2 * ((size_t)k * M + m)] = R[(size_t)k * M + best].real();
                residues_out[2 * ((size_t)k * M + m) + 1] = R[(size_t)k * M + best].imag();
            }
        }
        return AFSBEM_OK;
    });
}

int afsbem_vf_eval(int32_t M, const double *poles, int64_t n_fun, const double *residues, int32_t n_s, const double *s,
                   double *f_out) {
    return guarded_d([&] {
        AFS_REQUIRE(M >= 1 && n_fun >= 1 && n_s >= 0 && poles && residues && s && f_out, AFSBEM_EINVAL,
                    "vf_eval: bad sizes or null pointers");
        for (int64_t k = 0; k < n_fun; ++k)
            for (int j = 0; j < n_s; ++j) {
                cplx acc = 0.0;
                const cplx sj(s[2 * j], s[2 * j + 1]);
                for (int m = 0; m < M; ++m)
                    acc += cplx(residues[2 * ((size_t)k * M + m)], residues[2 * ((size_t)k * M + m) + 1]) /
                           (sj - cplx(poles[2 * m], poles[2 * m + 1]));
                f_out[2 * ((size_t)k * n_s + j)] = acc.real();
                f_out[2 * ((size_t)k * n_s + j) + 1] = acc.imag();
            }
        return AFSBEM_OK;
    });
}

int afsbem_vf_eval_time(int32_t M, const double *poles, int64_t n_fun, const double *residues, int32_t n_t,
                        const double *t, double *f_out) {
    return guarded_d([&] {
        AFS_REQUIRE(M >= 1 && n_fun >= 1 && n_t >= 0 && poles && residues && t && f_out, AFSBEM_EINVAL,
                    "vf_eval_time: bad sizes or null pointers");
        for (int64_t k = 0; k < n_fun; ++k)
            for (int i = 0; i < n_t; ++i) {
                cplx acc = 0.0;
                for (int m = 0; m < M; ++m)
                    acc += cplx(residues[2 * ((size_t)k * M + m)], residues[2 * ((size_t)k * M + m) + 1]) *
                           std::exp(cplx(poles[2 * m], poles[2 * m + 1]) * t[i]);
                f_out[(size_t)k * n_t + i] = acc.real();
            }
        return AFSBEM_OK;
    });
}

int afsbem_time_synthesis_device(int32_t M, const double *poles, int32_t J, const double *s, int64_t N,
                                 const void *d_X, int32_t Nt, const double *t, void *d_h, void *hip_stream) {
    return guarded_d([&] {
        AFS_REQUIRE(M >= 1 && J >= 1 && N >= 0 && Nt >= 0, AFSBEM_EINVAL, "bad sizes");
        AFS_REQUIRE(poles && s && (N == 0 || d_X) && (Nt == 0 || t) && (N == 0 || Nt == 0 || d_h), AFSBEM_EINVAL,
                    "null pointer argument");
        if (N == 0 || Nt == 0)
            return (int)AFSBEM_OK;
        AFS_REQUIRE((reinterpret_cast<uintptr_t>(d_X) & 15) == 0 && (reinterpret_cast<uintptr_t>(d_h) & 7) == 0,
                    AFSBEM_EINVAL, "d_X must be 16-byte aligned and d_h 8-byte aligned");
        std::vector<cplx> sv(J), pv(M);
        for (int j = 0; j < J; ++j)
            sv[j] = cplx(s[2 * j], s[2 * j + 1]);
        for (int m = 0; m < M; ++m)
            pv[m] = cplx(poles[2 * m], poles[2 * m + 1]);
        AFS_REQUIRE(group_poles(pv).dim() <= 2 * J, AFSBEM_EINVAL, "more poles than real samples (2 J)");
        const int Kpad = (2 * J + 3) / 4 * 4;
        const std::vector<double> K = synthesis_matrix(sv, pv, t, Nt, Kpad);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        double *dK = nullptr;
        AFS_HIP(hipMallocAsync((void **)&dK, K.size() * 8, st));
        AFS_HIP(hipMemcpyAsync(dK, K.data(), K.size() * 8, hipMemcpyHostToDevice, st));
        launch_synthesis(N, J, Kpad, Nt, static_cast<const double *>(d_X), dK, static_cast<double *>(d_h), st);
        AFS_HIP(hipFreeAsync(dK, st));
        AFS_HIP(hipStreamSynchronize(st));  // K lives on this host frame until the copy has run
        return (int)AFSBEM_OK;
    });
}

int afsbem_model_sample_device(int32_t M, const double *poles, int32_t J, const double *s, int64_t N,
                               const void *d_X, int32_t n_z, const double *z, void *d_H, void *hip_stream) {
    return guarded_d([&] {
        AFS_REQUIRE(M >= 1 && J >= 1 && N >= 0 && n_z >= 0, AFSBEM_EINVAL, "bad sizes");
        AFS_REQUIRE(poles && s && (N == 0 || d_X) && (n_z == 0 || z) && (N == 0 || n_z == 0 || d_H), AFSBEM_EINVAL,
                    "null pointer argument");
        AFS_REQUIRE(n_z <= (1 << 24), AFSBEM_EINVAL, "too many frequencies (at most 2^24)");  // 2 n_z columns
        if (N == 0 || n_z == 0)
            return (int)AFSBEM_OK;
        AFS_REQUIRE((reinterpret_cast<uintptr_t>(d_X) & 15) == 0 && (reinterpret_cast<uintptr_t>(d_H) & 7) == 0,
                    AFSBEM_EINVAL, "d_X must be 16-byte aligned and d_H 8-byte aligned");
        std::vector<cplx> sv(J), pv(M), zv(n_z);
        for (int j = 0; j < J; ++j)
            sv[j] = cplx(s[2 * j], s[2 * j + 1]);
        for (int m = 0; m < M; ++m)
            pv[m] = cplx(poles[2 * m], poles[2 * m + 1]);
        for (int k = 0; k < n_z; ++k)
            zv[k] = cplx(z[2 * k], z[2 * k + 1]);
        AFS_REQUIRE(group_poles(pv).dim() <= 2 * J, AFSBEM_EINVAL, "more poles than real samples (2 J)");
        const int Kpad = (2 * J + 3) / 4 * 4;
        const std::vector<double> K = sampling_matrix(sv, pv, zv, Kpad);
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        double *dK = nullptr;
        AFS_HIP(hipMallocAsync((void **)&dK, K.size() * 8, st));
        AFS_HIP(hipMemcpyAsync(dK, K.data(), K.size() * 8, hipMemcpyHostToDevice, st));
        launch_synthesis(N, J, Kpad, 2 * n_z, static_cast<const double *>(d_X), dK, static_cast<double *>(d_H), st);
        AFS_HIP(hipFreeAsync(dK, st));
        AFS_HIP(hipStreamSynchronize(st));  // K lives on this host frame until the copy has run
        return (int)AFSBEM_OK;
    });
}

int afsbem_fsm_invert_device(double P, double eta, int32_t Ns, int window, int64_t n_sig, const void *d_H,
                             void *d_h, void *hip_stream) {
    return guarded_d([&] {
        AFS_REQUIRE(P > 0 && std::isfinite(P) && std::isfinite(eta) && n_sig >= 0, AFSBEM_EINVAL,
                    "fsm_invert_device needs P > 0 and n_sig >= 0");
        AFS_REQUIRE(Ns >= 2 && Ns <= (1 << kFsmMaxLog2) && (Ns & (Ns - 1)) == 0, AFSBEM_EINVAL,
                    "fsm_invert_device: Ns must be a power of two in [2, 4096]");
        AFS_REQUIRE(window == 0 || window == 1, AFSBEM_EINVAL, "window must be 0 (none) or 1 (Hann)");
        AFS_REQUIRE(n_sig == 0 || (d_H && d_h), AFSBEM_EINVAL, "null pointer argument");
        if (n_sig == 0)
            return (int)AFSBEM_OK;
        AFS_REQUIRE((reinterpret_cast<uintptr_t>(d_H) & 15) == 0 && (reinterpret_cast<uintptr_t>(d_h) & 7) == 0,
                    AFSBEM_EINVAL, "d_H must be 16-byte aligned and d_h 8-byte aligned");
        int L = 0;
        while ((1 << L) < Ns)
            ++L;
        // tables: W[m] = e^{2 pi i m / Ns}; E[n] = e^{eta t_n} / P, t_n = n P / Ns
        std::vector<double> tab((size_t)3 * Ns);
        for (int m = 0; m < Ns; ++m) {
            const cplx w = unit_root(m, Ns);
            tab[2 * m] = w.real();
            tab[2 * m + 1] = w.imag();
            tab[(size_t)2 * Ns + m] = std::exp(eta * (m * P / Ns)) / P;
        }
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        double *dT = nullptr;
        AFS_HIP(hipMallocAsync((void **)&dT, tab.size() * 8, st));
        AFS_HIP(hipMemcpyAsync(dT, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st));
        launch_fsm(L, n_sig, window, static_cast<const double *>(d_H), dT, dT + 2 * Ns, static_cast<double *>(d_h), st);
        AFS_HIP(hipFreeAsync(dT, st));
        AFS_HIP(hipStreamSynchronize(st));  // the tables live on this host frame until the copy has run
        return (int)AFSBEM_OK;
    });
}

int afsbem_afs_params_default(afsbem_afs_params *p) {
    if (!p) {
        set_error("null params");
        return AFSBEM_EINVAL;
    }
    p->T = 1.0;
    p->eta = 3.0 * std::log(10.0);
    p->Ns = 256;
    p->J0 = 16;
    p->alpha_H = 2.0;
    p->alpha_L = 2.3;
    p->E1_bar = 1e-4;
    p->E2_bar = 2e-3;
    p->Jc = 3;
    p->max_Nc = 0;
    p->grid_pts = 2048;
    p->n_iter = 10;
    p->q = 1;
    return AFSBEM_OK;
}

static void check_afs_params(const afsbem_afs_params *P, int32_t K, int32_t Kt) {
    AFS_REQUIRE(P, AFSBEM_EINVAL, "null params");
    AFS_REQUIRE(P->T > 0 && P->Ns >= 4 && P->J0 >= 4 && P->alpha_H >= 1.0 && P->alpha_L > P->alpha_H &&
                    P->Jc >= 0 && P->grid_pts >= 16 && P->n_iter >= 1 && std::isfinite(P->eta) && P->q >= 1 &&
                    P->q <= 1024,
                AFSBEM_EINVAL, "invalid AFS parameters");
    AFS_REQUIRE(K >= 1 && Kt >= K, AFSBEM_EINVAL, "need 1 <= K <= Kt");
}

int afsbem_afs_run(const afsbem_afs_params *P, int32_t K, int32_t Kt, afsbem_response_fn fn, void *user,
                   afsbem_afs_result **out) {
    return guarded_d([&] {
        check_afs_params(P, K, Kt);
        AFS_REQUIRE(fn && out, AFSBEM_EINVAL, "null callback or output");
        auto *res = new afsbem_afs_result();
        try {
            ResponseFn resp = [&](const std::vector<cplx> &s, std::vector<cplx> &f, const VfModel *) {
                std::vector<double> sv(2 * s.size()), fv(2 * s.size() * Kt);
                for (size_t i = 0; i < s.size(); ++i) {
                    sv[2 * i] = s[i].real();
                    sv[2 * i + 1] = s[i].imag();
                }
                const int rc = fn((int32_t)s.size(), sv.data(), Kt, fv.data(), user);
                AFS_REQUIRE(rc == 0, AFSBEM_EINVAL, "response callback returned " + std::to_string(rc));
                f.resize(s.size() * Kt);
                for (size_t i = 0; i < f.size(); ++i)
                    f[i] = cplx(fv[2 * i], fv[2 * i + 1]);
            };
            afs_run_impl(*P, K, Kt, resp, res->r);
        } catch (...) {
            delete res;
            throw;
        }
        *out = res;
        return AFSBEM_OK;
    });
}


int afsbem_afs_run_problem(afsbem_problem *p, const afsbem_afs_params *params, const double *bc_shape, int load_kind,
                           const int64_t *dof_idx, int32_t K, int32_t Kt, const afsbem_solve_opts *opts,
                           afsbem_afs_result **out) {
    return guarded_d([&] {
        check_afs_params(params, K, Kt);
        AFS_REQUIRE(p && bc_shape && dof_idx && out, AFSBEM_EINVAL, "null pointer argument");
        AFS_REQUIRE(load_kind == 0 || load_kind == 1, AFSBEM_EINVAL, "load_kind must be 0 (Heaviside) or 1");
        int64_t nt = 0;
        if (afsbem_problem_info(p, &nt, nullptr, nullptr, nullptr) != AFSBEM_OK)
            throw Error{AFSBEM_EINVAL, "invalid problem"};
        const int64_t N = 3 * nt;
        for (int32_t k = 0; k < Kt; ++k)
            AFS_REQUIRE(dof_idx[k] >= 0 && dof_idx[k] < N, AFSBEM_EINVAL, "dof index out of range");
        afsbem_solve_opts o;
        afsbem_solve_opts_default(&o);
        if (opts)
            o = *opts;
        hipStream_t st = nullptr;
        AFS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        std::vector<void *> bufs;
        auto dmalloc = [&](size_t bytes) {
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, bytes);
            if (e != hipSuccess)
                throw Error{AFSBEM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
            bufs.push_back(q);
            return q;
        };
        std::vector<std::pair<cplx, double *>> solved;  // (s, device solution)
        auto *res = new afsbem_afs_result();
        try {
            ResponseFn resp = [&](const std::vector<cplx> &s, std::vector<cplx> &f, const VfModel *model) {
                const int n = (int)s.size();
                std::vector<double> hb((size_t)n * N * 2), sv(2 * n);
                for (int i = 0; i < n; ++i) {
                    const cplx ld = load_kind == 0 ? 1.0 / s[i] : cplx(1.0, 0.0);
                    sv[2 * i] = s[i].real();
                    sv[2 * i + 1] = s[i].imag();
                    for (int64_t q = 0; q < N; ++q) {
                        hb[2 * ((size_t)i * N + q)] = bc_shape[q] * ld.real();
                        hb[2 * ((size_t)i * N + q) + 1] = bc_shape[q] * ld.imag();
                    }
                }
                double *dbc = (double *)dmalloc(hb.size() * 8);
                double *da = (double *)dmalloc(hb.size() * 8);
                AFS_HIP(hipMemcpyAsync(dbc, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, st));
                afsbem_solve_opts oo = o;
                const double *x0 = nullptr;
                const bool warm = o.warm_start != AFSBEM_WARM_NONE;
                const int M = model ? (int)model->poles.size() : 0;
                const bool use_model = warm && o.warm_start == AFSBEM_WARM_MODEL && M > 0 && (int)solved.size() > M;
                if (warm && !solved.empty()) {
                    // one start per requested frequency: the current rational model's prediction for every
                    // unknown, or the nearest sampled solution (residual-optimal scaling inside the solve)
                    double *xs = (double *)dmalloc((size_t)n * N * 16);
                    std::vector<cplx> sj(solved.size()), al, be;
                    for (size_t q = 0; q < solved.size(); ++q)
                        sj[q] = solved[q].first;
                    for (int i = 0; i < n; ++i) {
                        double *xi = xs + 2 * (size_t)i * N;
                        if (use_model) {
                            vf_prediction_weights(sj, model->poles, s[i], al, be);
                            AFS_HIP(hipMemsetAsync(xi, 0, (size_t)N * 16, st));
                            for (size_t q = 0; q < solved.size(); ++q)
                                vec_axpy_conj(N, al[q].real(), al[q].imag(), be[q].real(), be[q].imag(),
                                              solved[q].second, xi, st);
                        } else {
                            size_t best = 0;
                            for (size_t q = 1; q < solved.size(); ++q)
                                if (std::abs(solved[q].first - s[i]) < std::abs(solved[best].first - s[i]))
                                    best = q;
                            AFS_HIP(hipMemcpyAsync(xi, solved[best].second, (size_t)N * 16, hipMemcpyDeviceToDevice,
                                                   st));
                        }
                    }
                    x0 = xs;
                    // learned: the network's prediction combined with the nearest solution (the first
                    // frequency's "previous" vector; later ones in the call follow their predecessor)
                    oo.warm_start = o.warm_start == AFSBEM_WARM_LEARNED ? AFSBEM_WARM_LEARNED : AFSBEM_WARM_USER;
                } else if (n > 1 && warm) {
                    // the initial round: each from the one before (learned: trained as the round goes)
                    oo.warm_start = o.warm_start == AFSBEM_WARM_LEARNED ? AFSBEM_WARM_LEARNED : AFSBEM_WARM_PREV;
                } else {
                    oo.warm_start = o.warm_start == AFSBEM_WARM_LEARNED ? AFSBEM_WARM_LEARNED : AFSBEM_WARM_NONE;
                }
                std::vector<afsbem_solve_stats> stats(n);
                const int rc = afsbem_solve_device(p, n, sv.data(), dbc, x0, da, nullptr, nullptr, &oo, stats.data(),
                                                   st);
                if (rc != AFSBEM_OK && rc != AFSBEM_ENOCONV)
                    throw Error{rc, std::string("solve failed: ") + afsbem_last_error()};
                for (const auto &q : stats) {
                    res->r.matvecs += q.iters;
                    // a sample that missed the tolerance is kept (best iterate) but counted: the
                    // result does not report convergence when any sample missed it
                    if (!(q.rel_res_fp64 <= o.tol))
                        ++res->r.unconverged;
                    if (!(q.rel_res_fp64 <= res->r.worst_rel_res))
                        res->r.worst_rel_res = q.rel_res_fp64;
                }
                std::vector<double> ha(hb.size());
                AFS_HIP(hipMemcpyAsync(ha.data(), da, ha.size() * 8, hipMemcpyDeviceToHost, st));
                AFS_HIP(hipStreamSynchronize(st));
                f.resize((size_t)n * Kt);
                for (int i = 0; i < n; ++i) {
                    for (int32_t k = 0; k < Kt; ++k) {
                        const size_t q = (size_t)i * N + dof_idx[k];
                        f[(size_t)i * Kt + k] = cplx(ha[2 * q], ha[2 * q + 1]);
                    }
                    solved.push_back({s[i], da + 2 * (size_t)i * N});
                }
            };
            afs_run_impl(*params, K, Kt, resp, res->r);
            if (res->r.unconverged > 0)
                res->r.converged = 0;
        } catch (...) {
            delete res;
            (void)hipStreamSynchronize(st);
            for (void *q : bufs)
                (void)hipFree(q);
            (void)hipStreamDestroy(st);
            throw;
        }
        (void)hipStreamSynchronize(st);
        for (void *q : bufs)
            (void)hipFree(q);
        (void)hipStreamDestroy(st);
        *out = res;
        return AFSBEM_OK;
    });
}

int afsbem_afs_result_info(const afsbem_afs_result *r, int32_t *Nc, int32_t *M, int32_t *n_steps, int32_t *converged) {
    return guarded_d([&] {
        AFS_REQUIRE(r, AFSBEM_EINVAL, "null result");
        if (Nc)
            *Nc = (int32_t)r->r.s.size();
        if (M)
            *M = (int32_t)r->r.model.poles.size();
        if (n_steps)
            *n_steps = (int32_t)r->r.E1.size();
        if (converged)
            *converged = r->r.converged;
        return AFSBEM_OK;
    });
}

int afsbem_afs_result_work(const afsbem_afs_result *r, int64_t *matvecs) {
    return guarded_d([&] {
        AFS_REQUIRE(r && matvecs, AFSBEM_EINVAL, "null argument");
        *matvecs = r->r.matvecs;
        return AFSBEM_OK;
    });
}

int afsbem_afs_result_status(const afsbem_afs_result *r, int32_t *capped, int32_t *unconverged_solves,
                             double *worst_rel_res) {
    return guarded_d([&] {
        AFS_REQUIRE(r, AFSBEM_EINVAL, "null result");
        if (capped)
            *capped = r->r.capped;
        if (unconverged_solves)
            *unconverged_solves = r->r.unconverged;
        if (worst_rel_res)
            *worst_rel_res = r->r.worst_rel_res;
        return AFSBEM_OK;
    });
}

int afsbem_afs_result_get(const afsbem_afs_result *r, double *s_out, double *F_out, double *poles_out,
                          double *residues_out, double *E1_out, double *E2_out) {
    return guarded_d([&] {
        AFS_REQUIRE(r, AFSBEM_EINVAL, "null result");
        const AfsResult &R = r->r;
        for (size_t i = 0; s_out && i < R.s.size(); ++i) {
            s_out[2 * i] = R.s[i].real();
            s_out[2 * i + 1] = R.s[i].imag();
        }
        for (size_t i = 0; F_out && i < R.F.size(); ++i) {
            F_out[2 * i] = R.F[i].real();
            F_out[2 * i + 1] = R.F[i].imag();
        }
        for (size_t i = 0; poles_out && i < R.model.poles.size(); ++i) {
            poles_out[2 * i] = R.model.poles[i].real();
            poles_out[2 * i + 1] = R.model.poles[i].imag();
        }
        for (size_t i = 0; residues_out && i < R.model.res.size(); ++i) {
            residues_out[2 * i] = R.model.res[i].real();
            residues_out[2 * i + 1] = R.model.res[i].imag();
        }
        for (size_t i = 0; E1_out && i < R.E1.size(); ++i)
            E1_out[i] = R.E1[i];
        for (size_t i = 0; E2_out && i < R.E2.size(); ++i)
            E2_out[i] = R.E2[i];
        return AFSBEM_OK;
    });
}

int afsbem_afs_result_destroy(afsbem_afs_result *r) {
    delete r;
    return AFSBEM_OK;
}

}  // extern "C"
