"""Pins of the FP64 oracle against what mathematics fixes independently of it:
closed forms, identities, brute-force quadrature and library routines.  Each
test is chosen so that a plausible mistake in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong weight) fails it."""
import numpy as np
import pytest

from oracle import bem
from synth import meshgen as mg
from tests import analytic

MAT = bem.DEFAULT_MATERIAL
LAM, CS, CP, BETA = bem.material_constants(MAT)


# ----------------------------------------------------------------- kernels
@pytest.mark.parametrize("x", [0.3 + 0.2j, 0.9 + 0.5j, 1.2 - 0.3j, 0.5 + 1.0j, 1.4 + 0.0j, 0.05 + 0.7j])
def test_series_equals_closed_form(x):
    a = bem.radial(x, BETA, 1)
    b = bem.radial(x, BETA, 2)
    assert np.max(np.abs(a - b) / np.abs(b)) < 1e-11


def test_static_limit_is_kelvin():
    x = np.zeros(3)
    y = np.array([0.3, -0.2, 0.5])
    U, _ = bem.kernel(0.0, x, y, np.array([0, 0, 1.0]))
    assert np.max(np.abs(U - analytic.kelvin_U(x, y, MAT[0], MAT[1]))) < 1e-15
    # and the small-s limit approaches it continuously
    U2, _ = bem.kernel(1e-7 + 1e-7j, x, y, np.array([0, 0, 1.0]))
    assert np.max(np.abs(U2 - analytic.kelvin_U(x, y, MAT[0], MAT[1]))) < 1e-7


def test_symmetries():
    s = 0.4 + 2.1j
    x = np.array([0.1, 0.2, -0.3])
    y = np.array([-0.5, 0.9, 0.4])
    n = np.array([0, 0, 1.0])
    U1, _ = bem.kernel(s, x, y, n)
    U2, _ = bem.kernel(s, y, x, n)
    assert np.max(np.abs(U1 - U1.T)) < 1e-16
    assert np.max(np.abs(U1 - U2)) < 1e-16


def _U(s, x, y):
    return bem.kernel(s, x, y, np.array([0, 0, 1.0]))[0]


def test_radial_derivatives_by_finite_differences():
    s = 0.3 + 1.7j
    for r in [0.2, 0.7, 1.9]:
        def psi_chi(rr):
            f = bem.radial(s * rr / CS, BETA)
            return f[0] / rr, f[1] / rr
        h = 1e-3
        p2, c2 = psi_chi(r + 2 * h)
        p1, c1 = psi_chi(r + h)
        p0, c0 = psi_chi(r - h)
        pm, cm = psi_chi(r - 2 * h)
        f = bem.radial(s * r / CS, BETA)
        dp = (-p2 + 8 * p1 - 8 * p0 + pm) / (12 * h)
        dc = (-c2 + 8 * c1 - 8 * c0 + cm) / (12 * h)
        assert abs(dp - f[2] / r ** 2) < 1e-8 * max(1, abs(f[2] / r ** 2))
        assert abs(dc - f[3] / r ** 2) < 1e-8 * max(1, abs(f[3] / r ** 2))


@pytest.mark.parametrize("s", [0.25 + 0.0j, 0.25 + 2.0j, 1.5 + 4.0j])
def test_navier_equation_residual(s):
    """mu lap U + (lam+mu) grad div U - rho s^2 U = 0 away from the source,
    4th-order central differences on every column of U."""
    x = np.zeros(3)
    y0 = np.array([0.4, -0.3, 0.5])
    h = 2e-3
    e = np.eye(3)

    def d2(i, j):
        if i == j:
            return (-_U(s, x, y0 + 2 * h * e[i]) + 16 * _U(s, x, y0 + h * e[i]) - 30 * _U(s, x, y0)
                    + 16 * _U(s, x, y0 - h * e[i]) - _U(s, x, y0 - 2 * h * e[i])) / (12 * h * h)
        w = {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}
        return sum(w[a] * w[b] * _U(s, x, y0 + a * h * e[i] + b * h * e[j])
                   for a in w for b in w) / (144 * h * h)

    D = [[d2(i, j) for j in range(3)] for i in range(3)]
    U0 = _U(s, x, y0)
    mu, rho = MAT[0], MAT[2]
    # U[f, j]: component j of the field of a force along f
    res = np.zeros((3, 3), complex)
    for f in range(3):
        for j in range(3):
            lap = sum(D[k][k][f, j] for k in range(3))
            gdiv = sum(D[j][l][f, l] for l in range(3))
            res[f, j] = mu * lap + (LAM + mu) * gdiv - rho * s * s * U0[f, j]
    scale = np.max(np.abs(D[0][0]))
    assert np.max(np.abs(res)) < 1e-7 * scale


@pytest.mark.parametrize("s", [0.0, 0.25 + 1.0j, 0.8 + 5.0j])
def test_traction_is_hooke_of_grad_U(s):
    x = np.array([0.05, 0.1, -0.02])
    y = np.array([0.5, -0.3, 0.35])
    n = np.array([0.3, -0.5, 0.8])
    n = n / np.linalg.norm(n)
    h = 1e-5
    g = np.zeros((3, 3, 3), complex)  # g[f, j, l] = d U_fj / d y_l
    for l in range(3):
        d = np.zeros(3)
        d[l] = h
        g[:, :, l] = (_U(s, x, y + d) - _U(s, x, y - d)) / (2 * h)
    mu = MAT[0]
    T_fd = np.zeros((3, 3), complex)
    for f in range(3):
        eps = 0.5 * (g[f] + g[f].T)
        sig = LAM * np.trace(g[f]) * np.eye(3) + 2 * mu * eps
        T_fd[f] = sig @ n
    _, T = bem.kernel(s, x, y, n)
    assert np.max(np.abs(T - T_fd)) < 1e-7 * np.max(np.abs(T))


def test_static_traction_flux_balances_unit_force():
    """Equilibrium of a ball around the source: the tractions of the static
    solution on the outward normal integrate to -I."""
    x = np.array([0.1, 0.0, -0.2])
    R = 0.7
    ct, wt = np.polynomial.legendre.leggauss(40)
    nphi = 64
    acc = np.zeros((3, 3))
    for c, w in zip(ct, wt):
        st = np.sqrt(1 - c * c)
        for k in range(nphi):
            ph = 2 * np.pi * k / nphi
            nrm = np.array([st * np.cos(ph), st * np.sin(ph), c])
            _, T = bem.kernel(0.0, x, x + R * nrm, nrm)
            acc += w * (2 * np.pi / nphi) * R * R * T.real
    assert np.max(np.abs(acc + np.eye(3))) < 1e-12


# -------------------------------------------------------------- quadrature
def test_radon7_is_exact_to_degree_5():
    from math import factorial
    bary, w = bem.radon7()
    assert abs(w.sum() - 1) < 1e-15
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                q = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
                exact = 2 * factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 2)
                assert abs(q - exact) < 1e-15, (a, b, c)


@pytest.mark.parametrize("n", [3, 8, 16, 24])
def test_gauss_legendre_matches_library(n):
    x, w = bem.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    o = np.argsort(x)
    assert np.max(np.abs(x[o] - xr)) < 1e-14
    assert np.max(np.abs(w[o] - wr)) < 1e-14


def _duffy(P, x, nq, f):
    u, wu = np.polynomial.legendre.leggauss(nq)
    u = 0.5 * (u + 1)
    wu = 0.5 * wu
    acc = 0
    for a in range(3):
        pa, pb = P[a] - x, P[(a + 1) % 3] - x
        J = np.linalg.norm(np.cross(pa, pb))
        for i in range(nq):
            for j in range(nq):
                acc = acc + wu[i] * wu[j] * u[i] * J * f(x + u[i] * ((1 - u[j]) * pa + u[j] * pb))
    return acc


def test_self_element_against_duffy_brute_force():
    """Self integrals by an independent scheme: Duffy maps of the three
    sub-triangles for G and for T - T0, a fine angular sum for the CPV."""
    m = mg.cavity(1)
    cen, nrm, _, _ = bem.geometry(m)
    e = 5
    P = m.xyz[m.tri[e]]
    x, n = cen[e], nrm[e]
    s = 0.25 + 1.3j
    G, H = bem.blocks(m, s, [(e, e)])
    Gref = _duffy(P, x, 24, lambda y: bem.kernel(s, x, y, n)[0])
    assert np.max(np.abs(G[0] - Gref)) < 1e-9 * np.max(np.abs(Gref))

    def T0(y):
        rv = y - x
        r = np.linalg.norm(rv)
        rh = rv / r
        return BETA ** 2 / (4 * np.pi * r * r) * (np.outer(rh, n) - np.outer(n, rh))
    Hreg = _duffy(P, x, 24, lambda y: bem.kernel(s, x, y, n)[1] - T0(y))
    e1 = (P[0] - x) / np.linalg.norm(P[0] - x)
    e2 = np.cross(n, e1)
    nth = 20000
    cpv = np.zeros((3, 3))
    for t in (np.arange(nth) + 0.5) * 2 * np.pi / nth:
        eh = np.cos(t) * e1 + np.sin(t) * e2
        R = np.inf
        for a in range(3):
            pa, pb = P[a] - x, P[(a + 1) % 3] - x
            M = np.array([eh, -(pb - pa)]).T
            sol = np.linalg.lstsq(M, pa, rcond=None)[0]
            if sol[0] > 0 and -1e-9 <= sol[1] <= 1 + 1e-9:
                R = min(R, sol[0])
        cpv += (np.outer(eh, n) - np.outer(n, eh)) * np.log(R)
    cpv *= BETA ** 2 / (4 * np.pi) * (2 * np.pi / nth)
    Href = Hreg + cpv + 0.5 * np.eye(3)
    assert np.max(np.abs(H[0] - Href)) < 1e-7 * np.max(np.abs(Href))


def test_near_pair_subdivision_converges():
    """A near pair (adjacent elements) under the default policy agrees with a
    much finer policy (far ratio 6, deeper subdivision) to the 7-point rule's
    accuracy, and the coarse far rule alone is visibly worse."""
    m = mg.cavity(1)
    s = 0.25 + 1.0j
    cen, _, _, h = bem.geometry(m)
    d = np.linalg.norm(cen[:, None] - cen[None], axis=2)
    d[np.arange(len(d)), np.arange(len(d))] = np.inf
    mm, nn = np.unravel_index(np.argmin(d), d.shape)
    G0, H0 = bem.blocks(m, s, [(mm, nn)])
    G1, H1 = bem.blocks(m, s, [(mm, nn)], policy=(6.0, 12, 16, 16))
    Gf, Hf = bem.blocks(m, s, [(mm, nn)], policy=(0.0, 0, 16, 16))
    err = np.max(np.abs(H0 - H1)) / np.max(np.abs(H1))
    err_far = np.max(np.abs(Hf - H1)) / np.max(np.abs(H1))
    assert err < 2e-4
    assert err_far > 10 * err
    assert np.max(np.abs(G0 - G1)) / np.max(np.abs(G1)) < 2e-5


def test_rigid_body_row_sums_exterior():
    """Static rigid translation, exterior domain: sum_n H_mn = I."""
    rs = bem.rowsum_H_static(mg.cavity(2))
    assert np.max(np.abs(rs - np.eye(3))) < 2e-6


def test_rigid_body_row_sums_interior():
    """Static rigid translation, bounded domain: sum_n H_mn = 0."""
    rs = bem.rowsum_H_static(mg.rod(2.0, 1.0, 3, 6))
    assert np.max(np.abs(rs)) < 5e-5


# ------------------------------------------------------------------ solves
def test_cavity_closed_form_itself():
    """The analytic cavity field satisfies the radial Navier equation and the
    pressure condition (finite differences), and its static limit is Pa/(4mu)."""
    s = 0.3 + 0.8j
    u = analytic.cavity_field(s)
    h = 1e-4
    mu, nu, rho = MAT
    for r in [1.3, 2.0]:
        d1 = (u(r + h) - u(r - h)) / (2 * h)
        d2 = (u(r + h) - 2 * u(r) + u(r - h)) / (h * h)
        res = (LAM + 2 * mu) * (d2 + 2 * d1 / r - 2 * u(r) / r ** 2) - rho * s * s * u(r)
        assert abs(res) < 1e-5 * abs(rho * s * s * u(r))
    d1 = (u(1 + h) - u(1 - h)) / (2 * h)
    assert abs((LAM + 2 * mu) * d1 + 2 * LAM * u(1.0) + 1 / s) < 1e-7
    assert abs(1e-9 * analytic.cavity_ur(1e-9 + 0j) - 0.25) < 1e-6
    # the explicit rational form at the unit material
    for sv in [0.25 + 0.5j, 1 + 2j]:
        assert abs(analytic.cavity_ur(sv) - (1 + sv / np.sqrt(3)) / (sv * (sv * sv + 4 * sv / np.sqrt(3) + 4))) < 1e-14


def test_cavity_solution_converges_to_closed_form():
    s = 0.25 + 1.0j
    ur = analytic.cavity_ur(s)
    errs = []
    for L in (1, 2, 3):
        m = mg.cavity(L)
        _, u, _ = bem.solve(m, s)
        _, nrm, _, _ = bem.geometry(m)
        un = np.einsum("ij,ij->i", u, -nrm)
        errs.append(np.max(np.abs(un - ur)) / abs(ur))
    # measured: 0.106, 0.049, 0.022 (first order in h for flat facets)
    assert errs[2] < 0.03
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8


def test_point_source_manufactured_solution():
    """u = U(x0, .) e_z from a source inside the cavity is an exact exterior
    field; prescribing its traction must return its displacement."""
    s = 0.25 + 1.0j
    x0 = np.array([0.1, -0.05, 0.08])
    errs = []
    for L in (1, 2, 3):
        m = mg.cavity(L)
        c, nrm, _, _ = bem.geometry(m)
        uex = np.array([bem.kernel(s, x0, c[i], nrm[i])[0][2] for i in range(len(c))])
        tex = np.array([bem.kernel(s, x0, c[i], nrm[i])[1][2] for i in range(len(c))])
        a, _, _ = bem.solve(m, s, tex)
        errs.append(np.linalg.norm(a - uex.reshape(-1)) / np.linalg.norm(uex))
    # measured: 0.042, 0.0144, 0.0059
    assert errs[2] < 0.008
    assert errs[0] / errs[1] > 2.2 and errs[1] / errs[2] > 2.2


def test_rod_mixed_bc_closed_form():
    """nu = 0 rod: fixed end, step traction at the other end (1D solution)."""
    mat = (1.0, 0.0, 1.0)
    s = 0.5 + 0.3j
    errs = []
    for nw, nl in [(2, 6), (4, 12), (6, 18)]:
        m = mg.rod(3.0, 1.0, nw, nl)
        cen, _, _, _ = bem.geometry(m)
        _, u, t = bem.solve(m, s, mat=mat)
        free = m.bc_kind == 0
        uz = analytic.rod_uz(cen[:, 2], s, 3.0)
        errs.append(np.linalg.norm(u[free, 2] - uz[free]) / np.linalg.norm(uz[free]))
        fixed = m.bc_kind == 1
        tz = analytic.rod_t_fixed(s, 3.0)
        assert np.sqrt(np.mean(np.abs(t[fixed, 2] - tz) ** 2)) / abs(tz) < 0.04
    # measured: 0.027, 0.0127, 0.0081
    assert errs[2] < 0.01 and errs[0] > errs[1] > errs[2]


def test_gmres_matches_lu():
    m = mg.cavity(2)
    s = 0.25 + 2.0j
    A, b = bem.assemble(m, s)
    x_lu = bem.solve_dense(A, b)
    Dinv = bem.block_jacobi(A)
    x, it, hist = bem.gmres(lambda v: A @ v, b, tol=1e-12, restart=20,
                            precond=lambda v: bem.apply_block(Dinv, v))
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-10
    assert hist[-1] <= 1e-12
    assert it < 60
