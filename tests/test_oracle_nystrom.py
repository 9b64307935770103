"""Pins of the Nystrom oracle (curved quadratic triangles, the paper's own
discretisation in Section 2.1) against what mathematics fixes independently
of it: the rule's exactness, interpolation identities, the element map,
brute-force quadrature, the flat-element oracle, rigid-body row sums and the
cavity closed form."""
from math import factorial

import numpy as np
import pytest

from oracle import bem
from oracle import nystrom as ny
from synth import meshgen as mg
from tests import analytic


def test_gauss6_is_exact_to_degree_4():
    pt, w = ny.gauss6()
    for p in range(5):
        for q in range(5 - p):
            exact = factorial(p) * factorial(q) / factorial(p + q + 2)
            assert abs(np.sum(w * pt[:, 0] ** p * pt[:, 1] ** q) - exact) < 1e-16
    assert np.all(w > 0) and np.all(pt > 0) and np.all(pt.sum(1) < 1)
    # and not to degree 5 (so it is the 6-point degree-4 rule, not a relabelled other one)
    assert abs(np.sum(w * pt[:, 0] ** 5) - factorial(5) / factorial(7)) > 1e-5


def test_lagrange_basis_interpolates_quadratics():
    pt, _ = ny.gauss6()
    C = ny.lagrange6()
    mono = lambda x, y: np.stack([np.ones_like(x), x, y, x * x, x * y, y * y])
    L_nodes = C @ mono(pt[:, 0], pt[:, 1])
    assert np.max(np.abs(L_nodes - np.eye(6))) < 1e-13
    rng = np.random.default_rng(3)
    z = rng.random((50, 2)) * 0.5
    L = C @ mono(z[:, 0], z[:, 1])                        # (6, 50)
    M_nodes = mono(pt[:, 0], pt[:, 1])                     # (6 monomials, 6 nodes)
    assert np.max(np.abs(M_nodes @ L - mono(z[:, 0], z[:, 1]))) < 1e-13


def test_element_map_nodes_flat_case_and_sphere_area():
    rng = np.random.default_rng(5)
    P = rng.random((6, 3))
    ref = np.array([[0, 0], [1, 0], [0, 1], [0.5, 0], [0.5, 0.5], [0, 0.5]], float)
    y, _, _ = ny.q6_map(P, ref)
    assert np.max(np.abs(y - P)) < 1e-15
    # straight sides: the affine map, J = 2 area, the flat normal
    V = rng.random((3, 3))
    Pf = np.vstack([V, 0.5 * (V[0] + V[1]), 0.5 * (V[1] + V[2]), 0.5 * (V[2] + V[0])])
    z = rng.random((10, 2)) * 0.5
    y, n, J = ny.q6_map(Pf, z)
    cr = np.cross(V[1] - V[0], V[2] - V[0])
    assert np.max(np.abs(y - (V[0] + z[:, :1] * (V[1] - V[0]) + z[:, 1:] * (V[2] - V[0])))) < 1e-15
    assert np.max(np.abs(J - np.linalg.norm(cr))) < 1e-14
    assert np.max(np.abs(n - cr / np.linalg.norm(cr))) < 1e-14
    # curved sphere: area converges to 4 pi at the quadratic-geometry rate
    errs = [abs(ny.nodes(mg.cavity_quadratic(L))[2].sum() - 4 * np.pi) for L in (0, 1, 2)]
    assert errs[2] < 2e-3 and errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10


def _duffy(n):
    """n x n collapsed Gauss rule on the reference triangle (points, weights)."""
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (x + 1), 0.5 * w
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * U
    return np.stack([U * (1 - V), U * V], -1).reshape(-1, 2), W.reshape(-1)


def test_near_rule_against_brute_force_with_quadratic_density():
    """sum_b f(pt_b) int K L_b dG equals int K f dG for a quadratic density f;
    the right side by a 48x48 collapsed Gauss rule and the point kernel."""
    s = 0.4 + 0.9j
    P = np.array([[0, 0, 0], [1, 0, 0.1], [0, 1, 0.05], [0.5, 0, 0.1], [0.5, 0.5, 0.13], [0, 0.5, 0.07]], float)
    x = np.array([0.3, 0.25, 0.35])                       # above the element, d/h ~ 0.25
    pt, _ = ny.gauss6()
    f = lambda z: np.stack([1 + z[:, 0] - 2 * z[:, 1] ** 2, z[:, 0] * z[:, 1], 0.5 - z[:, 0] ** 2], -1)
    z, w = _duffy(48)                                     # converged to 2e-14 (against 200x200)
    y, n, J = ny.q6_map(P, z)
    fz = f(z)
    ru = np.zeros(3, complex)
    rt = np.zeros(3, complex)
    for k in range(len(w)):
        U, T = bem.kernel(s, x, y[k], n[k])
        ru += w[k] * J[k] * (U @ fz[k])
        rt += w[k] * J[k] * (T @ fz[k])
    # the default policy's leaves (7-point rule at d/h >= 2) leave 3e-8 (U) and
    # 4e-7 (T); a stricter far ratio converges to the brute force
    for policy, tol in (((2.0, 8, 16, 16), 1e-6), ((8.0, 10, 16, 16), 1e-9)):
        G, H = ny.element_blocks(P, x, s, policy=policy)
        lhs_u = np.einsum("bij,bj->i", G, f(pt))
        lhs_t = np.einsum("bij,bj->i", H, f(pt))
        assert np.max(np.abs(lhs_u - ru)) < tol * np.max(np.abs(ru))
        assert np.max(np.abs(lhs_t - rt)) < tol * np.max(np.abs(rt))


def test_far_point_subdivision_rule_reduces_to_the_nystrom_weights():
    """Seen from a distant point the locally corrected weights int K L_b dG
    approach the rule's own w_b J_b K(x, y_b): on a flat element the gap is
    the 6-point rule's error on K L_b and shrinks at third order with the
    element (a misplaced basis function or Jacobian would leave O(1))."""
    s = 0.3 + 0.6j
    V = np.array([[0, 0, 0], [1, 0, 0.1], [0, 1, 0.05]], float)
    P0 = np.vstack([V, 0.5 * (V[0] + V[1]), 0.5 * (V[1] + V[2]), 0.5 * (V[2] + V[0])])
    x = np.array([3.0, -2.0, 4.0])
    pt, w = ny.gauss6()
    errs = []
    for c in (0.5, 0.25):
        P = c * P0
        G, H = ny.element_blocks(P, x, s)
        y, n, J = ny.q6_map(P, pt)
        e = 0.0
        for b in range(6):
            U, T = bem.kernel(s, x, y[b], n[b])
            e = max(e, np.max(np.abs(G[b] - w[b] * J[b] * U)) / np.max(np.abs(w[b] * J[b] * U)),
                    np.max(np.abs(H[b] - w[b] * J[b] * T)) / np.max(np.abs(w[b] * J[b] * T)))
        errs.append(e)
    # measured: 8.9e-5, 1.1e-5
    assert errs[0] < 2e-4 and errs[1] < 2e-5 and errs[0] / errs[1] > 5


@pytest.mark.parametrize("b0", [0, 4])
def test_self_rule_on_a_flat_element_against_the_flat_oracle(b0):
    """On a straight-sided element the self rule summed over the basis
    functions is 1/2 I + PV int_e T and int_e U at the node.  The flat oracle
    gives the same integrals from a decomposition of the element: a small
    homothetic triangle centred on the node (its centroid rule) plus six
    triangles filling the rest (regular rule with subdivision)."""
    s = 0.35 + 0.8j
    V = np.array([[0.1, 0.0, 0.2], [1.3, 0.2, 0.0], [0.2, 1.1, 0.4]])
    Pf = np.vstack([V, 0.5 * (V[0] + V[1]), 0.5 * (V[1] + V[2]), 0.5 * (V[2] + V[0])])
    pt, _ = ny.gauss6()
    x = V[0] + pt[b0, 0] * (V[1] - V[0]) + pt[b0, 1] * (V[2] - V[0])
    c = V.mean(0)
    k = 0.15
    Tk = x + k * (V - c)                                  # centroid x, edges parallel to the element's
    xyz = np.vstack([Tk, V])
    tri = [(0, 1, 2)]
    for a in range(3):
        b = (a + 1) % 3
        tri += [(3 + a, 3 + b, b), (3 + a, b, a)]
    flat = mg.Mesh(xyz, np.array(tri, np.int32), np.zeros(7, np.int8), np.zeros((7, 3)))
    nrm = bem.geometry(flat)[1]
    assert np.max(np.abs(nrm - nrm[0])) < 1e-12         # one plane, one orientation
    Gf, Hf = bem.blocks(flat, s, [(0, n) for n in range(7)], policy=(4.0, 12, 32, 32))
    # default 16 x 16 per half sub-triangle: 1e-6 at the points near an edge
    # (orbit b); 32 x 32: 1e-9
    for policy, tol in (((2.0, 8, 16, 16), 2e-6), ((2.0, 8, 32, 32), 1e-8)):
        G, H = ny.element_blocks(Pf, None, s, b0=b0, policy=policy)
        assert np.max(np.abs(G.sum(0) - Gf.sum(0))) < tol * np.max(np.abs(Gf.sum(0)))
        assert np.max(np.abs(H.sum(0) - Hf.sum(0))) < tol * np.max(np.abs(Hf.sum(0)))


def test_rigid_body_row_sums():
    """Static rigid translation: sum_j H_ij = I for the exterior (cavity)
    problem and 0 for the bounded one (a solid ball)."""
    rs = ny.rowsum_H_static(mg.cavity_quadratic(1))
    assert np.max(np.abs(rs - np.eye(3))) < 5e-6
    xyz, tri6 = mg.quadratic_sphere(1, inward=False)
    ball = mg.QuadMesh(xyz, tri6, np.zeros(len(tri6), np.int8), np.ones(len(tri6)))
    rs = ny.rowsum_H_static(ball)
    assert np.max(np.abs(rs)) < 5e-6


def test_cavity_converges_to_closed_form():
    s = 0.25 + 1.0j
    ur = analytic.cavity_ur(s)
    errs = []
    for L in (0, 1, 2):
        m = mg.cavity_quadratic(L)
        _, nrm, _ = ny.nodes(m)
        u = ny.solve(m, s).reshape(-1, 3)
        errs.append(np.max(np.abs(np.einsum("ij,ij->i", u, -nrm) - ur)) / abs(ur))
    # measured: 1.8e-2, 1.5e-3, 9.9e-5 (flat elements: 0.106, 0.049, 0.022 at L = 1, 2, 3)
    assert errs[2] < 2e-4
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8


def test_mixed_conditions_manufactured_solution():
    """u = U(x0, .) e_z from a point force inside the cavity is an exact
    exterior field: prescribing its traction on half the elements and its
    displacement on the other half must return the other halves (both column
    kinds and both right-hand-side terms)."""
    s = 0.25 + 1.0j
    x0 = np.array([0.1, -0.05, 0.08])
    errs = []
    for L in (0, 1):
        m = mg.cavity_quadratic(L)
        m.bc_kind = (np.arange(m.n_tri) % 2).astype(np.int8)
        y, n, _ = ny.nodes(m)
        ue = np.array([bem.kernel(s, x0, y[i], n[i])[0][2] for i in range(len(y))])
        te = np.array([bem.kernel(s, x0, y[i], n[i])[1][2] for i in range(len(y))])
        kind = np.repeat(m.bc_kind, 6)
        bc = np.where(kind[:, None] == 0, te, ue)
        want = np.where(kind[:, None] == 0, ue, te)
        a = ny.solve(m, s, bc).reshape(-1, 3)
        errs.append(np.linalg.norm(a - want) / np.linalg.norm(want))
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 4, errs


def test_rigid_body_row_sums_on_a_box_with_edges():
    """A bounded box from straight-sided six-node elements: the static row
    sums vanish at every point, including points beside the box's edges and
    corners (subdivision across a sharp edge, the self rule on flat elements).
    Measured: at most 2.5e-7 (48 elements) and 4.8e-7 (108)."""
    for n in (2, 3):
        xyz, tri, _ = mg.box((0, 0, 0), (1, 1, 1), n, n, n)
        pts, cache = [p for p in xyz], {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                pts.append(0.5 * (xyz[a] + xyz[b]))
                cache[key] = len(pts) - 1
            return cache[key]

        tri6 = np.array([(a, b, c, mid(a, b), mid(b, c), mid(c, a)) for a, b, c in tri], np.int32)
        m = mg.QuadMesh(np.array(pts), tri6, np.zeros(len(tri6), np.int8), np.ones(len(tri6)))
        rs = ny.rowsum_H_static(m)
        assert np.max(np.abs(rs)) < 2e-6, n
