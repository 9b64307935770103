"""Oracle for the paper's own discretisation (Section 2.1): curved quadratic
triangles and the locally-corrected Nystrom method, the unknowns at the six
points of the 6-point Gauss rule on every element.

Test infrastructure.  The element integrals and the assembly run in the C
library (``bem_oracle.c``, FP64): far elements by the rule itself, near
elements by recursive subdivision of the parameter triangle, the element that
holds the target node in polar coordinates about it with the strongly singular
part taken as a principal value.  Solving is plain numpy/LAPACK.
"""
from __future__ import annotations

import numpy as np

from ._clib import lib
from .bem import DEFAULT_MATERIAL, DEFAULT_POLICY, _f64, _p


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def gauss6():
    """Rule points (6, 2) in (xi, eta) and weights (6,) (summing to 1/2)."""
    pt = np.zeros(12)
    w = np.zeros(6)
    lib().orc_gauss6(_p(pt), _p(w))
    return pt.reshape(6, 2), w


def lagrange6():
    """C (6, 6): L_b = sum_k C[b, k] m_k, m = (1, xi, eta, xi^2, xi eta, eta^2)."""
    C = np.zeros(36)
    lib().orc_lagrange6(_p(C))
    return C.reshape(6, 6)


def q6_map(P, xieta):
    """Points, unit normals, Jacobians of the quadratic map of element P (6, 3)."""
    xieta = _f64(np.asarray(xieta).reshape(-1, 2))
    out = np.zeros((xieta.shape[0], 8))
    lib().orc_q6_map(_p(_f64(P)), xieta.shape[0], _p(xieta), _p(out))
    return out[:, 0:3], out[:, 3:6], out[:, 6]


def nodes(mesh):
    """Node points (n_k, 3), unit normals (n_k, 3), weights w_q J_q (n_k,)."""
    out = np.zeros((mesh.n_nodes, 8))
    lib().orc_nys_nodes(_p(_f64(mesh.xyz)), mesh.n_tri, _p(_i32(mesh.tri6)), _p(out))
    return out[:, 0:3], out[:, 3:6], out[:, 6]


def element_blocks(P, x, s, b0=-1, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """G_b, H_b (6, 3, 3) of one element: polar rule about rule point b0 when
    b0 >= 0 (H with the free term), else the subdivision rule seen from x."""
    G = np.zeros(108)
    H = np.zeros(108)
    lib().orc_nys_element(_p(_f64(P)), _p(_f64(np.zeros(3) if x is None else x)), int(b0), float(np.real(s)),
                          float(np.imag(s)), _p(_f64(mat)), _p(_f64(policy)), _p(G), _p(H))
    return (G[0::2] + 1j * G[1::2]).reshape(6, 3, 3), (H[0::2] + 1j * H[1::2]).reshape(6, 3, 3)


def pressure_bc(mesh, s, nrm=None):
    """Prescribed traction -p n / s at every node (Heaviside pressure)."""
    if nrm is None:
        _, nrm, _ = nodes(mesh)
    p = np.repeat(np.asarray(mesh.pressure, np.float64), 6)
    return -(p[:, None] * nrm) / s


def assemble(mesh, s, bc_val, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY, rows=None):
    """Rows of the Nystrom system; ``rows`` lists target nodes (default all):
    A [3 len(rows), 3 n_k], b [3 len(rows)], complex128."""
    nk = mesh.n_nodes
    bc = np.ascontiguousarray(np.asarray(bc_val, np.complex128).reshape(nk, 3)).view(np.float64)
    if rows is None:
        nr, rp = nk, None
    else:
        rows = np.ascontiguousarray(np.asarray(rows, np.int64))
        nr, rp = rows.shape[0], _p(rows)
    A = np.zeros((3 * nr, 3 * nk), np.complex128)
    b = np.zeros(3 * nr, np.complex128)
    lib().orc_nys_assemble_rows(_p(_f64(mesh.xyz)), mesh.n_tri, _p(_i32(mesh.tri6)),
                                _p(np.ascontiguousarray(mesh.bc_kind, np.int8)), _p(bc), float(np.real(s)),
                                float(np.imag(s)), _p(_f64(mat)), _p(_f64(policy)), nr, rp, _p(A), _p(b))
    return A, b


def rowsum_H_static(mesh, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """sum over all nodes of H at s = 0, per target node (n_k, 3, 3)."""
    out = np.zeros((mesh.n_nodes, 9))
    lib().orc_nys_rowsum_H_static(_p(_f64(mesh.xyz)), mesh.n_tri, _p(_i32(mesh.tri6)), _p(_f64(mat)),
                                  _p(_f64(policy)), _p(out))
    return out.reshape(-1, 3, 3)


def solve(mesh, s, bc_val=None, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """Assemble and solve by LU; returns the unknown vector (n_k * 3,)."""
    if bc_val is None:
        bc_val = pressure_bc(mesh, s)
    A, b = assemble(mesh, s, bc_val, mat, policy)
    return np.linalg.solve(A, b)
