"""Oracle for the per-frequency boundary-element solve (paper Section 2.1).

Test infrastructure.  Element integrals and assembly run in the C library
(``bem_oracle.c``, FP64); the linear algebra is plain numpy/LAPACK in FP64.

The discrete problem is the collocation system A(s) a(s) = b(s) of Eq. 2 for
flat triangles with constant u, t and the centroid as collocation point; its
exact solution is what every faster path must reproduce.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._clib import lib

DEFAULT_MATERIAL = (1.0, 0.25, 1.0)            # mu, nu, rho
DEFAULT_POLICY = (2.0, 8, 16, 16)              # far_ratio, max_subdiv, n_theta, n_rho


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def material_constants(mat=DEFAULT_MATERIAL):
    """lambda, c_s, c_p, beta = c_s/c_p (Section 2.1, with c_p = sqrt((lambda+2mu)/rho))."""
    mu, nu, rho = mat
    lam = 2 * mu * nu / (1 - 2 * nu)
    cs = np.sqrt(mu / rho)
    cp = np.sqrt((lam + 2 * mu) / rho)
    return lam, cs, cp, cs / cp


def radial(x, beta, mode=0):
    """(r psi, r chi, r^2 psi', r^2 chi') at x = s r / c_s; mode 0 auto, 1 series, 2 closed."""
    out = np.zeros(8)
    lib().orc_radial(float(np.real(x)), float(np.imag(x)), float(beta), int(mode), _p(out))
    return out[0::2] + 1j * out[1::2]


def kernel(s, x, y, n, mat=DEFAULT_MATERIAL, mode=0):
    """U_ij(x,y;s), T_ij(x,y,n;s) as 3x3 complex arrays (i: force direction at x)."""
    U = np.zeros(18)
    T = np.zeros(18)
    lib().orc_kernel(float(np.real(s)), float(np.imag(s)), _p(_f64(mat)), _p(_f64(x)), _p(_f64(y)),
                     _p(_f64(n)), int(mode), _p(U), _p(T))
    return (U[0::2] + 1j * U[1::2]).reshape(3, 3), (T[0::2] + 1j * T[1::2]).reshape(3, 3)


def radon7():
    bary = np.zeros(21)
    w = np.zeros(7)
    lib().orc_radon7(_p(bary), _p(w))
    return bary.reshape(7, 3), w


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(int(n), _p(x), _p(w))
    return x, w


def geometry(mesh):
    """centroid (nt,3), unit normal (nt,3), area (nt,), longest edge (nt,)."""
    nt = mesh.tri.shape[0]
    out = np.zeros((nt, 8))
    lib().orc_geometry(_p(_f64(mesh.xyz)), nt, _p(np.ascontiguousarray(mesh.tri, np.int32)), _p(out))
    return out[:, 0:3], out[:, 3:6], out[:, 6], out[:, 7]


def blocks(mesh, s, pairs, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """G_mn, H_mn (3x3 complex each, H with the free term on m == n) for a list of (m, n)."""
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    k = pairs.shape[0]
    G = np.zeros((k, 18))
    H = np.zeros((k, 18))
    lib().orc_blocks(_p(_f64(mesh.xyz)), mesh.tri.shape[0], _p(np.ascontiguousarray(mesh.tri, np.int32)),
                     float(np.real(s)), float(np.imag(s)), _p(_f64(mat)), _p(_f64(policy)), k,
                     _p(pairs), _p(G), _p(H))
    return (G[:, 0::2] + 1j * G[:, 1::2]).reshape(k, 3, 3), (H[:, 0::2] + 1j * H[:, 1::2]).reshape(k, 3, 3)


def heaviside_bc(mesh, s):
    """Prescribed boundary values at s for a unit step load: bc_shape / s."""
    return np.asarray(mesh.bc_shape, dtype=np.complex128) / s


def assemble(mesh, s, bc_val=None, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY, rows=None):
    """Rows of A(s) and b(s) (Eq. 2).  ``rows`` lists collocation elements
    (default: all); returns A [3*len(rows), 3*nt] and b [3*len(rows)], complex128."""
    nt = mesh.tri.shape[0]
    if bc_val is None:
        bc_val = heaviside_bc(mesh, s)
    bc = np.ascontiguousarray(np.asarray(bc_val, np.complex128).reshape(nt, 3)).view(np.float64)
    if rows is None:
        nr, rp = nt, None
    else:
        rows = np.ascontiguousarray(np.asarray(rows, np.int64))
        nr, rp = rows.shape[0], _p(rows)
    A = np.zeros((3 * nr, 3 * nt), np.complex128)
    b = np.zeros(3 * nr, np.complex128)
    lib().orc_assemble_rows(_p(_f64(mesh.xyz)), nt, _p(np.ascontiguousarray(mesh.tri, np.int32)),
                            _p(np.ascontiguousarray(mesh.bc_kind, np.int8)), _p(bc),
                            float(np.real(s)), float(np.imag(s)), _p(_f64(mat)), _p(_f64(policy)),
                            nr, rp, _p(A), _p(b))
    return A, b


def rowsum_H_static(mesh, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """sum_n H_mn at s = 0 for every row block m, shape (nt, 3, 3)."""
    nt = mesh.tri.shape[0]
    out = np.zeros((nt, 9))
    lib().orc_rowsum_H_static(_p(_f64(mesh.xyz)), nt, _p(np.ascontiguousarray(mesh.tri, np.int32)),
                              _p(_f64(mat)), _p(_f64(policy)), _p(out))
    return out.reshape(nt, 3, 3)


def solve_dense(A, b):
    """Exact discrete solution x = A^{-1} b by LU with partial pivoting (LAPACK)."""
    return np.linalg.solve(A, b)


def block_jacobi(A):
    """Inverses of the 3x3 diagonal blocks (one per collocation point), the
    block-diagonal preconditioner of Section 4."""
    nt = A.shape[0] // 3
    D = np.stack([A[3 * m:3 * m + 3, 3 * m:3 * m + 3] for m in range(nt)])
    return np.linalg.inv(D)


def apply_block(Dinv, v):
    nt = Dinv.shape[0]
    return np.einsum("mij,mj->mi", Dinv, v.reshape(nt, 3)).reshape(-1)


def gmres(matvec, b, tol=1e-8, restart=50, max_iter=2000, precond=None, x0=None):
    """Right-preconditioned restarted GMRES(m) with modified Gram-Schmidt and
    Givens rotations; stops on the true relative residual ||b - A x|| / ||b||.

    Returns (x, iterations, relative residual history)."""
    n = b.shape[0]
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, np.complex128)
    bnorm = np.linalg.norm(b)
    hist = []
    it = 0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol or it >= max_iter:
            return x, it, hist
        V = np.zeros((restart + 1, n), np.complex128)
        Hm = np.zeros((restart + 1, restart), np.complex128)
        cs = np.zeros(restart, np.complex128)
        sn = np.zeros(restart, np.complex128)
        g = np.zeros(restart + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            w = matvec(M(V[j]))
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -np.conj(sn[i]) * Hm[i, j] + np.conj(cs[i]) * Hm[i + 1, j]
                Hm[i, j] = t
            # complex Givens rotation [[c, s], [-conj(s), conj(c)]] zeroing H[j+1, j]
            a, c = Hm[j, j], Hm[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            if a == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(c) / den
            Hm[j, j] = cs[j] * a + sn[j] * c
            Hm[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if abs(g[j + 1]) / bnorm <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(Hm[:k, :k]), g[:k])
        x = x + M(V[:k].T @ y)


def solution_fields(mesh, a, bc_val):
    """Split the solution vector into element displacements u and tractions t
    (nt, 3) each, using the prescribed values for the known half."""
    nt = mesh.tri.shape[0]
    a = a.reshape(nt, 3)
    bc_val = np.asarray(bc_val).reshape(nt, 3)
    trac = (np.asarray(mesh.bc_kind) == 0)[:, None]
    u = np.where(trac, a, bc_val)
    t = np.where(trac, bc_val, a)
    return u, t


def solve(mesh, s, bc_val=None, mat=DEFAULT_MATERIAL, policy=DEFAULT_POLICY):
    """Assemble and solve at one s by LU; returns (a, u, t)."""
    if bc_val is None:
        bc_val = heaviside_bc(mesh, s)
    A, b = assemble(mesh, s, bc_val, mat, policy)
    a = solve_dense(A, b)
    u, t = solution_fields(mesh, a, bc_val)
    return a, u, t
