"""Oracle: vector fitting of K frequency responses with common poles (paper
Section 2.3, Eq. 5 and Eq. 6; the method of Gustavsen and Semlyen that the
paper cites).  Test infrastructure; numpy least squares and eigenvalues.

Model (Eq. 5): f_k(s) = sum_m r_km / (s - a_m), strictly proper, poles shared by
all K functions, real-coefficient structure (a complex pole comes with its
conjugate and conjugate residues).

Steps, in the paper's order:
 1. initial poles equally spaced over the band (Section 2.3): pairs
    -b_m/100 +- i b_m with b_m equally spaced in (0, Omega];
    for odd M one extra real pole -Omega/100;
 2. pole identification, repeated: with sigma(s) = 1 + sum_m c~_m phi_m(s),
    solve the linear least-squares problem
        sum_m c_km phi_m(s_j) - F_kj sum_m c~_m phi_m(s_j) = F_kj   (all k, j)
    in the real basis phi = {1/(s-a) + 1/(s-a*), i/(s-a) - i/(s-a*)} for a pair
    and 1/(s-a) for a real pole, real and imaginary parts stacked; the zeros
    of sigma are the new poles = eig(Ahat - bhat c~^T) with Ahat the real block
    form of the poles and bhat = (2, 0) per pair, 1 per real pole.  Unstable
    poles are kept unchanged (Section 2.3: flipping them gave large errors);
 3. residue identification with the poles fixed (Section 2.3), one
    least-squares matrix and K right-hand sides;
 4. f(s) from Eq. 5; the time response of each rational term, whose exact
    inverse Laplace transform is r e^{a t} (reading: Eq. 6 prints e^{-a t},
    which would contradict Eq. 5's 1/(s - a)).
"""
from __future__ import annotations

import numpy as np


def initial_poles(M, omega_max):
    npair = M // 2
    b = omega_max * np.arange(1, npair + 1) / npair if npair else np.array([])
    poles = []
    for bm in b:
        poles += [complex(-bm / 100, bm), complex(-bm / 100, -bm)]
    if M % 2:
        poles.append(complex(-omega_max / 100, 0.0))
    return np.array(poles, np.complex128)


def _structure(poles, tol=1e-12):
    """Group poles into (index, 'pair') with positive-imaginary representative,
    or (index, 'real').  Pairs are assumed to be present with both members."""
    items = []
    used = np.zeros(len(poles), bool)
    for i, a in enumerate(poles):
        if used[i]:
            continue
        if abs(a.imag) <= tol * max(1.0, abs(a)):
            items.append((complex(a.real, 0.0), "real"))
            used[i] = True
        else:
            # find the conjugate partner
            j = np.argmin(np.abs(poles - np.conj(a)) + used * 1e300)
            used[i] = used[j] = True
            items.append((complex(a.real, abs(a.imag)), "pair"))
    return items


def basis(s, items):
    """Real-coefficient basis matrix Phi[j, col] (complex values)."""
    s = np.asarray(s, np.complex128)
    cols = []
    for a, kind in items:
        if kind == "real":
            cols.append(1.0 / (s - a))
        else:
            cols.append(1.0 / (s - a) + 1.0 / (s - np.conj(a)))
            cols.append(1j / (s - a) - 1j / (s - np.conj(a)))
    return np.stack(cols, axis=1) if cols else np.zeros((len(s), 0), np.complex128)


def _realify(M):
    return np.concatenate([M.real, M.imag], axis=0)


def _poles_from_items(items):
    out = []
    for a, kind in items:
        if kind == "real":
            out.append(a)
        else:
            out += [a, np.conj(a)]
    return np.array(out, np.complex128)


def identify_poles(s, F, poles):
    """One pole-identification pass: returns the zeros of sigma as new poles."""
    F = np.atleast_2d(np.asarray(F, np.complex128))     # [K, J]
    K, J = F.shape
    items = _structure(poles)
    Phi = basis(s, items)                                # [J, M]
    M = Phi.shape[1]
    # unknowns: c_1 .. c_K (M each), then c~ (M)
    A = np.zeros((K * 2 * J, K * M + M))
    rhs = np.zeros(K * 2 * J)
    for k in range(K):
        rows = slice(k * 2 * J, (k + 1) * 2 * J)
        A[rows, k * M:(k + 1) * M] = _realify(Phi)
        A[rows, K * M:] = _realify(-F[k][:, None] * Phi)
        rhs[rows] = _realify(F[k][:, None])[:, 0]
    sol = np.linalg.lstsq(A, rhs, rcond=None)[0]
    ct = sol[K * M:]
    # real block realisation of the poles and the zeros of sigma
    Ahat = np.zeros((M, M))
    bhat = np.zeros(M)
    c = 0
    for a, kind in items:
        if kind == "real":
            Ahat[c, c] = a.real
            bhat[c] = 1.0
            c += 1
        else:
            Ahat[c:c + 2, c:c + 2] = [[a.real, a.imag], [-a.imag, a.real]]
            bhat[c] = 2.0
            c += 2
    new = np.linalg.eigvals(Ahat - np.outer(bhat, ct))
    # enforce exact conjugate pairs (eigenvalues of a real matrix)
    return _clean_conjugates(new)


def _clean_conjugates(p, tol=1e-10):
    p = np.array(p, np.complex128)
    out = []
    used = np.zeros(len(p), bool)
    for i in np.argsort(-p.imag):
        if used[i]:
            continue
        a = p[i]
        if abs(a.imag) <= tol * max(1.0, abs(a)):
            out.append(complex(a.real, 0.0))
            used[i] = True
        else:
            cand = np.where(~used)[0]
            j = cand[np.argmin(np.abs(p[cand] - np.conj(a)))]
            used[i] = used[j] = True
            ar, ai = 0.5 * (a.real + p[j].real), 0.5 * (abs(a.imag) + abs(p[j].imag))
            out += [complex(ar, ai), complex(ar, -ai)]
    return np.array(out, np.complex128)


def identify_residues(s, F, poles):
    """Residues r[k, m] (complex, aligned with the returned pole order) for fixed poles."""
    F = np.atleast_2d(np.asarray(F, np.complex128))
    items = _structure(poles)
    Phi = basis(s, items)
    A = _realify(Phi)
    B = np.concatenate([F.real.T, F.imag.T], axis=0)     # [2J, K]
    C = np.linalg.lstsq(A, B, rcond=None)[0]             # [M, K]
    res = []
    c = 0
    for a, kind in items:
        if kind == "real":
            res.append(C[c] + 0j)
            c += 1
        else:
            r = C[c] + 1j * C[c + 1]
            res += [r, np.conj(r)]
            c += 2
    return _poles_from_items(items), np.array(res).T       # [M], [K, M]


def fit(s, F, M, n_iter=10, init_poles=None, omega_max=None):
    """Full vector fitting: returns (poles [M], residues [K, M], rms)."""
    s = np.asarray(s, np.complex128)
    if init_poles is None:
        init_poles = initial_poles(M, omega_max if omega_max is not None else np.max(s.imag))
    poles = np.array(init_poles, np.complex128)
    for _ in range(n_iter):
        new = identify_poles(s, F, poles)
        if len(new) == len(poles) and np.max(np.abs(np.sort_complex(new) - np.sort_complex(poles))) <= \
                1e-10 * max(1.0, np.max(np.abs(poles))):
            poles = new
            break
        poles = new
    poles, res = identify_residues(s, F, poles)
    Fhat = evaluate(s, poles, res)
    F2 = np.atleast_2d(F)
    rms = np.sqrt(np.mean(np.abs(Fhat - F2) ** 2))
    return poles, res, rms


def evaluate(s, poles, res):
    """f_k(s) = sum_m r_km / (s - a_m); res [K, M] -> [K, len(s)]."""
    s = np.asarray(s, np.complex128)
    return np.atleast_2d(res) @ (1.0 / (s[None, :] - poles[:, None]))


def time_response(t, poles, res):
    """Inverse Laplace transform of the model: sum_m r_km e^{a_m t} (real part)."""
    t = np.asarray(t, np.float64)
    return np.real(np.atleast_2d(res) @ np.exp(np.outer(poles, t)))


def fit_error(f_model, f_data):
    """E_vf of Section 4.1: relative discrete L2 misfit over the samples."""
    return np.sqrt(np.sum(np.abs(f_model - f_data) ** 2) / np.sum(np.abs(f_data) ** 2))
