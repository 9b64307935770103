"""Oracle: adaptive frequency sampling (paper Section 3, Eq. 7-14 and the
Algorithm of Section 3.4).  Test infrastructure; drives any response
function (a real BEM solve or a synthetic rational mock).

Readings of the paper used here:
 * initial frequencies (Section 3.4): w_j = Omega [1 - cos(j pi / (2 (J0 - 1)))],
   j = 0..J0-1 (the printed formula lacks the pi and would span only
   [0, 0.12 Omega]); s_j = eta + i w_j; Omega = pi Ns / T;
 * fitting orders (Eq. 10): M_H = floor(J / alpha_H), M_L = floor(J / alpha_L);
 * "s in [0, Omega]" (Eq. 7-9) means w in [0, Omega] on Re s = eta; maxima
   are taken over a uniform grid of G points; grid points within dw/4 of an
   existing sample are excluded for s_new; ties go to the smallest w;
 * e_k (Eq. 8) is evaluated for every test function; k_max ranges over the
   ORFs I_o (Eq. 9) and E2 over the test set I_t, which contains I_o (Eq. 13);
   the test functions use the ORF poles of each order (residue identification);
 * E1 (Eq. 12) compares the order-M_H time responses (Eq. 11) of consecutive
   steps; E1 at step 0 is +infinity; the integrals over [0, T] use composite
   Simpson on 4 Ns + 1 points;
 * convergence (Eq. 14): E1 < E1_bar and E2 < E2_bar, then Jc further steps
   that must all pass, otherwise sampling resumes (stage 3 of the Algorithm);
 * safety cap: at most Ns/2 + 1 samples (the cost of the FSM); a run that
   reaches the cap, also in the middle of the Jc validation steps, is
   reported as not converged ("capped");
 * multi-point steps (q new frequencies per analysis, an extension the paper
   does not make: it inserts one): the first is the argmax above; each further
   one is the next largest local maximum of the same masked discrepancy that
   lies at least dw/4 from every sample and every earlier pick; fewer than q
   when no such maximum is left.  The Jc validation steps still add one
   frequency each (the paper's convergence check unchanged).  q = 1 is the
   paper's rule.
"""
from __future__ import annotations

import numpy as np

from . import vf


def initial_frequencies(eta, omega, J0):
    j = np.arange(J0)
    return eta + 1j * omega * (1 - np.cos(j * np.pi / (2 * (J0 - 1))))


def orders(J, alpha_H=2.0, alpha_L=2.3):
    return int(np.floor(J / alpha_H)), int(np.floor(J / alpha_L))


def simpson(y, t):
    """Composite Simpson rule on a uniform grid with an even number of intervals."""
    h = t[1] - t[0]
    return h / 3 * (y[..., 0] + y[..., -1] + 4 * y[..., 1:-1:2].sum(-1) + 2 * y[..., 2:-1:2].sum(-1))


def select_new(d, wgrid, taken_w, dw, q):
    """Indices into wgrid of up to q new frequencies from the discrepancy d on
    the grid: grid points within dw/4 of a sampled frequency (taken_w) are
    excluded; the first pick is the largest remaining value (smallest w on
    ties), then the remaining local maxima (d[i] > d[i-1], d[i] >= d[i+1],
    one-sided at the ends) in decreasing order (smallest w on ties), each at
    least dw/4 from every earlier pick."""
    d = np.array(d, np.float64)
    taken = np.zeros(len(wgrid), bool)
    for w in taken_w:
        taken |= np.abs(wgrid - w) < dw / 4
    d[taken] = -1.0
    picks = [int(np.argmax(d))]
    if q > 1:
        n = len(d)
        cands = []
        for i in range(n):
            if taken[i]:
                continue
            left = d[i] > d[i - 1] if i > 0 else True
            right = d[i] >= d[i + 1] if i < n - 1 else True
            if left and right:
                cands.append(i)
        cands.sort(key=lambda i: (-d[i], i))
        for i in cands:
            if len(picks) >= q:
                break
            if all(abs(wgrid[i] - wgrid[j]) >= dw / 4 for j in picks):
                picks.append(i)
    return picks


def fit_discrepancy(fH, fL):
    """e_k of Eq. 8 for every function k: the largest |f_kH - f_kL| over the
    frequency grid divided by the largest |f_kH| over the same grid.
    fH, fL: [Kt, G] values of the two fits on the grid -> e [Kt]."""
    fH = np.atleast_2d(fH)
    fL = np.atleast_2d(fL)
    return np.abs(fH - fL).max(axis=1) / np.abs(fH).max(axis=1)


def stop_E2(e):
    """E2 of Eq. 13: the largest e_k over the test set."""
    return float(np.max(e))


def stop_E1(td, prev_td, tgrid):
    """E1 of Eq. 12: for every test function the integral over [0, T] of the
    squared change of its time response (Eq. 11) between two consecutive steps,
    divided by the integral of the square of the current response; the largest
    of these ratios.  td, prev_td: [Kt, len(tgrid)] responses on the uniform
    grid tgrid (composite Simpson); prev_td None (step 0) gives +infinity."""
    if prev_td is None:
        return np.inf
    num = simpson((td - prev_td) ** 2, tgrid)
    den = simpson(td ** 2, tgrid)
    return float(np.max(num / den))


def _fit_pair(S, F, K, J, omega, alpha_H, alpha_L, n_iter):
    MH, ML = orders(J, alpha_H, alpha_L)
    out = []
    for M in (MH, ML):
        p, _, _ = vf.fit(S, F[:, :K].T, M, n_iter=n_iter, omega_max=omega)
        p, r = vf.identify_residues(S, F.T, p)
        out.append((p, r))
    return out, (MH, ML)


def run(response, K, Kt, T, eta, Ns, J0=16, alpha_H=2.0, alpha_L=2.3, E1_bar=1e-4, E2_bar=2e-3, Jc=3,
        max_Nc=None, grid_pts=2048, n_iter=10, q=1):
    """response(s) -> array [len(s), Kt] of complex values (columns < K are the ORFs).
    q: new frequencies per analysis step (select_new).
    Returns a dict with the samples, the final order-M_H model and the histories."""
    omega = np.pi * Ns / T
    dw = 2 * np.pi / T
    max_Nc = (Ns // 2 + 1) if max_Nc is None else max_Nc
    wgrid = np.linspace(0.0, omega, grid_pts)
    sgrid = eta + 1j * wgrid
    tgrid = np.linspace(0.0, T, 4 * Ns + 1)
    S = list(initial_frequencies(eta, omega, J0))
    F = np.asarray(response(np.array(S)), np.complex128).reshape(len(S), Kt)
    hist = {"E1": [], "E2": [], "J": [], "s_new": [], "MH": [], "ML": []}
    prev_td = None

    def analyse():
        nonlocal prev_td
        Sa = np.array(S)
        J = len(S)
        ((pH, rH), (pL, rL)), (MH, ML) = _fit_pair(Sa, F, K, J, omega, alpha_H, alpha_L, n_iter)
        fH = vf.evaluate(sgrid, pH, rH)
        fL = vf.evaluate(sgrid, pL, rL)
        diff = np.abs(fH - fL)
        e = fit_discrepancy(fH, fL)
        E2 = stop_E2(e)
        td = vf.time_response(tgrid, pH, rH)
        E1 = stop_E1(td, prev_td, tgrid)
        prev_td = td
        kmax = int(np.argmax(e[:K]))
        s_new = sgrid[select_new(diff[kmax], wgrid, Sa.imag, dw, q)]
        hist["E1"].append(E1)
        hist["E2"].append(E2)
        hist["J"].append(J)
        hist["s_new"].append(s_new)
        hist["MH"].append(MH)
        hist["ML"].append(ML)
        return E1, E2, s_new, (pH, rH)

    def add(s_new):
        nonlocal F
        s_new = np.asarray(s_new)[: max_Nc - len(S)]
        S.extend(s_new)
        F = np.concatenate([F, np.asarray(response(s_new), np.complex128).reshape(len(s_new), Kt)])

    E1, E2, s_new, model = analyse()
    converged = capped = False
    while True:
        if E1 < E1_bar and E2 < E2_bar:
            # stage 3: Jc further steps, one frequency each, must all pass
            passed = 0
            while passed < Jc and len(S) < max_Nc:
                add(s_new[:1])
                E1, E2, s_new, model = analyse()
                if not (E1 < E1_bar and E2 < E2_bar):
                    break
                passed += 1
            if passed == Jc:
                converged = True
                break
            if len(S) >= max_Nc:
                # the cap cut the validation short: not converged (Eq. 14 asks for all Jc steps)
                capped = True
                break
            continue
        if len(S) >= max_Nc:
            capped = True
            break
        add(s_new)
        E1, E2, s_new, model = analyse()
    return {"s": np.array(S), "F": F, "poles": model[0], "residues": model[1], "converged": converged,
            "capped": capped, "Nc": len(S), "history": hist}
