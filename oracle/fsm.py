"""Oracle: Fourier-series-method inversion of the Laplace transform by direct
summation (paper Section 2.2, Eq. 3 and Eq. 4).  Test infrastructure.

The Bromwich integral (Eq. 3) along Re s = eta, with s = eta + i w, is
    h(t) = (e^{eta t} / (2 pi)) int h(eta + i w) e^{i w t} dw,
truncated to |w| <= Omega = Ns dw / 2 and evaluated with the trapezoidal
rule on w_k = k dw, dw = 2 pi / P (P the period).  For a real time signal
h(eta - i w) = conj(h(eta + i w)), so only k = 0..Ns/2 are needed (Section 2.2:
Nc = Ns/2 + 1 frequency solves).  The end points k = +-Ns/2 carry the half
trapezoid weight.  An optional Hann window W_k = (1 + cos(2 pi k / Ns))/2
multiplies each term (Section 2.2).

Readings: Eq. 4 is printed without the factor dw / (2 pi) = 1 / P; it is
included here.  The damping abscissa eta = kappa ln(10) / T (Section 2.2) is an
input.
"""
from __future__ import annotations

import numpy as np


def grid(P, eta, Ns):
    """s_k = eta + i 2 pi k / P, k = 0..Ns/2."""
    return eta + 1j * 2 * np.pi * np.arange(Ns // 2 + 1) / P


def hann(Ns):
    k = np.arange(Ns // 2 + 1)
    return 0.5 * (1 + np.cos(2 * np.pi * k / Ns))


def invert_direct(P, eta, Ns, H, t, window=False):
    """h(t) at arbitrary times t from H[..., k] = h(s_k), k = 0..Ns/2, by the
    trapezoidal sum over k = -Ns/2..Ns/2 (direct, no FFT)."""
    H = np.asarray(H, np.complex128)
    t = np.asarray(t, np.float64)
    half = Ns // 2
    k = np.arange(half + 1)
    w = np.ones(half + 1)
    w[half] = 0.5                      # trapezoid end point (the k = -Ns/2 twin adds the other half)
    if window:
        w = w * hann(Ns)
    dw = 2 * np.pi / P
    phase = np.exp(1j * np.outer(t, k * dw))          # [nt, half+1]
    # positive and negative frequencies: term(k) + conj(term(k)) for k > 0, once for k = 0
    mult = np.where(k == 0, 1.0, 2.0)
    terms = (H[..., None, :] * (w * mult)) * phase     # [..., nt, half+1]
    total = np.real(terms.sum(axis=-1))
    return np.exp(eta * t) * total / P


def time_grid(P, Ns):
    return np.arange(Ns) * P / Ns
