"""Closed-form solutions used to pin the oracle.  Written independently of
the oracle (nothing here calls it), from the governing equations:

* Kelvin's static point-force solution (textbook);
* the pressurised spherical cavity in full space: radially symmetric outgoing
  (decaying) P-wave field u(r) = C (1 + k r) e^{-k r} / r^2, k = s / c_p,
  with sigma_rr(a) = -p(s);
* the nu = 0 prismatic rod (the paper's first example reduces to 1D):
  E u'' = rho s^2 u, u(0) = 0, E u'(L) = p(s).
"""
import numpy as np


def lame(mu, nu):
    return 2 * mu * nu / (1 - 2 * nu)


def kelvin_U(x, y, mu, nu):
    rv = np.asarray(y, float) - np.asarray(x, float)
    r = np.linalg.norm(rv)
    rh = rv / r
    return ((3 - 4 * nu) * np.eye(3) + np.outer(rh, rh)) / (16 * np.pi * mu * (1 - nu) * r)


def cavity_field(s, a=1.0, mu=1.0, nu=0.25, rho=1.0, P=1.0):
    """Radial displacement u(r, s) outside a cavity of radius a under internal
    pressure P/s (Heaviside), as a callable of r."""
    lam = lame(mu, nu)
    cp = np.sqrt((lam + 2 * mu) / rho)
    k = s / cp
    pbar = P / s
    # u = C f(r), f = (1 + k r) e^{-k r} / r^2
    # sigma_rr = (lam + 2mu) u' + 2 lam u / r; f'(r) = -e^{-kr}(k^2 r^2 + 2 k r + 2)/r^3
    fa = (1 + k * a) * np.exp(-k * a) / a ** 2
    dfa = -np.exp(-k * a) * (k * k * a * a + 2 * k * a + 2) / a ** 3
    C = -pbar / ((lam + 2 * mu) * dfa + 2 * lam * fa / a)
    return lambda r: C * (1 + k * r) * np.exp(-k * r) / r ** 2


def cavity_ur(s, a=1.0, mu=1.0, nu=0.25, rho=1.0, P=1.0):
    return cavity_field(s, a, mu, nu, rho, P)(a)


def cavity_ur_time(t):
    """Inverse transform of cavity_ur for a = mu = rho = P = 1, nu = 1/4
    (partial fractions of (1 + s/sqrt3)/(s(s^2 + 4 s/sqrt3 + 4)))."""
    t = np.asarray(t, float)
    w = np.sqrt(8.0 / 3.0)
    return 0.25 * (1 - np.exp(-2 * t / np.sqrt(3)) * (np.cos(w * t) - np.sin(w * t) / np.sqrt(2)))


def rod_uz(z, s, L, E=2.0, rho=1.0, P=1.0):
    c = np.sqrt(E / rho)
    k = s / c
    pbar = P / s
    return pbar * np.sinh(k * z) / (E * k * np.cosh(k * L))


def rod_t_fixed(s, L, E=2.0, rho=1.0, P=1.0):
    """z-traction on the fixed face z = 0 (outward normal -e_z)."""
    c = np.sqrt(E / rho)
    k = s / c
    return -(P / s) / np.cosh(k * L)
