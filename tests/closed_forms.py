"""Closed forms and independent constructions that pin the oracle.

Nothing here imports the oracle: each function is written from textbook physics
or from a different route to the same quantity (numerical differentiation,
adaptive quadrature), so that agreement with the oracle is evidence and not a
self-comparison.
"""
import math

import numpy as np
from scipy import integrate
from scipy.special import erf

BOHR = 0.529177210903
HARTREE = 27.211386245988


def lorentz_alpha(alpha0, c6, nu, w):
    """TS polarisability at imaginary frequency w (Ha): alpha0 nu / (1 + (w / w0)^2)."""
    w0 = 4.0 * c6 / (3.0 * alpha0 ** 2)
    return alpha0 * nu / (1.0 + (w / w0) ** 2)


def c6_casimir_polder(a1, w1, a2, w2):
    """(3/pi) int_0^inf a1(iw) a2(iw) dw for two single-Lorentzian oscillators.

    = (3/2) a1 a2 w1 w2 / (w1 + w2) (London formula); a = static polarisability.
    """
    return 1.5 * a1 * a2 * w1 * w2 / (w1 + w2)


def c9_atm(a1, w1, a2, w2, a3, w3):
    """(3/pi) int_0^inf a1 a2 a3 dw for three Lorentzian oscillators (ATM coefficient)."""
    return (3.0 * a1 * a2 * a3 * w1 * w2 * w3 * (w1 + w2 + w3)
            / (2.0 * (w1 + w2) * (w2 + w3) * (w3 + w1)))


def atm_geometry_factor(p1, p2, p3):
    """(1 + 3 cos a cos b cos c) / (r12 r23 r31)^3 for a triangle (bohr)."""
    r12, r23, r31 = p2 - p1, p3 - p2, p1 - p3
    d12, d23, d31 = (np.linalg.norm(v) for v in (r12, r23, r31))
    ca = np.dot(p2 - p1, p3 - p1) / (d12 * d31)
    cb = np.dot(p1 - p2, p3 - p2) / (d12 * d23)
    cc = np.dot(p1 - p3, p2 - p3) / (d31 * d23)
    return (1.0 + 3.0 * ca * cb * cc) / (d12 * d23 * d31) ** 3


def qho_dimer_energy(a1, w1, a2, w2, t_axes):
    """Zero-point energy change of two coupled isotropic Drude oscillators (Ha).

    Each axis with dipole coupling t gives normal modes Omega_+-^2 =
    (w1^2 + w2^2)/2 +- sqrt((w1^2 - w2^2)^2 / 4 + a1 a2 w1^2 w2^2 t^2); the energy is
    sum_axes (Omega_+ + Omega_- - w1 - w2) / 2.
    """
    e = 0.0
    for t in t_axes:
        c = a1 * a2 * w1 * w1 * w2 * w2 * t * t
        disc = math.sqrt((w1 * w1 - w2 * w2) ** 2 / 4.0 + c)
        op = math.sqrt((w1 * w1 + w2 * w2) / 2.0 + disc)
        om = math.sqrt((w1 * w1 + w2 * w2) / 2.0 - disc)
        e += 0.5 * (op + om - w1 - w2)
    return e


def dimer_series_energy(a1, w1, a2, w2, t_axes, n_max):
    """Dimer MBD energy truncated at body order n_max, by adaptive quadrature (Ha).

    For two atoms [G^n]_11 vanishes for odd n and equals (a1 a2 t^2)^m for n = 2m on
    each axis, so E = sum_axes sum_{m <= n_max/2} (-1/m) int dw/2pi (a1(w) a2(w) t^2)^m.
    """
    e = 0.0
    for t in t_axes:
        for m in range(1, n_max // 2 + 1):
            f = lambda w: (a1 / (1 + (w / w1) ** 2) * a2 / (1 + (w / w2) ** 2) * t * t) ** m
            val, _ = integrate.quad(f, 0.0, np.inf, epsabs=0, epsrel=1e-13, limit=400)
            e += -1.0 / m * val / (2.0 * math.pi)
    return e


def fermi(r, S, d=6.0):
    return 1.0 / (1.0 + math.exp(-d * (r / S - 1.0)))


def _hess_cd(fun, x, h):
    H = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            ea = np.eye(3)[a] * h
            eb = np.eye(3)[b] * h
            H[a, b] = (fun(x + ea + eb) - fun(x + ea - eb) - fun(x - ea + eb) + fun(x - ea - eb)) / (4 * h * h)
    return H


def numerical_hessian(fun, x, h=1e-3):
    """Central-difference Hessian of a scalar function of a 3-vector, with two
    Richardson steps (error O(h^6)); ``h`` is the largest step used."""
    h1, h2, h3 = _hess_cd(fun, x, h), _hess_cd(fun, x, h / 2), _hess_cd(fun, x, h / 4)
    r1 = (4 * h2 - h1) / 3
    r2 = (4 * h3 - h2) / 3
    return (16 * r2 - r1) / 15


def erf_coulomb(sigma):
    """phi(r) = erf(|r| / sigma) / |r|, the potential of a Gaussian charge."""
    return lambda v: erf(np.linalg.norm(v) / sigma) / np.linalg.norm(v)


def coulomb(v):
    return 1.0 / np.linalg.norm(v)


def sr_tensor_fd(rv, sigma, S, d=6.0):
    """Short-range dipole tensor from the numerical Hessian of erf(r/sigma)/r.

    T_SR,ij = (1 - f(r, S)) d/dr_i d/dr_j phi(|r_i - r_j|) = -(1 - f) Hess phi (r).
    """
    r = np.linalg.norm(rv)
    H = numerical_hessian(erf_coulomb(sigma), rv, h=1e-2 * min(r, sigma))
    return -(1.0 - fermi(r, S, d)) * H


def smooth_cutoff(r, rc, rb):
    """The C1 switch from 1 to 0 over the buffer [rc - rb, rc] (Sec. III.A/III.B cutoff functions).

    Built as the unique cubic with value 1 and zero slope at rc - rb and value 0
    and zero slope at rc (Hermite conditions, solved numerically here in the
    basis 1, s, s^2, s^3 of s = r - rc + rb), so it is an independent
    construction of the buffer polynomial rather than a retyping of it; 1 below
    the buffer, 0 beyond.
    """
    if r < rc - rb:
        return 1.0
    if r >= rc:
        return 0.0
    M = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0],
                  [1.0, rb, rb * rb, rb ** 3], [0.0, 1.0, 2 * rb, 3 * rb * rb]])
    c = np.linalg.solve(M, np.array([1.0, 0.0, 0.0, 0.0]))
    s = r - rc + rb
    return c[0] + c[1] * s + c[2] * s * s + c[3] * s ** 3


def l2_projection_poly(f, a, b, degree):
    """The continuous least-squares (unit weight) polynomial of the given degree
    for f on [a, b], from its Legendre coefficients (2j+1)/2 int_{-1}^{1} f(c + h x)
    P_j(x) dx computed by adaptive quadrature; returned as a callable."""
    from scipy import integrate, special
    h, c = 0.5 * (b - a), 0.5 * (b + a)
    cl = []
    for j in range(degree + 1):
        val, _ = integrate.quad(lambda x: f(c + h * x) * special.eval_legendre(j, x), -1.0, 1.0,
                                epsabs=1e-14, epsrel=1e-12, limit=200)
        cl.append((2 * j + 1) / 2.0 * val)

    def p(lam):
        x = (np.asarray(lam, dtype=np.float64) - c) / h
        return sum(cj * special.eval_legendre(j, x) for j, cj in enumerate(cl))
    return p
