"""Whole-system MBD with whole-system SCS: plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is the non-local
model that lMBD approximates (Sec. II.B): one 3N x 3N SCS solve with the
short-range tensor of every pair (no f_SR, no K2 shell), SCS radii, the damped
long-range tensor of every pair (no f_LR), and the energy
E = int_0^inf dw/2pi Tr ln(1 - A_LR(w) T_LR), evaluated in its symmetric form
sqrt(A) T sqrt(A) by eigen-decomposition, or as the truncated series
sum_n c_n Tr G^n.  Open boundary only.  Written independently of ``lmbd.py``:
the two share no helper, so the limit test that compares them is not a
self-comparison.
"""
import math

import numpy as np
from scipy.special import erf

BOHR_A = 0.529177210903
HARTREE_EV = 27.211386245988


def _free(species_table, species, nu, omegas):
    tab = np.asarray(species_table, dtype=np.float64)
    a0, c6, r0 = tab[species, 0], tab[species, 1], tab[species, 2]
    wi = 4.0 * c6 / (3.0 * a0 * a0)
    abar = (a0 * nu)[:, None] / (1.0 + (np.asarray(omegas)[None, :] / wi[:, None]) ** 2)
    sig = (np.sqrt(2.0 / np.pi) * abar / 3.0) ** (1.0 / 3.0)
    return a0, r0, abar, sig, r0 * nu ** (1.0 / 3.0)


def full_scs(pos, species, nu, species_table, omegas, beta=0.83, damp_d=6.0):
    """Whole-system SCS polarisabilities alpha~_iso (N, nw): B~ alpha~ = d with d_i = I."""
    x = np.asarray(pos, dtype=np.float64) / BOHR_A
    n = x.shape[0]
    a0, r0, abar, sig, R = _free(species_table, species, nu, omegas)
    nw = abar.shape[1]
    out = np.zeros((n, nw))
    rvec = x[:, None, :] - x[None, :, :]
    r = np.linalg.norm(rvec, axis=-1)
    np.fill_diagonal(r, 1.0)
    S = beta * (R[:, None] + R[None, :])
    fdamp = 1.0 / (1.0 + np.exp(-damp_d * (r / S - 1.0)))
    rr = rvec[:, :, :, None] * rvec[:, :, None, :]
    Tdip = (3.0 * rr - (r ** 2)[:, :, None, None] * np.eye(3)) / (r ** 5)[:, :, None, None]
    for w in range(nw):
        s_ij = np.sqrt(sig[:, w][:, None] ** 2 + sig[:, w][None, :] ** 2)
        u = r / s_ij
        g = erf(u) - 2.0 / np.sqrt(np.pi) * u * np.exp(-u * u)
        h = 4.0 / np.sqrt(np.pi) * u ** 3 * np.exp(-u * u)
        blk = (1.0 - fdamp)[:, :, None, None] * (-Tdip * g[:, :, None, None]
                                                 + h[:, :, None, None] * rr / (r ** 5)[:, :, None, None])
        for i in range(n):
            blk[i, i] = np.eye(3) / abar[i, w]
        B = blk.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
        d = np.tile(np.eye(3), (n, 1))
        X = np.linalg.solve(B, d).reshape(n, 3, 3)
        out[:, w] = np.trace(X, axis1=1, axis2=2) / 3.0
    return out


def full_mbd(pos, species, nu, species_table, omega, weight, n_max=None, c_n=None,
             beta=0.83, damp_d=6.0):
    """Total MBD energy (eV) and per-atom shares Tr[ln(1 - G~)]_ii (or series shares).

    omega/weight: quadrature of int_0^inf d omega.  n_max None => exact logarithm.
    """
    x = np.asarray(pos, dtype=np.float64) / BOHR_A
    n = x.shape[0]
    omegas = np.concatenate([[0.0], np.asarray(omega, dtype=np.float64)])
    a0, r0, abar, sig, R = _free(species_table, species, nu, omegas)
    alpha = full_scs(pos, species, nu, species_table, omegas, beta, damp_d)
    Rs = r0 * (alpha[:, 0] / a0) ** (1.0 / 3.0)
    rvec = x[:, None, :] - x[None, :, :]
    r = np.linalg.norm(rvec, axis=-1)
    np.fill_diagonal(r, 1.0)
    S = beta * (Rs[:, None] + Rs[None, :])
    fdamp = 1.0 / (1.0 + np.exp(-damp_d * (r / S - 1.0)))
    rr = rvec[:, :, :, None] * rvec[:, :, None, :]
    Tdip = (3.0 * rr - (r ** 2)[:, :, None, None] * np.eye(3)) / (r ** 5)[:, :, None, None]
    blk = fdamp[:, :, None, None] * Tdip
    for i in range(n):
        blk[i, i] = 0.0
    T = blk.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)
    if n_max is not None and c_n is None:
        c_n = np.array([0.0, 0.0] + [-1.0 / m for m in range(2, n_max + 1)])
    shares = np.zeros(n)
    for q in range(len(omega)):
        s = np.repeat(np.sqrt(alpha[:, q + 1]), 3)
        G = s[:, None] * T * s[None, :]
        if n_max is None:
            lam, V = np.linalg.eigh(G)
            diag = (V ** 2) @ np.log1p(-lam)
        else:
            diag = np.zeros(3 * n)
            P = np.eye(3 * n)
            for m in range(1, n_max + 1):
                P = P @ G
                diag += c_n[m] * np.diag(P)
        shares += weight[q] * diag.reshape(n, 3).sum(1)
    shares *= HARTREE_EV / (2.0 * math.pi)
    return float(shares.sum()), shares
