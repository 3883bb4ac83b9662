"""Per-atom lMBD energies and exact forces: plain float64 torch on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every step follows the
paper's statement of the method in its order; nothing is blocked, fused or
reordered beyond what the equations say.  Section and equation names refer to
Muhli, Ala-Nissila & Caro, "Atom-wise formulation of the many-body dispersion
problem for linear-scaling van der Waals corrections" (2024).

Readings taken where the paper is silent or ambiguous (each is listed in the
design notes of the repository):
  * sign: E_k = (1/2pi) int dw sum_n c_n Tr[G~^n]_kk with c_n = -1/n, the series
    of ln(1 - x); the energy is negative (Sec. II.B MBD energy, Sec. III.A
    series expansion and polynomial-fit form).
  * frequencies are imaginary-axis; the quadrature (omega, weight) is an input;
    by default the SCS is solved exactly at omega = 0 and at every quadrature
    node.  With scs_freq = "lorentz" it is solved at omega = 0 and omega_ref
    only, and the blended polarisabilities at the nodes follow the two-point
    Lorentzian of Sec. III.C (Eqs. alpha_SCS_freq and char-freq), applied to the
    blended alpha~_i of the frame.
  * one cutoff per role: K1 = B(r_scs), K2 = B(2 r_scs) \\ B(r_scs) for the SCS
    (Sec. III.B), K = B(r_nbr) for the energy, f_LR cut at r_mbd1 for pairs that
    touch the central atom and r_mbd2 otherwise (Sec. III.A cutoff function);
    optionally separate radii r_2b1 / r_2b2 for the n = 2 term (Sec. III.A, the
    two-body cutoffs): its T_LR is cut at r_2b1 / r_2b2 instead.
  * balls are open: r < r_c is inside.
  * S~ in T_LR uses the blended static polarisability alpha~_i(0) of the frame.
  * periodic images are explicit sites carrying their base atom's data.
  * forces are the exact gradient -d(sum_k w_k E_k)/dR with Hirshfeld ratios
    held fixed (including the central-polarisability terms that the paper's
    approximate force drops).
"""
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

BOHR = 0.529177210903      # Angstrom per bohr (CODATA 2018)
HARTREE = 27.211386245988  # eV per hartree (CODATA 2018)

_DT = torch.float64


@dataclass
class OracleParams:
    """Method parameters.  Lengths in Angstrom, frequencies in hartree."""
    r_scs: float
    r_nbr: float
    r_mbd1: float
    r_mbd2: float
    omega: np.ndarray             # quadrature nodes (imaginary frequency), Ha
    weight: np.ndarray            # quadrature weights for int_0^inf d omega
    beta: float = 0.83
    damp_d: float = 6.0
    r_buf: float = 0.5
    r_inner: float = 2.0
    n_max: Optional[int] = 6      # None => exact block logarithm (infinite body order)
    c_n: Optional[np.ndarray] = None  # length n_max + 1; None => c_n = -1/n for n >= 2
    scs_freq: str = "exact"       # "exact": SCS at every node; "lorentz": two-point model (Sec. III.C)
    c_n_mode: str = "series"      # "series": fixed c_n; "fit": per atom and node, a least-squares
                                  # polynomial of ln(1 - x) over the spectrum of G~ (Sec. III.A)
    fit_nodes: int = 32           # Gauss-Legendre nodes of the discrete least-squares fit
    lanczos_steps: Optional[int] = 20  # Lanczos steps for the spectrum bounds; None => exact extremes
    coef_fixed: Optional[dict] = None  # "fit" mode: {atom: (n_nodes, n_max + 1) array} used instead
                                       # of refitting (the coefficients held fixed)
    omega_ref: Optional[float] = None  # reference frequency of the two-point model, Ha
    r_2b1: Optional[float] = None  # two-body radii (Sec. III.A): the n = 2 term's T_LR is cut at r_2b1
    r_2b2: Optional[float] = None  #   (pairs touching k) and r_2b2 (others); None: the MBD radii

    def two_body_radii(self):
        return (self.r_mbd1 if self.r_2b1 is None else self.r_2b1,
                self.r_mbd2 if self.r_2b2 is None else self.r_2b2)

    def separate_two_body(self):
        return self.two_body_radii() != (self.r_mbd1, self.r_mbd2)

    def scs_omegas(self):
        """Frequencies at which the local SCS systems are solved (omega = 0 first)."""
        if self.scs_freq == "exact":
            return np.concatenate([[0.0], self.omega])
        if self.scs_freq == "lorentz":
            assert self.omega_ref is not None and self.omega_ref > 0.0
            return np.array([0.0, float(self.omega_ref)])
        raise ValueError(f"unknown scs_freq {self.scs_freq!r}")

    def coefficients(self):
        if self.n_max is None:
            return None
        if self.c_n is not None:
            c = np.asarray(self.c_n, dtype=np.float64).copy()
            assert c.shape[0] == self.n_max + 1
            c[:2] = 0.0  # the n = 0 and n = 1 terms vanish (zero diagonal of G)
            return c
        c = np.zeros(self.n_max + 1)
        for n in range(2, self.n_max + 1):
            c[n] = -1.0 / n
        return c


def make_params(cutoffs: dict, omega, weight, **kw) -> OracleParams:
    return OracleParams(r_scs=cutoffs["r_scs"], r_nbr=cutoffs["r_nbr"], r_mbd1=cutoffs["r_mbd1"],
                        r_mbd2=cutoffs["r_mbd2"], omega=np.asarray(omega, dtype=np.float64),
                        weight=np.asarray(weight, dtype=np.float64), r_2b1=cutoffs.get("r_2b1"),
                        r_2b2=cutoffs.get("r_2b2"), **kw)


# ----------------------------------------------------------------------------
# Neighbourhoods (balls around the central atom, Sec. III.A and III.B)
# ----------------------------------------------------------------------------

def _image_shifts(pos, cell, pbc, rmax):
    if cell is None or not np.any(pbc):
        return np.zeros((1, 3), dtype=np.int64)
    cell = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(cell))
    frac = pos @ np.linalg.inv(cell)
    ranges = []
    for d in range(3):
        if not pbc[d]:
            ranges.append([0])
            continue
        e, f = [(d + 1) % 3, (d + 2) % 3]
        spacing = vol / np.linalg.norm(np.cross(cell[e], cell[f]))
        spread = frac[:, d].max() - frac[:, d].min()
        m = int(math.ceil(rmax / spacing + spread))
        ranges.append(range(-m, m + 1))
    return np.array([(a, b, c) for a in ranges[0] for b in ranges[1] for c in ranges[2]],
                    dtype=np.int64)


class _Images:
    """All periodic images of the atoms within reach, with a k-d tree over them."""

    def __init__(self, pos, cell, pbc, rmax):
        from scipy.spatial import cKDTree
        self.pos = np.asarray(pos, dtype=np.float64)
        self.shifts = _image_shifts(self.pos, cell, pbc, rmax)
        tvec = (self.shifts @ np.asarray(cell, dtype=np.float64) if cell is not None
                else np.zeros((1, 3)))
        n = self.pos.shape[0]
        self.img = (self.pos[None, :, :] + tvec[:, None, :]).reshape(-1, 3)
        self.img_base = np.tile(np.arange(n), len(self.shifts))
        self.img_shift = np.repeat(self.shifts, n, axis=0)
        self.tree = cKDTree(self.img)


def neighbourhood(pos, cell, pbc, k, rmax, images=None):
    """All sites (atoms and periodic images) strictly within rmax (Angstrom) of atom k.

    Returns (base, shift, dist): base atom index, integer lattice shift and
    distance; the central atom itself comes first, the rest by increasing
    distance (ties broken by base index, then shift).
    """
    if images is None:
        images = _Images(pos, cell, pbc, rmax)
    cand = np.asarray(images.tree.query_ball_point(images.pos[k], rmax), dtype=np.int64)
    rel = images.img[cand] - images.pos[k]
    dist = np.sqrt(np.einsum("na,na->n", rel, rel))
    keep = dist < rmax
    cand, d = cand[keep], dist[keep]
    j_idx = images.img_base[cand]
    sh = images.img_shift[cand]
    is_self = (j_idx == k) & np.all(sh == 0, axis=1)
    order = np.lexsort((sh[:, 2], sh[:, 1], sh[:, 0], j_idx, d, ~is_self))
    return j_idx[order], sh[order], d[order]


# ----------------------------------------------------------------------------
# Free-atom quantities (Sec. II.B: TS polarisability, attenuation length, radii)
# ----------------------------------------------------------------------------

def free_atom_terms(species_table, species, nu, omegas):
    """Per-atom, position-independent inputs of the screening.

    omega_i = 4 C6 / (3 alpha0^2);  abar_i(w) = alpha0 nu / (1 + (w / omega_i)^2);
    sigma_i(w) = (sqrt(2/pi) abar_i(w) / 3)^(1/3);  R_i = R0 nu^(1/3).
    Returns dict of numpy arrays: abar (N, nw), sigma (N, nw), R (N,), alpha0 (N,),
    r0 (N,), omega_i (N,).
    """
    tab = np.asarray(species_table, dtype=np.float64)
    a0 = tab[species, 0]
    c6 = tab[species, 1]
    r0 = tab[species, 2]
    om = 4.0 * c6 / (3.0 * a0 ** 2)
    w = np.asarray(omegas, dtype=np.float64)
    if isinstance(nu, torch.Tensor):   # volume ratios as a differentiable torch tensor
        lor = torch.as_tensor(1.0 / (1.0 + (w[None, :] / om[:, None]) ** 2), dtype=_DT)
        abar = (torch.as_tensor(a0, dtype=_DT) * nu)[:, None] * lor
        R = torch.as_tensor(r0, dtype=_DT) * nu ** (1.0 / 3.0)
    else:
        abar = (a0 * nu)[:, None] / (1.0 + (w[None, :] / om[:, None]) ** 2)
        R = r0 * np.asarray(nu, dtype=np.float64) ** (1.0 / 3.0)
    sigma = (math.sqrt(2.0 / math.pi) * abar / 3.0) ** (1.0 / 3.0)
    return dict(abar=abar, sigma=sigma, R=R, alpha0=a0, r0=r0, omega_i=om)


# ----------------------------------------------------------------------------
# Pair tensors
# ----------------------------------------------------------------------------

def _dipole_T(rv):
    """T_ij = (3 r r^T - r^2 I) / r^5 for a batch of separation vectors (..., 3)."""
    r2 = (rv * rv).sum(-1)
    r = torch.sqrt(r2)
    eye = torch.eye(3, dtype=_DT)
    outer = rv[..., :, None] * rv[..., None, :]
    return (3.0 * outer - r2[..., None, None] * eye) / r[..., None, None] ** 5


def _fermi(r, S, d):
    """Fermi damping f(r, S) = 1 / (1 + exp(-d (r / S - 1)))."""
    return 1.0 / (1.0 + torch.exp(-d * (r / S - 1.0)))


def _cutoff_poly(r, rc, rb):
    """1 below rc - rb, 1 - 3 x^2 + 2 x^3 with x = (r - rc + rb) / rb in the buffer, 0 beyond."""
    x = (r - rc + rb) / rb
    mid = 1.0 - 3.0 * x * x + 2.0 * x ** 3
    one = torch.ones_like(r)
    zero = torch.zeros_like(r)
    return torch.where(r < rc - rb, one, torch.where(r < rc, mid, zero))


def _t_sr(rv, sig, S, rc, rb, d):
    """Short-range dipole tensor with the SR cutoff (Sec. II.B T_SR, g and h; Sec. III.B f_SR).

    rv: (P, 3) separations [bohr]; sig: (P, nw) pair attenuation lengths; S: (P,)
    unscreened vdW radii sums.  Returns (P, nw, 3, 3):
      f_SR(r) (1 - f(r, S)) { -T g(r, sigma) + h(r, sigma) }.
    """
    r = torch.sqrt((rv * rv).sum(-1))                       # (P,)
    u = r[:, None] / sig                                    # (P, nw)
    ex = torch.exp(-u * u)
    g = torch.erf(u) - 2.0 / math.sqrt(math.pi) * u * ex
    T = _dipole_T(rv)                                       # (P, 3, 3)
    rr = rv[:, :, None] * rv[:, None, :] / r[:, None, None] ** 5
    h = (4.0 / math.sqrt(math.pi) * u ** 3 * ex)[:, :, None, None] * rr[:, None, :, :]
    core = -T[:, None, :, :] * g[:, :, None, None] + h
    pref = _cutoff_poly(r, rc, rb) * (1.0 - _fermi(r, S, d))
    return pref[:, None, None, None] * core


# ----------------------------------------------------------------------------
# Local SCS (Sec. III.B, local polarisability system B~_K alpha~_K = d_K)
# ----------------------------------------------------------------------------

class _Frame:
    """Geometry of the neighbourhood of one central atom, differentiable in positions."""

    def __init__(self, st, k, prm, images):
        r_big = max(2.0 * prm.r_scs, prm.r_nbr)
        base, sh, dist = neighbourhood(st["pos"], st["cell"], st["pbc"], k, r_big, images)
        self.k = k
        self.base = base
        self.shift = sh
        self.dist = dist
        self.n1 = int(np.sum(dist < prm.r_scs))
        self.n12 = int(np.sum(dist < 2.0 * prm.r_scs))
        self.nK = int(np.sum(dist < prm.r_nbr))

    def positions(self, pos_t, cell_t):
        """Site positions relative to the central atom, in bohr, as a torch tensor."""
        p = pos_t[self.base] - pos_t[self.k]
        if cell_t is not None:
            p = p + torch.as_tensor(self.shift, dtype=_DT) @ cell_t
        return p / BOHR


def _scs_solve(frame, p, fa, prm):
    """Solve the local SCS system of one frame at every frequency.

    B~_ij = delta_ij / abar_i + T_SR,ij (i, j in K1);
    d_i = 1 - sum_{j in K2} f_inner(r_ij) T_SR,ij abar_j;  X = B~^{-1} d;
    alpha~_K,i = Tr(X_i) / 3.
    Returns alpha_loc as a (nw, n1) tensor.
    """
    n1, n12 = frame.n1, frame.n12
    b1 = frame.base[:n1]
    abar = torch.as_tensor(fa["abar"], dtype=_DT)
    sigma = torch.as_tensor(fa["sigma"], dtype=_DT)
    Rv = torch.as_tensor(fa["R"], dtype=_DT)
    nw = abar.shape[1]
    rc, rb, rin = prm.r_scs / BOHR, prm.r_buf / BOHR, prm.r_inner / BOHR

    # B~ over K1 x K1
    I, J = np.nonzero(~np.eye(n1, dtype=bool))
    rv = p[I] - p[J]
    bi, bj = frame.base[I], frame.base[J]
    sig = torch.sqrt(sigma[bi] ** 2 + sigma[bj] ** 2)
    S = prm.beta * (Rv[bi] + Rv[bj])
    tsr = _t_sr(rv, sig, S, rc, rb, prm.damp_d)                       # (P, nw, 3, 3)
    blocks = torch.zeros((n1, n1, nw, 3, 3), dtype=_DT)
    blocks = blocks.index_put((torch.as_tensor(I), torch.as_tensor(J)), tsr)
    B = blocks.permute(2, 0, 3, 1, 4).reshape(nw, 3 * n1, 3 * n1)
    B = B + torch.diag_embed((1.0 / abar[b1]).T.repeat_interleave(3, dim=1))
    eye = torch.eye(3, dtype=_DT)

    # right-hand side d over K1, coupled to the uncoupled shell K2
    rhs = eye.expand(nw, n1, 3, 3).clone()
    if n12 > n1:
        ii, jj = np.meshgrid(np.arange(n1), np.arange(n1, n12), indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
        with torch.no_grad():
            rr = torch.sqrt(((p[ii] - p[jj]) ** 2).sum(-1))
        keep = (rr < rc).numpy()
        ii, jj = ii[keep], jj[keep]
        if ii.size:
            rv2 = p[ii] - p[jj]
            bi, bj = frame.base[ii], frame.base[jj]
            sig2 = torch.sqrt(sigma[bi] ** 2 + sigma[bj] ** 2)
            S2 = prm.beta * (Rv[bi] + Rv[bj])
            t2 = _t_sr(rv2, sig2, S2, rc, rb, prm.damp_d)           # (P2, nw, 3, 3)
            r2 = torch.sqrt((rv2 * rv2).sum(-1))
            x = r2 / rin
            finner = torch.where(r2 < rin, 3.0 * x * x - 2.0 * x ** 3, torch.ones_like(r2))
            contrib = finner[:, None, None, None] * t2 * abar[bj][:, :, None, None]
            acc = torch.zeros((n1, nw, 3, 3), dtype=_DT).index_add(0, torch.as_tensor(ii), contrib)
            rhs = rhs - acc.permute(1, 0, 2, 3)
    rhs = rhs.reshape(nw, 3 * n1, 3)
    X = torch.linalg.solve(B, rhs)                                   # (nw, 3 n1, 3)
    Xb = X.reshape(nw, n1, 3, 3)
    return torch.diagonal(Xb, dim1=-2, dim2=-1).sum(-1) / 3.0        # (nw, n1)


# ----------------------------------------------------------------------------
# Eigenvalue-bounded polynomial (Sec. III.A, Eqs. diagonal_appr, eigendecomp and
# polynomial-fit)
# ----------------------------------------------------------------------------

class PolarisationCatastrophe(ValueError):
    """The spectrum of G~_K reaches 1: ln(1 - x) has no real value there."""


_M64 = (1 << 64) - 1


def _splitmix64(z):
    """The output function of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) on the
    64-bit counter z: add the golden-ratio increment, then two xor-shift-multiply
    rounds and a final xor-shift."""
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def lanczos_start(k, base, shift):
    """Start vector of the Lanczos iteration of frame k (unnormalised, 3 entries per
    site): entry (site, c) = U(k, base atom, lattice shift, c), uniform in [-1/2, 1/2),
    keyed on the site's identity so that it does not depend on the order of the sites
    (a vector built from the geometry alone would be symmetric in a symmetric frame
    and could miss the extreme eigenvectors).  With s = the lattice shift packed as
    three 8-bit fields biased by 128:
        U = (SM(SM(k * 2^32 + base) + 4 s + c) >> 11) * 2^-53 - 1/2   (SM = SplitMix64)."""
    out = np.empty(3 * len(base))
    for i, (j, sh) in enumerate(zip(base, shift)):
        s = ((int(sh[0]) + 128) << 16) | ((int(sh[1]) + 128) << 8) | (int(sh[2]) + 128)
        h = _splitmix64((int(k) << 32) + int(j))
        for c in range(3):
            z = _splitmix64((h + 4 * s + c) & _M64)
            out[3 * i + c] = (z >> 11) * 2.0 ** -53 - 0.5
    return out


def lanczos_bounds(G, v1, steps, tol=1e-10):
    """Estimates of the smallest and largest eigenvalue of the symmetric G (Sec.
    III.A: Lanczos on the symmetrised matrix): `steps` Lanczos steps from v1 without
    reorthogonalisation, then the extreme eigenvalues of the tridiagonal matrix.
    Step j: w = G v_j - beta_j v_{j-1}, alpha_j = <v_j, w>, w -= alpha_j v_j,
    beta_{j+1} = |w|; the iteration stops early where beta_{j+1} <= tol (|alpha_j| +
    beta_j) (an invariant subspace: its Ritz values are exact)."""
    G = np.asarray(G, dtype=np.float64)
    v = np.asarray(v1, dtype=np.float64) / np.linalg.norm(v1)
    v_prev = np.zeros_like(v)
    beta = 0.0
    al, be = [], []
    for j in range(steps):
        w = G @ v - beta * v_prev
        alpha = float(v @ w)
        w = w - alpha * v
        al.append(alpha)
        if j == steps - 1:
            break
        beta_next = float(np.linalg.norm(w))
        if beta_next <= tol * (abs(alpha) + beta):
            break
        be.append(beta_next)
        v_prev, v, beta = v, w / beta_next, beta_next
    Tm = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    lam = np.linalg.eigvalsh(Tm)
    return float(lam[0]), float(lam[-1])


def log_fit_coefficients(lam_min, lam_max, n_max, n_nodes=32, f=None):
    """Coefficients c_0 .. c_{n_max} of the degree-n_max polynomial that fits
    f(x) = ln(1 - x) (or the given f) in the least-squares sense on the interval
    [lam_min, lam_max] (Eq. diagonal_appr): the sum over the n_nodes Gauss-Legendre
    nodes of the interval of the quadrature-weighted squared residual is minimised
    (the continuous fit with unit weight, discretised).  Solved by numpy's least
    squares on the weighted Vandermonde matrix in x / s, s = max(|lam_min|,
    |lam_max|), then scaled back.  An interval narrower than 1e-12 (no coupling)
    leaves the fit undetermined: the Taylor coefficients -1/n are returned, the limit
    of the fit as the interval shrinks to the origin."""
    if f is None:
        if lam_max >= 1.0:
            raise PolarisationCatastrophe(f"largest eigenvalue {lam_max} >= 1")
        f = lambda x: np.log1p(-x)
    if lam_max - lam_min <= 1e-12:
        return np.array([0.0] + [-1.0 / n for n in range(1, n_max + 1)])
    x, w = np.polynomial.legendre.leggauss(n_nodes)
    h, c = 0.5 * (lam_max - lam_min), 0.5 * (lam_max + lam_min)
    lam = c + h * x
    sc = max(abs(lam_min), abs(lam_max))
    V = (lam / sc)[:, None] ** np.arange(n_max + 1)[None, :]
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(sw[:, None] * V, sw * f(lam), rcond=None)
    return coef / sc ** np.arange(n_max + 1)


def spectrum_bounds(G):
    """Smallest and largest eigenvalue of the symmetric matrix G (the values the
    Lanczos iteration converges to)."""
    lam = np.linalg.eigvalsh(np.asarray(G, dtype=np.float64))
    return float(lam[0]), float(lam[-1])


def frame_bounds(frame, p, alpha_loc, alpha_cen_K, fa, prm):
    """(n_nodes, 2) bounds [lambda_min, lambda_max] of G~_K at every node: Lanczos
    with prm.lanczos_steps steps, or the exact extremes if that is None."""
    with torch.no_grad():
        A, T = _mbd_operators(frame, p, alpha_loc, alpha_cen_K, fa, prm)
        v1 = lanczos_start(frame.k, frame.base[:frame.nK], frame.shift[:frame.nK])
        out = []
        for q in range(len(prm.omega)):
            s = torch.sqrt(A[:, q + 1]).repeat_interleave(3)
            G = (s[:, None] * T * s[None, :]).numpy()
            if prm.lanczos_steps is None:
                out.append(spectrum_bounds(G))
            else:
                out.append(lanczos_bounds(G, v1, prm.lanczos_steps))
    return np.array(out)


def fitted_coefficients(frame, p, alpha_loc, alpha_cen_K, fa, prm):
    """(n_nodes, n_max + 1) fitted coefficients of one frame, one row per node."""
    bounds = frame_bounds(frame, p, alpha_loc, alpha_cen_K, fa, prm)
    return np.array([log_fit_coefficients(a, b, prm.n_max, prm.fit_nodes) for a, b in bounds])


# ----------------------------------------------------------------------------
# Local MBD energy (Sec. III.A symmetrised local energy; Sec. III.B blend)
# ----------------------------------------------------------------------------

def lorentz_polarisabilities(a0, a_ref, omega, omega_ref):
    """Two-point Lorentzian model of Sec. III.C: (..., len(omega)) polarisabilities.

    Eq. (char-freq): the characteristic frequency omega~ = omega_ref /
    sqrt(alpha~(0)/alpha~(omega_ref) - 1); Eq. (alpha_SCS_freq): alpha~(omega) =
    alpha~(0) / (1 + (omega/omega~)^2).  Needs alpha~(0) >= alpha~(omega_ref) > 0
    (a real characteristic frequency); ValueError otherwise.
    """
    if bool(torch.any(a_ref <= 0.0)) or bool(torch.any(a0 < a_ref)):
        raise ValueError("SCS polarisability not decreasing between 0 and omega_ref")
    om_t = omega_ref / torch.sqrt(a0 / a_ref - 1.0)
    w = torch.as_tensor(np.asarray(omega, dtype=np.float64), dtype=_DT)
    return a0[..., None] / (1.0 + (w / om_t[..., None]) ** 2)


def _mbd_operators(frame, p, alpha_loc, alpha_cen_K, fa, prm, two_body=False):
    """Blended polarisabilities A (nK, 1 + n_nodes: omega = 0, then the nodes) and
    T_LR (3 nK x 3 nK) of one frame; with two_body also the n = 2 term's T_LR, cut at
    the two-body radii.

    alpha_loc: (nw, n1) local polarisabilities of the frame; alpha_cen_K: (nK, nw)
    central polarisabilities of the base atoms of the first nK sites.
    """
    nK, n1 = frame.nK, frame.n1
    rscs = prm.r_scs / BOHR
    rb = prm.r_buf / BOHR
    a0 = torch.as_tensor(fa["alpha0"], dtype=_DT)[frame.base[:nK]]
    r0 = torch.as_tensor(fa["r0"], dtype=_DT)[frame.base[:nK]]
    pk = p[:nK]

    # blended polarisabilities alpha~_i(w), i in K
    alphas = []
    for s in range(nK):
        if s < n1:
            if s == 0:
                alphas.append(alpha_loc[:, 0])  # f_SCS(0) = 0: the central atom's own value
            else:
                r = torch.sqrt((pk[s] * pk[s]).sum())
                x = r / rscs
                f = 3.0 * x * x - 2.0 * x ** 3
                alphas.append((1.0 - f) * alpha_loc[:, s] + f * alpha_cen_K[s])
        else:
            alphas.append(alpha_cen_K[s])
    A = torch.stack(alphas, 0)                                        # (nK, nw)
    if prm.scs_freq == "lorentz":
        # columns: omega = 0, then the nodes from the two-point model
        A = torch.cat([A[:, :1], lorentz_polarisabilities(A[:, 0], A[:, 1], prm.omega, prm.omega_ref)], 1)

    # SCS vdW radii and T_LR (Sec. II.B scaled radii; Sec. III.A f_LR)
    Rt = r0 * (A[:, 0] / a0) ** (1.0 / 3.0)
    I, J = np.nonzero(~np.eye(nK, dtype=bool))
    rv = pk[I] - pk[J]
    r = torch.sqrt((rv * rv).sum(-1))
    St = prm.beta * (Rt[I] + Rt[J])
    central = (I == 0) | (J == 0)
    damped = _fermi(r, St, prm.damp_d)[:, None, None] * _dipole_T(rv)

    def t_lr(r1, r2):   # f_LR with p = 1 at r1 for pairs touching k, p = 2 at r2 for the others
        rcut = torch.as_tensor(np.where(central, r1, r2) / BOHR, dtype=_DT)
        x = (r - rcut + rb) / rb
        flr = torch.where(r < rcut - rb, torch.ones_like(r),
                          torch.where(r < rcut, 1.0 - 3.0 * x * x + 2.0 * x ** 3, torch.zeros_like(r)))
        blocks = torch.zeros((nK, nK, 3, 3), dtype=_DT).index_put(
            (torch.as_tensor(I), torch.as_tensor(J)), flr[:, None, None] * damped)
        return blocks.permute(0, 2, 1, 3).reshape(3 * nK, 3 * nK)

    T = t_lr(prm.r_mbd1, prm.r_mbd2)
    if not two_body:
        return A, T
    return A, T, (t_lr(*prm.two_body_radii()) if prm.separate_two_body() else T)


def _mbd_energy(frame, p, alpha_loc, alpha_cen_K, fa, prm):
    """Energy of one central atom in eV (Sec. III.A, the symmetrised local energy)."""
    nK = frame.nK
    A, T, T2 = _mbd_operators(frame, p, alpha_loc, alpha_cen_K, fa, prm, two_body=True)
    sep = prm.separate_two_body()
    coef = prm.coefficients()
    if sep and coef is None:
        raise ValueError("separate two-body radii need a finite body order")
    cfit = None
    if prm.c_n_mode == "fit":
        # per node: c_n fitted over [lambda_min, lambda_max] of G~ (held fixed under
        # differentiation: the forces treat the coefficients as constants, as the
        # force expression of Sec. III.D does); the n = 0 and n = 1 terms are dropped
        if prm.coef_fixed is not None and frame.k in prm.coef_fixed:
            cfit = np.asarray(prm.coef_fixed[frame.k], dtype=np.float64)
        else:
            cfit = fitted_coefficients(frame, p, alpha_loc, alpha_cen_K, fa, prm)
    e_freq = []
    for q in range(len(prm.omega)):
        s = torch.sqrt(A[:, q + 1]).repeat_interleave(3)
        G = s[:, None] * T * s[None, :]                               # sqrt(A) T sqrt(A)
        if cfit is not None:
            coef = cfit[q].copy()
            coef[:2] = 0.0
        if coef is None:
            lam, V = torch.linalg.eigh(G)
            e_freq.append((torch.log1p(-lam) * (V[:3, :] ** 2).sum(0)).sum())
        else:
            u = torch.zeros((3 * nK, 3), dtype=_DT)
            u[:3, :3] = torch.eye(3, dtype=_DT)
            acc = torch.zeros((), dtype=_DT)
            for n in range(1, prm.n_max + 1):
                u = G @ u
                if coef[n] != 0.0 and not (sep and n == 2):
                    acc = acc + coef[n] * torch.trace(u[:3, :])
            if sep:   # the n = 2 term with the two-body T_LR: Tr[G2 G2]_kk over the central block row
                g2 = s[:3, None] * T2[:3, :] * s[None, :]
                acc = acc + coef[2] * (g2 * g2).sum()
            e_freq.append(acc)
    wq = torch.as_tensor(prm.weight, dtype=_DT)
    return (wq * torch.stack(e_freq)).sum() / (2.0 * math.pi) * HARTREE


def _paper_force_functional(frame, p, alpha_loc, alpha_cen_K, fa, prm):
    """A scalar whose gradient with respect to the central atom is the paper's
    approximate force on it (Sec. III.D, Eqs. cent-appr-step and cent-appr), eV.

    The force is minus the gradient of the total energy the central atom k sees,
    E^tot_k = int dw/2pi sum_n c_n Tr(G~^n) over the whole neighbourhood, with
    two approximations: the central polarisabilities do not move (Eq.
    full-pol-grad; the caller passes them as constants), and for n >= 3 only the
    block row and column of k in dG~ are kept, which makes the n-th term's
    derivative n Tr(G~^(n-1) dG~) = 2 n Tr(g~_k G~^(n-2) dg~_k^T).  The n = 2 term
    is differentiated in full.  So the functional is
        int dw/2pi [ c_2 Tr(G~^2) + sum_{n>=3} c_n n Tr(g~_k B_n g~_k^T) ],
    B_n = G~^(n-2) held fixed, g~_k the block row of k.  Its value is not an
    energy; only its gradient with respect to r_k is used.  With the fitted
    coefficients (prm.c_n_mode == "fit") each node takes the frame's own c_n,
    held fixed.  With separate two-body radii the n = 2 trace uses their T_LR
    (r_2b1 on the pairs touching k, r_2b2 on the others).
    """
    nK = frame.nK
    A, T, T2 = _mbd_operators(frame, p, alpha_loc, alpha_cen_K, fa, prm, two_body=True)
    coef = prm.coefficients()
    assert coef is not None, "the approximate forces need a finite n_max"
    cfit = fitted_coefficients(frame, p, alpha_loc, alpha_cen_K, fa, prm) if prm.c_n_mode == "fit" else None
    vals = []
    for q in range(len(prm.omega)):
        s = torch.sqrt(A[:, q + 1]).repeat_interleave(3)
        G = s[:, None] * T * s[None, :]
        if cfit is not None:
            coef = cfit[q]
        G2 = s[:, None] * T2 * s[None, :]                 # the n = 2 term's G (two-body radii)
        acc = coef[2] * (G2 * G2).sum()                   # Tr(G^2) of the symmetric G
        g = G[:3, :]                                      # block row of the central atom
        Gf = G.detach()
        for n in range(3, prm.n_max + 1):
            B = torch.linalg.matrix_power(Gf, n - 2)      # held fixed
            acc = acc + coef[n] * n * torch.trace(g @ B @ g.T)
        vals.append(acc)
    wq = torch.as_tensor(prm.weight, dtype=_DT)
    return (wq * torch.stack(vals)).sum() / (2.0 * math.pi) * HARTREE


def lmbd_paper_forces(structure, prm, species_table, weights=None, atoms=None):
    """Per-atom energies (eV) and the paper's approximate forces (eV/A): for each
    atom k, F_k = -w_k d/dr_k of the functional of _paper_force_functional in
    k's own neighbourhood, with k's own local SCS solve differentiated and the
    central polarisabilities of the other atoms held fixed (Sec. III.D).  With
    SCS switched off and cutoffs covering the whole structure this is the exact
    force of the total energy; in general it is not the gradient of sum_k E_k.
    ``atoms`` restricts the atoms whose forces are formed (others are zero)."""
    st, fa, images = _prepare(structure, prm, species_table)
    N = structure.n
    w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
    ks = list(range(N)) if atoms is None else list(atoms)
    e = lmbd_energies(structure, prm, species_table, atoms=ks)
    frames = {k: _Frame(st, k, prm, images) for k in ks}
    needed = sorted({int(b) for k in ks for b in frames[k].base[:frames[k].nK]})
    central = scs_central(structure, prm, species_table, needed)
    cell_t = _cell_tensor(st)
    f = np.zeros((N, 3))
    for k in ks:
        fr = frames[k]
        pos_t = torch.tensor(st["pos"], dtype=_DT, requires_grad=True)
        p = fr.positions(pos_t, cell_t)
        aloc = _scs_solve(fr, p, fa, prm)
        acen = torch.as_tensor(central[fr.base[:fr.nK]], dtype=_DT)   # d alpha~_I ~ 0
        val = _paper_force_functional(fr, p, aloc, acen, fa, prm)
        if val.requires_grad:
            (grad,) = torch.autograd.grad(val, pos_t)
            f[k] = -w[k] * grad[k].numpy()
    return e, f


# ----------------------------------------------------------------------------
# Drivers
# ----------------------------------------------------------------------------

def _prepare(structure, prm, species_table):
    st = dict(pos=np.asarray(structure.pos, dtype=np.float64), cell=structure.cell,
              pbc=np.asarray(structure.pbc, dtype=bool))
    fa = free_atom_terms(species_table, structure.species, structure.nu, prm.scs_omegas())
    images = _Images(st["pos"], st["cell"], st["pbc"], max(2.0 * prm.r_scs, prm.r_nbr))
    return st, fa, images


def _cell_tensor(st):
    return None if st["cell"] is None else torch.as_tensor(st["cell"], dtype=_DT)


def scs_central(structure, prm, species_table, atoms=None):
    """Central SCS polarisabilities alpha~_I,k(w) at the SCS frequencies: (N, nw) array.

    The central polarisability of atom k is the k-th entry of its own local
    SCS solution (Sec. III.B, the central/local blend).
    """
    st, fa, images = _prepare(structure, prm, species_table)
    N = structure.n
    nw = len(prm.scs_omegas())
    out = np.zeros((N, nw))
    pos_t = torch.as_tensor(st["pos"], dtype=_DT)
    cell_t = _cell_tensor(st)
    for k in (range(N) if atoms is None else atoms):
        fr = _Frame(st, k, prm, images)
        with torch.no_grad():
            out[k] = _scs_solve(fr, fr.positions(pos_t, cell_t), fa, prm)[:, 0].numpy()
    return out


def lmbd_energies(structure, prm, species_table, atoms=None, central=None):
    """Per-atom lMBD energies in eV (array of length N; atoms not requested are 0).

    Two stages as in the paper's flowchart: every central polarisability first,
    then each atom's local SCS, blend and series energy.
    """
    st, fa, images = _prepare(structure, prm, species_table)
    N = structure.n
    if central is None:
        needed = None
        if atoms is not None:
            needed = set()
            for k in atoms:
                fr = _Frame(st, k, prm, images)
                needed.update(int(b) for b in fr.base[:fr.nK])
            needed = sorted(needed)
        central = scs_central(structure, prm, species_table, needed)
    pos_t = torch.as_tensor(st["pos"], dtype=_DT)
    cell_t = _cell_tensor(st)
    e = np.zeros(N)
    with torch.no_grad():
        for k in (range(N) if atoms is None else atoms):
            fr = _Frame(st, k, prm, images)
            p = fr.positions(pos_t, cell_t)
            aloc = _scs_solve(fr, p, fa, prm)
            acen = torch.as_tensor(central[fr.base[:fr.nK]], dtype=_DT)
            e[k] = float(_mbd_energy(fr, p, aloc, acen, fa, prm))
    return e


def lmbd_spectrum_bounds(structure, prm, species_table, atoms=None):
    """(N, n_nodes, 2) bounds [lambda_min, lambda_max] of G~_K of every atom at every
    quadrature node (Lanczos estimates, or exact with prm.lanczos_steps = None); the
    rows of atoms not requested are 0.  A largest eigenvalue of 1 or more is the
    polarisation catastrophe of Sec. III.A (1 - G~_K is then not positive definite)."""
    st, fa, images = _prepare(structure, prm, species_table)
    N = structure.n
    needed = set()
    for k in (range(N) if atoms is None else atoms):
        fr = _Frame(st, k, prm, images)
        needed.update(int(b) for b in fr.base[:fr.nK])
    central = scs_central(structure, prm, species_table, sorted(needed))
    pos_t = torch.as_tensor(st["pos"], dtype=_DT)
    cell_t = _cell_tensor(st)
    out = np.zeros((N, len(prm.omega), 2))
    with torch.no_grad():
        for k in (range(N) if atoms is None else atoms):
            fr = _Frame(st, k, prm, images)
            p = fr.positions(pos_t, cell_t)
            aloc = _scs_solve(fr, p, fa, prm)
            acen = torch.as_tensor(central[fr.base[:fr.nK]], dtype=_DT)
            out[k] = frame_bounds(fr, p, aloc, acen, fa, prm)
    return out


def lmbd_energy_forces(structure, prm, species_table, weights=None, atoms=None, timings=None, want_dv=False):
    """Per-atom energies (eV) and exact forces -d(sum_k w_k E_k)/dR (eV/A).

    With ``want_dv`` a third array is returned: d(sum_k w_k E_k)/d nu (eV), the
    derivative with respect to the Hirshfeld-volume ratios, which enter through
    the TS polarisabilities, attenuation lengths and radii (Sec. II.B); the same
    two reverse passes carry it.

    Reverse mode in two passes, mirroring the two stages: pass B differentiates
    each atom's MBD stage (its own local SCS included) and collects the
    gradients of the central polarisabilities it used; pass C pushes those
    through each atom's own SCS solve.  ``atoms`` restricts the sum over k
    (for timing a bounded sample); the forces are then those of that partial sum.
    If ``timings`` is a dict, the wall time and the number of atoms of the
    central pass (A), pass B and pass C are stored in it.
    """
    import time
    t0 = time.perf_counter()
    st, fa, images = _prepare(structure, prm, species_table)
    N = structure.n
    nw = len(prm.scs_omegas())
    nu_t = None
    if want_dv:
        nu_t = torch.tensor(np.asarray(structure.nu, dtype=np.float64), dtype=_DT, requires_grad=True)

    def fa_graph():   # free-atom terms; with want_dv a fresh graph from nu for every backward pass
        return fa if nu_t is None else free_atom_terms(species_table, structure.species, nu_t, prm.scs_omegas())
    w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
    ks = list(range(N)) if atoms is None else list(atoms)
    frames = {}

    def frame(k):
        if k not in frames:
            frames[k] = _Frame(st, k, prm, images)
        return frames[k]

    needed = sorted({int(b) for k in ks for b in frame(k).base[:frame(k).nK]})
    t1 = time.perf_counter()
    central = scs_central(structure, prm, species_table, needed)
    t2 = time.perf_counter()
    cell_t = _cell_tensor(st)
    pos_t = torch.tensor(st["pos"], dtype=_DT, requires_grad=True)
    abar_c = np.zeros((N, nw))
    e = np.zeros(N)
    for k in ks:  # pass B
        fr = frame(k)
        p = fr.positions(pos_t, cell_t)
        fk = fa_graph()
        aloc = _scs_solve(fr, p, fk, prm)
        acen = torch.tensor(central[fr.base[:fr.nK]], dtype=_DT, requires_grad=True)
        ek = _mbd_energy(fr, p, aloc, acen, fk, prm)
        e[k] = float(ek.detach())
        if ek.requires_grad:
            (w[k] * ek).backward()
        if acen.grad is not None:   # an atom with no neighbour in K uses no central polarisability
            np.add.at(abar_c, fr.base[:fr.nK], acen.grad.numpy())
    t3 = time.perf_counter()
    n_c = 0
    for a in range(N):  # pass C
        if not np.any(abar_c[a] != 0.0):
            continue
        n_c += 1
        fr = frame(a)
        p = fr.positions(pos_t, cell_t)
        aloc = _scs_solve(fr, p, fa_graph(), prm)
        (aloc[:, 0] * torch.as_tensor(abar_c[a], dtype=_DT)).sum().backward()
    t4 = time.perf_counter()
    if timings is not None:
        timings.update(prepare_s=t1 - t0, central_s=t2 - t1, central_atoms=len(needed), pass_b_s=t3 - t2,
                       pass_b_atoms=len(ks), pass_c_s=t4 - t3, pass_c_atoms=n_c)
    f = np.zeros_like(st["pos"]) if pos_t.grad is None else -pos_t.grad.numpy().copy()
    if want_dv:   # (no gradient: no energy depends on a volume ratio)
        dv = np.zeros(N) if nu_t.grad is None else nu_t.grad.numpy().copy()
        return e, f, dv
    return e, f
