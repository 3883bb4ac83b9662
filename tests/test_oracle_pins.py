"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test compares the oracle with a closed form, a limit, an invariance or an
independent construction (numerical Hessians, adaptive quadrature, the
whole-system model) so that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import lmbd as L
from workloads import SPECIES_TABLE, SPECIES_INDEX, frequency_grid, Structure
from workloads import configs as C
from tests import closed_forms as cf

GRID12 = frequency_grid(12)
GRID200 = frequency_grid(200)

C_IDX = SPECIES_INDEX["C"]


def _open(pos, species=None, nu=None):
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    sp = np.full(n, C_IDX, dtype=np.int32) if species is None else np.asarray(species, np.int32)
    nu = np.full(n, 0.85) if nu is None else np.asarray(nu, np.float64)
    return Structure(pos, sp, nu, None, np.zeros(3, bool))


def _params(r_scs, r_nbr, grid=GRID12, **kw):
    return oracle.make_params(dict(r_scs=r_scs, r_nbr=r_nbr, r_mbd1=r_nbr, r_mbd2=r_nbr),
                              grid[0], grid[1], **kw)


def _rand_cluster(n, seed, box=7.0, dmin=1.6, hcno=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    from workloads.structures import rsa_cube_open, hcno_species
    pos = rsa_cube_open(n, box, dmin, rng)
    sp = hcno_species(n, rng) if hcno else np.full(n, C_IDX, np.int32)
    nu = rng.uniform(0.6, 1.0, n)
    return Structure(pos, sp, nu, None, np.zeros(3, bool))


def _free(st):
    tab = SPECIES_TABLE[st.species]
    a = tab[:, 0] * st.nu
    w = 4.0 * tab[:, 1] / (3.0 * tab[:, 0] ** 2)
    R = tab[:, 2] * st.nu ** (1.0 / 3.0)
    return a, w, R


# SCS switched off: K1 = {k}, K2 empty (2 r_scs below every distance), so the
# polarisabilities stay at their TS values; all MBD pairs inside r_nbr - r_b.
NO_SCS = 0.6


# --------------------------------------------------------------------------- P1

def test_quadrature_reproduces_casimir_polder():
    """(3/pi) int abar_i abar_j dw on the 12-point grid equals the London formula."""
    om, wt = GRID12
    worst = 0.0
    for i in range(4):
        for j in range(4):
            for nui, nuj in ((1.0, 1.0), (0.6, 0.9)):
                fi = oracle.free_atom_terms(SPECIES_TABLE, np.array([i, j]), np.array([nui, nuj]), om)
                num = 3.0 / math.pi * np.sum(wt * fi["abar"][0] * fi["abar"][1])
                a0 = SPECIES_TABLE[[i, j], 0] * [nui, nuj]
                w0 = 4 * SPECIES_TABLE[[i, j], 1] / (3 * SPECIES_TABLE[[i, j], 0] ** 2)
                ref = cf.c6_casimir_polder(a0[0], w0[0], a0[1], w0[1])
                worst = max(worst, abs(num / ref - 1.0))
                if i == j and nui == nuj:
                    # the free-atom C6 comes back, scaled by nu^2
                    assert abs(ref / (SPECIES_TABLE[i, 1] * nui ** 2) - 1) < 1e-13
    assert worst < 5e-8
    om2, wt2 = GRID200
    fi = oracle.free_atom_terms(SPECIES_TABLE, np.array([0, 3]), np.array([0.7, 0.9]), om2)
    num = 3.0 / math.pi * np.sum(wt2 * fi["abar"][0] * fi["abar"][1])
    a0 = SPECIES_TABLE[[0, 3], 0] * [0.7, 0.9]
    w0 = 4 * SPECIES_TABLE[[0, 3], 1] / (3 * SPECIES_TABLE[[0, 3], 0] ** 2)
    assert abs(num / cf.c6_casimir_polder(a0[0], w0[0], a0[1], w0[1]) - 1) < 1e-12


# ---------------------------------------------------------------- pair tensors

def test_dipole_tensor_is_hessian_of_coulomb():
    import torch
    rng = np.random.default_rng(3)
    for _ in range(5):
        rv = rng.normal(size=3) * 3
        T = L._dipole_T(torch.as_tensor(rv)[None]).numpy()[0]
        H = cf.numerical_hessian(cf.coulomb, rv, h=1e-2 * np.linalg.norm(rv))
        assert np.allclose(T, H, rtol=1e-8, atol=1e-8 * np.abs(H).max())


def test_short_range_tensor_is_screened_erf_hessian():
    """T_SR = (1 - f) d/dr_i d/dr_j [erf(r/sigma)/r] with the f_SR cutoff equal to 1."""
    import torch
    rng = np.random.default_rng(4)
    for _ in range(6):
        rv = rng.normal(size=3)
        rv *= rng.uniform(1.0, 7.0) / np.linalg.norm(rv)
        sig = rng.uniform(1.0, 3.0)
        S = rng.uniform(4.0, 7.0)
        got = L._t_sr(torch.as_tensor(rv)[None], torch.tensor([[sig]], dtype=torch.float64),
                      torch.tensor([S], dtype=torch.float64),
                      100.0, 1.0, 6.0).numpy()[0, 0]
        ref = cf.sr_tensor_fd(rv, sig, S)
        assert np.allclose(got, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_cutoff_polynomial_is_c1_smooth():
    import torch
    r = torch.linspace(3.0, 6.0, 3001, dtype=torch.float64)
    f = L._cutoff_poly(r, 5.0, 0.5).numpy()
    assert f[0] == 1.0 and f[-1] == 0.0
    assert np.all(np.diff(f) <= 1e-15)
    assert np.max(np.abs(np.diff(f))) < 4e-3   # no jump; slope bounded by 1.5 / r_b


# --------------------------------------------------------------- SCS (P6, P7, P8)

def _sigma(a):
    return (math.sqrt(2.0 / math.pi) * a / 3.0) ** (1.0 / 3.0)


def _solve_scs_fd(centers_bohr, abar, R, fixed=None, beta=0.83, finner=None, rc=None, rb=None):
    """Independent small SCS solve with tensors from numerical Hessians.

    centers: coupled atoms (n, 3) bohr; abar/R: their TS values; fixed: list of
    (pos, abar_j, R_j) uncoupled atoms entering the right-hand side, with the
    optional inner-buffer weight finner(r).  Pairs at or beyond rc (bohr) do not
    couple.  Without rb the constructions keep every coupled pair clear of the
    cutoff buffer; with rb (bohr) every tensor is scaled by the C1 cubic switch
    over [rc - rb, rc].
    """
    n = len(centers_bohr)
    B = np.zeros((3 * n, 3 * n))
    couples = lambda rv: rc is None or np.linalg.norm(rv) < rc
    fsr = lambda rv: 1.0 if rb is None else cf.smooth_cutoff(np.linalg.norm(rv), rc, rb)
    for i in range(n):
        B[3 * i:3 * i + 3, 3 * i:3 * i + 3] = np.eye(3) / abar[i]
        for j in range(n):
            if i != j and couples(centers_bohr[i] - centers_bohr[j]):
                rv = centers_bohr[i] - centers_bohr[j]
                sig = math.hypot(_sigma(abar[i]), _sigma(abar[j]))
                B[3 * i:3 * i + 3, 3 * j:3 * j + 3] = fsr(rv) * cf.sr_tensor_fd(rv, sig, beta * (R[i] + R[j]))
    d = np.tile(np.eye(3), (n, 1))
    for (pj, aj, Rj) in (fixed or []):
        for i in range(n):
            rv = centers_bohr[i] - pj
            r = np.linalg.norm(rv)
            if not couples(rv):
                continue
            sig = math.hypot(_sigma(abar[i]), _sigma(aj))
            w = (1.0 if finner is None else finner(r)) * fsr(rv)
            d[3 * i:3 * i + 3] -= w * cf.sr_tensor_fd(rv, sig, beta * (R[i] + Rj)) * aj
    X = np.linalg.solve(B, d)
    return np.array([np.trace(X[3 * i:3 * i + 3]) / 3.0 for i in range(n)])


def test_scs_dimer_matches_independent_solve():
    st = _open([[0, 0, 0], [1.2, 1.0, 0.4]], species=[C_IDX, SPECIES_INDEX["O"]], nu=[0.8, 0.95])
    prm = _params(5.0, 5.0)
    got = oracle.scs_central(st, prm, SPECIES_TABLE)
    a0, w0, R = _free(st)
    omegas = np.concatenate([[0.0], prm.omega])
    x = st.pos / cf.BOHR
    for q, w in enumerate(omegas):
        ab = a0 / (1.0 + (w / w0) ** 2)
        ref = _solve_scs_fd(x, ab, R)
        assert np.allclose(got[:, q], ref, rtol=1e-7)
    # screening raises the polarisability along a bonded pair at this distance
    assert np.all(got[:, 0] != a0)


def test_scs_isolated_atom_keeps_ts_polarisability():
    st = _open([[0, 0, 0], [20.0, 0, 0]], nu=[0.7, 0.9])
    prm = _params(5.0, 5.0)
    got = oracle.scs_central(st, prm, SPECIES_TABLE)
    fa = oracle.free_atom_terms(SPECIES_TABLE, st.species, st.nu, np.concatenate([[0.0], prm.omega]))
    assert np.allclose(got, fa["abar"], rtol=1e-15, atol=0)


def test_scs_uncoupled_shell_and_inner_buffer():
    """K2 atoms enter only the right-hand side, with TS polarisability and f_inner."""
    # k at the origin, i inside r_scs, j in the shell [r_scs, 2 r_scs) of k but 1.49 A from i
    st = _open([[0, 0, 0], [2.0, 0, 0], [3.4, 0.5, 0.0]], nu=[0.9, 0.8, 0.7],
               species=[C_IDX, C_IDX, SPECIES_INDEX["N"]])
    prm = _params(3.0, 3.0)
    got = oracle.scs_central(st, prm, SPECIES_TABLE)
    a0, w0, R = _free(st)
    x = st.pos / cf.BOHR
    rin = 2.0 / cf.BOHR
    rc = 3.0 / cf.BOHR
    finner = lambda r: 3 * (r / rin) ** 2 - 2 * (r / rin) ** 3 if r < rin else 1.0
    for q, w in enumerate(np.concatenate([[0.0], prm.omega])):
        ab = a0 / (1.0 + (w / w0) ** 2)
        # frame of atom 0: K1 = {0, 1}, K2 = {2}
        ref0 = _solve_scs_fd(x[:2], ab[:2], R[:2], fixed=[(x[2], ab[2], R[2])], finner=finner, rc=rc)[0]
        # frame of atom 1: all three inside r_scs, no shell
        ref1 = _solve_scs_fd(x, ab, R, rc=rc)[1]
        assert abs(got[0, q] / ref0 - 1) < 1e-7
        assert abs(got[1, q] / ref1 - 1) < 1e-7


def test_full_cutoff_local_scs_is_whole_system_scs():
    st = _rand_cluster(16, 11)
    prm = _params(16.0, 16.0)  # covers the cluster diameter plus the buffer
    got = oracle.scs_central(st, prm, SPECIES_TABLE)
    ref = oracle.full_scs(st.pos, st.species, st.nu, SPECIES_TABLE, np.concatenate([[0.0], prm.omega]))
    assert np.allclose(got, ref, rtol=1e-12)


# ------------------------------------------------------------ MBD (P2, P3, P4)

def test_second_order_is_damped_pairwise_c6():
    st = _rand_cluster(8, 21, box=6.0, dmin=1.5)
    prm = _params(NO_SCS, 30.0, grid=GRID200, n_max=2)
    e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    a, w, R = _free(st)
    x = st.pos / cf.BOHR
    ref = np.zeros(st.n)
    for i in range(st.n):
        for j in range(st.n):
            if i != j:
                r = np.linalg.norm(x[i] - x[j])
                f = cf.fermi(r, 0.83 * (R[i] + R[j]) / cf.BOHR * cf.BOHR)
                f = cf.fermi(r, 0.83 * (R[i] + R[j]))
                ref[i] += -0.5 * cf.c6_casimir_polder(a[i], w[i], a[j], w[j]) * f * f / r ** 6
    assert np.allclose(e, ref * cf.HARTREE, rtol=1e-11, atol=0)


def test_third_order_is_axilrod_teller_muto():
    pos = np.array([[0.0, 0.0, 0.0], [3.1, 0.0, 0.0], [1.2, 2.6, 0.7]])
    st = _open(pos, species=[C_IDX, SPECIES_INDEX["N"], SPECIES_INDEX["H"]], nu=[0.9, 0.75, 0.8])
    e2 = oracle.lmbd_energies(st, _params(NO_SCS, 30.0, grid=GRID200, n_max=2), SPECIES_TABLE).sum()
    e3 = oracle.lmbd_energies(st, _params(NO_SCS, 30.0, grid=GRID200, n_max=3), SPECIES_TABLE).sum()
    a, w, R = _free(st)
    x = pos / cf.BOHR
    f = 1.0
    for i, j in ((0, 1), (1, 2), (2, 0)):
        f *= cf.fermi(np.linalg.norm(x[i] - x[j]), 0.83 * (R[i] + R[j]))
    ref = cf.c9_atm(a[0], w[0], a[1], w[1], a[2], w[2]) * f * cf.atm_geometry_factor(*x)
    assert abs((e3 - e2) / (ref * cf.HARTREE) - 1.0) < 1e-10


def _dimer_couplings(st):
    a, w, R = _free(st)
    r = np.linalg.norm(st.pos[1] - st.pos[0]) / cf.BOHR
    f = cf.fermi(r, 0.83 * (R[0] + R[1]))
    return a, w, [2.0 * f / r ** 3, -f / r ** 3, -f / r ** 3]


def test_coupled_oscillator_dimer_log_limit():
    st = _open([[0, 0, 0], [2.3, 1.1, -0.6]], species=[C_IDX, SPECIES_INDEX["O"]], nu=[0.8, 0.9])
    e = oracle.lmbd_energies(st, _params(NO_SCS, 30.0, grid=GRID200, n_max=None), SPECIES_TABLE)
    a, w, t = _dimer_couplings(st)
    ref = cf.qho_dimer_energy(a[0], w[0], a[1], w[1], t) * cf.HARTREE
    assert abs(e.sum() / ref - 1) < 1e-10
    assert abs(e[0] - e[1]) < 1e-12 * abs(ref)


def test_dimer_truncated_series_matches_adaptive_quadrature():
    st = _open([[0, 0, 0], [1.9, 0.0, 0.9]], species=[C_IDX, C_IDX], nu=[0.7, 1.0])
    e = oracle.lmbd_energies(st, _params(NO_SCS, 30.0, grid=GRID200, n_max=6), SPECIES_TABLE)
    a, w, t = _dimer_couplings(st)
    ref = cf.dimer_series_energy(a[0], w[0], a[1], w[1], t, 6) * cf.HARTREE
    assert abs(e.sum() / ref - 1) < 1e-10


def test_series_converges_to_block_logarithm():
    st = _rand_cluster(10, 31, box=7.0, dmin=2.0)
    e_log = oracle.lmbd_energies(st, _params(4.0, 6.0, n_max=None), SPECIES_TABLE)
    e_40 = oracle.lmbd_energies(st, _params(4.0, 6.0, n_max=40), SPECIES_TABLE)
    e_2 = oracle.lmbd_energies(st, _params(4.0, 6.0, n_max=2), SPECIES_TABLE)
    assert np.allclose(e_40, e_log, rtol=1e-9, atol=1e-13)
    assert not np.allclose(e_2, e_log, rtol=1e-4)


# ---------------------------------------- cutoff buffers and the two MBD radii

def _radii_params(r_scs, r_nbr, r_mbd1, r_mbd2, grid=GRID200, **kw):
    return oracle.make_params(dict(r_scs=r_scs, r_nbr=r_nbr, r_mbd1=r_mbd1, r_mbd2=r_mbd2),
                              grid[0], grid[1], **kw)


def _at_distance(r_A, direction=(0.3, -0.8, 0.52)):
    d = np.asarray(direction, dtype=np.float64)
    return d * (r_A / np.linalg.norm(d))


def test_cutoff_polynomial_is_the_c1_hermite_cubic():
    """The SR buffer function equals the unique cubic that leaves 1 and reaches 0
    with zero slope at both ends of the buffer (Sec. III.B f_SR)."""
    import torch
    rc, rb = 5.0, 0.5
    r = np.linspace(4.2, 5.2, 201)
    got = L._cutoff_poly(torch.as_tensor(r), rc, rb).numpy()
    ref = np.array([cf.smooth_cutoff(x, rc, rb) for x in r])
    assert np.allclose(got, ref, rtol=0, atol=1e-13)


def test_buffered_dimer_second_order():
    """SCS off, n_max = 2, the pair inside the f_LR buffer of r_MBD,1: every pair of a
    dimer touches the central atom, so each atom's energy is -C6 f^2 f_LR(r)^2 / (2 r^6)
    with f_LR cut at r_MBD,1 (Sec. III.A), whatever r_MBD,2 is."""
    r1, rb = 4.0, 0.5
    for r_A, r2 in ((3.55, 2.5), (3.7, 4.0), (3.93, 1.0)):
        st = _open([[0, 0, 0], _at_distance(r_A)], species=[C_IDX, SPECIES_INDEX["N"]], nu=[0.8, 0.95])
        e = oracle.lmbd_energies(st, _radii_params(NO_SCS, 4.5, r1, r2, n_max=2), SPECIES_TABLE)
        a, w, R = _free(st)
        r = r_A / cf.BOHR
        f = cf.fermi(r, 0.83 * (R[0] + R[1]))
        flr = cf.smooth_cutoff(r_A, r1, rb)
        assert 0.0 < flr < 1.0
        ref = -0.5 * cf.c6_casimir_polder(a[0], w[0], a[1], w[1]) * (f * flr) ** 2 / r ** 6 * cf.HARTREE
        assert np.allclose(e, [ref, ref], rtol=1e-11, atol=0)


def test_two_radius_trimer_third_order_shares():
    """SCS off, a triangle with r_MBD,1 above every edge plus the buffer, edge a-b inside
    the f_LR buffer of r_MBD,2 and the other edges below it.  In the frames of a and b
    the a-b pair touches the central atom (p = 1, no cut); in the frame of c it does
    not (p = 2, Sec. III.A).  Each atom's third-order term is one third of the ATM
    energy, times f_LR(r_ab; r_MBD,2) for c only."""
    pos = np.array([[0.0, 0.0, 0.0], [3.62, 0.0, 0.0], [1.6, 2.4, 0.5]])
    r1, r2, rb = 5.0, 4.0, 0.5
    st = _open(pos, species=[C_IDX, SPECIES_INDEX["O"], SPECIES_INDEX["H"]], nu=[0.85, 0.7, 0.9])
    e2 = oracle.lmbd_energies(st, _radii_params(NO_SCS, 5.0, r1, r2, n_max=2), SPECIES_TABLE)
    e3 = oracle.lmbd_energies(st, _radii_params(NO_SCS, 5.0, r1, r2, n_max=3), SPECIES_TABLE)
    a, w, R = _free(st)
    x = pos / cf.BOHR
    f = 1.0
    for i, j in ((0, 1), (1, 2), (2, 0)):
        f *= cf.fermi(np.linalg.norm(x[i] - x[j]), 0.83 * (R[i] + R[j]))
    atm = cf.c9_atm(a[0], w[0], a[1], w[1], a[2], w[2]) * f * cf.atm_geometry_factor(*x) * cf.HARTREE
    phi = cf.smooth_cutoff(np.linalg.norm(pos[1] - pos[0]), r2, rb)
    assert 0.05 < phi < 0.95
    assert np.linalg.norm(pos[2] - pos[0]) < r2 - rb and np.linalg.norm(pos[2] - pos[1]) < r2 - rb
    assert np.allclose(e3 - e2, np.array([1.0, 1.0, phi]) * atm / 3.0, rtol=1e-10, atol=0)


def test_scs_dimer_inside_the_short_range_buffer():
    """Two atoms inside the f_SR buffer of r_SCS: the independent solve with the tensor
    scaled by the C1 cubic switch reproduces the oracle's local SCS (Sec. III.B f_SR)."""
    rs, rb = 3.0, 0.5
    for r_A in (2.62, 2.86):
        st = _open([[0, 0, 0], _at_distance(r_A)], species=[C_IDX, SPECIES_INDEX["N"]], nu=[0.8, 0.95])
        prm = _params(rs, rs)
        got = oracle.scs_central(st, prm, SPECIES_TABLE)
        a0, w0, R = _free(st)
        x = st.pos / cf.BOHR
        for q, w in enumerate(np.concatenate([[0.0], prm.omega])):
            ab = a0 / (1.0 + (w / w0) ** 2)
            ref = _solve_scs_fd(x, ab, R, rc=rs / cf.BOHR, rb=rb / cf.BOHR)
            assert np.allclose(got[:, q], ref, rtol=1e-8)
            if q == 0:   # the buffer matters here (at high frequency the screening fades)
                unbuffered = _solve_scs_fd(x, ab, R, rc=rs / cf.BOHR)
                assert np.all(np.abs(unbuffered / ref - 1.0) > 1e-4)


# ------------------------------------------------------------------ limits (P5)

def test_full_cutoff_lmbd_is_full_mbd_series_and_log():
    s, _ = C.config_small_open()
    sub = Structure(s.pos[:24], s.species[:24], s.nu[:24], None, np.zeros(3, bool))
    big = 22.0
    for n_max in (6, None):
        prm = _params(big, big, n_max=n_max)
        e = oracle.lmbd_energies(sub, prm, SPECIES_TABLE)
        E, shares = oracle.full_mbd(sub.pos, sub.species, sub.nu, SPECIES_TABLE, prm.omega, prm.weight,
                                    n_max=n_max)
        assert abs(e.sum() / E - 1) < 1e-12
        assert np.allclose(e, shares, rtol=1e-10, atol=1e-14)


def test_blend_uses_local_and_central_polarisabilities():
    """Three atoms in a row: the middle atom's polarisability in the first atom's
    frame is the f_SCS blend of the two-atom-plus-shell solve and its own three-atom
    solve (Sec. III.B, the range-separated combination)."""
    pos = np.array([[0.0, 0, 0], [2.4, 0, 0], [4.8, 0.3, 0]])
    st = _open(pos, nu=[0.8, 0.9, 0.7])
    rs = 3.0
    grid = frequency_grid(40)
    prm = _params(rs, 10.0, grid=grid, n_max=2)
    e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    a0, w0, R = _free(st)
    x = pos / cf.BOHR
    omegas = np.concatenate([[0.0], grid[0]])
    rin = 2.0 / cf.BOHR
    finner = lambda r: 3 * (r / rin) ** 2 - 2 * (r / rin) ** 3 if r < rin else 1.0
    alpha = np.zeros((len(omegas), 3))
    for q, w in enumerate(omegas):
        ab = a0 / (1.0 + (w / w0) ** 2)
        rc = rs / cf.BOHR
        loc0 = _solve_scs_fd(x[:2], ab[:2], R[:2], fixed=[(x[2], ab[2], R[2])], finner=finner, rc=rc)
        cen1 = _solve_scs_fd(x, ab, R, rc=rc)[1]
        cen2 = _solve_scs_fd(x[1:], ab[1:], R[1:], fixed=[(x[0], ab[0], R[0])], finner=finner,
                             rc=rc)[1]
        fs = 3 * (2.4 / rs) ** 2 - 2 * (2.4 / rs) ** 3
        alpha[q] = [loc0[0], (1 - fs) * loc0[1] + fs * cen1, cen2]
    atom0 = st.species[0]
    r0 = SPECIES_TABLE[st.species, 2]
    Rt = r0 * (alpha[0] / SPECIES_TABLE[st.species, 0]) ** (1.0 / 3.0)
    ref = 0.0
    for j in (1, 2):
        rv = x[0] - x[j]
        r = np.linalg.norm(rv)
        f = cf.fermi(r, 0.83 * (Rt[0] + Rt[j]))
        T = cf.numerical_hessian(cf.coulomb, rv, h=1e-2 * r) * f
        tr = np.trace(T @ T)
        ref += -0.5 * np.sum(grid[1] * alpha[1:, 0] * alpha[1:, j]) * tr / (2 * math.pi)
    assert abs(e[0] / (ref * cf.HARTREE) - 1) < 2e-7


# ---------------------------------------------------------- invariances (P9, P12)

def test_rotation_translation_permutation_invariance():
    st = _rand_cluster(14, 41)
    prm = _params(3.5, 4.5)
    e0, f0 = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    perm = rng.permutation(st.n)
    st2 = Structure(st.pos[perm] @ Q.T + np.array([1.3, -7.2, 0.4]), st.species[perm], st.nu[perm],
                    None, np.zeros(3, bool))
    e1, f1 = oracle.lmbd_energy_forces(st2, prm, SPECIES_TABLE)
    assert np.allclose(e1, e0[perm], rtol=1e-10, atol=1e-14)
    assert np.allclose(f1, f0[perm] @ Q.T, rtol=1e-8, atol=1e-11)


def test_lattice_shift_and_supercell_invariance():
    st = C.carbon_box(24, 7, g_cm3=1.2, dmin=1.4)
    prm = _params(3.5, 3.5)
    e0 = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    shifted = st.copy()
    shifted.pos[3] += st.cell[1] - 2 * st.cell[2]
    e1 = oracle.lmbd_energies(shifted, prm, SPECIES_TABLE)
    assert np.allclose(e1, e0, rtol=1e-11, atol=1e-15)
    reps = [st.pos + np.array([a, b, c]) @ st.cell for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    sup = Structure(np.concatenate(reps), np.tile(st.species, 8), np.tile(st.nu, 8), 2 * st.cell,
                    np.ones(3, bool))
    e2 = oracle.lmbd_energies(sup, prm, SPECIES_TABLE, atoms=list(range(st.n)))
    assert np.allclose(e2[:st.n], e0, rtol=1e-11, atol=1e-15)


def test_size_consistency_of_distant_fragments():
    a = _rand_cluster(6, 51, box=4.0)
    b = _rand_cluster(5, 52, box=4.0)
    prm = _params(3.0, 4.0)
    far = np.array([30.0, 0, 0])
    ab = Structure(np.concatenate([a.pos, b.pos + far]), np.concatenate([a.species, b.species]),
                   np.concatenate([a.nu, b.nu]), None, np.zeros(3, bool))
    e = oracle.lmbd_energies(ab, prm, SPECIES_TABLE)
    ea = oracle.lmbd_energies(a, prm, SPECIES_TABLE)
    eb = oracle.lmbd_energies(b, prm, SPECIES_TABLE)
    assert np.allclose(e, np.concatenate([ea, eb]), rtol=1e-12, atol=1e-16)


# ----------------------------------------------------------------- forces (P10)

def _lists_equal(st, prm, pos2):
    r_big = max(2 * prm.r_scs, prm.r_nbr)
    s2 = st.copy()
    s2.pos = pos2
    for k in range(st.n):
        b1, s1, d1 = oracle.neighbourhood(st.pos, st.cell, st.pbc, k, r_big)
        b2, sh2, d2 = oracle.neighbourhood(pos2, st.cell, st.pbc, k, r_big)
        if len(b1) != len(b2):
            return False
        for rc in (prm.r_scs, prm.r_nbr):
            if np.sum(d1 < rc) != np.sum(d2 < rc):
                return False
    return True


def _fd_check(st, prm, comps, h=1e-4, tol=2e-6):
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    assert np.allclose(f.sum(0), 0.0, atol=1e-10 * max(1.0, np.abs(f).max()))
    checked = 0
    for (a, g) in comps:
        pp, pm = st.pos.copy(), st.pos.copy()
        pp[a, g] += h
        pm[a, g] -= h
        if not (_lists_equal(st, prm, pp) and _lists_equal(st, prm, pm)):
            continue  # a neighbour set changes inside the stencil: skip this draw
        sp_, sm_ = st.copy(), st.copy()
        sp_.pos, sm_.pos = pp, pm
        ep = oracle.lmbd_energies(sp_, prm, SPECIES_TABLE).sum()
        em = oracle.lmbd_energies(sm_, prm, SPECIES_TABLE).sum()
        fd = -(ep - em) / (2 * h)
        assert abs(fd - f[a, g]) < tol * max(1.0, abs(f[a, g])) + 1e-8, (a, g, fd, f[a, g])
        checked += 1
    assert checked >= len(comps) // 2


def test_forces_finite_difference_open_cluster():
    st = _rand_cluster(12, 61, box=5.5, dmin=1.4)
    prm = _params(3.0, 4.0)
    _fd_check(st, prm, [(0, 0), (3, 1), (7, 2), (11, 0)])


def test_forces_with_an_isolated_atom():
    """An atom with no neighbour inside the cutoffs has zero energy and zero
    force, and its presence changes nothing for the others (its central
    polarisability enters no energy, so its adjoint is zero, not missing)."""
    a = _rand_cluster(6, 71, box=4.0)
    prm = _params(3.0, 4.0)
    far = np.array([[25.0, 0.0, 0.0]])
    st = Structure(np.concatenate([a.pos, far]), np.concatenate([a.species, a.species[:1]]),
                   np.concatenate([a.nu, a.nu[:1]]), None, np.zeros(3, bool))
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    ea, fa = oracle.lmbd_energy_forces(a, prm, SPECIES_TABLE)
    assert e[-1] == 0.0 and np.all(f[-1] == 0.0)
    assert np.allclose(e[:-1], ea, rtol=1e-12, atol=1e-16)
    assert np.allclose(f[:-1], fa, rtol=1e-10, atol=1e-14)
    assert np.allclose(f.sum(0), 0.0, atol=1e-12)
    lone = Structure(far.copy(), a.species[:1], a.nu[:1], None, np.zeros(3, bool))
    e1, f1 = oracle.lmbd_energy_forces(lone, prm, SPECIES_TABLE)
    assert e1[0] == 0.0 and np.all(f1 == 0.0)


@pytest.mark.slow
def test_forces_finite_difference_periodic_box():
    st = C.hcno_box(20, 9, g_cm3=1.0)
    prm = _params(3.2, 3.5)
    _fd_check(st, prm, [(1, 0), (5, 2), (13, 1)])


# ------------------------------------------------ volume-ratio derivatives

def test_volume_ratio_derivative_of_the_pairwise_dimer():
    """SCS off, n_max = 2: E_a + E_b = -C6 f^2 / r^6 with C6 proportional to nu_a nu_b
    and S = beta (R0_a nu_a^(1/3) + R0_b nu_b^(1/3)) (the screened radii reduce to the
    TS ones); its nu-derivative in closed form."""
    st = _open([[0, 0, 0], _at_distance(2.9)], species=[C_IDX, SPECIES_INDEX["O"]], nu=[0.8, 0.9])
    prm = _params(NO_SCS, 8.0, grid=GRID200, n_max=2)
    w = np.array([0.7, 1.3])
    e, f, dv = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=w, want_dv=True)
    a, om, R = _free(st)
    r = 2.9 / cf.BOHR
    S = 0.83 * (R[0] + R[1])
    fe = cf.fermi(r, S)
    c6 = cf.c6_casimir_polder(a[0], om[0], a[1], om[1])
    share = -0.5 * c6 * fe * fe / r ** 6 * cf.HARTREE    # each atom's energy
    assert np.allclose(e, [share, share], rtol=1e-11)
    dfdS = -6.0 * r * fe * (1 - fe) / S ** 2
    for b in range(2):
        dS = 0.83 * R[b] / (3.0 * st.nu[b])
        d_share = share * (1.0 / st.nu[b] + 2.0 * dfdS * dS / fe)
        assert abs(dv[b] / (w.sum() * d_share) - 1.0) < 1e-10


def test_volume_ratio_derivative_finite_difference():
    """Screened H/C/N/O cluster (shell, inner buffer and blend active): d(sum_k w_k
    E_k)/d nu against central differences of the energies."""
    st = _rand_cluster(12, 91, box=5.5, dmin=1.4)
    prm = _params(3.0, 4.0)
    rng = np.random.default_rng(92)
    w = rng.uniform(0.5, 1.5, st.n)
    e, f, dv = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=w, want_dv=True)
    e2, f2 = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=w)
    assert np.allclose(e, e2, rtol=1e-13, atol=0) and np.allclose(f, f2, rtol=1e-11, atol=1e-15)
    h = 1e-5
    for b in (0, 4, 9):
        sp_, sm_ = st.copy(), st.copy()
        sp_.nu = st.nu.copy()
        sm_.nu = st.nu.copy()
        sp_.nu[b] += h
        sm_.nu[b] -= h
        fd = (w @ oracle.lmbd_energies(sp_, prm, SPECIES_TABLE) - w @ oracle.lmbd_energies(sm_, prm, SPECIES_TABLE)) / (2 * h)
        assert abs(fd - dv[b]) < 1e-7 * max(1.0, abs(dv[b])), (b, fd, dv[b])


# ------------------------------------------- the paper's approximate forces

def test_paper_forces_are_exact_without_screening_and_with_full_cutoffs():
    """SCS off and every frame covering the whole cluster: no polarisability moves
    and T_LR,ij with i, j != k does not depend on r_k, so the central-atom
    approximation is exact and E^tot_k is the total energy: the paper's force on
    k (Sec. III.D) is minus the gradient of sum_j E_j, checked against central
    differences of the total energy and against the exact adjoint."""
    st = _rand_cluster(7, 101, box=5.0, dmin=1.5)
    prm = _params(NO_SCS, 30.0, n_max=6)
    e, f = oracle.lmbd_paper_forces(st, prm, SPECIES_TABLE)
    e_ex, f_ex = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    assert np.allclose(e, e_ex, rtol=1e-13, atol=0)
    assert np.allclose(f, f_ex, rtol=1e-9, atol=1e-13)
    h = 1e-4
    for a, g in ((0, 0), (3, 1), (6, 2)):
        sp_, sm_ = st.copy(), st.copy()
        sp_.pos[a, g] += h
        sm_.pos[a, g] -= h
        fd = -(oracle.lmbd_energies(sp_, prm, SPECIES_TABLE).sum()
               - oracle.lmbd_energies(sm_, prm, SPECIES_TABLE).sum()) / (2 * h)
        assert abs(fd - f[a, g]) < 1e-7 * max(1.0, abs(fd)), (a, g, fd, f[a, g])


def test_paper_forces_are_an_approximation_with_screening():
    """With local SCS the central polarisabilities are held fixed and, for n >= 3, only
    the central atom's row and column of dG~ are kept: the result is close to, but
    not, the exact force, and it is not momentum-conserving."""
    st = _rand_cluster(12, 61, box=5.5, dmin=1.4)
    prm = _params(3.0, 4.0)
    e, f = oracle.lmbd_paper_forces(st, prm, SPECIES_TABLE)
    e_ex, f_ex = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    assert np.array_equal(e, oracle.lmbd_energies(st, prm, SPECIES_TABLE))
    d = np.abs(f - f_ex).max()
    assert 1e-7 < d < 0.5 * np.abs(f_ex).max()
    assert np.abs(f.sum(0)).max() > 1e-9


# ------------------------------------------- two-point Lorentzian SCS model

OMEGA_REF = 0.5


def test_lorentz_model_is_exact_for_unscreened_atoms():
    """Without SCS coupling every polarisability is the TS Lorentzian, whose
    characteristic frequency the two-point model recovers exactly (Sec. III.C,
    Eqs. alpha_SCS_freq and char-freq), for any reference frequency."""
    st = _rand_cluster(10, 81, box=6.0, dmin=1.5)
    e0, f0 = oracle.lmbd_energy_forces(st, _params(NO_SCS, 4.0), SPECIES_TABLE)
    for om_ref in (0.3, 1.7):
        e, f = oracle.lmbd_energy_forces(st, _params(NO_SCS, 4.0, scs_freq="lorentz", omega_ref=om_ref),
                                         SPECIES_TABLE)
        assert np.allclose(e, e0, rtol=1e-12, atol=0)
        assert np.allclose(f, f0, rtol=1e-10, atol=1e-14)


def test_lorentz_model_interpolates_the_exact_solves():
    """A quadrature with the single node omega_ref: the model takes the solved
    alpha~(0) and alpha~(omega_ref) unchanged, so it equals the exact frequency
    treatment, energies and forces (screened cluster, blend active)."""
    st = _rand_cluster(12, 83, box=5.5, dmin=1.4)
    grid = (np.array([OMEGA_REF]), np.array([0.9]))
    e0, f0 = oracle.lmbd_energy_forces(st, _params(3.0, 4.0, grid=grid), SPECIES_TABLE)
    e, f = oracle.lmbd_energy_forces(st, _params(3.0, 4.0, grid=grid, scs_freq="lorentz",
                                                 omega_ref=OMEGA_REF), SPECIES_TABLE)
    assert np.all(e0 != 0.0)
    assert np.allclose(e, e0, rtol=1e-12, atol=0)
    assert np.allclose(f, f0, rtol=1e-10, atol=1e-14)


def test_lorentz_model_second_order_is_casimir_polder_of_screened_lorentzians():
    """Screened dimer, n_max = 2: each atom's energy is -C6 f^2 / (2 r^6) with C6
    the Casimir-Polder integral of the two model Lorentzians, whose static values
    and characteristic frequencies come from independent SCS solves at 0 and
    omega_ref (Eq. char-freq) and whose damping uses the screened radii."""
    st = _open([[0, 0, 0], [1.6, 1.1, 0.5]], species=[C_IDX, SPECIES_INDEX["N"]], nu=[0.8, 0.95])
    prm = _params(5.0, 8.0, grid=GRID200, n_max=2, scs_freq="lorentz", omega_ref=OMEGA_REF)
    e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    a0, w0, R = _free(st)
    x = st.pos / cf.BOHR
    s0 = _solve_scs_fd(x, a0, R)
    sr = _solve_scs_fd(x, a0 / (1.0 + (OMEGA_REF / w0) ** 2), R)
    assert np.all(s0 > sr)
    wt = OMEGA_REF / np.sqrt(s0 / sr - 1.0)
    Rt = SPECIES_TABLE[st.species, 2] * (s0 / SPECIES_TABLE[st.species, 0]) ** (1.0 / 3.0)
    r = np.linalg.norm(x[0] - x[1])
    c6 = cf.c6_casimir_polder(s0[0], wt[0], s0[1], wt[1])
    ref = -0.5 * c6 * cf.fermi(r, 0.83 * (Rt[0] + Rt[1])) ** 2 / r ** 6 * cf.HARTREE
    assert np.allclose(e, [ref, ref], rtol=1e-10, atol=0)
    # the exact frequency treatment differs: the screened dimer is not one Lorentzian
    ex = oracle.lmbd_energies(st, _params(5.0, 8.0, grid=GRID200, n_max=2), SPECIES_TABLE)
    assert abs(ex[0] / e[0] - 1.0) > 1e-6


def test_lorentz_model_rejects_rising_polarisability():
    """A real characteristic frequency needs alpha~(0) >= alpha~(omega_ref) > 0."""
    import torch
    a0 = torch.tensor([10.0, 5.0], dtype=torch.float64)
    with pytest.raises(ValueError):
        L.lorentz_polarisabilities(a0, torch.tensor([9.0, 6.0], dtype=torch.float64), [0.1], 0.5)
    with pytest.raises(ValueError):
        L.lorentz_polarisabilities(a0, torch.tensor([9.0, -1.0], dtype=torch.float64), [0.1], 0.5)


def test_lorentz_model_forces_finite_difference():
    st = _rand_cluster(12, 61, box=5.5, dmin=1.4)
    prm = _params(3.0, 4.0, scs_freq="lorentz", omega_ref=OMEGA_REF)
    _fd_check(st, prm, [(0, 0), (3, 1), (7, 2), (11, 0)])


# ------------------------------------------------------------------ neighbours

def test_neighbourhood_matches_brute_force_images():
    st = C.carbon_box(10, 3, g_cm3=1.0, dmin=1.2)   # L ~ 5.8 A, so many images are in reach
    rmax = 7.3
    for k in (0, 4, 9):
        base, sh, d = oracle.neighbourhood(st.pos, st.cell, st.pbc, k, rmax)
        ref = set()
        for a in range(-4, 5):
            for b in range(-4, 5):
                for c in range(-4, 5):
                    for j in range(st.n):
                        v = st.pos[j] + np.array([a, b, c]) @ st.cell - st.pos[k]
                        if np.linalg.norm(v) < rmax:
                            ref.add((j, a, b, c))
        got = {(int(j), *map(int, s)) for j, s in zip(base, sh)}
        assert got == ref
        assert base[0] == k and np.all(sh[0] == 0) and np.all(np.diff(d[1:]) >= 0)


# ------------------------- eigenvalue-bounded polynomial fit of ln(1 - x)

def test_splitmix64_reproduces_its_published_outputs():
    """The start vector's generator: the first five outputs of SplitMix64 seeded with
    1234567 as published with the generator."""
    g, m = 0x9E3779B97F4A7C15, (1 << 64) - 1
    out = [L._splitmix64((1234567 + i * g) & m) for i in range(5)]
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
                   16408922859458223821]
    v = L.lanczos_start(3, [3, 5, 5], [[0, 0, 0], [0, 0, 0], [1, -1, 0]])
    assert np.all(np.abs(v) <= 0.5) and len(set(np.round(v, 15))) == 9   # images keyed apart
    w = L.lanczos_start(3, [5, 3], [[1, -1, 0], [0, 0, 0]])
    assert np.array_equal(w[:3], v[6:]) and np.array_equal(w[3:], v[:3])   # keyed on identity


def test_log_fit_is_the_discretised_continuous_projection():
    """The fit reproduces a polynomial of degree <= n_max exactly and equals the
    continuous least-squares polynomial (Legendre projection by adaptive
    quadrature) up to the discretisation of the 32-node rule."""
    cub = lambda x: 0.3 - 1.2 * x + 0.5 * x ** 2 - 2.0 * x ** 3
    c = L.log_fit_coefficients(-0.7, 0.45, 6, f=cub)
    assert np.allclose(c, [0.3, -1.2, 0.5, -2.0, 0.0, 0.0, 0.0], atol=1e-12)
    lam = np.linspace(-0.7, 0.45, 301)
    for (a, b, n) in ((-0.7, 0.45, 6), (-0.2, 0.05, 4), (-0.9, 0.8, 10)):
        c = L.log_fit_coefficients(a, b, n)
        ref = cf.l2_projection_poly(lambda x: np.log1p(-x), a, b, n)
        lam = np.linspace(a, b, 301)
        assert np.abs(np.polyval(c[::-1], lam) - ref(lam)).max() < 1e-11, (a, b, n)
        # a fit, not an interpolant: the residual alternates and is small against the series
        series = -sum(lam ** k / k for k in range(1, n + 1))
        assert np.abs(np.polyval(c[::-1], lam) - np.log1p(-lam)).max() < np.abs(series - np.log1p(-lam)).max()
    # an interval of no width (no coupling): the Taylor coefficients
    assert np.allclose(L.log_fit_coefficients(0.0, 0.0, 4), [0.0, -1.0, -0.5, -1 / 3, -0.25])
    with pytest.raises(L.PolarisationCatastrophe):
        L.log_fit_coefficients(-0.5, 1.0, 6)


def test_lanczos_bounds_reach_the_extreme_eigenvalues():
    """Ritz extremes lie inside the spectrum, move outwards with the step count and
    reach the exact extremes once the Krylov space is the whole space; an invariant
    subspace stops the iteration with exact values."""
    rng = np.random.default_rng(3)
    lam = np.sort(rng.uniform(-0.8, 0.6, 40))
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    G = Q @ np.diag(lam) @ Q.T
    v1 = rng.uniform(-0.5, 0.5, 40)
    prev = (np.inf, -np.inf)
    for m in (3, 6, 10, 20):
        lo, hi = L.lanczos_bounds(G, v1, m)
        assert lam[0] - 1e-12 <= lo <= prev[0] + 1e-12 and prev[1] - 1e-12 <= hi <= lam[-1] + 1e-12
        prev = (lo, hi)
    lo, hi = L.lanczos_bounds(G, v1, 40)
    assert abs(lo - lam[0]) < 1e-10 and abs(hi - lam[-1]) < 1e-10
    # four distinct eigenvalues (a dimer's spectrum): stops after four steps, exact
    D = np.diag([0.7, -0.7, 0.3, 0.3, -0.3, -0.3])
    Q6, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    lo, hi = L.lanczos_bounds(Q6 @ D @ Q6.T, rng.uniform(-0.5, 0.5, 6), 20)
    assert abs(lo + 0.7) < 1e-13 and abs(hi - 0.7) < 1e-13


def _fit_params(r_scs, r_nbr, n_max, grid=GRID12, steps=20, **kw):
    prm = _params(r_scs, r_nbr, grid=grid, n_max=n_max, **kw)
    prm.c_n_mode = "fit"
    prm.lanczos_steps = steps
    return prm


def test_fitted_dimer_energy_closed_form():
    """Dimer without screening: G~ has the eigenvalues +-t_a per axis (t_z = 2 x,
    t_x = t_y = -x, x = sqrt(alpha_1 alpha_2) f / r^3), so the bounds are +-2x and
    sum_{n>=2} c_n Tr[G~^n]_kk = sum_axes [(p(t_a) + p(-t_a)) / 2 - p(0)] with p the
    least-squares polynomial of ln(1 - x) on [-2x, 2x], here from adaptive quadrature."""
    st = _open([[0, 0, 0], [1.7, 0.9, -0.4]], species=[C_IDX, SPECIES_INDEX["N"]], nu=[0.8, 0.95])
    prm = _fit_params(NO_SCS, 30.0, 6, grid=GRID12)
    e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    b = oracle.lmbd_spectrum_bounds(st, prm, SPECIES_TABLE)
    a, w, t = _dimer_couplings(st)
    om, wq = GRID12
    ref = 0.0
    for q in range(len(om)):
        ai = a / (1.0 + (om[q] / w) ** 2)
        x = math.sqrt(ai[0] * ai[1])
        ts = [x * ti for ti in t]
        lo, hi = -2.0 * abs(ts[1]), 2.0 * abs(ts[1])
        assert abs(b[0, q, 0] - lo) < 1e-13 and abs(b[0, q, 1] - hi) < 1e-13
        p = cf.l2_projection_poly(lambda y: np.log1p(-y), lo, hi, 6)
        ref += wq[q] * sum(0.5 * (p(ta) + p(-ta)) - p(0.0) for ta in ts)
    ref *= cf.HARTREE / (2.0 * math.pi)
    assert abs(e[0] / ref - 1.0) < 1e-9 and abs(e[1] / ref - 1.0) < 1e-9


def test_fitted_energy_is_the_polynomial_of_the_eigendecomposition():
    """Eq. eigendecomp: sum_{n>=2} c_n Tr[G~^n]_kk equals the central 3x3 block's trace
    of V p(Lambda) V^T, less c_0 times 3 (the n = 0 term; the n = 1 term is zero)."""
    import torch
    st = _rand_cluster(9, 17, box=5.0, dmin=1.5)
    prm = _fit_params(3.0, 4.5, 5)
    stp, fa, images = L._prepare(st, prm, SPECIES_TABLE)
    central = oracle.scs_central(st, prm, SPECIES_TABLE)
    pos_t = torch.as_tensor(st.pos, dtype=torch.float64)
    e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    for k in (0, 4, 8):
        fr = L._Frame(stp, k, prm, images)
        p = fr.positions(pos_t, None)
        with torch.no_grad():
            aloc = L._scs_solve(fr, p, fa, prm)
            acen = torch.as_tensor(central[fr.base[:fr.nK]], dtype=torch.float64)
            A, T = L._mbd_operators(fr, p, aloc, acen, fa, prm)
        coef = L.fitted_coefficients(fr, p, aloc, acen, fa, prm)
        tot = 0.0
        for q in range(len(prm.omega)):
            s = np.sqrt(A[:, q + 1].numpy()).repeat(3)
            G = s[:, None] * T.numpy() * s[None, :]
            lam, V = np.linalg.eigh(G)
            pl = np.polyval(coef[q][::-1], lam)
            tot += prm.weight[q] * ((V[:3, :] ** 2).sum(0) @ pl - 3.0 * coef[q][0])
        assert abs(tot * cf.HARTREE / (2.0 * math.pi) / e[k] - 1.0) < 1e-11


def test_fit_converges_faster_than_the_series():
    """Fig. convergence: at the same body order the fitted polynomial is much closer
    to the block logarithm than the truncated series, and it converges with n_max."""
    st = _rand_cluster(14, 5, box=6.0, dmin=1.5, hcno=False)
    e_log = oracle.lmbd_energies(st, _params(3.5, 5.0, n_max=None), SPECIES_TABLE)
    errs = []
    for n in (4, 6, 8):
        e_s = oracle.lmbd_energies(st, _params(3.5, 5.0, n_max=n), SPECIES_TABLE)
        e_f = oracle.lmbd_energies(st, _fit_params(3.5, 5.0, n, steps=None), SPECIES_TABLE)
        es, ef = np.abs(e_s - e_log).max(), np.abs(e_f - e_log).max()
        assert ef < 0.2 * es, (n, ef, es)
        errs.append(ef)
    assert errs[2] < errs[1] < errs[0]


def test_fit_forces_hold_the_coefficients_fixed():
    """The forces treat the fitted c_n as constants: they are the central differences
    of the energy evaluated with the coefficients of the unperturbed geometry."""
    st = _rand_cluster(8, 23, box=5.0, dmin=1.5)
    prm = _fit_params(3.0, 4.0, 6, steps=12)
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    import torch
    stp, fa, images = L._prepare(st, prm, SPECIES_TABLE)
    central = oracle.scs_central(st, prm, SPECIES_TABLE)
    pos_t = torch.as_tensor(st.pos, dtype=torch.float64)
    fixed = {}
    for k in range(st.n):
        fr = L._Frame(stp, k, prm, images)
        p = fr.positions(pos_t, None)
        with torch.no_grad():
            aloc = L._scs_solve(fr, p, fa, prm)
        acen = torch.as_tensor(central[fr.base[:fr.nK]], dtype=torch.float64)
        fixed[k] = L.fitted_coefficients(fr, p, aloc, acen, fa, prm)
    pf = _fit_params(3.0, 4.0, 6, steps=12)
    pf.coef_fixed = fixed
    assert np.allclose(oracle.lmbd_energies(st, pf, SPECIES_TABLE), e, rtol=0, atol=1e-14)
    h = 1e-4
    for (a, g) in ((0, 0), (3, 1), (6, 2)):
        sp_, sm_ = st.copy(), st.copy()
        sp_.pos = st.pos.copy()
        sm_.pos = st.pos.copy()
        sp_.pos[a, g] += h
        sm_.pos[a, g] -= h
        if not (_lists_equal(st, prm, sp_.pos) and _lists_equal(st, prm, sm_.pos)):
            continue
        fd = -(oracle.lmbd_energies(sp_, pf, SPECIES_TABLE).sum() - oracle.lmbd_energies(sm_, pf, SPECIES_TABLE).sum()) / (2 * h)
        assert abs(fd - f[a, g]) < 2e-6 * max(1.0, abs(f[a, g])), (a, g, fd, f[a, g])
    # refitting at every geometry moves the energy by the coefficients' own change:
    # not the gradient of the refitted energy (the paper's forces neglect that term)
    sp_ = st.copy()
    sp_.pos = st.pos.copy()
    sp_.pos[0, 0] += 1e-3
    assert not np.allclose(oracle.lmbd_energies(sp_, pf, SPECIES_TABLE), oracle.lmbd_energies(sp_, prm, SPECIES_TABLE),
                           rtol=0, atol=1e-15)


def test_polarisation_catastrophe_is_detected():
    """Strongly polarisable atoms at short range: the largest eigenvalue of G~ passes
    1, ln(1 - x) has no fit there, and the fit mode refuses with an error (the
    series mode computes a number, the spectrum bounds show the catastrophe)."""
    tab = np.array(SPECIES_TABLE, copy=True)
    tab[C_IDX] = [600.0, 2000.0, 4.0]
    st = _open([[0, 0, 0], [3.0, 0.2, 0.1], [1.2, 2.7, 0.4]])
    prm = _fit_params(NO_SCS, 10.0, 6, steps=20)
    b = oracle.lmbd_spectrum_bounds(st, prm, tab)
    assert b[:, 0, 1].max() >= 1.0
    with pytest.raises(oracle.PolarisationCatastrophe):
        oracle.lmbd_energies(st, prm, tab)
    assert np.all(np.isfinite(oracle.lmbd_energies(st, _params(NO_SCS, 10.0, n_max=6), tab)))


# ------------------------------------------------------------- separate two-body radii

def test_two_body_radii_dimer():
    """SCS off, a dimer beyond r_MBD,1 but inside the f_LR buffer of the two-body radius
    r_2b,1 (Sec. III.A): the MBD T_LR has no coupling, so every term n >= 3 is zero,
    while the n = 2 term is the pairwise -C6 f^2 f_LR(r; r_2b,1)^2 / (2 r^6) for any
    n_max; with r_2b,1 = r_MBD,1 the dimer has no energy at all."""
    rb = 0.5
    for r_A in (4.62, 4.8):
        st = _open([[0, 0, 0], _at_distance(r_A)], species=[C_IDX, SPECIES_INDEX["N"]], nu=[0.8, 0.95])
        cut = dict(r_scs=NO_SCS, r_nbr=5.5, r_mbd1=3.0, r_mbd2=3.0, r_2b1=5.0, r_2b2=2.0)
        a, w, R = _free(st)
        r = r_A / cf.BOHR
        f = cf.fermi(r, 0.83 * (R[0] + R[1]))
        flr = cf.smooth_cutoff(r_A, 5.0, rb)
        assert 0.0 < flr < 1.0
        ref = -0.5 * cf.c6_casimir_polder(a[0], w[0], a[1], w[1]) * (f * flr) ** 2 / r ** 6 * cf.HARTREE
        for n_max in (2, 6):
            e = oracle.lmbd_energies(st, oracle.make_params(cut, GRID200[0], GRID200[1], n_max=n_max),
                                     SPECIES_TABLE)
            assert np.allclose(e, [ref, ref], rtol=1e-11, atol=0), (r_A, n_max)
        same = dict(cut, r_2b1=3.0, r_2b2=3.0)
        e0 = oracle.lmbd_energies(st, oracle.make_params(same, GRID200[0], GRID200[1], n_max=6), SPECIES_TABLE)
        assert np.all(e0 == 0.0)


def test_two_body_radii_trimer_splits_the_orders():
    """SCS off, a triangle: with separate two-body radii the second-order energy is the
    pairwise sum with f_LR at r_2b,1 on the pairs touching each central atom, and the
    third-order share is still one third of the ATM energy with the MBD radii's
    factors (edge a-b in the buffer of r_MBD,2, so c's share carries it)."""
    pos = np.array([[0.0, 0.0, 0.0], [3.62, 0.0, 0.0], [1.6, 2.4, 0.5]])
    r1, r2, rb = 5.0, 4.0, 0.5
    st = _open(pos, species=[C_IDX, SPECIES_INDEX["O"], SPECIES_INDEX["H"]], nu=[0.85, 0.7, 0.9])
    # r_2b,1 = 4 A: the a-b edge (3.62 A) inside its buffer, the other edges below it
    cut = dict(r_scs=NO_SCS, r_nbr=5.0, r_mbd1=r1, r_mbd2=r2, r_2b1=4.0, r_2b2=1.0)
    p2 = oracle.make_params(cut, GRID200[0], GRID200[1], n_max=2)
    p3 = oracle.make_params(cut, GRID200[0], GRID200[1], n_max=3)
    e2 = oracle.lmbd_energies(st, p2, SPECIES_TABLE)
    e3 = oracle.lmbd_energies(st, p3, SPECIES_TABLE)
    a, w, R = _free(st)
    x = pos / cf.BOHR
    pair = {}
    for i, j in ((0, 1), (1, 2), (2, 0)):
        r = np.linalg.norm(x[i] - x[j])
        c6 = cf.c6_casimir_polder(a[i], w[i], a[j], w[j])
        fl = cf.smooth_cutoff(np.linalg.norm(pos[i] - pos[j]), 4.0, rb)
        pair[(i, j)] = pair[(j, i)] = -0.5 * c6 * (cf.fermi(r, 0.83 * (R[i] + R[j])) * fl) ** 2 / r ** 6 * cf.HARTREE
    assert 0.05 < cf.smooth_cutoff(np.linalg.norm(pos[1] - pos[0]), 4.0, rb) < 0.95
    ref2 = [pair[(0, 1)] + pair[(0, 2)], pair[(1, 0)] + pair[(1, 2)], pair[(2, 0)] + pair[(2, 1)]]
    assert np.allclose(e2, ref2, rtol=1e-11, atol=0)
    f = 1.0
    for i, j in ((0, 1), (1, 2), (2, 0)):
        f *= cf.fermi(np.linalg.norm(x[i] - x[j]), 0.83 * (R[i] + R[j]))
    atm = cf.c9_atm(a[0], w[0], a[1], w[1], a[2], w[2]) * f * cf.atm_geometry_factor(*x) * cf.HARTREE
    phi = cf.smooth_cutoff(np.linalg.norm(pos[1] - pos[0]), r2, rb)
    assert np.allclose(e3 - e2, np.array([1.0, 1.0, phi]) * atm / 3.0, rtol=1e-10, atol=0)


def test_two_body_radii_forces_finite_difference():
    """Exact forces with separate two-body radii (a larger r_2b,1 than r_MBD,1) against
    central differences of the energy."""
    st = _rand_cluster(10, 71, box=5.5, dmin=1.4)
    cut = dict(r_scs=3.0, r_nbr=5.0, r_mbd1=3.5, r_mbd2=3.0, r_2b1=5.0, r_2b2=4.0)
    prm = oracle.make_params(cut, GRID12[0], GRID12[1], n_max=5)
    _fd_check(st, prm, [(0, 0), (4, 1), (9, 2)])


def test_two_body_radii_paper_forces_exact_limit():
    """The approximate forces with separate two-body radii: without screening and with
    every frame holding the whole structure they are the exact forces (the n = 2 term
    of the frame's total trace moves with r_k only through its central pairs, whatever
    r_2b,2 is)."""
    st = _rand_cluster(8, 19, box=4.5, dmin=1.3)
    cut = dict(r_scs=NO_SCS, r_nbr=12.0, r_mbd1=9.0, r_mbd2=8.5, r_2b1=12.0, r_2b2=2.5)
    prm = oracle.make_params(cut, GRID12[0], GRID12[1], n_max=5)
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    ep, fp = oracle.lmbd_paper_forces(st, prm, SPECIES_TABLE)
    assert np.allclose(ep, e, rtol=0, atol=1e-14)
    assert np.allclose(fp, f, rtol=0, atol=1e-12 * max(1.0, np.abs(f).max()))
