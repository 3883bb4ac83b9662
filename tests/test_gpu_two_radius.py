"""The two-radius MBD regime (Sec. III.A: K = B(r_MBD,1 + r_MBD,2); pairs that touch
the central atom couple up to r_MBD,1, all others up to r_MBD,2) with neighbourhoods
larger than the SCS spheres, against the oracle on sampled atoms.

216 C atoms in a periodic box at 2.0 g/cm^3 (L = 12.9 A, so K holds periodic images
of most atoms), r_SCS = 4 A, r_MBD,1 = 5 A, r_MBD,2 = 3.5 A: K has 258 sites on
average (up to 270).  Energies of three atoms and the forces of a weighted sum of
their energies; FP64 to 1e-8 eV/atom and 1e-8 eV/A, mixed to 1e-5 and 1e-4.
"""
import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from tests.gpu_common import gpu_run, oracle_params

pytestmark = pytest.mark.gpu

CUT = dict(r_scs=4.0, r_nbr=8.5, r_mbd1=5.0, r_mbd2=3.5)
ATOMS = [0, 77, 150]


@pytest.fixture(scope="module")
def case():
    st = C.carbon_box(216, 21, g_cm3=2.0)
    nk = max(len(oracle.neighbourhood(st.pos, st.cell, st.pbc, k, CUT["r_nbr"])[0]) for k in ATOMS)
    w = np.zeros(st.n)
    w[ATOMS] = [1.0, 0.5, -0.7]
    e, f = oracle.lmbd_energy_forces(st, oracle_params(CUT), SPECIES_TABLE, weights=w, atoms=ATOMS)
    return st, w, e[ATOMS], f, nk


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_radius_regime_matches_oracle(case, precision):
    st, w, e_ref, f_ref, nk = case
    print(f"case C216 two-radius {CUT} nK up to {nk}, {precision}", flush=True)
    assert nk > 160
    g = gpu_run(st, CUT, weights=w, precision=precision)
    de = np.abs(g["energies"][ATOMS] - e_ref).max()
    df = np.abs(g["forces"] - f_ref).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A (max |F| {np.abs(f_ref).max():.3e})", flush=True)
    e_tol, f_tol = (1e-8, 1e-8) if precision == "fp64" else (1e-5, 1e-4)
    assert de < e_tol and df < f_tol
