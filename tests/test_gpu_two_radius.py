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


def _ctx(mode):
    from paper_2407_06409_amd import Context
    ctx = Context(0)
    ctx.set_mbd_product(mode)
    return ctx


@pytest.mark.parametrize("mode", ["dense", "sparse"])
def test_two_radius_regime_both_product_forms(case, mode):
    """The automatic choice takes the sparse form here; both forms forced."""
    st, w, e_ref, f_ref, nk = case
    print(f"case C216 two-radius, MBD products {mode}", flush=True)
    g = gpu_run(st, CUT, weights=w, ctx=_ctx(mode))
    de = np.abs(g["energies"][ATOMS] - e_ref).max()
    df = np.abs(g["forces"] - f_ref).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A", flush=True)
    assert de < 1e-8 and df < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sparse_form_where_every_pair_couples(precision):
    """Sparse products forced on a single-radius box, r_MBD,1 = r_MBD,2 = r_nbr (every
    block row couples to every site of K): energies and forces, hence the sparse
    adjoint (pair contraction, screened radii and blend terms) on full rows, against
    the oracle."""
    st = C.carbon_box(96, 11, g_cm3=2.0)
    cut = dict(r_scs=4.0, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)
    print(f"case C96 {cut} sparse MBD products forced, {precision}", flush=True)
    g = gpu_run(st, cut, precision=precision, ctx=_ctx("sparse"))
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut), SPECIES_TABLE)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A", flush=True)
    e_tol, f_tol = (1e-8, 1e-8) if precision == "fp64" else (1e-5, 1e-4)
    assert de < e_tol and df < f_tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sparse_form_on_a_small_two_radius_box(precision):
    """Sparse products forced with r_MBD,2 = 3 A below r_nbr = r_MBD,1 = 4.5 A: the
    pairs that do not touch the central atom are cut at the smaller radius."""
    st = C.carbon_box(96, 11, g_cm3=2.0)
    cut = dict(r_scs=4.0, r_nbr=4.5, r_mbd1=4.5, r_mbd2=3.0)
    print(f"case C96 {cut} sparse MBD products forced, {precision}", flush=True)
    g = gpu_run(st, cut, precision=precision, ctx=_ctx("sparse"))
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut), SPECIES_TABLE)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A", flush=True)
    e_tol, f_tol = (1e-8, 1e-8) if precision == "fp64" else (1e-5, 1e-4)
    assert de < e_tol and df < f_tol


def test_sparse_form_with_two_point_model_and_energy_only():
    from workloads.configs import OMEGA_REF
    st, cut = C.config_small_open()
    print(f"case C64 open sparse forced, two-point model, energies only", flush=True)
    lor = dict(scs_freq="lorentz", omega_ref=OMEGA_REF)
    g = gpu_run(st, cut, forces=False, ctx=_ctx("sparse"), **lor)
    e = oracle.lmbd_energies(st, oracle_params(cut, **lor), SPECIES_TABLE)
    de = np.abs(g["energies"] - e).max()
    print(f"  max |dE| {de:.3e} eV/atom", flush=True)
    assert de < 1e-8


def test_unknown_product_form_is_an_argument_error():
    from paper_2407_06409_amd import Context, load_library
    ctx = Context(0)
    assert load_library().lmbd_set_mbd_product(ctx.handle, 7) == 1
    assert load_library().lmbd_set_mbd_product(None, 0) == 1


def test_product_form_is_chosen_per_structure():
    """A two-radius structure (sparse form) and a single-radius one (dense form) in
    one call: each result is bitwise that of the structure evaluated alone."""
    from paper_2407_06409_amd import compute_batch
    from tests.gpu_common import method_params
    a = C.carbon_box(216, 21, g_cm3=2.0)
    b = C.carbon_box(96, 11, g_cm3=2.0)
    reqs = [dict(pos=a.pos, species=a.species, v_ratio=a.nu, cell=a.cell, pbc=(1, 1, 1), cutoffs=CUT),
            dict(pos=b.pos, species=b.species, v_ratio=b.nu, cell=b.cell, pbc=(1, 1, 1),
                 cutoffs=dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0))]
    mp = method_params()
    print("case C216 two-radius + C96 single radius in one call", flush=True)
    both = compute_batch(reqs, mp, SPECIES_TABLE)
    for r, got in zip(reqs, both):
        alone = compute_batch([r], mp, SPECIES_TABLE)[0]
        assert np.array_equal(alone["energies"], got["energies"])
        assert np.array_equal(alone["forces"], got["forces"])


# ---------------------------------------------------------------- neighbourhoods beyond LDS
# 128 C atoms at 2.0 g/cm^3 (L = 10.9 A), r_SCS = 4, r_MBD,1 = 6, r_MBD,2 = 4, K = B(10 A):
# about 420 sites per neighbourhood, more than the per-site arrays of the MBD stage can
# keep in LDS, so the sparse form with its site arrays in the workspace runs.
BIG_CUT = dict(r_scs=4.0, r_nbr=10.0, r_mbd1=6.0, r_mbd2=4.0)
BIG_ATOMS = [0, 41, 99]


@pytest.fixture(scope="module")
def big_case():
    st = C.carbon_box(128, 31, g_cm3=2.0)
    nk = min(len(oracle.neighbourhood(st.pos, st.cell, st.pbc, k, BIG_CUT["r_nbr"])[0]) for k in BIG_ATOMS)
    w = np.zeros(st.n)
    w[BIG_ATOMS] = [1.0, -0.6, 0.8]
    e, f = oracle.lmbd_energy_forces(st, oracle_params(BIG_CUT), SPECIES_TABLE, weights=w, atoms=BIG_ATOMS)
    return st, w, e[BIG_ATOMS], f, nk


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_neighbourhoods_beyond_lds_match_oracle(big_case, precision):
    st, w, e_ref, f_ref, nk = big_case
    print(f"case C128 {BIG_CUT}, nK at least {nk}, {precision}", flush=True)
    assert nk > 400
    g = gpu_run(st, BIG_CUT, weights=w, precision=precision)
    de = np.abs(g["energies"][BIG_ATOMS] - e_ref).max()
    df = np.abs(g["forces"] - f_ref).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A (max |F| {np.abs(f_ref).max():.3e})", flush=True)
    e_tol, f_tol = (1e-8, 1e-8) if precision == "fp64" else (1e-5, 1e-4)
    assert de < e_tol and df < f_tol
    assert np.abs(g["forces"].sum(0)).max() < 1e-9


def test_neighbourhoods_beyond_lds_need_the_sparse_form(big_case):
    """Forcing the dense products on such neighbourhoods is refused; energies of every
    atom are finite and the same with the automatic and the forced sparse choice."""
    from paper_2407_06409_amd import LmbdError
    st, w, e_ref, f_ref, nk = big_case
    with pytest.raises(LmbdError) as ei:
        gpu_run(st, BIG_CUT, forces=False, ctx=_ctx("dense"))
    assert ei.value.code == "LMBD_E_UNSUPPORTED"
    a = gpu_run(st, BIG_CUT, forces=False)
    b = gpu_run(st, BIG_CUT, forces=False, ctx=_ctx("sparse"))
    assert np.all(np.isfinite(a["energies"])) and np.array_equal(a["energies"], b["energies"])
