"""Two-point Lorentzian SCS frequency model (Sec. III.C) on the GPU against the
oracle's same model, through the C ABI.

The local SCS systems are solved at omega = 0 and omega_ref only; the blended
polarisabilities at the quadrature nodes follow the Lorentzian fixed by those two
values.  FP64 bars as for the exact frequency treatment (1e-8 eV/atom, 1e-8 eV/A);
the mixed path to 1e-5 eV/atom and 1e-4 eV/A.
"""
import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from workloads.configs import OMEGA_REF
from tests.gpu_common import gpu_run, oracle_params

pytestmark = pytest.mark.gpu

LOR = dict(scs_freq="lorentz", omega_ref=OMEGA_REF)


def _cases():
    return {
        "open64": C.config_small_open(),
        "box96": (C.carbon_box(96, 11, g_cm3=2.0), dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0)),
        "hcno72": (C.hcno_box(72, 12), dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)),
    }


@pytest.mark.parametrize("case", ["open64", "box96", "hcno72"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_point_model_against_oracle(case, precision):
    st, cut = _cases()[case]
    print(f"case {case} n={st.n} two-point SCS, {precision}", flush=True)
    g = gpu_run(st, cut, precision=precision, **LOR)
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut, **LOR), SPECIES_TABLE)
    de = np.abs(g["energies"] - e).max()
    df = np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A (sum E {e.sum():.6f})", flush=True)
    e_tol, f_tol = (1e-8, 1e-8) if precision == "fp64" else (1e-5, 1e-4)
    assert de < e_tol and df < f_tol


def test_two_point_model_general_radii_and_weights():
    st = C.hcno_cluster(40, 13)
    cut = dict(r_scs=3.5, r_nbr=6.0, r_mbd1=6.0, r_mbd2=4.0)
    w = np.random.default_rng(0).uniform(-1, 2, st.n)
    print(f"case hcno_cluster40 n={st.n} two-point SCS, radii {cut}", flush=True)
    g = gpu_run(st, cut, weights=w, **LOR)
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut, **LOR), SPECIES_TABLE, weights=w)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e}, max |dF| {df:.3e}", flush=True)
    assert de < 1e-8 and df < 1e-8


def test_two_point_model_with_the_single_node_omega_ref_is_the_exact_treatment():
    """With the quadrature node omega_ref alone, the model passes the solved
    polarisabilities through unchanged (rho = 1: d alpha/d alpha(0) = 0 and
    d alpha/d alpha(omega_ref) = 1), so both treatments give the same energies and
    forces on the GPU."""
    st, cut = C.carbon_box(96, 11, g_cm3=2.0), dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0)
    grid = (np.array([OMEGA_REF]), np.array([0.9]))
    print(f"case box96 single node omega_ref={OMEGA_REF}", flush=True)
    a = gpu_run(st, cut, grid=grid)
    b = gpu_run(st, cut, grid=grid, **LOR)
    de = np.abs(a["energies"] - b["energies"]).max()
    df = np.abs(a["forces"] - b["forces"]).max()
    print(f"  max |dE| {de:.3e}, max |dF| {df:.3e}", flush=True)
    assert np.abs(a["energies"]).min() > 0.0
    assert de < 1e-12 * np.abs(a["energies"]).max() and df < 1e-12 * max(1.0, np.abs(a["forces"]).max())


def test_two_point_model_differs_from_exact_treatment_by_a_model_error():
    """The model is an approximation: on the 12-node grid it moves the energies by
    a small fraction of themselves (printed), and its central static polarisabilities
    are the exact ones (both solve the same SCS system at omega = 0)."""
    st, cut = C.carbon_box(96, 11, g_cm3=2.0), dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0)
    a = gpu_run(st, cut)
    b = gpu_run(st, cut, **LOR)
    rel = np.abs(b["energies"] / a["energies"] - 1.0)
    print(f"  model vs exact frequency treatment: max rel dE {rel.max():.3e}, mean {rel.mean():.3e}", flush=True)
    assert np.allclose(a["alpha_scs0"], b["alpha_scs0"], rtol=1e-13, atol=0)
    assert 0.0 < rel.max() < 0.1


def test_two_point_model_rejects_bad_reference_frequency():
    from paper_2407_06409_amd import LmbdError
    st, cut = C.config_small_open()
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(LmbdError) as ei:
            gpu_run(st, cut, scs_freq="lorentz", omega_ref=bad)
        assert ei.value.code == "LMBD_E_INVALID_ARG"
