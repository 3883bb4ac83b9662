"""GPU (HIP, gfx950) against the FP64 CPU oracle, through the C ABI.

Energies must agree within 1e-8 eV/atom and forces within 1e-8 eV/A (FP64
path); both sides evaluate the same definition with different summation order
and different linear solvers, so the expected differences are at round-off.
"""
import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE, Structure
from workloads import configs as C
from tests.gpu_common import gpu_run, oracle_params

pytestmark = pytest.mark.gpu

E_TOL = 1e-8   # eV per atom
F_TOL = 1e-8   # eV / A


def _check(st, cut, n_max=6, forces=True, weights=None):
    print(f"case {st.name or 'structure'} n={st.n} cut={cut['r_scs']} n_max={n_max}", flush=True)
    g = gpu_run(st, cut, n_max=n_max, forces=forces, weights=weights)
    prm = oracle_params(cut, n_max=n_max)
    if forces:
        e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=weights)
        err_f = np.abs(g["forces"] - f).max()
        print(f"  max |dF| = {err_f:.3e} eV/A (max |F| {np.abs(f).max():.3e})", flush=True)
        assert err_f < F_TOL
    else:
        e = oracle.lmbd_energies(st, prm, SPECIES_TABLE)
    err_e = np.abs(g["energies"] - e).max()
    print(f"  max |dE| = {err_e:.3e} eV (sum E {e.sum():.6f})", flush=True)
    assert err_e < E_TOL
    return g, e


def test_open_cluster_energy_forces():
    st, cut = C.config_small_open()
    _check(st, cut)


def test_periodic_carbon_box_with_images():
    st = C.carbon_box(96, 11, g_cm3=2.0)
    _check(st, dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0))


def test_periodic_hcno_box():
    st = C.hcno_box(72, 12)
    _check(st, dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5))


def test_general_radii_and_weights():
    st = C.hcno_cluster(40, 13)
    rng = np.random.default_rng(0)
    _check(st, dict(r_scs=3.5, r_nbr=6.0, r_mbd1=6.0, r_mbd2=4.0), weights=rng.uniform(-1, 2, st.n))
    _check(st, dict(r_scs=4.0, r_nbr=3.0, r_mbd1=3.0, r_mbd2=3.0))


@pytest.mark.parametrize("n_max", [2, 3, 5, 8])
def test_series_orders(n_max):
    st, cut = C.config_small_open()
    _check(st, cut, n_max=n_max, forces=(n_max == 3))


def test_edge_cases_isolated_and_dimer():
    iso = Structure(np.array([[0.0, 0, 0], [30.0, 0, 0]]), np.array([1, 0], np.int32),
                    np.array([0.9, 0.8]), None, np.zeros(3, bool), "isolated")
    g = gpu_run(iso, dict(r_scs=5.0, r_nbr=5.0, r_mbd1=5.0, r_mbd2=5.0))
    assert np.all(g["energies"] == 0.0) and np.all(g["forces"] == 0.0)
    one = Structure(np.array([[1.0, 2, 3]]), np.array([1], np.int32), np.array([0.9]), None,
                    np.zeros(3, bool), "single")
    g = gpu_run(one, dict(r_scs=5.0, r_nbr=5.0, r_mbd1=5.0, r_mbd2=5.0))
    assert g["energies"][0] == 0.0
    dimer = Structure(np.array([[0.0, 0, 0], [1.9, 0.4, 0.2]]), np.array([1, 3], np.int32),
                      np.array([0.9, 0.8]), None, np.zeros(3, bool), "dimer")
    _check(dimer, dict(r_scs=5.0, r_nbr=5.0, r_mbd1=5.0, r_mbd2=5.0))


def test_deterministic_and_batch_independent():
    import torch
    from paper_2407_06409_amd import compute_batch
    from tests.gpu_common import method_params
    a = C.carbon_box(64, 21, g_cm3=2.0)
    b = C.hcno_cluster(50, 22)
    cut_a = dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0)
    cut_b = dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)
    dev = torch.device("cuda:0")

    def desc(st, cut):
        return dict(pos=torch.as_tensor(st.pos, device=dev), species=torch.as_tensor(st.species, device=dev),
                    v_ratio=torch.as_tensor(st.nu, device=dev), cell=st.cell, pbc=tuple(int(x) for x in st.pbc),
                    cutoffs=cut)

    alone = compute_batch([desc(a, cut_a)], method_params(), SPECIES_TABLE)[0]
    again = compute_batch([desc(a, cut_a)], method_params(), SPECIES_TABLE)[0]
    mixed = compute_batch([desc(b, cut_b), desc(a, cut_a)], method_params(), SPECIES_TABLE)
    torch.cuda.synchronize()
    assert torch.equal(alone["energies"], again["energies"]) and torch.equal(alone["forces"], again["forces"])
    assert torch.equal(alone["energies"], mixed[1]["energies"])
    assert torch.equal(alone["forces"], mixed[1]["forces"])


def test_forces_sum_to_zero_and_autograd():
    import torch
    from paper_2407_06409_amd import LMBDEnergy
    from tests.gpu_common import method_params
    st = C.carbon_box(80, 31, g_cm3=2.0)
    cut = dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)
    g = gpu_run(st, cut)
    assert np.abs(g["forces"].sum(0)).max() < 1e-12 * max(1.0, np.abs(g["forces"]).max() * st.n)
    dev = torch.device("cuda:0")
    pos = torch.tensor(st.pos, device=dev, requires_grad=True)
    e = LMBDEnergy.apply(pos, torch.as_tensor(st.species, device=dev), torch.as_tensor(st.nu, device=dev),
                         st.cell, cut, method_params(), SPECIES_TABLE)
    (e * torch.arange(st.n, device=dev, dtype=torch.float64)).sum().backward()
    w = np.arange(st.n, dtype=np.float64)
    gw = gpu_run(st, cut, weights=w)
    assert np.allclose(pos.grad.cpu().numpy(), -gw["forces"], rtol=0, atol=1e-12)
    assert np.allclose(e.detach().cpu().numpy(), g["energies"], rtol=0, atol=0)


def test_invalid_inputs_raise():
    from paper_2407_06409_amd import LmbdError
    st, cut = C.config_small_open()
    bad = st.copy()
    bad.pos[3, 1] = np.nan
    with pytest.raises(LmbdError) as ei:
        gpu_run(bad, cut)
    assert ei.value.code == "LMBD_E_INVALID_ARG"
    with pytest.raises(LmbdError) as ei:
        gpu_run(st, dict(r_scs=0.4, r_nbr=5.0, r_mbd1=5.0, r_mbd2=5.0))
    assert ei.value.code == "LMBD_E_INVALID_ARG"
    bad = st.copy()
    bad.nu[0] = -1.0
    with pytest.raises(LmbdError) as ei:
        gpu_run(bad, cut)
    assert ei.value.code == "LMBD_E_INVALID_ARG"
