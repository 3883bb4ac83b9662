"""The eigenvalue-bounded polynomial coefficients (Sec. III.A, cn_mode = "fit") and
the spectrum-bound output on the GPU, through the C ABI, against the oracle's
own Lanczos bounds and least-squares fit (same start vector, same step count):

* energies and exact forces (coefficients held fixed) of an open cluster and a
  periodic box, FP64 within 1e-8 and mixed precision within 1e-5 eV/atom and
  1e-4 eV/A; the spectrum bounds of every atom and node;
* the fit with the two-point frequency model and with the approximate forces;
* the sparse MBD products (two-radius regime) with the fit;
* the spectrum output in the series mode leaves the results untouched;
* a polarisation catastrophe (largest bound >= 1) is an error with the atom's
  index in the fit mode, and shows in the bounds in the series mode.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE, SPECIES_INDEX, Structure
from workloads import configs as C
from tests.gpu_common import oracle_params, method_params

pytestmark = pytest.mark.gpu

STEPS = 20


def _oprm(cut, **kw):
    prm = oracle_params(cut, **kw)
    prm.c_n_mode = "fit"
    prm.lanczos_steps = STEPS
    return prm


def _run(st, cut, precision="fp64", cn_mode="fit", forces=True, weights=None, spectrum=True, ctx=None,
         table=SPECIES_TABLE, **kw):
    import torch
    from paper_2407_06409_amd import compute
    dev = torch.device("cuda:0")
    prm = dataclasses.replace(method_params(precision=precision, **{k: v for k, v in kw.items()
                                                                     if k in ("scs_freq", "omega_ref")}),
                              cn_mode=cn_mode, lanczos_steps=STEPS,
                              **{k: v for k, v in kw.items() if k == "force_model"})
    w = None if weights is None else torch.as_tensor(weights, device=dev)
    out = compute(torch.as_tensor(st.pos, device=dev), torch.as_tensor(st.species, device=dev),
                  torch.as_tensor(st.nu, device=dev), cutoffs=cut, params=prm, species_table=table,
                  cell=st.cell, pbc=tuple(int(x) for x in st.pbc), e_weight=w, forces=forces, ctx=ctx,
                  want_spectrum=spectrum)
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}


CASES = {
    "cluster40": lambda: (C.hcno_cluster(40, 13), dict(r_scs=3.5, r_nbr=5.0, r_mbd1=5.0, r_mbd2=4.0)),
    "hcno72": lambda: (C.hcno_box(72, 12), dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fit_against_oracle(case):
    st, cut = CASES[case]()
    w = np.random.default_rng(11).uniform(0.5, 1.5, st.n)
    prm = _oprm(cut)
    print(f"case {case} n={st.n} fitted c_n, {STEPS} Lanczos steps", flush=True)
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=w)
    b = oracle.lmbd_spectrum_bounds(st, prm, SPECIES_TABLE)
    g = _run(st, cut, weights=w)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    db = np.abs(g["spectrum"] - b).max()
    print(f"  FP64: max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A, max |d bound| {db:.3e} "
          f"(bounds in [{b[..., 0].min():.3f}, {b[..., 1].max():.3f}])", flush=True)
    assert de < 1e-8 and df < 1e-8 and db < 1e-10
    s = _run(st, cut, cn_mode="series", weights=w, spectrum=False)
    print(f"  fit - series: max |dE| {np.abs(g['energies'] - s['energies']).max():.3e} eV", flush=True)
    m = _run(st, cut, precision="mixed", weights=w)
    de_m, df_m = np.abs(m["energies"] - e).max(), np.abs(m["forces"] - f).max()
    db_m = np.abs(m["spectrum"] - b).max()
    print(f"  mixed: max |dE| {de_m:.3e} eV, max |dF| {df_m:.3e} eV/A, max |d bound| {db_m:.3e}", flush=True)
    assert de_m < 1e-5 and df_m < 1e-4 and db_m < 1e-5


def test_fit_with_lorentz_model_and_paper_forces():
    st, cut = CASES["cluster40"]()
    print(f"case cluster40 fit + two-point model (omega_ref 0.5 Ha)", flush=True)
    prm = _oprm(cut, scs_freq="lorentz", omega_ref=0.5)
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE)
    g = _run(st, cut, scs_freq="lorentz", omega_ref=0.5)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A", flush=True)
    assert de < 1e-8 and df < 1e-8
    print(f"case cluster40 fit + approximate forces", flush=True)
    e, f = oracle.lmbd_paper_forces(st, _oprm(cut), SPECIES_TABLE)
    g = _run(st, cut, force_model="paper")
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    print(f"  max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A", flush=True)
    assert de < 1e-8 and df < 1e-8


def test_fit_with_sparse_products():
    from paper_2407_06409_amd import Context
    st = C.hcno_box(72, 12)
    cut = dict(r_scs=4.0, r_nbr=6.0, r_mbd1=6.0, r_mbd2=2.5)
    ctx = Context(0)
    ctx.set_mbd_product("sparse")
    print(f"case hcno72 two-radius {cut}, sparse products, fit", flush=True)
    prm = _oprm(cut)
    atoms = list(range(0, 72, 9))
    w = np.zeros(st.n)
    w[atoms] = 1.0
    e, f = oracle.lmbd_energy_forces(st, prm, SPECIES_TABLE, weights=w, atoms=atoms)
    b = oracle.lmbd_spectrum_bounds(st, prm, SPECIES_TABLE, atoms=atoms)
    g = _run(st, cut, weights=w, ctx=ctx)
    de = np.abs(g["energies"][atoms] - e[atoms]).max()
    df = np.abs(g["forces"] - f).max()
    db = np.abs(g["spectrum"][atoms] - b[atoms]).max()
    print(f"  FP64: max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A, max |d bound| {db:.3e}", flush=True)
    assert de < 1e-8 and df < 1e-8 and db < 1e-10
    m = _run(st, cut, precision="mixed", weights=w, ctx=ctx)
    de_m, df_m = np.abs(m["energies"][atoms] - e[atoms]).max(), np.abs(m["forces"] - f).max()
    print(f"  mixed: max |dE| {de_m:.3e} eV, max |dF| {df_m:.3e} eV/A", flush=True)
    assert de_m < 1e-5 and df_m < 1e-4


def test_spectrum_output_leaves_the_series_results_unchanged():
    st, cut = C.config_small_open()
    print(f"case open64 series with and without the spectrum output", flush=True)
    a = _run(st, cut, cn_mode="series", spectrum=False)
    b = _run(st, cut, cn_mode="series", spectrum=True)
    assert np.array_equal(a["energies"], b["energies"]) and np.array_equal(a["forces"], b["forces"])
    ref = oracle.lmbd_spectrum_bounds(st, _oprm(cut), SPECIES_TABLE)
    assert np.abs(b["spectrum"] - ref).max() < 1e-10
    assert np.all(b["spectrum"][..., 0] < 0) and np.all(b["spectrum"][..., 1] > 0)


def test_polarisation_catastrophe_is_reported():
    """Strongly polarisable atoms at short range (a made-up species of 600 bohr^3): the
    largest bound passes 1; the fit mode fails with the lowest such atom, the series
    mode evaluates and reports the bounds.  Atoms 0-2 are far from the cluster 3-5."""
    from paper_2407_06409_amd import LmbdError
    tab = np.array(SPECIES_TABLE, copy=True)
    tab[SPECIES_INDEX["C"]] = [600.0, 2000.0, 4.0]
    ci, hi = SPECIES_INDEX["C"], SPECIES_INDEX["H"]
    pos = np.array([[0.0, 0, 0], [1.1, 0, 0], [0, 1.1, 0], [30.0, 0, 0], [33.0, 0.2, 0.1], [31.2, 2.7, 0.4]])
    st = Structure(pos, np.array([hi, hi, hi, ci, ci, ci], np.int32), np.full(6, 0.9), None, np.zeros(3, bool),
                   "catastrophe")
    cut = dict(r_scs=0.6, r_nbr=10.0, r_mbd1=10.0, r_mbd2=10.0)
    ob = oracle.lmbd_spectrum_bounds(st, _oprm(cut), tab)
    assert ob[3:, 0, 1].max() >= 1.0 and ob[:3, :, 1].max() < 1.0
    for precision in ("fp64", "mixed"):
        with pytest.raises(LmbdError) as ei:
            _run(st, cut, precision=precision, table=tab)
        print(f"  {precision}: {ei.value}", flush=True)
        assert ei.value.code == "LMBD_E_POLARISATION" and "atom 3" in str(ei.value)
    s = _run(st, cut, cn_mode="series", table=tab)
    assert np.all(np.isfinite(s["energies"])) and np.abs(s["spectrum"] - ob).max() < 1e-10
