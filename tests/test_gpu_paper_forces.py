"""The paper's approximate forces (Sec. III.D, force_model = "paper") on the GPU
against the oracle's own evaluation of them (oracle.lmbd_paper_forces), through
the C ABI: FP64 within 1e-8 eV/A, mixed precision within 1e-4 eV/A; energies
are those of the exact mode.  Where the approximations are exact (no
screening, every neighbourhood the whole structure) the GPU's approximate and
exact forces agree."""
import dataclasses

import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from tests.gpu_common import oracle_params, method_params, GRID

pytestmark = pytest.mark.gpu


def _run(st, cut, precision="fp64", force_model="paper", weights=None, want_dv=False):
    import torch
    from paper_2407_06409_amd import compute
    dev = torch.device("cuda:0")
    prm = dataclasses.replace(method_params(precision=precision), force_model=force_model)
    w = None if weights is None else torch.as_tensor(weights, device=dev)
    out = compute(torch.as_tensor(st.pos, device=dev), torch.as_tensor(st.species, device=dev),
                  torch.as_tensor(st.nu, device=dev), cutoffs=cut, params=prm, species_table=SPECIES_TABLE,
                  cell=st.cell, pbc=tuple(int(x) for x in st.pbc), e_weight=w, forces=True, want_dv=want_dv)
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}


CASES = {
    "open64": lambda: C.config_small_open(),
    "cluster40": lambda: (C.hcno_cluster(40, 13), dict(r_scs=3.5, r_nbr=5.0, r_mbd1=5.0, r_mbd2=4.0)),
    "hcno72": lambda: (C.hcno_box(72, 12), dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_paper_forces_against_oracle(case):
    st, cut = CASES[case]()
    w = np.random.default_rng(3).uniform(0.5, 1.5, st.n)
    print(f"case {case} n={st.n} approximate forces", flush=True)
    e, f = oracle.lmbd_paper_forces(st, oracle_params(cut), SPECIES_TABLE, weights=w)
    g = _run(st, cut, weights=w)
    de, df = np.abs(g["energies"] - e).max(), np.abs(g["forces"] - f).max()
    ex = _run(st, cut, force_model="exact", weights=w)
    print(f"  FP64: max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A (max |F| {np.abs(f).max():.3e}); "
          f"approximate vs exact forces: max {np.abs(g['forces'] - ex['forces']).max():.3e} eV/A", flush=True)
    assert de < 1e-8 and df < 1e-8
    assert np.array_equal(g["energies"], ex["energies"])
    m = _run(st, cut, precision="mixed", weights=w)
    de_m, df_m = np.abs(m["energies"] - e).max(), np.abs(m["forces"] - f).max()
    print(f"  mixed: max |dE| {de_m:.3e} eV, max |dF| {df_m:.3e} eV/A", flush=True)
    assert de_m < 1e-5 and df_m < 1e-4


def test_paper_forces_equal_exact_where_the_approximations_are_exact():
    st = C.hcno_cluster(12, 17, dmin=1.3)
    cut = dict(r_scs=0.6, r_nbr=30.0, r_mbd1=30.0, r_mbd2=30.0)   # 2 r_scs below d_min: no screening; every frame sees all
    a, b = _run(st, cut), _run(st, cut, force_model="exact")
    d = np.abs(a["forces"] - b["forces"]).max()
    print(f"  approximate vs exact forces without screening: {d:.3e} eV/A", flush=True)
    assert d < 1e-10 * max(1.0, np.abs(b["forces"]).max())


def test_paper_forces_reject_volume_ratio_derivatives():
    from paper_2407_06409_amd import LmbdError
    st, cut = C.config_small_open()
    with pytest.raises(LmbdError) as ei:
        _run(st, cut, want_dv=True)
    assert ei.value.code == "LMBD_E_INVALID_ARG"
