"""Mixed-precision path (FP32 pair tensors, FP32 MFMA factorisation and GEMMs, FP64
refinement of the SCS solve and FP64 accumulation) against the FP64 oracle and the
FP64 GPU path.  Bound: 1e-5 eV/atom on energies; force errors are reported and held
to 1e-4 eV/A."""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from tests.gpu_common import gpu_run, oracle_params

pytestmark = pytest.mark.gpu

E_TOL = 1e-5
F_TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fullsize.json")


@pytest.mark.parametrize("case", ["open64", "box96", "hcno72"])
def test_mixed_small_against_oracle(case):
    if case == "open64":
        st, cut = C.config_small_open()
    elif case == "box96":
        st, cut = C.carbon_box(96, 11, g_cm3=2.0), dict(r_scs=4.0, r_nbr=4.0, r_mbd1=4.0, r_mbd2=4.0)
    else:
        st, cut = C.hcno_box(72, 12), dict(r_scs=4.5, r_nbr=4.5, r_mbd1=4.5, r_mbd2=4.5)
    print(f"case {case} n={st.n} mixed", flush=True)
    g = gpu_run(st, cut, precision="mixed")
    e, f = oracle.lmbd_energy_forces(st, oracle_params(cut), SPECIES_TABLE)
    de = np.abs(g["energies"] - e).max()
    df = np.abs(g["forces"] - f).max()
    print(f"  mixed vs oracle: max |dE| {de:.3e} eV/atom, max |dF| {df:.3e} eV/A", flush=True)
    assert de < E_TOL and df < F_TOL


def test_mixed_c13824_against_oracle_and_fp64_gpu():
    with open(GOLDEN) as fh:
        gold = json.load(fh)["C13824_pbc"]
    st, cut = C.config_mixed_pbc()
    print(f"case C13824 n={st.n} mixed vs fp64", flush=True)
    m = gpu_run(st, cut, precision="mixed")
    atoms = gold["energies"]["atoms"]
    de_o = np.abs(m["energies"][atoms] - np.array(gold["energies"]["energies_eV"])).max()
    d = gpu_run(st, cut, precision="fp64")
    de = np.abs(m["energies"] - d["energies"])
    df = np.abs(m["forces"] - d["forces"])
    print(f"  mixed vs oracle (sampled): max |dE| {de_o:.3e} eV/atom", flush=True)
    print(f"  mixed vs FP64 GPU (all atoms): max |dE| {de.max():.3e}, mean {de.mean():.3e} eV/atom; "
          f"max |dF| {df.max():.3e}, mean {df.mean():.3e} eV/A", flush=True)
    assert de_o < E_TOL and de.max() < E_TOL and df.max() < F_TOL
