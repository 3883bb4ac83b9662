"""Write the stored oracle values used by the full-size GPU parity tests.

Every number in the files written here comes from the CPU oracle (``oracle/``)
on the seeded workloads of ``workloads/``; nothing is taken from the GPU path.

    python tests/golden/make_golden.py                        # all fixtures
    python tests/golden/make_golden.py --only C1728_pbc_6p8A    # some, merged into the file
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import SPECIES_TABLE, DEFAULT_PARAMS, frequency_grid  # noqa: E402
from workloads import configs as C  # noqa: E402


def params(cut):
    g = frequency_grid(DEFAULT_PARAMS["n_freq"])
    return oracle.make_params(cut, g[0], g[1], n_max=DEFAULT_PARAMS["n_max"], beta=DEFAULT_PARAMS["beta"],
                              damp_d=DEFAULT_PARAMS["damp_d"], r_buf=DEFAULT_PARAMS["r_buf"],
                              r_inner=DEFAULT_PARAMS["r_inner"])


def sample(n, m, seed):
    return sorted(int(x) for x in np.random.Generator(np.random.PCG64(seed)).choice(n, m, replace=False))


# The oracle evaluates one central atom at a time; the fixtures split their atoms
# over worker processes (one torch thread each).  A force fixture of a partial sum
# is the sum of the single-atom terms' forces (the forces are linear in the
# weights), added in atom order.
_JOB = {}


def _init_worker():
    import torch
    torch.set_num_threads(1)


def _energy_of(k):
    st, cut = _JOB["st"], _JOB["cut"]
    return float(oracle.lmbd_energies(st, params(cut), SPECIES_TABLE, atoms=[k])[k])


def _forces_of(k):
    st, cut = _JOB["st"], _JOB["cut"]
    w = np.zeros(st.n)
    w[k] = 1.0
    e, f = oracle.lmbd_energy_forces(st, params(cut), SPECIES_TABLE, weights=w, atoms=[k])
    return float(e[k]), f


def _pool_map(fn, st, cut, items):
    import multiprocessing as mp
    _JOB.update(st=st, cut=cut)
    ctx = mp.get_context("fork")
    with ctx.Pool(min(len(items), os.cpu_count() or 1), initializer=_init_worker) as pool:
        return pool.map(fn, items, chunksize=1)


def energies_fixture(name, st, cut, atoms):
    t = time.time()
    e = _pool_map(_energy_of, st, cut, list(atoms))
    print(f"{name}: energies of {len(atoms)} atoms in {time.time() - t:.1f} s", flush=True)
    return {"atoms": list(atoms), "energies_eV": e}


def forces_fixture(name, st, cut, atoms):
    """Forces of the partial sum sum_{k in atoms} E_k (weights 1 on the sample, 0 elsewhere)."""
    t = time.time()
    parts = _pool_map(_forces_of, st, cut, list(atoms))
    f = np.zeros((st.n, 3))
    for _, fk in parts:
        f += fk
    nz = np.nonzero(np.any(f != 0.0, axis=1))[0]
    print(f"{name}: forces of the {len(atoms)}-atom partial sum in {time.time() - t:.1f} s "
          f"({len(nz)} atoms with nonzero force)", flush=True)
    return {"weighted_atoms": list(atoms), "force_atoms": [int(a) for a in nz],
            "forces_eV_per_A": [[float(x) for x in f[a]] for a in nz]}


def whole_fixture(name, st, cut):
    """Every atom's energy and the forces of the whole energy (all weights 1)."""
    t = time.time()
    parts = _pool_map(_forces_of, st, cut, list(range(st.n)))
    f = np.zeros((st.n, 3))
    for _, fk in parts:
        f += fk
    print(f"{name}: energies and forces of all {st.n} atoms in {time.time() - t:.1f} s", flush=True)
    return {"energies_eV": [e for e, _ in parts], "forces_eV_per_A": [[float(x) for x in fa] for fa in f]}


def cutoff_6p8A():
    """The 1,728-atom carbon box with every radius at 6.8 A: 132 K1 sites per atom
    on average and up to 154 (N = 3 n1 up to 462), the large-neighbourhood end
    of the solves."""
    st, cut = C.config_plain_pbc()
    return st, {k: (6.8 if k.startswith("r_") else v) for k, v in cut.items()}


def two_radius_6_3():
    """The 1,728-atom carbon box in the two-radius regime of Sec. III.A: r_SCS =
    r_MBD,1 = 6 A, r_MBD,2 = 3 A and K = B(r_MBD,1 + r_MBD,2) = B(9 A), about 305
    sites per neighbourhood, of which a block row other than the central atom's
    couples to about 11."""
    st, _ = C.config_plain_pbc()
    return st, dict(r_scs=6.0, r_nbr=9.0, r_mbd1=6.0, r_mbd2=3.0)


def two_radius_10_8():
    """The 1,728-atom carbon box at production two-radius settings of Sec. III.A/IV:
    r_SCS = 6 A, r_MBD,1 = 10 A, r_MBD,2 = 8 A and K = B(18 A), about 2,450 sites
    per neighbourhood (periodic images included), each row other than the central
    atom's coupled to about 220 of them."""
    st, _ = C.config_plain_pbc()
    return st, dict(r_scs=6.0, r_nbr=18.0, r_mbd1=10.0, r_mbd2=8.0)


def small_hcno_box(n, rc):
    """Periodic H/C/N/O cube at 1.0 g/cm^3 small enough that every atom's own
    periodic images lie inside its SCS shell (edge below 2 r_SCS), as the
    smallest periodic requests of the serving workload are."""
    return C.hcno_box(n, 7000 + n), dict(r_scs=rc, r_nbr=rc, r_mbd1=rc, r_mbd2=rc)


def fixture(name):
    if name == "C1728_pbc":
        st, cut = C.config_plain_pbc()
        return {"cutoffs": cut,
                "energies": energies_fixture("C1728", st, cut, sample(st.n, 64, 7)),
                "forces": forces_fixture("C1728", st, cut, sample(st.n, 16, 8))}
    if name == "HCNO4096_pbc":
        st, cut = C.config_diff_hcno()
        return {"cutoffs": cut, "energies": energies_fixture("HCNO4096", st, cut, sample(st.n, 64, 9)),
                "forces": forces_fixture("HCNO4096", st, cut, sample(st.n, 16, 15))}
    if name == "C13824_pbc":
        st, cut = C.config_mixed_pbc()
        return {"cutoffs": cut, "energies": energies_fixture("C13824", st, cut, sample(st.n, 64, 10))}
    if name in ("HCNO50_pbc_5A", "HCNO100_pbc_6A"):
        n, rc = (50, 5.0) if name == "HCNO50_pbc_5A" else (100, 6.0)
        st, cut = small_hcno_box(n, rc)
        return {"cutoffs": cut, "box_A": float(st.cell[0, 0]), "whole": whole_fixture(name, st, cut)}
    if name == "C1728_pbc_6p8A":
        st, cut = cutoff_6p8A()
        return {"cutoffs": cut,
                "energies": energies_fixture("C1728 6.8A", st, cut, sample(st.n, 4, 11)),
                "forces": forces_fixture("C1728 6.8A", st, cut, sample(st.n, 1, 12))}
    if name == "C1728_pbc_two_radius":
        st, cut = two_radius_6_3()
        return {"cutoffs": cut,
                "energies": energies_fixture("C1728 two-radius", st, cut, sample(st.n, 4, 13)),
                "forces": forces_fixture("C1728 two-radius", st, cut, sample(st.n, 1, 14))}
    if name == "HCNO512_pbc_8A":
        # the paper's SCS cutoff (8 A) on a molecular-liquid-like box: K1 of about 180 sites
        st = C.hcno_box(512, 8512)
        cut = dict(r_scs=8.0, r_nbr=8.0, r_mbd1=8.0, r_mbd2=8.0)
        return {"cutoffs": cut,
                "energies": energies_fixture("HCNO512 8 A", st, cut, sample(st.n, 4, 18)),
                "forces": forces_fixture("HCNO512 8 A", st, cut, sample(st.n, 1, 19))}
    if name == "C216_pbc_15p10A":
        # the paper's 15 + 10 A production radii (Sec. IV): K = B(25 A), about 6,600 sites with images
        st = C.carbon_box(216, 41, g_cm3=2.0)
        cut = dict(r_scs=6.0, r_nbr=25.0, r_mbd1=15.0, r_mbd2=10.0)
        return {"cutoffs": cut, "energies": energies_fixture("C216 15+10 A", st, cut, sample(st.n, 4, 20))}
    if name == "C1728_pbc_10p8A":
        st, cut = two_radius_10_8()
        return {"cutoffs": cut,
                "energies": energies_fixture("C1728 10+8 A", st, cut, sample(st.n, 8, 16)),
                "forces": forces_fixture("C1728 10+8 A", st, cut, sample(st.n, 1, 17))}
    raise KeyError(name)




NAMES = ["C1728_pbc", "HCNO4096_pbc", "C13824_pbc", "C1728_pbc_6p8A", "C1728_pbc_two_radius", "HCNO50_pbc_5A",
         "HCNO100_pbc_6A", "C1728_pbc_10p8A", "HCNO512_pbc_8A", "C216_pbc_15p10A"]


def main():
    """All fixtures, or (--only a,b) only the named ones, merged into the stored file."""
    path = os.path.join(HERE, "oracle_fullsize.json")
    names = NAMES
    out = {"source": "CPU FP64 oracle (oracle/lmbd.py) on the seeded workloads; written by "
                     "tests/golden/make_golden.py",
           "params": DEFAULT_PARAMS}
    if "--only" in sys.argv:
        names = sys.argv[sys.argv.index("--only") + 1].split(",")
        with open(path) as fh:
            out = json.load(fh)
    for name in names:
        out[name] = fixture(name)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
