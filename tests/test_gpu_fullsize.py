"""Full-size workloads on the GPU against stored oracle values and finite differences.

The stored values (tests/golden/oracle_fullsize.json) are written by
tests/golden/make_golden.py, which calls only the CPU oracle.
"""
import json
import os

import numpy as np
import pytest

from workloads import configs as C
from tests.gpu_common import gpu_run

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fullsize.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_c1728_energies_and_partial_forces_match_oracle():
    g = golden()["C1728_pbc"]
    st, cut = C.config_plain_pbc()
    print(f"case C1728 n={st.n}", flush=True)
    full = gpu_run(st, cut, forces=True)
    atoms = g["energies"]["atoms"]
    de = np.abs(full["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    print(f"  max |dE| on {len(atoms)} sampled atoms: {de:.3e} eV", flush=True)
    assert de < 1e-8
    f = full["forces"]
    assert np.abs(f.sum(0)).max() < 1e-10
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    part = gpu_run(st, cut, forces=True, weights=w)
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    df = np.abs(part["forces"] - ref).max()
    print(f"  max |dF| of the weighted partial sum over all atoms: {df:.3e} eV/A "
          f"(max |F| {np.abs(ref).max():.3e})", flush=True)
    assert df < 1e-8


def test_c1728_cutoff_6p8A_large_neighbourhoods_match_oracle():
    """Up to 154 K1 sites per atom (N = 3 n1 up to 462): the solves' second row
    slot (rows 256 and up of the 256-thread workgroups) and the larger LDS
    layouts, against stored oracle energies and the forces of a one-atom sum."""
    g = golden()["C1728_pbc_6p8A"]
    st, _ = C.config_plain_pbc()
    cut = g["cutoffs"]
    print(f"case C1728 cutoff 6.8 A n={st.n}", flush=True)
    full = gpu_run(st, cut, forces=False)
    atoms = g["energies"]["atoms"]
    de = np.abs(full["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    print(f"  max |dE| on {len(atoms)} sampled atoms: {de:.3e} eV", flush=True)
    assert de < 1e-8
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    part = gpu_run(st, cut, forces=True, weights=w)
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    df = np.abs(part["forces"] - ref).max()
    print(f"  max |dF| of the weighted one-atom sum over all atoms: {df:.3e} eV/A "
          f"(max |F| {np.abs(ref).max():.3e})", flush=True)
    assert df < 1e-8
    # the mixed path (FP32 factors and solves, FP64 refinement) at the same sizes
    mixed = gpu_run(st, cut, forces=True, weights=w, precision="mixed")
    de_m = np.abs(mixed["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    df_m = np.abs(mixed["forces"] - ref).max()
    print(f"  mixed: max |dE| {de_m:.3e} eV/atom, max |dF| {df_m:.3e} eV/A", flush=True)
    assert de_m < 1e-5 and df_m < 1e-4


@pytest.mark.parametrize("mode", ["sparse", "dense"])
def test_c1728_two_radius_regime_matches_oracle(mode):
    """The two-radius regime at full size (r_MBD,1 = r_SCS = 6 A, r_MBD,2 = 3 A, K =
    B(9 A), about 305 sites per neighbourhood), in the product form the automatic
    choice takes (sparse) and in the dense one, against stored oracle energies and
    the forces of a one-atom sum; the mixed path with the sparse form too."""
    from paper_2407_06409_amd import Context
    g = golden()["C1728_pbc_two_radius"]
    st, _ = C.config_plain_pbc()
    cut = g["cutoffs"]
    ctx = Context(0)
    ctx.set_mbd_product(mode)
    print(f"case C1728 two-radius {cut} n={st.n}, MBD products {mode}", flush=True)
    atoms = g["energies"]["atoms"]
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    full = gpu_run(st, cut, forces=False, ctx=ctx)
    de = np.abs(full["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    part = gpu_run(st, cut, forces=True, weights=w, ctx=ctx)
    df = np.abs(part["forces"] - ref).max()
    print(f"  max |dE| on {len(atoms)} sampled atoms {de:.3e} eV, max |dF| of the one-atom sum {df:.3e} eV/A "
          f"(max |F| {np.abs(ref).max():.3e})", flush=True)
    assert de < 1e-8 and df < 1e-8
    if mode == "sparse":
        mixed = gpu_run(st, cut, forces=True, weights=w, precision="mixed", ctx=ctx)
        de_m = np.abs(mixed["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
        df_m = np.abs(mixed["forces"] - ref).max()
        print(f"  mixed: max |dE| {de_m:.3e} eV/atom, max |dF| {df_m:.3e} eV/A", flush=True)
        assert de_m < 1e-5 and df_m < 1e-4


def test_hcno4096_energies_and_partial_forces_match_oracle():
    """Sampled energies and the forces of a 16-atom weighted partial sum (every atom
    whose force it moves) against stored oracle values."""
    g = golden()["HCNO4096_pbc"]
    st, cut = C.config_diff_hcno()
    print(f"case HCNO4096 n={st.n}", flush=True)
    out = gpu_run(st, cut, forces=False)
    atoms = g["energies"]["atoms"]
    de = np.abs(out["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    print(f"  max |dE| on {len(atoms)} sampled atoms: {de:.3e} eV", flush=True)
    assert de < 1e-8
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    part = gpu_run(st, cut, forces=True, weights=w)
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    df = np.abs(part["forces"] - ref).max()
    print(f"  max |dF| of the {len(g['forces']['weighted_atoms'])}-atom partial sum over all atoms: {df:.3e} eV/A "
          f"(max |F| {np.abs(ref).max():.3e})", flush=True)
    assert df < 1e-8


def test_c13824_energies_match_oracle_fp64():
    g = golden()["C13824_pbc"]
    st, cut = C.config_mixed_pbc()
    print(f"case C13824 n={st.n}", flush=True)
    out = gpu_run(st, cut, forces=False)
    atoms = g["energies"]["atoms"]
    de = np.abs(out["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    print(f"  max |dE| {de:.3e} eV", flush=True)
    assert de < 1e-8


def _crosses(st, a, g, h, radii):
    """True if moving atom a by +-h along g changes any neighbour-set membership."""
    L = st.cell[0, 0]
    for sgn in (-1.0, 1.0):
        p = st.pos[a].copy()
        p[g] += sgn * h
        d0 = st.pos - st.pos[a]
        d0 -= L * np.round(d0 / L)
        d1 = st.pos - p
        d1 -= L * np.round(d1 / L)
        r0 = np.linalg.norm(d0, axis=1)
        r1 = np.linalg.norm(d1, axis=1)
        for rc in radii:
            if np.any((r0 < rc) != (r1 < rc)):
                return True
    return False


def test_hcno4096_adjoint_forces_match_central_differences():
    """F = -dE/dR of the GPU adjoint vs central differences of the GPU energy (h = 1e-4 A)
    on 32 seeded (atom, component) draws; draws whose stencil changes a neighbour set
    (the method's hard membership switches) are skipped and replaced."""
    st, cut = C.config_diff_hcno()
    print(f"case HCNO4096 FD n={st.n}", flush=True)
    full = gpu_run(st, cut, forces=True)
    rng = np.random.Generator(np.random.PCG64(4242))
    radii = [cut["r_scs"], 2 * cut["r_scs"], cut["r_nbr"]]
    h = 1e-4
    checked, worst = 0, 0.0
    while checked < 32:
        a = int(rng.integers(st.n))
        g = int(rng.integers(3))
        if _crosses(st, a, g, h, radii):
            continue
        sp, sm = st.copy(), st.copy()
        sp.pos[a, g] += h
        sm.pos[a, g] -= h
        ep = gpu_run(sp, cut, forces=False)["energies"].sum()
        em = gpu_run(sm, cut, forces=False)["energies"].sum()
        fd = -(ep - em) / (2 * h)
        err = abs(fd - full["forces"][a, g])
        worst = max(worst, err)
        assert err < 1e-7 + 1e-6 * abs(fd), (a, g, fd, full["forces"][a, g])
        checked += 1
    print(f"  32 FD components, max |F_adj - F_fd| = {worst:.3e} eV/A", flush=True)


def test_c1728_production_two_radius_matches_oracle():
    """The paper's production radii (r_MBD,1 = 10 A, r_MBD,2 = 8 A, K = B(18 A), about
    2,450 sites per neighbourhood with periodic images; r_SCS = 6 A) on the 1,728-atom
    box: the sparse MBD form with its site arrays in the workspace, against stored oracle
    energies of sampled atoms and the forces of a one-atom sum, FP64 and mixed."""
    import torch
    from paper_2407_06409_amd import Context, release_default_context
    # a call of about 126 GiB (FP64 with forces): nothing held from the earlier tests
    release_default_context()
    torch.cuda.empty_cache()
    g = golden()["C1728_pbc_10p8A"]
    st, _ = C.config_plain_pbc()
    cut = g["cutoffs"]
    atoms = g["energies"]["atoms"]
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    ctx = Context(0)
    try:
        print(f"case C1728 production radii {cut} n={st.n}, energies", flush=True)
        full = gpu_run(st, cut, forces=False, ctx=ctx)
        de = np.abs(full["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
        print(f"  max |dE| on {len(atoms)} sampled atoms {de:.3e} eV", flush=True)
        part = gpu_run(st, cut, forces=True, weights=w, ctx=ctx)
        df = np.abs(part["forces"] - ref).max()
        print(f"  max |dF| of the one-atom sum {df:.3e} eV/A (max |F| {np.abs(ref).max():.3e})", flush=True)
        assert de < 1e-8 and df < 1e-8
        mixed = gpu_run(st, cut, forces=True, weights=w, precision="mixed", ctx=ctx)
        de_m = np.abs(mixed["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
        df_m = np.abs(mixed["forces"] - ref).max()
        print(f"  mixed: max |dE| {de_m:.3e} eV/atom, max |dF| {df_m:.3e} eV/A", flush=True)
        assert de_m < 1e-5 and df_m < 1e-4
    finally:
        ctx.close()


def test_hcno512_scs_cutoff_8A_matches_oracle():
    """The paper's SCS cutoff r_SCS = 8 A on a 512-atom H/C/N/O box at 1.0 g/cm^3: K1 of
    up to 205 sites (N = 3 n1 up to 615, beyond the two rows per thread of the 256-thread
    solves: three rows per thread run), against stored oracle energies of sampled atoms
    and the forces of a one-atom sum, FP64 and mixed."""
    g = golden()["HCNO512_pbc_8A"]
    st = C.hcno_box(512, 8512)
    cut = g["cutoffs"]
    atoms = g["energies"]["atoms"]
    w = np.zeros(st.n)
    w[g["forces"]["weighted_atoms"]] = 1.0
    ref = np.zeros((st.n, 3))
    ref[g["forces"]["force_atoms"]] = np.array(g["forces"]["forces_eV_per_A"])
    print(f"case HCNO512 r_SCS 8 A n={st.n}", flush=True)
    part = gpu_run(st, cut, forces=True, weights=w)
    de = np.abs(part["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    df = np.abs(part["forces"] - ref).max()
    print(f"  FP64: max |dE| {de:.3e} eV, max |dF| {df:.3e} eV/A (max |F| {np.abs(ref).max():.3e})", flush=True)
    assert de < 1e-8 and df < 1e-8
    mixed = gpu_run(st, cut, forces=True, weights=w, precision="mixed")
    de_m = np.abs(mixed["energies"][atoms] - np.array(g["energies"]["energies_eV"])).max()
    df_m = np.abs(mixed["forces"] - ref).max()
    print(f"  mixed: max |dE| {de_m:.3e} eV/atom, max |dF| {df_m:.3e} eV/A", flush=True)
    assert de_m < 1e-5 and df_m < 1e-4
