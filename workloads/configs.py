"""The five seeded workloads of the hot path, plus scaled-down variants for tests.

1. 64 C atoms, open 12 A cube, RSA d_min 1.3 A, nu ~ U[0.7, 1.0], cutoff 5 A.
2. 1,728 C atoms, periodic cube at 2.0 g/cm^3 (L = 25.83 A), d_min 1.3 A,
   nu ~ U[0.6, 1.0], cutoff 6 A.
3. 4,096 H/C/N/O (50/30/10/10) atoms, periodic cube at 1.0 g/cm^3, d_min 0.9 A,
   nu ~ U[0.6, 1.0], cutoff 6 A.
4. 13,824 C atoms, as 2 at the larger size.
5. 256 requests, sizes log-uniform in [50, 5000] atoms, H/C/N/O as 3, half open
   spheres and half periodic cubes at 1.0 g/cm^3, cutoff ~ U[5, 6] A, Poisson
   arrival times (in units of the mean inter-arrival time).

A single cutoff r_c sets r_SCS = r_nbr = r_MBD,1 = r_MBD,2 = r_c.
"""
import numpy as np

from .structures import (Structure, number_density, rsa_box, rsa_cube_open, rsa_sphere_open,
                         hcno_species)
from .species import SPECIES_INDEX
from .grid import frequency_grid

# Method parameters that the workloads fix (values as inputs; each side builds its own struct).
DEFAULT_PARAMS = dict(beta=0.83, damp_d=6.0, r_buf=0.5, r_inner=2.0, n_max=6, n_freq=12)
# reference frequency of the two-point SCS frequency model (Ha): the scale of the
# frequency grid, which has half of its nodes below it
OMEGA_REF = 0.5

HCNO = {"H": 0.5, "C": 0.3, "N": 0.1, "O": 0.1}


def cutoffs(rc):
    return dict(r_scs=rc, r_nbr=rc, r_mbd1=rc, r_mbd2=rc)


def _carbon(n, rng):
    return np.full(n, SPECIES_INDEX["C"], dtype=np.int32)


def carbon_box(n, seed, g_cm3=2.0, dmin=1.3, nu_lo=0.6, nu_hi=1.0):
    """n C atoms in a periodic cube at the given mass density."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = number_density(g_cm3, {"C": 1.0})
    length = (n / rho) ** (1.0 / 3.0)
    pos = rsa_box(n, length, dmin, rng)
    nu = rng.uniform(nu_lo, nu_hi, size=n)
    return Structure(pos, _carbon(n, rng), nu, np.eye(3) * length, np.ones(3, dtype=bool),
                     f"C{n}-pbc-{g_cm3}gcc")


def hcno_box(n, seed, g_cm3=1.0, dmin=0.9, nu_lo=0.6, nu_hi=1.0):
    """n H/C/N/O atoms in a periodic cube at the given mass density."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = number_density(g_cm3, HCNO)
    length = (n / rho) ** (1.0 / 3.0)
    pos = rsa_box(n, length, dmin, rng)
    sp = hcno_species(n, rng)
    nu = rng.uniform(nu_lo, nu_hi, size=n)
    return Structure(pos, sp, nu, np.eye(3) * length, np.ones(3, dtype=bool), f"HCNO{n}-pbc")


def carbon_slab(n, seed, length, thickness, pbc=(1, 1, 0), dmin=1.3, nu_lo=0.6, nu_hi=1.0):
    """n C atoms periodic along the directions with pbc set (edge ``length``) and
    confined to [0, thickness) along the others (a slab for pbc (1, 1, 0), a wire
    for (1, 0, 0)).  The rows of the cell along non-periodic directions carry a
    tilt: they only fix the fractional frame, never an image."""
    rng = np.random.Generator(np.random.PCG64(seed))
    span = [length if pbc[d] else thickness for d in range(3)]
    box = [length if pbc[d] else thickness + 4.0 * length for d in range(3)]   # no clash across the gap
    from .structures import _rsa
    pos = _rsa(n, lambda r: r.uniform(0.0, 1.0, size=3) * np.array(span), dmin, (0, 0, 0), box, True, rng)
    nu = rng.uniform(nu_lo, nu_hi, size=n)
    cell = np.diag([length if pbc[d] else thickness + 20.0 for d in range(3)])
    for d in range(3):
        if not pbc[d]:
            cell[d, (d + 1) % 3] = 3.0
            cell[d, (d + 2) % 3] = -2.0
    return Structure(pos, _carbon(n, rng), nu, cell, np.array([bool(x) for x in pbc]),
                     f"C{n}-pbc{''.join(str(int(x)) for x in pbc)}")


def hcno_cluster(n, seed, g_cm3=1.0, dmin=0.9, nu_lo=0.6, nu_hi=1.0):
    """n H/C/N/O atoms in an open sphere at the given mass density."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = number_density(g_cm3, HCNO)
    radius = (3.0 * n / (4.0 * np.pi * rho)) ** (1.0 / 3.0)
    pos = rsa_sphere_open(n, radius, dmin, rng)
    sp = hcno_species(n, rng)
    nu = rng.uniform(nu_lo, nu_hi, size=n)
    return Structure(pos, sp, nu, None, np.zeros(3, dtype=bool), f"HCNO{n}-open")


def config_small_open(seed=1001):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rsa_cube_open(64, 12.0, 1.3, rng)
    nu = rng.uniform(0.7, 1.0, size=64)
    s = Structure(pos, _carbon(64, rng), nu, None, np.zeros(3, dtype=bool), "C64-open")
    return s, cutoffs(5.0)


def config_plain_pbc(seed=1002):
    return carbon_box(1728, seed), cutoffs(6.0)


def config_diff_hcno(seed=1003):
    return hcno_box(4096, seed), cutoffs(6.0)


def config_mixed_pbc(seed=1004):
    return carbon_box(13824, seed), cutoffs(6.0)


def serving_requests(n_requests=256, seed_base=5000, arrival_seed=5999, lo=50, hi=5000):
    """Request list for the serving workload.

    Returns a list of dicts {"structure", "cutoffs", "arrival"} where ``arrival``
    is the arrival time in units of the mean inter-arrival time (Poisson stream).
    """
    arng = np.random.Generator(np.random.PCG64(arrival_seed))
    gaps = arng.exponential(1.0, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        rng = np.random.Generator(np.random.PCG64(seed_base + i))
        n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        rc = float(rng.uniform(5.0, 6.0))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        if i % 2 == 0:
            s = hcno_cluster(n, sub_seed)
        else:
            s = hcno_box(n, sub_seed)
        out.append({"structure": s, "cutoffs": cutoffs(rc), "arrival": float(arrivals[i])})
    return out
