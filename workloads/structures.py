"""Seeded random structures built by random sequential addition (RSA).

Positions are drawn uniformly and a candidate is rejected when it lies closer
than ``dmin`` to an accepted atom (minimum image for periodic boxes).  All
generators take a numpy ``Generator`` so that every workload is reproducible.
"""
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .species import SPECIES_INDEX

AMU_G = 1.66053906660e-24  # g per atomic mass unit
MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999}


@dataclass
class Structure:
    pos: np.ndarray                 # (N, 3) float64, Angstrom
    species: np.ndarray             # (N,) int32 index into the species table
    nu: np.ndarray                  # (N,) float64 Hirshfeld-volume ratios
    cell: Optional[np.ndarray] = None   # (3, 3) float64 rows = lattice vectors, or None (open)
    pbc: np.ndarray = field(default_factory=lambda: np.zeros(3, dtype=bool))
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def copy(self) -> "Structure":
        return Structure(self.pos.copy(), self.species.copy(), self.nu.copy(),
                         None if self.cell is None else self.cell.copy(), self.pbc.copy(), self.name)


def number_density(g_cm3: float, fractions: dict) -> float:
    """Atoms per cubic Angstrom for a mass density and a composition."""
    mean_mass = sum(MASS[s] * f for s, f in fractions.items())
    return g_cm3 / (mean_mass * AMU_G) * 1e-24


def _rsa(n, sampler, dmin, lo, hi, periodic, rng, max_tries=200000):
    """Accept candidates from ``sampler`` that keep ``dmin`` to every accepted atom.

    The overlap test looks only at the 27 buckets (edge >= dmin) around the
    candidate; it is plain Python on floats, which is much faster than numpy on
    three-element arrays and takes the same decisions.
    """
    lo = [float(x) for x in lo]
    box = [float(hi[d]) - lo[d] for d in range(3)]
    nc = [max(1, int(math.floor(box[d] / dmin))) for d in range(3)]
    h = [box[d] / nc[d] for d in range(3)]
    offsets = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    buckets = {}
    acc = []
    d2min = dmin * dmin
    tries = 0
    while len(acc) < n:
        tries += 1
        if tries > max_tries + 50 * n:
            raise RuntimeError("RSA failed to place all atoms; density too high for dmin")
        p = sampler(rng).tolist()
        key = []
        for d in range(3):
            c = math.floor((p[d] - lo[d]) / h[d])
            key.append(c % nc[d] if periodic else min(max(c, 0), nc[d] - 1))
        clash = False
        for off in offsets:
            q = [key[0] + off[0], key[1] + off[1], key[2] + off[2]]
            if periodic:
                q = (q[0] % nc[0], q[1] % nc[1], q[2] % nc[2])
            elif min(q) < 0 or q[0] >= nc[0] or q[1] >= nc[1] or q[2] >= nc[2]:
                continue
            for j in buckets.get(tuple(q), ()):
                x = acc[j]
                dx, dy, dz = x[0] - p[0], x[1] - p[1], x[2] - p[2]
                if periodic:
                    dx -= box[0] * round(dx / box[0])
                    dy -= box[1] * round(dy / box[1])
                    dz -= box[2] * round(dz / box[2])
                if dx * dx + dy * dy + dz * dz < d2min:
                    clash = True
                    break
            if clash:
                break
        if clash:
            continue
        buckets.setdefault(tuple(key), []).append(len(acc))
        acc.append(p)
    return np.array(acc, dtype=np.float64).reshape(n, 3)


def rsa_box(n, length, dmin, rng):
    """n atoms in a periodic cube of edge ``length`` Angstrom."""
    sampler = lambda r: r.uniform(0.0, length, size=3)
    return _rsa(n, sampler, dmin, (0, 0, 0), (length,) * 3, True, rng)


def rsa_cube_open(n, length, dmin, rng):
    """n atoms in an open cube of edge ``length`` Angstrom (no periodic images)."""
    sampler = lambda r: r.uniform(0.0, length, size=3)
    return _rsa(n, sampler, dmin, (0, 0, 0), (length,) * 3, False, rng)


def rsa_sphere_open(n, radius, dmin, rng):
    """n atoms uniformly inside an open sphere of the given radius (Angstrom)."""

    def sampler(r):
        while True:
            p = r.uniform(-radius, radius, size=3)
            if p @ p <= radius * radius:
                return p

    return _rsa(n, sampler, dmin, (-radius,) * 3, (radius,) * 3, False, rng)


def hcno_species(n, rng):
    """Species indices for an H/C/N/O 50/30/10/10 mixture, shuffled.

    Counts: N and O are round(0.1 n), C is floor(0.3 n), H takes the rest.
    """
    n_n = int(round(0.1 * n))
    n_o = int(round(0.1 * n))
    n_c = int(np.floor(0.3 * n))
    n_h = n - n_n - n_o - n_c
    sp = np.concatenate([
        np.full(n_h, SPECIES_INDEX["H"]), np.full(n_c, SPECIES_INDEX["C"]),
        np.full(n_n, SPECIES_INDEX["N"]), np.full(n_o, SPECIES_INDEX["O"]),
    ]).astype(np.int32)
    rng.shuffle(sp)
    return sp
