"""Seeded random structures built by random sequential addition (RSA).

Positions are drawn uniformly and a candidate is rejected when it lies closer
than ``dmin`` to an accepted atom (minimum image for periodic boxes).  All
generators take a numpy ``Generator`` so that every workload is reproducible.
"""
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


class _Grid:
    """Bucket grid used only to speed up the RSA overlap test."""

    def __init__(self, lo, hi, cell_size, periodic):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.span = np.asarray(hi, dtype=np.float64) - self.lo
        self.nc = np.maximum(1, np.floor(self.span / cell_size).astype(int))
        self.h = self.span / self.nc
        self.periodic = periodic
        self.buckets = {}

    def key(self, p):
        c = np.floor((p - self.lo) / self.h).astype(int)
        if self.periodic:
            c %= self.nc
        else:
            c = np.clip(c, 0, self.nc - 1)
        return tuple(c)

    def near(self, p):
        c = np.array(self.key(p))
        out = []
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    q = c + (dx, dy, dz)
                    if self.periodic:
                        q %= self.nc
                    elif np.any(q < 0) or np.any(q >= self.nc):
                        continue
                    out.extend(self.buckets.get(tuple(q), ()))
        return out

    def add(self, idx, p):
        self.buckets.setdefault(self.key(p), []).append(idx)


def _rsa(n, sampler, dmin, lo, hi, periodic, rng, max_tries=200000):
    box = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    grid = _Grid(lo, hi, dmin, periodic)
    pos = np.empty((n, 3), dtype=np.float64)
    count = 0
    tries = 0
    d2min = dmin * dmin
    while count < n:
        tries += 1
        if tries > max_tries + 50 * n:
            raise RuntimeError("RSA failed to place all atoms; density too high for dmin")
        p = sampler(rng)
        cand = grid.near(p)
        if cand:
            d = pos[cand] - p
            if periodic:
                d -= box * np.round(d / box)
            if np.min(np.einsum("ij,ij->i", d, d)) < d2min:
                continue
        pos[count] = p
        grid.add(count, p)
        count += 1
    return pos


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
