"""Seeded synthetic inputs for the lMBD hot path.

This package only *generates inputs*: atomic structures (positions, species,
Hirshfeld-volume ratios, cells), the free-atom parameter tables, and the
frequency quadrature grid that the caller hands to the method.  It contains
none of the method's arithmetic, so both the CPU oracle and the GPU path can
use it without sharing any computation.
"""
from .structures import Structure, rsa_box, rsa_cube_open, rsa_sphere_open, hcno_species
from .species import SPECIES_TABLE, SPECIES_INDEX
from .grid import frequency_grid
from .configs import (config_small_open, config_plain_pbc, config_diff_hcno, config_mixed_pbc,
                      serving_requests, DEFAULT_PARAMS)

__all__ = [
    "Structure", "rsa_box", "rsa_cube_open", "rsa_sphere_open", "hcno_species",
    "SPECIES_TABLE", "SPECIES_INDEX", "frequency_grid",
    "config_small_open", "config_plain_pbc", "config_diff_hcno", "config_mixed_pbc",
    "serving_requests", "DEFAULT_PARAMS",
]
