"""Free-atom parameters (alpha0 [bohr^3], C6 [Ha bohr^6], R0 [bohr]) for H, C, N, O.

These are the reference free-atom values of the Tkatchenko-Scheffler scheme that
the method starts from (Sec. II.B, the TS polarisability and vdW-radius
definitions); the numbers are the ones the workload definitions fix.
"""
import numpy as np

# index -> (symbol, alpha0, C6, R0)
_TABLE = [
    ("H", 4.5, 6.5, 3.10),
    ("C", 12.0, 46.6, 3.59),
    ("N", 7.4, 24.2, 3.34),
    ("O", 5.4, 15.6, 3.19),
]

SPECIES_INDEX = {sym: i for i, (sym, *_rest) in enumerate(_TABLE)}
# (n_species, 3) float64: alpha0, c6, r0
SPECIES_TABLE = np.array([[a, c, r] for (_s, a, c, r) in _TABLE], dtype=np.float64)
