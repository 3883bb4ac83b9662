"""Plain FP64 CPU oracle for the atom-wise (linear-scaling) MBD method.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct reference
that the GPU path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2407_06409_amd``) never imports, calls or links anything here, and this
package shares no code with it.

Modules
-------
lmbd      per-atom lMBD energies and exact forces (torch, float64, CPU autograd);
          the paper's approximate forces (Sec. III.D) as a separate function;
          the eigenvalue-bounded polynomial fit of ln(1 - x) (Sec. III.A) with its
          Lanczos spectrum bounds
full_mbd  whole-system MBD with whole-system SCS (numpy, float64): the limit
          that lMBD must reach when the cutoffs cover the whole molecule
"""
from .lmbd import (OracleParams, make_params, neighbourhood, free_atom_terms, lmbd_energies,
                   lmbd_energy_forces, lmbd_paper_forces, lmbd_spectrum_bounds, scs_central,
                   PolarisationCatastrophe, BOHR, HARTREE)
from .full_mbd import full_mbd, full_scs

__all__ = ["OracleParams", "make_params", "neighbourhood", "free_atom_terms", "lmbd_energies",
           "lmbd_energy_forces", "lmbd_paper_forces", "lmbd_spectrum_bounds",
           "PolarisationCatastrophe", "scs_central", "full_mbd", "full_scs", "BOHR", "HARTREE"]
