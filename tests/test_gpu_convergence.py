"""lMBD converges to full MBD as the cutoff grows (Sec. III.A: r_MBD is the central
convergence parameter; Sec. IV).  Config 1 (64 carbon atoms in an open 12 A cube,
largest interatomic distance 16.1 A): the GPU's total lMBD energy at
r_SCS = r_MBD = r_c for r_c from 5 to 22 A, against the oracle's whole-system MBD
(whole-system SCS, the same series order n_max = 6, and the exact log-det for
context).  From r_c = 18 A on every neighbourhood is the whole system, clear of
the buffers, so the two agree to round-off; the curve is printed for the record."""
import numpy as np
import pytest

import oracle
from workloads import SPECIES_TABLE
from workloads import configs as C
from tests.gpu_common import gpu_run, GRID

pytestmark = pytest.mark.gpu

RADII = [5.0, 6.0, 8.0, 10.0, 12.0, 14.0, 16.0, 18.0, 20.0, 22.0]


def test_lmbd_converges_to_full_mbd():
    st, _ = C.config_small_open()
    span = np.linalg.norm(st.pos[:, None] - st.pos[None], axis=-1).max()
    assert span < RADII[-1] - 1.0
    e_series, _ = oracle.full_mbd(st.pos, st.species, st.nu, SPECIES_TABLE, GRID[0], GRID[1], n_max=6)
    e_log, _ = oracle.full_mbd(st.pos, st.species, st.nu, SPECIES_TABLE, GRID[0], GRID[1], n_max=None)
    print(f"full MBD: series n_max = 6 {e_series:.10f} eV, log-det {e_log:.10f} eV", flush=True)
    errs = []
    for rc in RADII:
        cut = dict(r_scs=rc, r_nbr=rc, r_mbd1=rc, r_mbd2=rc)
        e = gpu_run(st, cut, forces=False)["energies"].sum()
        errs.append(abs(e / e_series - 1.0))
        print(f"  r_c {rc:5.1f} A: lMBD {e:.10f} eV, relative difference from full MBD {errs[-1]:.3e}", flush=True)
    assert errs[-1] < 1e-10                    # whole-system neighbourhoods: full MBD
    assert max(errs[-4:]) < min(errs[:3])      # the large cutoffs are closer than the small ones
