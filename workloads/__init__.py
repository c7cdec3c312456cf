"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package is the only code both sides use.  It produces the data the
method takes as given (Appendix A of the paper: quasiparticle energies, the
dipole matrix in a smooth gauge, the wavefunctions the kernel is built from,
and the driving fields), here from small lattice models that stand in for the
paper's ab initio MoS2 inputs.  It holds none of the method's arithmetic:
no kernel elements, no SVD, no equation of motion, no field evaluation and
no observables.
"""

from .models import (  # noqa: F401
    multiband_model, flat_band_model, diagonal_band_model,
    HARTREE_EV, FS_AU, BOHR_NM, EFIELD_AU_V_PER_CM,
    Model, mp_grid, dirac_model, tb4_model, load_tb4_table,
)
from .fields import FieldTable  # noqa: F401
from .configs import CONFIGS, get_config, Workload  # noqa: F401
