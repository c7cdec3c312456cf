"""FP64 CPU oracle for TD-aGW propagation with a dense or SVD-compressed kernel.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the HIP library is checked against.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the library never
does, and this package imports nothing from the library (the two share only
the seeded inputs in ``workloads``).

Modules, each following the paper's definitions step by step:
  kernel.py      direct (screened) electron-hole kernel on the lattice model
                 (Eq. sigma-from-k, Eq. bse-direct-def in its single-G limit)
  compress.py    K = K_diag + U M V^H truncated SVD (Eq. svd_diag_offdiag) and the
                 channel-wise truncated SVD (Eq. svd-channel-wise)
  propagate.py   RK4 integration of the TD-aGW equation of motion
                 (Eq. tdagw with Eq. sigma-from-k or Eq. svd_acc)
  observables.py polarisation, current, band occupation (Sec. SVD acceleration)
  bse.py         linearised operator (Bethe-Salpeter Hamiltonian) and the
                 linear-response solution used as a brute-force pin
  spectra.py     absorption and high-harmonic spectra from time series
  adjoint.py     reverse-mode derivative of the discrete RK4 propagation
                 (not in the paper; the exact gradient of the scheme above)
  intraband.py   intraband part of the length-gauge field coupling: covariant
                 k-derivative with parallel-transport links (Eq. tdagw, App. A.1)
"""

from .kernel import (  # noqa: F401
    pair_table, rytova_keldysh, cell_average_w0, fold_q, coulomb_matrix, build_kernel,
    kernel_element,
)
from .compress import (  # noqa: F401
    split_diag, svd_offdiag, choose_rank, compress, randomized_compress, channel_blocks, compress_channelwise,
)
from .propagate import field_at, DenseOp, LowRankOp, ChannelOp, propagate, rho_equilibrium  # noqa: F401
from .observables import observables  # noqa: F401
from .bse import linear_operator, linear_response  # noqa: F401
from .spectra import absorption, hhg  # noqa: F401
from .adjoint import propagate_adjoint, harmonic_loss, field_param_derivs  # noqa: F401
from .intraband import transport_links, covariant_derivative, polar_unitary, grid_spacing  # noqa: F401
