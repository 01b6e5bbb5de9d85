"""Plain FP64 CPU oracle of the divide-and-conquer DFT SCF step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls it, and it shares no code, table or constant generator with the
HIP library: both follow the paper (Sec. 2.2, Eqs. (1)-(5); the DC-LCFO
post-processing of Sec. 2.3, Eqs. (6)-(9)) and the readings
listed in the design notes, independently.

Layout conventions: global arrays are numpy arrays of shape (Nz, Ny, Nx)
(x fastest in memory); fragment orbital blocks have shape (m, nz, ny, nx).
Inner products carry the volume element: <x, y> = dV * sum(x * y).

Parity status of each function is stated in its docstring; functions without
an independent pin say "parity unpinned".
"""
from .rng import splitmix64_uniform, initial_orbitals  # noqa: F401
from .grid import (fd_second_derivative_coefficients, laplacian_periodic,  # noqa: F401
                   FragmentMap, build_fragments)
from .model import (local_potential, kb_projectors, fragment_projectors,  # noqa: F401
                    lda_pz81)
from .solver import (apply_h, apply_h_local, kb_project, cholesky_orthonormalize,  # noqa: F401
                     cg_eigensolver, core_weights, fermi_occupation,
                     fermi_level, fragment_density)
from .scf import (poisson_fd, poisson_fd_cg, OracleSCF, total_energy)  # noqa: F401
from .grad import band_energy, band_energy_grad  # noqa: F401
from .lcfo import lcfo_basis, lcfo_hamiltonian  # noqa: F401
