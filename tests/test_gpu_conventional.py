"""Conventional Kohn-Sham DFT on the same kernels: one fragment covering the cell
with no buffer (the core is the whole cell, so Eqs. (2)-(4) reduce to the ordinary
density and the fragment Hamiltonian to the global one), ceil(1.2 N_e / 2) orbitals.
The oracle in this configuration is pinned to an independent dense-diagonalisation
SCF (tests/test_oracle_scf.py); here the GPU follows it step by step.  Tolerances
as for the SCF step (FP64), and 1e-5 Ha per atom for the mixed path's energy."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import l1_over_ne, require_gpu
import workloads

pytestmark = pytest.mark.gpu


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


@pytest.mark.parametrize("cells,steps", [((1, 1, 1), 8), ((2, 2, 1), 3)])
def test_conventional_steps_match_oracle(cells, steps):
    require_gpu()
    cfg = workloads.si_cells_config(cells)
    assert cfg.n_fragments == 1 and cfg.fragment_shape == tuple(cfg.n_grid)
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg) as d:
        for k in range(steps):
            ri, gi = o.step(), d.dcdft_scf_step()
            print(cfg.name, k, ri["mu"], gi["mu"], ri["residual_paper"])
            assert abs(ri["mu"] - gi["mu"]) < 1e-10
            eps, w = d.dcdft_eigenvalues(0)
            np.testing.assert_allclose(eps, o.eps[0], rtol=0, atol=1e-10)
            # the core is the whole cell: every core weight is 1
            np.testing.assert_allclose(w, np.ones_like(w), rtol=0, atol=1e-12)
            assert l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne) < 1e-9
            assert abs(ri["e_total"] - gi["e_total"]) < 1e-8 * max(1.0, abs(ri["e_total"]))


def test_conventional_mixed_precision():
    require_gpu()
    cfg = workloads.si_cells_config((2, 2, 1))
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg, precision=1) as d:
        for k in range(3):
            ri, gi = o.step(), d.dcdft_scf_step()
            de = abs(ri["e_total"] - gi["e_total"]) / cfg.system.n_atoms
            print(f"mixed conventional step {k}: dE/atom {de:.2e}")
            assert de <= 1e-5


def test_orbital_limit_is_reported():
    """More than 80 orbitals in a fragment is outside the kernels' register and LDS
    tiles: setup reports it as an argument error rather than running."""
    require_gpu()
    from paper_2606_21125_amd.binding import DcdftError
    cfg = workloads.si_cells_config((2, 2, 2))       # 154 orbitals in one fragment
    with pytest.raises(DcdftError):
        _gpu(cfg)
