"""Checkpoint and resume of the SCF state through the C ABI (orbitals, rho_tot^in and
every rho_alpha^in): a context restored from a checkpoint continues the iteration
of the context that wrote it.  The restored context's chemical-potential solver
starts from its own previous value, so the results agree to rounding (the FP64
parity bounds), not bit for bit."""
import numpy as np
import pytest

from tests.gpu_common import require_gpu
from tests.test_gpu_parity import _ragged_tiny

pytestmark = pytest.mark.gpu


def test_checkpoint_resume_continues_the_iteration(tmp_path):
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    cfg = _ragged_tiny()
    path = str(tmp_path / "state.npz")
    with DCDFT.from_config(cfg) as a:
        for _ in range(3):
            a.dcdft_scf_step()
        a.save_state(path)
        with DCDFT.from_config(cfg) as b:
            b.load_state(path)
            for k in range(3):
                ia, ib = a.dcdft_scf_step(), b.dcdft_scf_step()
                assert abs(ia["mu"] - ib["mu"]) < 1e-10, k
                assert abs(ia["e_total"] - ib["e_total"]) < 1e-9, k
                for f in range(cfg.n_fragments):
                    np.testing.assert_allclose(b.dcdft_eigenvalues(f)[0],
                                               a.dcdft_eigenvalues(f)[0], rtol=0, atol=1e-10)
                ra, rb = a.dcdft_density(), b.dcdft_density()
                assert np.abs(ra - rb).sum() * float(np.prod(cfg.system.cell)) / ra.size \
                    / cfg.system.n_electrons < 1e-9


def test_checkpoint_of_another_shape_is_refused(tmp_path):
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    cfg = _ragged_tiny()
    path = str(tmp_path / "state.npz")
    with DCDFT.from_config(cfg) as a:
        a.save_state(path)
    cfg2 = _ragged_tiny()
    cfg2.nstate_frag = np.array([9, 12, 7, 16], dtype=np.int32)
    with DCDFT.from_config(cfg2) as b:
        with pytest.raises(ValueError):
            b.load_state(path)
