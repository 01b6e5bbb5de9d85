"""Pulay mixing with a Kerker preconditioner on the GPU against the oracle's
(dcdft_set_mixer / OracleSCF.set_mixer), through the C ABI.

Both run the same SCF from the same start with the same mixer, free running:
per step every fragment's eigenvalues (1e-10 Ha), mu (1e-10 Ha), the density
(dV sum |d rho| / N_e <= 1e-9) and the paper's residual agree in FP64; the
mixed-precision path's energy stays within 1e-5 Ha per atom.  A failed step
restores the mixer's history with the rest of the state, and the retry matches a
context that never failed.  Argument checks of dcdft_set_mixer.
"""
import numpy as np
import pytest

import oracle
from tests.gpu_common import l1_over_ne, require_gpu
from tests.helpers import tiny_config
import workloads

pytestmark = pytest.mark.gpu


def _ragged():
    cfg = tiny_config(n_grid=(12, 12, 10), cell=(7.2, 7.2, 6.0), n_atoms=5, nstate=9,
                      num_fragment=(2, 2, 1), buffer=(2, 3, 0), smearing=0.05, valence=2.0)
    cfg.nstate_frag = np.array([9, 12, 7, 17], dtype=np.int32)
    return cfg


@pytest.mark.parametrize("which,steps", [("config1", 8), ("ragged", 10)])
def test_pulay_kerker_follows_the_oracle(which, steps):
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    cfg = workloads.config(1) if which == "config1" else _ragged()
    o = oracle.OracleSCF(cfg)
    o.set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
    with DCDFT.from_config(cfg) as d:
        d.dcdft_set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
        for k in range(steps):
            r, gi = o.step(), d.dcdft_scf_step()
            de = max(float(np.abs(d.dcdft_eigenvalues(f)[0] - o.eps[f]).max())
                     for f in range(cfg.n_fragments))
            l1 = l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne)
            print(which, k, f"R_paper {r['residual_paper']:.3e} {gi['residual_paper']:.3e} "
                  f"|d mu| {abs(r['mu'] - gi['mu']):.1e} |d eps| {de:.1e} L1 {l1:.1e}",
                  flush=True)
            assert abs(r["mu"] - gi["mu"]) <= 1e-10
            assert de <= 1e-10 and l1 <= 1e-9
            assert abs(r["residual_paper"] - gi["residual_paper"]) <= 1e-9 * max(
                1e-3, r["residual_paper"])
        rin = d.dcdft_get_field(2)
        assert l1_over_ne(rin, o.rho_in, o.dv, o.ne) <= 1e-9


def test_pulay_mixed_precision_energy():
    require_gpu()
    from paper_2606_21125_amd import DCDFT, PREC_MIXED
    cfg = workloads.config(1)
    o = oracle.OracleSCF(cfg)
    o.set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
    with DCDFT.from_config(cfg, precision=PREC_MIXED) as d:
        d.dcdft_set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
        for k in range(6):
            r, gi = o.step(), d.dcdft_scf_step()
            de = abs(r["e_total"] - gi["e_total"]) / cfg.system.n_atoms
            print("mixed", k, f"dE/atom {de:.2e}", flush=True)
            assert de <= 1e-5


def test_failed_step_restores_the_mixer_history():
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    from paper_2606_21125_amd.binding import DcdftError
    cfg = _ragged()
    with DCDFT.from_config(cfg) as d, DCDFT.from_config(cfg) as ref:
        for x in (d, ref):
            x.dcdft_set_mixer("pulay", alpha=0.3, q0=0.8, history=4)
        for _ in range(3):
            d.dcdft_scf_step()
            ref.dcdft_scf_step()
        good = d.dcdft_get_orbitals(1)
        bad = good.copy()
        bad[2] = 0.0
        d.dcdft_set_orbitals(1, bad)
        with pytest.raises(DcdftError) as e:
            d.dcdft_scf_step()
        assert e.value.status == -4
        d.dcdft_set_orbitals(1, good)
        for _ in range(3):
            gi, ri = d.dcdft_scf_step(), ref.dcdft_scf_step()
            for k in ("mu", "e_total", "residual_paper", "residual_out_in"):
                assert gi[k] == ri[k], k
        assert np.array_equal(d.dcdft_density(), ref.dcdft_density())


def test_set_mixer_arguments():
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    from paper_2606_21125_amd.binding import DcdftError
    cfg = tiny_config()
    with DCDFT.from_config(cfg) as d:
        for args in ((5, 0.3, 0.8, 8), (1, 0.0, 0.8, 8), (1, 1.5, 0.8, 8), (1, 0.3, -1.0, 8),
                     (1, 0.3, 0.8, 0), (1, 0.3, 0.8, 17), (1, 0.3, float("nan"), 8)):
            with pytest.raises(DcdftError) as e:
                d.dcdft_set_mixer(*args)
            assert e.value.status == -1
        d.dcdft_set_mixer("pulay", 0.3, 0.0, 3)
        d.dcdft_scf_step()
        d.dcdft_set_mixer("linear", 0.2)
        d.dcdft_scf_step()
