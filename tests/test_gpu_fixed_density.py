"""Fixed-density DC (Sec. 2.6, third usage; Sec. 3.2) on the GPU against the FP64
oracle in the same mode: both read the same frozen density (atom-centred Gaussians,
a stand-in for a density file), then iterate the fragment eigensolvers in its
potential without Poisson, V_eff or mixing updates.

Tolerances as for the SCF step (FP64 path): eigenvalues and mu 1e-10 Ha, core
weights 1e-9, density dV sum |d rho| / N_e <= 1e-9; the frozen rho^in must come
back bitwise, and the paper's residual must be exactly 0.  Mixed path: E_tot
within 1e-5 Ha per atom.
"""
import numpy as np
import pytest

import oracle
from oracle.scf import poisson_fd
from tests.gpu_common import l1_over_ne, require_gpu
from tests.test_gpu_parity import _ragged_tiny
import workloads

pytestmark = pytest.mark.gpu


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


def _frozen(cfg):
    return workloads.superposed_density(cfg.system, cfg.n_grid)


def _compare(o, d, ri, gi, cfg, tag, fixed=True):
    print(tag, ri["mu"], gi["mu"], ri["e_total"], gi["e_total"], gi["residual_out_in"])
    if fixed:
        assert gi["residual_paper"] == 0.0
    else:
        assert abs(ri["residual_paper"] - gi["residual_paper"]) < 1e-9
    assert abs(ri["mu"] - gi["mu"]) < 1e-10
    assert abs(gi["charge"] - o.ne) < 1e-9 * o.ne
    for frag in range(cfg.n_fragments):
        eps, w = d.dcdft_eigenvalues(frag)
        np.testing.assert_allclose(eps, o.eps[frag], rtol=0, atol=1e-10)
        np.testing.assert_allclose(w, o.w[frag], rtol=0, atol=1e-9)
    assert l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne) < 1e-9
    assert abs(ri["e_total"] - gi["e_total"]) < 1e-8 * max(1.0, abs(ri["e_total"]))
    assert abs(ri["residual_out_in"] - gi["residual_out_in"]) < 1e-9


@pytest.mark.parametrize("which,steps", [("ragged", 5), ("config1", 3)])
def test_fixed_density_steps_match_oracle(which, steps):
    require_gpu()
    from paper_2606_21125_amd.binding import FFIELD_RHO_IN, FIELD_RHO_IN, FIELD_VH
    cfg = workloads.config(1) if which == "config1" else _ragged_tiny()
    rho = _frozen(cfg)
    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.set_density(rho)
    vh_ref = poisson_fd(rho, o.h)
    with _gpu(cfg) as d:
        d.dcdft_set_density(rho)
        d.dcdft_fix_density(True)
        frag_in = [d.dcdft_get_fragment_field(f, FFIELD_RHO_IN) for f in range(cfg.n_fragments)]
        for f in range(cfg.n_fragments):
            assert np.array_equal(frag_in[f], o.rho_frag_in[f]), f
        vh0 = d.dcdft_get_field(FIELD_VH)
        assert np.abs(vh0 - vh_ref).max() < 1e-11 * max(1.0, np.abs(vh_ref).max())
        for k in range(steps):
            _compare(o, d, o.step(), d.dcdft_scf_step(), cfg, f"{which} step {k}")
            assert np.array_equal(d.dcdft_get_field(FIELD_RHO_IN), rho)
            assert np.array_equal(d.dcdft_get_field(FIELD_VH), vh0)
            for f in range(cfg.n_fragments):
                assert np.array_equal(d.dcdft_get_fragment_field(f, FFIELD_RHO_IN), frag_in[f])


def test_fix_and_release_after_scf_steps():
    """Fixing after ordinary SCF steps freezes the density the last step mixed (its
    potentials are formed at the switch); releasing resumes the SCF iteration with
    Poisson and mixing.  The batched step graph is re-captured at each switch, and
    plain per-fragment launches give the same numbers bit for bit."""
    require_gpu()
    cfg = _ragged_tiny()
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg, batched=1) as d, _gpu(cfg, batched=0) as p:
        plan = [False, False, True, True, True, False, False]
        prev = None
        for k, fixed in enumerate(plan):
            if fixed != prev:
                o.fixed_density = fixed
                d.dcdft_fix_density(fixed)
                p.dcdft_fix_density(fixed)
                prev = fixed
            ri, gi, pi = o.step(), d.dcdft_scf_step(), p.dcdft_scf_step()
            if not fixed:
                assert abs(ri["residual_paper"] - cfg.mixing * ri["residual_out_in"]) < 1e-13
            _compare(o, d, ri, gi, cfg, f"step {k} fixed={fixed}", fixed)
            assert gi["mu"] == pi["mu"] and gi["e_total"] == pi["e_total"], k
            assert np.array_equal(d.dcdft_density(), p.dcdft_density()), k


def test_fixed_density_mixed_precision():
    require_gpu()
    cfg = workloads.config(1)
    rho = _frozen(cfg)
    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.set_density(rho)
    nat = cfg.system.n_atoms
    with _gpu(cfg, precision=1) as d:
        d.dcdft_set_density(rho)
        d.dcdft_fix_density(True)
        for k in range(4):
            ri, gi = o.step(), d.dcdft_scf_step()
            de = abs(ri["e_total"] - gi["e_total"]) / nat
            deps = max(np.abs(d.dcdft_eigenvalues(f)[0] - o.eps[f]).max()
                       for f in range(cfg.n_fragments))
            drho = l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne)
            print(f"mixed fixed step {k}: dE/atom {de:.2e} deps {deps:.2e} drho {drho:.2e}")
            assert gi["residual_paper"] == 0.0
            assert de <= 1e-5
            assert abs(ri["mu"] - gi["mu"]) <= 1e-4 and deps <= 1e-4 and drho <= 1e-4


def test_fix_density_rejects_bad_flag():
    """A flag other than 0 or 1 is an argument error and leaves the mode unchanged."""
    require_gpu()
    from paper_2606_21125_amd.binding import load_library
    cfg = _ragged_tiny()
    with _gpu(cfg) as d:
        lib = load_library()
        assert lib.dcdft_fix_density(d.ctx, 2) == -1
        assert lib.dcdft_fix_density(d.ctx, -1) == -1
        assert lib.dcdft_fix_density(None, 1) == -1
        info = d.dcdft_scf_step()
        assert info["residual_paper"] > 0.0
