"""Density-template potential V^alpha = (rho_alpha^in - rho_tot^in) / xi (Eq. (5)) on
the GPU against the FP64 oracle with the same xi: in the SCF iteration (where it
acts on buffer points) and in fixed-density mode with fragment densities that
differ from the total one everywhere.  Tolerances as for the SCF step: V_eff 1e-11
relative to its largest value, eigenvalues and mu 1e-10 Ha, density
dV sum |d rho| / N_e <= 1e-9."""
import math

import numpy as np
import pytest

import oracle
from tests.gpu_common import l1_over_ne, require_gpu
from tests.test_gpu_parity import _ragged_tiny
import workloads

pytestmark = pytest.mark.gpu


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


def _check_step(o, d, ri, gi, cfg, tag):
    print(tag, ri["mu"], gi["mu"], ri["e_total"], gi["e_total"])
    assert abs(ri["mu"] - gi["mu"]) < 1e-10
    for frag in range(cfg.n_fragments):
        eps, w = d.dcdft_eigenvalues(frag)
        np.testing.assert_allclose(eps, o.eps[frag], rtol=0, atol=1e-10)
        np.testing.assert_allclose(w, o.w[frag], rtol=0, atol=1e-9)
    assert l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne) < 1e-9
    assert abs(ri["e_total"] - gi["e_total"]) < 1e-8 * max(1.0, abs(ri["e_total"]))
    assert abs(ri["residual_paper"] - gi["residual_paper"]) < 1e-9


@pytest.mark.parametrize("which,steps", [("ragged", 5), ("config1", 3)])
def test_template_scf_steps_match_oracle(which, steps):
    require_gpu()
    from paper_2606_21125_amd.binding import FFIELD_VEFF
    cfg = workloads.config(1) if which == "config1" else _ragged_tiny()
    xi = 0.2
    o = oracle.OracleSCF(cfg)
    o.template_xi = xi
    with _gpu(cfg) as d:
        d.dcdft_set_template(xi)
        for k in range(steps):
            # the oracle's V_eff of this step, formed from its input densities
            v_h = oracle.scf.poisson_fd(o.rho_in, o.h)
            refs = [o.veff(frag, v_h) for frag in range(cfg.n_fragments)]
            ri, gi = o.step(), d.dcdft_scf_step()
            _check_step(o, d, ri, gi, cfg, f"{which} step {k}")
            for frag in range(cfg.n_fragments):
                got = d.dcdft_get_fragment_field(frag, FFIELD_VEFF)
                scale = max(1.0, np.abs(refs[frag]).max())
                assert np.abs(got - refs[frag]).max() < 1e-11 * scale, frag


def test_template_in_fixed_density_mode():
    """Frozen total density and fragment densities modulated against it: V_eff with
    the template term, then fixed-density steps, against the oracle."""
    require_gpu()
    from paper_2606_21125_amd.binding import FFIELD_VEFF
    cfg = _ragged_tiny()
    rho = workloads.superposed_density(cfg.system, cfg.n_grid)
    o = oracle.OracleSCF(cfg)
    rho_frag = []
    for a, f in enumerate(o.frags):
        t = np.arange(f.n) / f.n
        rho_frag.append(rho.ravel()[f.global_index] * (1.0 + 0.2 * np.sin(2 * math.pi * 7 * t + a)))
    xi = 0.1
    o.fixed_density = True
    o.template_xi = xi
    o.set_density(rho, rho_frag)
    with _gpu(cfg) as d:
        d.dcdft_set_density(rho, np.concatenate(rho_frag))
        d.dcdft_fix_density(True)
        d.dcdft_set_template(xi)
        v_h = oracle.scf.poisson_fd(rho, o.h)
        for frag in range(cfg.n_fragments):
            ref = o.veff(frag, v_h)
            got = d.dcdft_get_fragment_field(frag, FFIELD_VEFF)
            assert np.abs(got - ref).max() < 1e-11 * max(1.0, np.abs(ref).max()), frag
        for k in range(4):
            ri, gi = o.step(), d.dcdft_scf_step()
            assert gi["residual_paper"] == 0.0
            _check_step(o, d, ri, gi, cfg, f"fixed+template step {k}")
        # switching the template off in fixed-density mode re-forms V_eff at once
        d.dcdft_set_template(0.0)
        o.template_xi = 0.0
        for frag in range(cfg.n_fragments):
            ref = o.veff(frag, v_h)
            got = d.dcdft_get_fragment_field(frag, FFIELD_VEFF)
            assert np.abs(got - ref).max() < 1e-11 * max(1.0, np.abs(ref).max()), frag


def test_template_off_is_the_plain_step_and_bad_xi_is_rejected():
    require_gpu()
    from paper_2606_21125_amd.binding import load_library
    cfg = _ragged_tiny()
    with _gpu(cfg) as a, _gpu(cfg) as b:
        b.dcdft_set_template(0.3)
        b.dcdft_set_template(0.0)
        lib = load_library()
        assert lib.dcdft_set_template(b.ctx, -1.0) == -1
        assert lib.dcdft_set_template(b.ctx, float("nan")) == -1
        assert lib.dcdft_set_template(b.ctx, float("inf")) == -1
        for k in range(3):
            ia, ib = a.dcdft_scf_step(), b.dcdft_scf_step()
            assert ia["mu"] == ib["mu"] and ia["e_total"] == ib["e_total"], k
            assert np.array_equal(a.dcdft_density(), b.dcdft_density()), k
