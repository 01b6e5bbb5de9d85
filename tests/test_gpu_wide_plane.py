"""Fragment boxes whose x-y plane has more than 1024 points (one thread per point
no longer fits a workgroup): the stencil runs plane-tiled (32 x 16 point tiles
with a periodic halo), and the fused <x, Hx> of the CG sweep takes a pass of its
own.  Checked against the oracle on planes that are ragged against the tiles
(40 x 36 points):
  * H psi of a one-fragment cell, FP64 (relative 1e-12) and FP32 (2e-6);
  * DC SCF steps of two fragments with 40 x 36 x 12 boxes and 12 and 21 orbitals
    (two tile classes; FP64 step bounds, and the mixed path's energy);
  * one wide fragment with 90 orbitals (the large-orbital path on a tiled plane)."""
import numpy as np
import pytest

import oracle
from oracle import solver as osol
from paper_2606_21125_amd.binding import FFIELD_VEFF
from tests.gpu_common import l1_over_ne, require_gpu
from tests.helpers import tiny_config

pytestmark = pytest.mark.gpu


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


def _wide(nstate, num_fragment=(1, 1, 1), buffer=(0, 0, 0), n_grid=(40, 36, 8)):
    return tiny_config(n_grid=n_grid, cell=(20.0, 18.0, 0.5 * n_grid[2]), n_atoms=8,
                       nstate=nstate, num_fragment=num_fragment, buffer=buffer, valence=2.0,
                       smearing=0.05)


@pytest.mark.parametrize("prec", [0, 1])
def test_wide_plane_apply_h(prec):
    require_gpu()
    import torch
    cfg = _wide(12)
    o = oracle.OracleSCF(cfg)
    rng = np.random.default_rng(3)
    tdt, tol = (torch.float64, 1e-12) if prec == 0 else (torch.float32, 2e-6)
    with _gpu(cfg, precision=prec) as d:
        shape = o.frags[0].shape
        assert shape[1] * shape[2] > 1024
        veff = d.dcdft_get_fragment_field(0, FFIELD_VEFF).reshape(shape)
        m = 37                                   # a chunk of 16-vector tiles and a tail
        x = rng.normal(size=(m,) + shape)
        if prec == 1:
            x = x.astype(np.float32).astype(np.float64)
        ref = osol.apply_h(x, veff, o.fproj[0], o.h, o.dv).reshape(m, -1)
        xt = torch.tensor(x.reshape(m, -1), device="cuda", dtype=tdt)
        yt = torch.empty_like(xt)
        d.dcdft_apply_h(0, xt, yt, prec=prec)
        err = np.abs(yt.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"wide-plane H psi, prec {prec}: relative {err:.2e}", flush=True)
        assert err <= tol


@pytest.mark.parametrize("cfg_kind", ["dc", "large"])
def test_wide_plane_scf_steps_match_oracle(cfg_kind):
    require_gpu()
    if cfg_kind == "dc":
        cfg = _wide(12, num_fragment=(1, 1, 2), buffer=(0, 0, 2), n_grid=(40, 36, 16))
        cfg.nstate_frag = np.array([12, 21], dtype=np.int32)   # two tile classes
    else:
        cfg = _wide(90)
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg) as d:
        for k in range(3):
            ri, gi = o.step(), d.dcdft_scf_step()
            print(cfg_kind, k, ri["mu"], gi["mu"], flush=True)
            assert abs(ri["mu"] - gi["mu"]) < 1e-10
            for f in range(cfg.n_fragments):
                eps, w = d.dcdft_eigenvalues(f)
                np.testing.assert_allclose(eps, o.eps[f], rtol=0, atol=1e-10)
                np.testing.assert_allclose(w, o.w[f], rtol=0, atol=1e-9)
            assert l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne) < 1e-9
            assert abs(ri["e_total"] - gi["e_total"]) < 1e-8 * max(1.0, abs(ri["e_total"]))


def test_wide_plane_mixed_precision_energy():
    """The FP32 path on the wide DC boxes (tiled stencil and its dot pass in FP32):
    total energy within 1e-5 Ha per atom of the oracle over three steps."""
    require_gpu()
    cfg = _wide(12, num_fragment=(1, 1, 2), buffer=(0, 0, 2), n_grid=(40, 36, 16))
    cfg.nstate_frag = np.array([12, 21], dtype=np.int32)
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg, precision=1) as d:
        for k in range(3):
            ri, gi = o.step(), d.dcdft_scf_step()
            de = abs(ri["e_total"] - gi["e_total"]) / cfg.system.n_atoms
            print(f"wide mixed step {k}: dE/atom {de:.2e}", flush=True)
            assert de <= 1e-5
