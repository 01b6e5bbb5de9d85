"""Edge sizes of the fragment eigenproblem against the FP64 oracle: the largest
orbital count the kernels hold (80 = five 16-wide tiles), a single orbital (1 x 1
Gram, Cholesky and eigenproblem; capacity exactly N_e, so mu sits at the top of the
bracket, where mu itself is not unique and is not compared), and orbital counts on and next to tile boundaries in one batch.
Tolerances as for the SCF step."""
import numpy as np
import pytest

import oracle
from tests.gpu_common import l1_over_ne, require_gpu
from tests.helpers import tiny_config
import workloads

pytestmark = pytest.mark.gpu


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


def _follow(cfg, steps, check_mu=True):
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg) as d:
        for k in range(steps):
            ri, gi = o.step(), d.dcdft_scf_step()
            print(cfg.name, k, ri["mu"], gi["mu"])
            if check_mu:
                assert abs(ri["mu"] - gi["mu"]) < 1e-10
            for f in range(cfg.n_fragments):
                np.testing.assert_allclose(d.dcdft_eigenvalues(f)[0], o.eps[f], rtol=0,
                                           atol=1e-10)
            assert l1_over_ne(d.dcdft_density(), o.rho_out, o.dv, o.ne) < 1e-9
            assert abs(ri["e_total"] - gi["e_total"]) < 1e-8 * max(1.0, abs(ri["e_total"]))


def test_largest_orbital_count():
    require_gpu()
    _follow(workloads.config(1, nstate=80), 2)


def test_single_orbital_exact_capacity():
    require_gpu()
    cfg = tiny_config(n_grid=(12, 12, 12), cell=(7.2, 7.2, 7.2), n_atoms=1, nstate=1,
                      valence=2.0, smearing=0.05)
    # every mu far enough above the one eigenvalue gives N_e to rounding, so mu is
    # not unique here; the occupation (1 to rounding), density and energy are
    _follow(cfg, 3, check_mu=False)


def test_tile_boundary_counts_in_one_batch():
    require_gpu()
    cfg = tiny_config(n_grid=(12, 12, 10), cell=(7.2, 7.2, 6.0), n_atoms=5, nstate=16,
                      num_fragment=(2, 2, 1), buffer=(2, 3, 0), smearing=0.05, valence=2.0)
    cfg.nstate_frag = np.array([16, 32, 15, 33], dtype=np.int32)
    _follow(cfg, 3)


def test_no_atoms_reaches_the_closed_form_spectrum():
    """No atoms (an empty projector table and V_loc = 0), two electrons in the k = 0
    state: the density stays uniform, so V_H = 0 and V_xc is the constant of the
    uniform density, and the CG eigensolver must reach the closed-form spectrum of
    the nine-point Laplacian, eps(k) = sum_d (-c0 - 2 sum_j c_j cos(2 pi j k_d / n_d))
    / (2 h^2), shifted by that constant."""
    require_gpu()
    import math
    from oracle.grid import FD_COEFFS
    from oracle.model import lda_pz81
    from paper_2606_21125_amd import DCDFT
    from workloads.systems import SI
    n, L = 10, 5.0
    h = L / n
    c = FD_COEFFS
    lam1 = np.array([(-c[0] - 2 * sum(c[j] * math.cos(2 * math.pi * j * k / n)
                                      for j in range(1, 5))) / (2 * h * h) for k in range(n)])
    spec = np.sort((lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]).ravel())
    ne = 2.0
    _, vxc = lda_pz81(np.array([ne / L ** 3]))
    with DCDFT((n, n, n), (L, L, L), (1, 1, 1), (0, 0, 0), np.zeros((0, 3)),
               np.zeros(0, dtype=np.int32), [SI], np.array([7], dtype=np.int32), ne,
               smearing=0.05, cg_sweeps=6) as d:
        d.dcdft_fix_density(True)
        for _ in range(40):
            info = d.dcdft_scf_step()
        eps, w = d.dcdft_eigenvalues(0)
        np.testing.assert_allclose(eps, spec[:7] + vxc[0], rtol=0, atol=1e-10)
        np.testing.assert_allclose(w, np.ones(7), rtol=0, atol=1e-12)
        assert abs(info["charge"] - ne) < 1e-12


def test_shift_by_one_core_permutes_the_fragments():
    """Moving every atom and the frozen density by one core length along x maps
    fragment (ax, ay, az) onto ((ax + 1) mod 2, ay, az): after the fragment
    eigensolvers have converged in that fixed potential, each fragment's lowest
    eigenvalues equal those of its image (a check of the box geometry, periodic
    wrap, projector tables and gathers that needs no oracle)."""
    require_gpu()
    from paper_2606_21125_amd import DCDFT
    cfg = workloads.config(1)
    sysm = cfg.system
    nx = cfg.n_grid[0]
    ncore = nx // cfg.num_fragment[0]
    h = sysm.cell[0] / nx
    rho = workloads.superposed_density(sysm, cfg.n_grid)
    pos_s = sysm.positions.copy()
    pos_s[:, 0] = np.mod(pos_s[:, 0] + ncore * h, sysm.cell[0])
    rho_s = np.roll(rho, ncore, axis=2)
    eps = []
    for pos, rh in ((sysm.positions, rho), (pos_s, rho_s)):
        with DCDFT(cfg.n_grid, sysm.cell, cfg.num_fragment, cfg.num_rgrid_buffer, pos,
                   sysm.species_index, sysm.species, cfg.nstate_frag, sysm.n_electrons,
                   smearing=cfg.smearing, cg_sweeps=8) as d:
            d.dcdft_set_density(rh)
            d.dcdft_fix_density(True)
            for _ in range(30):
                d.dcdft_scf_step()
            eps.append([d.dcdft_eigenvalues(f)[0] for f in range(cfg.n_fragments)])
    for f in range(cfg.n_fragments):
        ax, ay, az = f % 2, (f // 2) % 2, f // 4
        fs = (ax + 1) % 2 + 2 * (ay + 2 * az)
        np.testing.assert_allclose(eps[1][fs][:48], eps[0][f][:48], rtol=0, atol=1e-8)


def test_fragment_hamiltonian_is_symmetric_on_the_gpu():
    """<x, H y> = <H x, y> for the fragment Hamiltonian applied by the library
    (periodic stencil, diagonal V_eff, symmetric rank-A projector term)."""
    require_gpu()
    import torch
    cfg = workloads.config(1)
    rng = np.random.default_rng(8)
    with _gpu(cfg) as d:
        d.dcdft_scf_step()
        for frag in (0, 5):
            info = d.dcdft_fragment_info(frag)
            n = int(np.prod(info["shape"]))
            x = torch.tensor(rng.normal(size=(2, n)), device="cuda")
            hx = torch.empty_like(x)
            d.dcdft_apply_h(frag, x, hx)
            a = float((x[0] * hx[1]).sum())
            b = float((hx[0] * x[1]).sum())
            assert abs(a - b) <= 1e-12 * max(abs(a), float((x[0] * hx[0]).sum()))


def test_projector_support_boundary_on_grid_points():
    """Atoms on grid points with a support radius of exactly three grid spacings
    (h = 0.5 bohr, R_cut = 1.5): 30 of each atom's 123 support points lie at
    r^2 = R_cut^2 exactly, where beta is still a third of its peak.  The GPU's
    support masks (FP64 r^2 = (dz^2 + dy^2) + dx^2 <= R_cut^2, the oracle's order)
    must keep the same points as the oracle: H psi on every fragment against the
    oracle at 1e-12 (FP64) and 1e-5 (FP32) relative, and two SCF steps followed."""
    require_gpu()
    import torch
    from workloads.systems import RunConfig, Species, System
    from paper_2606_21125_amd import PREC_MIXED
    sp = Species("X", 2.0, -3.0, 1.0, 1.0, 1.0, 1.5)
    pos = np.array([[1.5, 2.0, 3.0], [4.0, 4.5, 0.5]])
    sysm = System(np.array([6.0, 6.0, 6.0]), pos, np.zeros(2, dtype=np.int32), [sp])
    cfg = RunConfig("boundary", sysm, (12, 12, 12), (2, 2, 1), (2, 2, 0),
                    np.full(4, 8, dtype=np.int32), smearing=0.05, seed=3)
    o = oracle.OracleSCF(cfg)
    rng = np.random.default_rng(12)
    v_h = np.zeros_like(o.rho_in)
    with _gpu(cfg) as d:
        for f in range(cfg.n_fragments):
            shape = o.frags[f].shape
            psi = rng.normal(size=(5,) + shape)
            ref = oracle.apply_h(psi, o.veff(f, v_h).reshape(shape), o.fproj[f], o.h, o.dv)
            ref = ref.reshape(5, -1)
            for dt, tol in ((torch.float64, 1e-12), (torch.float32, 1e-5)):
                x = torch.tensor(psi.reshape(5, -1), device="cuda", dtype=dt)
                hx = torch.empty_like(x)
                d.dcdft_apply_h(f, x, hx, prec=0 if dt == torch.float64 else PREC_MIXED)
                err = np.abs(hx.double().cpu().numpy() - ref).max()
                assert err <= tol * np.abs(ref).max(), (f, dt, err)
    _follow(cfg, 2)
