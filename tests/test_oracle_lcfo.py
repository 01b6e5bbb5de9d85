"""Pins of the oracle's DC-LCFO basis and global Hamiltonian (Sec. 2.3, Eqs. (6)-(9)).

* One fragment covering the cell (b = 0): the core is everything, the selected
  orbitals are already orthonormal, so the basis spans them and the matrix of Eq.
  (9) has the Ritz eigenvalues of the selected orbitals as its spectrum.
* Buffers at least as wide as the stencil (4 points) and as two projector support
  radii (a support that meets a core stays inside the box), with V_xc taken from
  the total density: every H^alpha acts on
  a core-supported function as the global Hamiltonian does, so the assembled
  matrix equals Lambda^T H Lambda with H an independent dense global Hamiltonian.
* Narrow buffers (H^alpha differs from the global operator): the matrix is
  symmetric by construction of the neighbour blocks.
* The basis is orthonormal over the whole system (Eq. (7)), and its size per
  fragment is the number of overlap eigenvalues above lambda_cut, counted here
  from the singular values of the core-projected orbitals.
"""
import math

import numpy as np

import oracle
from oracle import grid as og
from oracle import model as om
from oracle.lcfo import lcfo_basis, lcfo_hamiltonian
from tests.helpers import dense_kinetic, tiny_config


def _fixed_state(cfg, rho, steps):
    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.set_density(rho)
    for _ in range(steps):
        o.step()
    return o


def _analytic_density(cfg):
    sysm = cfg.system
    nx, ny, nz = cfg.n_grid
    h = sysm.cell / np.array(cfg.n_grid)
    z, y, x = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0],
                          indexing="ij")
    rho = 1.0 + 0.3 * np.cos(2 * math.pi * x / sysm.cell[0]) \
        + 0.2 * np.sin(2 * math.pi * y / sysm.cell[1]) * np.cos(2 * math.pi * z / sysm.cell[2])
    return rho * sysm.n_electrons / (float(np.prod(h)) * rho.sum())


def _global(o, basis):
    rows = []
    for a, f in enumerate(o.frags):
        g = np.zeros((basis[a].shape[0], o.n_global))
        g[:, f.global_index] = basis[a]
        rows.append(g)
    return np.concatenate(rows)


def test_single_fragment_matrix_has_the_ritz_spectrum():
    cfg = tiny_config(n_grid=(10, 10, 10), cell=(6.0, 6.0, 6.0), n_atoms=2, nstate=8,
                      smearing=0.05, sweeps=4)
    o = _fixed_state(cfg, _analytic_density(cfg), 6)
    eps = o.eps[0]
    f = o.frags[0]
    for k in (8, 5):
        cut = 0.5 * (eps[k - 1] + eps[k]) if k < len(eps) else eps[-1] + 1.0
        basis = [lcfo_basis(o.psi[0], eps, f.core_mask.astype(float), o.dv, cut, 1e-7)]
        assert basis[0].shape[0] == k
        hm = lcfo_hamiltonian(o, basis, [o.veff_last[0]])
        np.testing.assert_allclose(np.linalg.eigvalsh(0.5 * (hm + hm.T)), eps[:k], rtol=0,
                                   atol=1e-10)
        lam = _global(o, basis)
        np.testing.assert_allclose(o.dv * lam @ lam.T, np.eye(k), rtol=0, atol=1e-12)


def test_wide_buffers_give_the_global_hamiltonian():
    # a projector meeting a core reaches at most two support radii past it: the
    # buffer (8 points) holds that (2 x 3.8 points) and the stencil (4 points)
    cfg = tiny_config(n_grid=(36, 8, 8), cell=(18.0, 4.0, 4.0), n_atoms=6, nstate=12,
                      num_fragment=(2, 1, 1), buffer=(8, 0, 0), smearing=0.05, valence=2.0,
                      kb_rcut=1.9)
    sysm = cfg.system
    rho = _analytic_density(cfg)
    o = _fixed_state(cfg, rho, 4)
    assert 2.0 * sysm.species[0].kb_rcut / o.h[0] < 8.0
    basis = []
    for a, f in enumerate(o.frags):
        cut = 0.5 * (o.eps[a][8] + o.eps[a][9])
        basis.append(lcfo_basis(o.psi[a], o.eps[a], f.core_mask.astype(float), o.dv, cut, 1e-7))
    hm = lcfo_hamiltonian(o, basis, [o.veff_last[a] for a in range(len(o.frags))])
    # independent dense global Hamiltonian with V_xc of the total density
    nx, ny, nz = cfg.n_grid
    ng = nx * ny * nz
    h = sysm.cell / np.array(cfg.n_grid)
    dv = float(np.prod(h))
    lap = -2.0 * dense_kinetic((nz, ny, nx), h, og.FD_COEFFS)
    vh = np.linalg.pinv(lap, rcond=1e-12, hermitian=True) @ (-4 * math.pi * (rho.ravel() - rho.mean()))
    vh -= vh.mean()
    _, vxc = om.lda_pz81(rho.ravel())
    hd = dense_kinetic((nz, ny, nx), h, og.FD_COEFFS) \
        + np.diag(om.local_potential(sysm, cfg.n_grid).ravel() + vh + vxc)
    for p in om.kb_projectors(sysm, cfg.n_grid):
        b = np.zeros(ng)
        b[p.index] = p.value
        hd += p.energy * dv * np.outer(b, b)
    lam = _global(o, basis)
    np.testing.assert_allclose(dv * lam @ lam.T, np.eye(lam.shape[0]), rtol=0, atol=1e-12)
    ref = dv * lam @ hd @ lam.T
    nb0 = basis[0].shape[0]
    assert np.abs(ref[:nb0, nb0:]).max() > 1e-3          # the neighbour blocks are not empty
    np.testing.assert_allclose(hm, ref, rtol=0, atol=1e-10)


def test_narrow_buffers_symmetric_matrix_and_basis_count():
    cfg = tiny_config(n_grid=(12, 12, 10), cell=(7.2, 7.2, 6.0), n_atoms=5, nstate=12,
                      num_fragment=(2, 2, 1), buffer=(2, 2, 0), smearing=0.05, valence=2.0)
    o = _fixed_state(cfg, _analytic_density(cfg), 3)
    basis, counts = [], []
    for a, f in enumerate(o.frags):
        core = f.core_mask.astype(float)
        cut = o.eps[a][-1] + 1.0                        # every orbital selected
        phibar = o.psi[a] * core[None, :]
        sv = np.linalg.svd(np.sqrt(o.dv) * phibar, compute_uv=False) ** 2
        lam_cut = float(np.sqrt(sv[2] * sv[3]))          # between the 3rd and 4th largest
        basis.append(lcfo_basis(o.psi[a], o.eps[a], core, o.dv, cut, lam_cut))
        counts.append(int(np.sum(sv > lam_cut)))
        assert basis[a].shape[0] == counts[a] == 3
    hm = lcfo_hamiltonian(o, basis, [o.veff_last[a] for a in range(len(o.frags))])
    off = np.concatenate([[0], np.cumsum(counts)])
    # neighbour blocks are symmetric by construction; same-fragment blocks to rounding
    np.testing.assert_allclose(hm, hm.T, rtol=0, atol=1e-12)
    assert np.abs(hm[off[0]:off[1], off[1]:off[2]]).max() > 1e-4
    lam = _global(o, basis)
    np.testing.assert_allclose(o.dv * lam @ lam.T, np.eye(lam.shape[0]), rtol=0, atol=1e-12)
