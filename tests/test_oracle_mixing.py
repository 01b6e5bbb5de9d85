"""Pins of the oracle's density mixers (CPU only).

* The Pulay weights equal numpy's solve of the bordered least-squares system, and
  dependent residuals are detected.
* The Kerker filter multiplies a single Fourier mode by q^2 / (q^2 + q0^2), with
  q^2 the eigenvalue of minus the nine-point Laplacian built as a dense matrix
  here, and removes the constant.
* On a linear fixed-point problem whose Jacobian has three distinct eigenvalues,
  Pulay mixing reaches the fixed point in a handful of steps (it is GMRES on
  linear problems; linear mixing needs hundreds).
* Pulay mixing with one history entry and no preconditioner is linear mixing,
  for the total and every fragment density, along a real DC SCF.
* Pulay mixing keeps the fragment densities equal to the total density on core
  points, and converges the one-fragment (conventional) SCF to the density of the
  independent dense-diagonalisation SCF (the fixed point does not move).
"""
import math

import numpy as np

import oracle
from oracle.mixing import PulayKerkerMixer, kerker_filter, pulay_weights
from tests.helpers import dense_second_derivative_1d, tiny_config
from tests.test_oracle_scf import conventional_config, conventional_reference
from oracle import grid as og


def test_pulay_weights_match_a_library_solve():
    rng = np.random.default_rng(4)
    for k in (1, 2, 5, 8):
        r = rng.normal(size=(k, 40))
        a = r @ r.T
        c, ok = pulay_weights(a)
        assert ok
        m = np.zeros((k + 1, k + 1))
        m[:k, :k] = a
        m[k, :k] = m[:k, k] = 1.0
        rhs = np.zeros(k + 1)
        rhs[k] = 1.0
        np.testing.assert_allclose(c, np.linalg.solve(m, rhs)[:k], rtol=1e-10, atol=1e-12)
        assert abs(c.sum() - 1.0) < 1e-12
    r = rng.normal(size=(3, 40))
    r[2] = r[1]
    _, ok = pulay_weights(r @ r.T)
    assert not ok


def test_kerker_filter_on_single_modes():
    n_grid, cell = (8, 6, 10), (5.0, 4.0, 7.5)
    h = np.array(cell) / np.array(n_grid)
    q0 = 0.7
    nz, ny, nx = n_grid[2], n_grid[1], n_grid[0]
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    for kx, ky, kz in ((1, 0, 0), (0, 2, 1), (3, 1, 4), (4, 3, 5)):
        mode = (np.cos(2 * math.pi * kx * x / nx) * np.cos(2 * math.pi * ky * y / ny)
                * np.sin(2 * math.pi * kz * z / nz + 0.3)) * np.ones((nz, ny, nx))
        # q^2 from the dense periodic nine-point Laplacian acting on the mode
        lap = np.zeros_like(mode)
        for ax, (n, hd) in zip((2, 1, 0), ((nx, h[0]), (ny, h[1]), (nz, h[2]))):
            d2 = dense_second_derivative_1d(n, hd, og.FD_COEFFS)
            lap += np.moveaxis(np.tensordot(d2, np.moveaxis(mode, ax, 0), axes=(1, 0)), 0, ax)
        q2 = float(-np.sum(lap * mode) / np.sum(mode * mode))
        np.testing.assert_allclose(-lap, q2 * mode, rtol=0, atol=1e-10 * abs(q2))
        out = kerker_filter(mode, n_grid, h, q0)
        np.testing.assert_allclose(out, q2 / (q2 + q0 * q0) * mode, rtol=0, atol=1e-13)
    assert np.abs(kerker_filter(np.full((nz, ny, nx), 3.0), n_grid, h, q0)).max() < 1e-14


def test_pulay_solves_a_linear_fixed_point_problem():
    rng = np.random.default_rng(9)
    shape = (4, 5, 6)
    star = rng.uniform(0.5, 1.5, size=shape)
    jac = rng.choice([0.5, 2.0, 5.0], size=shape)      # three distinct eigenvalues
    out_of = lambda rho: star + (1.0 - jac) * (rho - star)   # R = -J (rho - rho*)
    mix = PulayKerkerMixer((6, 5, 4), (1.0, 1.0, 1.0), alpha=0.3, q0=0.0, history=8)
    rho = np.ones(shape)
    errs = []
    for _ in range(6):
        rho, _ = mix.mix(rho, out_of(rho), [], [])
        errs.append(float(np.abs(rho - star).max()))
    assert errs[4] < 1e-10, errs
    # linear mixing with the same step is still far away
    lin = np.ones(shape)
    for _ in range(6):
        lin = lin + 0.3 * (out_of(lin) - lin)
    assert np.abs(lin - star).max() > 1e-2


def test_one_entry_pulay_without_kerker_is_linear_mixing():
    cfg = tiny_config(n_grid=(12, 12, 10), cell=(7.2, 7.2, 6.0), n_atoms=4, nstate=14,
                      num_fragment=(2, 1, 1), buffer=(2, 0, 0), smearing=0.05, valence=2.0)
    a, b = oracle.OracleSCF(cfg), oracle.OracleSCF(cfg)
    b.set_mixer("pulay", alpha=cfg.mixing, q0=0.0, history=1)
    for _ in range(4):
        ra, rb = a.step(), b.step()
        assert abs(ra["residual_paper"] - rb["residual_paper"]) < 1e-14
        assert np.abs(a.rho_in - b.rho_in).max() < 1e-14
        for x, y in zip(a.rho_frag_in, b.rho_frag_in):
            assert np.abs(x - y).max() < 1e-14


def test_pulay_keeps_core_densities_and_converges_the_conventional_scf():
    cfg = tiny_config(n_grid=(12, 12, 10), cell=(7.2, 7.2, 6.0), n_atoms=4, nstate=14,
                      num_fragment=(2, 1, 1), buffer=(2, 0, 0), smearing=0.05, valence=2.0)
    o = oracle.OracleSCF(cfg)
    o.set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
    for _ in range(6):
        o.step()
        flat = o.rho_in.ravel()
        for f, rf in zip(o.frags, o.rho_frag_in):
            assert np.abs(rf[f.core_mask] - flat[f.global_index[f.core_mask]]).max() < 1e-14
    # Pulay extrapolation assumes rho_out is a function of rho_in alone: with 12
    # CG sweeps per iteration the fragment orbitals follow rho_in closely enough
    conv = conventional_config(sweeps=12)
    ref = conventional_reference()
    c = oracle.OracleSCF(conv)
    c.set_mixer("pulay", alpha=0.3, q0=0.8, history=8)
    for _ in range(200):
        info = c.step()
        if info["residual_out_in"] < 1e-12:
            break
    assert info["residual_out_in"] < 1e-11
    assert c.dv * np.abs(c.rho_out - ref["rho"]).sum() / c.ne < 1e-9
    np.testing.assert_allclose(c.eps[0], ref["eps"], rtol=0, atol=1e-9)
