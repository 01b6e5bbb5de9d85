"""SCF-level pins of the oracle (CPU only).

* One fragment covering the whole cell (b = 0) is conventional DFT: its
  self-consistent density and eigenvalues must equal those of an independent
  dense-diagonalisation SCF written here (dense Kronecker Hamiltonian, LAPACK
  eigensolver, Brent root for mu, dense pseudo-inverse Poisson solve).
* Total charge of rho_tot^out equals N_e.
* At self-consistency the Harris-Foulkes energy equals the Kohn-Sham energy
  evaluated directly from the orbitals.
* The DC density approaches the conventional one as the buffer grows
  (Sec. 3.2 reports accuracy improving with the buffer thickness).
"""
import math

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import grid as og
from oracle import model as om
from oracle import solver as osol
from tests.helpers import dense_kinetic, dense_second_derivative_1d, tiny_config


def dense_scf(cfg, iters=300, tol=1e-12):
    sysm = cfg.system
    n_grid = cfg.n_grid
    shape = (n_grid[2], n_grid[1], n_grid[0])
    h = sysm.cell / np.array(n_grid)
    dv = float(np.prod(h))
    n = int(np.prod(n_grid))
    t = dense_kinetic(shape, h, og.FD_COEFFS)
    lap = -2.0 * t
    lap_pinv = np.linalg.pinv(lap, rcond=1e-12, hermitian=True)
    vloc = om.local_potential(sysm, n_grid).ravel()
    projs = om.kb_projectors(sysm, n_grid)
    vnl = np.zeros((n, n))
    for p in projs:
        b = np.zeros(n)
        b[p.index] = p.value
        vnl += p.energy * dv * np.outer(b, b)
    ne = sysm.n_electrons
    rho = np.full(n, ne / (n * dv))
    m = int(cfg.nstate_frag[0])
    for it in range(iters):
        vh = lap_pinv @ (-4 * math.pi * (rho - rho.mean()))
        vh -= vh.mean()
        _, vxc = om.lda_pz81(rho)
        hmat = t + vnl + np.diag(vloc + vh + vxc)
        e, u = np.linalg.eigh(hmat)
        e, u = e[:m], u[:, :m] / math.sqrt(dv)
        count = lambda mu: float(np.sum(2.0 / (1.0 + np.exp((e - mu) / cfg.smearing)))) - ne
        mu = scipy.optimize.brentq(count, e[0] - 5, e[-1] + 5, xtol=1e-15, rtol=1e-15)
        f = 1.0 / (1.0 + np.exp((e - mu) / cfg.smearing))
        rho_out = np.sum(2 * f[None, :] * u * u, axis=1)
        res = dv * np.sum(np.abs(rho_out - rho)) / ne
        rho = rho + cfg.mixing * (rho_out - rho)
        if res < tol:
            break
    return dict(rho=rho_out.reshape(shape), eps=e, mu=mu, f=f, u=u, vh=vh, vloc=vloc,
                t=t, vnl=vnl, dv=dv, res=res)


def run_oracle(cfg, iters=400, tol=1e-12):
    o = oracle.OracleSCF(cfg)
    info = None
    for _ in range(iters):
        info = o.step()
        if info["residual_out_in"] < tol:
            break
    return o, info


def test_single_fragment_is_conventional_dft():
    cfg = tiny_config(n_grid=(10, 10, 10), cell=(6.0, 6.0, 6.0), n_atoms=2, nstate=6,
                      smearing=0.05, mixing=0.3, sweeps=4)
    ref = dense_scf(cfg)
    assert ref["res"] < 1e-11
    o, info = run_oracle(cfg)
    assert info["residual_out_in"] < 1e-11
    np.testing.assert_allclose(o.eps[0], ref["eps"], rtol=0, atol=1e-9)
    assert abs(o.mu - ref["mu"]) < 1e-9
    assert o.dv * np.abs(o.rho_out - ref["rho"]).sum() / o.ne < 1e-9
    # charge of the assembled density
    assert abs(info["charge"] - o.ne) < 1e-10 * o.ne
    # Harris-Foulkes energy equals the Kohn-Sham energy at self-consistency
    u, f, dv = ref["u"], ref["f"], ref["dv"]
    rho = ref["rho"].ravel()
    e_one = float(np.sum(2 * f * np.einsum("li,lk,ki->i", u, ref["t"] + ref["vnl"] + np.diag(ref["vloc"]), u))) * dv
    exc, _ = om.lda_pz81(rho)
    ent = -float(np.sum(2 * (f * np.log(f) + (1 - f) * np.log(1 - f))))
    e_ks = e_one + 0.5 * dv * float(np.sum(rho * ref["vh"])) + dv * float(np.sum(rho * exc)) \
        - cfg.smearing * ent
    assert abs(info["e_total"] - e_ks) < 1e-8 * max(1.0, abs(e_ks))


def test_dc_density_approaches_conventional_with_buffer():
    errs = []
    # linear mixing 0.3 sloshes in this elongated cell; 0.1 converges
    base = dict(n_grid=(16, 8, 8), cell=(12.0, 6.0, 6.0), n_atoms=4, nstate=8,
                smearing=0.05, mixing=0.1, sweeps=4, valence=2.0)
    ref_cfg = tiny_config(**base, num_fragment=(1, 1, 1), buffer=(0, 0, 0))
    ref, rinfo = run_oracle(ref_cfg)
    assert rinfo["residual_out_in"] < 1e-11
    for b in (1, 2, 3):
        cfg = tiny_config(**base, num_fragment=(2, 1, 1), buffer=(b, 0, 0))
        o, info = run_oracle(cfg, iters=800, tol=1e-11)
        assert info["residual_out_in"] < 1e-9
        assert abs(info["charge"] - o.ne) < 1e-10 * o.ne
        errs.append(o.dv * np.abs(o.rho_out - ref.rho_out).sum() / o.ne)
    assert errs[0] > errs[1] > errs[2]


def test_dc_step_conserves_charge_and_mixes_consistently():
    cfg = tiny_config(n_grid=(12, 12, 12), cell=(7.2, 7.2, 7.2), n_atoms=4, nstate=10,
                      num_fragment=(2, 2, 1), buffer=(2, 2, 0), smearing=0.05)
    o = oracle.OracleSCF(cfg)
    prev = o.rho_in.copy()
    for _ in range(3):
        info = o.step()
        assert abs(info["charge"] - o.ne) < 1e-10 * o.ne
        # residual bookkeeping: R_paper = mixing * R_out,in
        assert abs(info["residual_paper"] - cfg.mixing * info["residual_out_in"]) < 1e-13
        # on every core point the fragment density equals the total density
        for f, rf in zip(o.frags, o.rho_frag_in):
            np.testing.assert_allclose(rf[f.core_mask], o.rho_in.ravel()[f.global_index[f.core_mask]],
                                       rtol=1e-13, atol=1e-15)
        prev = o.rho_in.copy()
