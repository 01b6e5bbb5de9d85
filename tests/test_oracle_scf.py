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
import scipy.linalg
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
        e, u = scipy.linalg.eigh(hmat, subset_by_index=[0, m - 1])
        u = u / math.sqrt(dv)
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


_CONVENTIONAL = {}


def conventional_config(sweeps=4):
    """Two atoms in a 6 bohr cube on a 10^3 grid, one fragment, no buffer."""
    return tiny_config(n_grid=(10, 10, 10), cell=(6.0, 6.0, 6.0), n_atoms=2, nstate=6,
                       smearing=0.05, mixing=0.3, sweeps=sweeps)


def conventional_reference():
    """dense_scf of conventional_config (independent of the CG sweep count), once."""
    if "ref" not in _CONVENTIONAL:
        _CONVENTIONAL["ref"] = dense_scf(conventional_config())
    return _CONVENTIONAL["ref"]


def run_oracle(cfg, iters=400, tol=1e-12):
    o = oracle.OracleSCF(cfg)
    info = None
    for _ in range(iters):
        info = o.step()
        if info["residual_out_in"] < tol:
            break
    return o, info


def test_single_fragment_is_conventional_dft():
    cfg = conventional_config()
    ref = conventional_reference()
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


# --- fixed-density DC (Sec. 2.6, third usage; Sec. 3.2) ----------------------------------

def _dense_poisson(shape, h, rho):
    """V_H of rho with the FD Laplacian as a dense matrix (pseudo-inverse, zero mean)."""
    lap = -2.0 * dense_kinetic(shape, h, og.FD_COEFFS)
    v = np.linalg.pinv(lap, rcond=1e-12, hermitian=True) @ (-4 * math.pi * (rho - rho.mean()))
    return v - v.mean()


def _fixed_steps(o, n_max=200, tol=1e-12):
    """Fixed-density iterations until no eigenvalue and no value of rho^out moves by
    more than tol (the orbitals converge only as the square root of the
    eigenvalues); checks on the way that nothing of the frozen density changes."""
    rho0 = o.rho_in.copy()
    frag0 = [r.copy() for r in o.rho_frag_in]
    prev = None
    for _ in range(n_max):
        info = o.step()
        assert info["residual_paper"] == 0.0
        assert np.array_equal(o.rho_in, rho0)
        assert all(np.array_equal(a, b) for a, b in zip(o.rho_frag_in, frag0))
        cur = np.concatenate(o.eps + [o.rho_out.ravel()])
        if prev is not None and np.abs(cur - prev).max() < tol:
            break
        prev = cur
    else:
        raise AssertionError("fixed-density iterations did not settle")
    return info


def test_fixed_density_at_conventional_density_reproduces_it():
    """One fragment (b = 0) frozen at the self-consistent density of the dense
    conventional SCF: the eigenvalues, mu and the output density are those of the
    dense solution, and rho^out reproduces the frozen density (the density error
    specific to DC is absent, Sec. 2.6)."""
    # two more states than the conventional test: a wider gap at the subspace edge
    # lets the orbitals (not only the eigenvalues) settle within the step budget
    cfg = tiny_config(n_grid=(10, 10, 10), cell=(6.0, 6.0, 6.0), n_atoms=2, nstate=8,
                      smearing=0.05, mixing=0.3, sweeps=4)
    ref = dense_scf(cfg)
    assert ref["res"] < 1e-11
    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.set_density(ref["rho"])
    info = _fixed_steps(o)
    np.testing.assert_allclose(o.eps[0], ref["eps"], rtol=0, atol=1e-9)
    assert abs(o.mu - ref["mu"]) < 1e-9
    assert info["residual_out_in"] < 1e-10
    np.testing.assert_allclose(o.v_h.ravel(), ref["vh"], rtol=0, atol=1e-10)


def test_fixed_density_dc_fragments_solve_the_frozen_potential():
    """Two buffered fragments frozen at an analytic density: every fragment's
    eigenvalues are the lowest of its own dense Hamiltonian, built here from the
    frozen density (kinetic on the periodic fragment box, V_loc + V_H + V_xc of the
    fragment's share of the density, global projectors restricted to the box without
    renormalisation, Eq. (5)); mu solves the weighted charge equation (Eq. (4))."""
    cfg = tiny_config(n_grid=(16, 8, 8), cell=(12.0, 6.0, 6.0), n_atoms=4, nstate=8,
                      num_fragment=(2, 1, 1), buffer=(2, 0, 0), smearing=0.05, valence=2.0)
    sysm = cfg.system
    nx, ny, nz = cfg.n_grid
    h = sysm.cell / np.array(cfg.n_grid)
    dv = float(np.prod(h))
    z, y, x = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0],
                          indexing="ij")
    shape_g = (nz, ny, nx)
    rho = 1.0 + 0.4 * np.sin(2 * math.pi * x / sysm.cell[0]) * np.cos(2 * math.pi * y / sysm.cell[1]) \
        + 0.2 * np.cos(2 * math.pi * z / sysm.cell[2])
    rho *= sysm.n_electrons / (dv * rho.sum())
    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.set_density(rho)
    _fixed_steps(o, n_max=400)

    vh = _dense_poisson(shape_g, h, rho.ravel())
    vloc = om.local_potential(sysm, cfg.n_grid).ravel()
    beta = []
    for p in om.kb_projectors(sysm, cfg.n_grid):
        b = np.zeros(nx * ny * nz)
        b[p.index] = p.value
        beta.append((p.energy, b))
    b_buf, ncore = 2, nx // 2
    lx = np.arange(ncore + 2 * b_buf)
    eps_all, w_all = [], []
    for alpha in range(2):
        gx = (alpha * ncore - b_buf + lx) % nx
        gidx = (gx[None, None, :] + nx * (np.arange(ny)[None, :, None]
                                          + ny * np.arange(nz)[:, None, None])).ravel()
        rf = rho.ravel()[gidx]
        _, vxc = om.lda_pz81(rf)
        hm = dense_kinetic((nz, ny, lx.size), h, og.FD_COEFFS) + np.diag(vloc[gidx] + vh[gidx] + vxc)
        for e, b in beta:
            bf = b[gidx]
            hm += e * dv * np.outer(bf, bf)
        ev = np.linalg.eigvalsh(hm)
        m = int(cfg.nstate_frag[alpha])
        assert ev[m] - ev[m - 1] > 1e-3      # a gap at the subspace edge
        np.testing.assert_allclose(o.eps[alpha], ev[:m], rtol=0, atol=1e-9)
        eps_all.append(o.eps[alpha])
        w_all.append(o.w[alpha])
    eps_all, w_all = np.concatenate(eps_all), np.concatenate(w_all)
    count = lambda mu: float(np.sum(2 * w_all / (1 + np.exp((eps_all - mu) / cfg.smearing)))) \
        - sysm.n_electrons
    mu = scipy.optimize.brentq(count, eps_all.min() - 5, eps_all.max() + 5, xtol=1e-15, rtol=1e-15)
    assert abs(o.mu - mu) < 1e-10


# --- density-template potential V^alpha (Eq. (5)) ----------------------------------------

def test_template_potential_enters_the_fragment_hamiltonian():
    """Frozen total and fragment densities that differ (each fragment's density is
    the total times its own modulation): with xi > 0 every fragment's eigenvalues are
    those of its dense Hamiltonian with V^alpha = (rho_alpha - rho_tot) / xi added on
    the diagonal; with rho_alpha equal to rho_tot the template changes nothing."""
    cfg = tiny_config(n_grid=(16, 8, 8), cell=(12.0, 6.0, 6.0), n_atoms=4, nstate=9,
                      num_fragment=(2, 1, 1), buffer=(2, 0, 0), smearing=0.05, valence=2.0)
    sysm = cfg.system
    nx, ny, nz = cfg.n_grid
    h = sysm.cell / np.array(cfg.n_grid)
    dv = float(np.prod(h))
    z, y, x = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0],
                          indexing="ij")
    rho = 1.0 + 0.3 * np.cos(2 * math.pi * x / sysm.cell[0]) + 0.1 * np.sin(2 * math.pi * z / sysm.cell[2])
    rho *= sysm.n_electrons / (dv * rho.sum())
    b_buf, ncore = 2, nx // 2
    lx = np.arange(ncore + 2 * b_buf)
    gidx = []
    for alpha in range(2):
        gx = (alpha * ncore - b_buf + lx) % nx
        gidx.append((gx[None, None, :] + nx * (np.arange(ny)[None, :, None]
                                               + ny * np.arange(nz)[:, None, None])).ravel())
    lxf = np.broadcast_to(lx[None, None, :], (nz, ny, lx.size)).ravel()
    rho_frag = [rho.ravel()[gidx[a]] * (1.0 + 0.25 * np.sin(2 * math.pi * lxf / lx.size + 1.3 * a))
                for a in range(2)]
    xi = 0.05

    o = oracle.OracleSCF(cfg)
    o.fixed_density = True
    o.template_xi = xi
    o.set_density(rho, rho_frag)
    _fixed_steps(o, n_max=400)

    vh = _dense_poisson((nz, ny, nx), h, rho.ravel())
    vloc = om.local_potential(sysm, cfg.n_grid).ravel()
    projs = om.kb_projectors(sysm, cfg.n_grid)
    for alpha in range(2):
        g = gidx[alpha]
        _, vxc = om.lda_pz81(rho_frag[alpha])
        vtemp = (rho_frag[alpha] - rho.ravel()[g]) / xi
        assert np.abs(vtemp).max() > 0.05      # the template term is not negligible
        hm = dense_kinetic((nz, ny, lx.size), h, og.FD_COEFFS) \
            + np.diag(vloc[g] + vh[g] + vxc + vtemp)
        for p in projs:
            bfull = np.zeros(nx * ny * nz)
            bfull[p.index] = p.value
            hm += p.energy * dv * np.outer(bfull[g], bfull[g])
        ev = np.linalg.eigvalsh(hm)
        m = int(cfg.nstate_frag[alpha])
        assert ev[m] - ev[m - 1] > 1e-3
        np.testing.assert_allclose(o.eps[alpha], ev[:m], rtol=0, atol=1e-9)

    # rho_alpha = rho_tot on every fragment point: V^alpha vanishes identically
    a = oracle.OracleSCF(cfg)
    b = oracle.OracleSCF(cfg)
    b.template_xi = xi
    for o2 in (a, b):
        o2.fixed_density = True
        o2.set_density(rho)
    for _ in range(2):
        ia, ib = a.step(), b.step()
        assert ia == ib


def test_template_potential_in_the_scf_acts_on_buffers_only():
    """From the uniform start every fragment density equals the total one, so the
    first step is unchanged by the template; mixing keeps them equal on core points
    only, so from the second step on V^alpha is nonzero exactly on buffer points."""
    cfg = tiny_config(n_grid=(12, 12, 12), cell=(7.2, 7.2, 7.2), n_atoms=4, nstate=10,
                      num_fragment=(2, 2, 1), buffer=(2, 2, 0), smearing=0.05)
    a = oracle.OracleSCF(cfg)
    b = oracle.OracleSCF(cfg)
    b.template_xi = 2.0
    assert a.step() == b.step()
    v_h = oracle.scf.poisson_fd(b.rho_in, b.h)
    for alpha, f in enumerate(b.frags):
        dvt = b.veff(alpha, v_h) - a.veff(alpha, v_h)
        assert np.array_equal(dvt[f.core_mask], np.zeros(int(f.core_mask.sum())))
        assert np.abs(dvt[~f.core_mask]).max() > 0.0
    ia, ib = a.step(), b.step()
    assert ia["e_band"] != ib["e_band"]
