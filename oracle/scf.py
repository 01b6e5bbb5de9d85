"""Hartree potential, total energy and the DC-DFT SCF iteration (test
infrastructure only).

One SCF iteration (Sec. 2.2; the loop runs "as in conventional DFT" over the
total density):
  1. V_H from the global Poisson equation of rho_tot^in, discretised with the
     same nine-point-per-axis Laplacian: L V_H = -4 pi (rho - mean rho),
     V_H with zero mean (jellium gauge).
  2. V_eff^alpha = V_loc + V_H (gathered from the global grid) + V_xc[rho_alpha^in]
     + V^alpha (Eq. (5): exchange-correlation from the fragment density; the
     density-template potential V^alpha = (rho_alpha^in - rho_tot^in) / xi when a
     xi > 0 is set, zero by default as in the paper).
  3. fragment eigensolver (``cg_eigensolver``), core weights.
  4. global mu (``fermi_level``).
  5. rho_alpha^out (Eq. (4)); rho_tot^out = sum_alpha core-projected rho_alpha
     (Eqs. (2)-(3)).
  6. Harris-Foulkes / Mermin free energy at rho^in (the ion-ion term, constant
     for a fixed geometry, is omitted).
  7. residuals: dV sum |rho_out - rho_in| / N_e and the paper's convergence
     measure dV sum |rho_k^in - rho_(k-1)^in| / N_e (Sec. 3.3).
  8. mixing: linear, rho^in <- rho^in + a (rho^out - rho^in), applied to the
     total density and to every fragment density; or, after set_mixer("pulay",
     ...), Pulay mixing with a Kerker preconditioner (``oracle.mixing``).

Fixed-density DC (Sec. 2.6, third usage; Sec. 3.2): rho_tot^in is a density
read in and stays frozen.  Every iteration re-solves the fragment eigenproblems
in the potential of that density (steps 1-7 unchanged) and assembles rho^out,
but step 8 is skipped: neither rho_tot^in nor any rho_alpha^in changes, so the
paper's residual is zero and rho^out - rho^in measures how far the fragment
solution is from reproducing the frozen density.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from .grid import FD_COEFFS, HALF_WIDTH, build_fragments, laplacian_periodic
from .model import (fragment_projectors, grid_spacing, kb_projectors, lda_pz81,
                    local_potential)
from .mixing import PulayKerkerMixer
from .rng import initial_orbitals
from .solver import (apply_h, cg_eigensolver, cholesky_orthonormalize, core_weights,
                     fermi_level, fermi_occupation, fragment_density)


def fd_symbol(n_grid, h) -> np.ndarray:
    """Eigenvalues of the periodic FD Laplacian on the Fourier modes, (Nz, Ny, Nx)."""
    lam = []
    for d in range(3):
        k = np.arange(n_grid[d])
        s = FD_COEFFS[0] + 2.0 * sum(FD_COEFFS[j] * np.cos(2.0 * math.pi * j * k / n_grid[d])
                                     for j in range(1, HALF_WIDTH + 1))
        lam.append(s / (h[d] * h[d]))
    return lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :]


def poisson_fd(rho: np.ndarray, h) -> np.ndarray:
    """Exact solution of L V = -4 pi (rho - mean rho) with mean V = 0, by
    diagonalising the circulant FD Laplacian with the FFT."""
    n_grid = (rho.shape[2], rho.shape[1], rho.shape[0])
    lam = fd_symbol(n_grid, h)
    rk = np.fft.fftn(rho)
    lam_safe = lam.copy()
    lam_safe[0, 0, 0] = 1.0
    vk = -4.0 * math.pi * rk / lam_safe
    vk[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(vk))


def poisson_fd_cg(rho: np.ndarray, h, tol: float = 1e-13, x0: Optional[np.ndarray] = None,
                  maxiter: int = 20000) -> np.ndarray:
    """The same equation by conjugate gradients on -L (SPD on zero-mean fields),
    stopping at ||r|| <= tol ||b||."""
    b = 4.0 * math.pi * (rho - rho.mean())
    x = np.zeros_like(rho) if x0 is None else x0 - x0.mean()
    r = b + laplacian_periodic(x, h)
    p = r.copy()
    rr = float(np.sum(r * r))
    bn = math.sqrt(float(np.sum(b * b)))
    for _ in range(maxiter):
        if math.sqrt(rr) <= tol * bn:
            break
        ap = -laplacian_periodic(p, h)
        alpha = rr / float(np.sum(p * ap))
        x = x + alpha * p
        r = r - alpha * ap
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x - x.mean()


def entropy_term(occ: np.ndarray, w: np.ndarray) -> float:
    """S = -sum 2 w [f ln f + (1 - f) ln(1 - f)], 0 ln 0 = 0."""
    f = np.asarray(occ)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(f > 0, f * np.log(np.where(f > 0, f, 1.0)), 0.0)
        t2 = np.where(f < 1, (1 - f) * np.log(np.where(f < 1, 1 - f, 1.0)), 0.0)
    return float(-np.sum(2.0 * w * (t1 + t2)))


def total_energy(e_band: float, rho_in: np.ndarray, v_h: np.ndarray, dv: float,
                 sigma: float, entropy: float) -> float:
    """E = E_band - dV sum rho_in (V_H + V_xc[rho_in]) + 1/2 dV sum rho_in V_H
           + dV sum rho_in eps_xc[rho_in] - sigma S."""
    exc, vxc = lda_pz81(rho_in)
    return (e_band - dv * float(np.sum(rho_in * (v_h + vxc))) + 0.5 * dv * float(np.sum(rho_in * v_h))
            + dv * float(np.sum(rho_in * exc)) - sigma * entropy)


_WORKER_LIMITS = None
_WORKER_PROJECTORS = None


def _worker_init(blas_threads: int, system=None, n_grid=None):
    """Pool worker set-up: BLAS thread count of the worker process and, when the
    system is given, its own copy of the global projectors (for _setup_fragment)."""
    global _WORKER_LIMITS, _WORKER_PROJECTORS
    try:
        from threadpoolctl import threadpool_limits
        _WORKER_LIMITS = threadpool_limits(limits=blas_threads)
    except ImportError:
        pass
    if system is not None:
        _WORKER_PROJECTORS = kb_projectors(system, n_grid)


def _setup_fragment(args):
    """Projectors restricted to one fragment and its orthonormalised initial
    orbitals (the per-fragment part of OracleSCF's set-up, run in a worker)."""
    frag, n_global, seed, m, dv = args
    proj = fragment_projectors(_WORKER_PROJECTORS, frag, n_global)
    raw = initial_orbitals(seed, frag.alpha, m, frag.shape).reshape(m, -1)
    return proj, cholesky_orthonormalize(raw, dv)[0]


def _solve_fragment(args):
    psi, veff, proj, h, dv, sweeps, shape = args
    m = psi.shape[0]
    hop = lambda x: apply_h(x.reshape((x.shape[0],) + shape), veff, proj, h, dv).reshape(x.shape[0], -1)
    return cg_eigensolver(psi, hop, sweeps, dv)


class OracleSCF:
    """State and iteration of the DC-DFT SCF on the CPU, FP64."""

    def __init__(self, cfg, workers: int = 1, blas_threads: int = 1, fragments=None):
        """fragments: None for the whole system, or a subset of fragment indices;
        only those fragments then get projectors and orbitals (for timing a sample
        of the fragment eigensolves with solve_fragments; step() needs them all)."""
        self.cfg = cfg
        sysm = cfg.system
        self.n_grid = tuple(int(v) for v in cfg.n_grid)
        self.h = grid_spacing(sysm.cell, self.n_grid)
        self.dv = float(np.prod(self.h))
        self.n_global = int(np.prod(self.n_grid))
        self.ne = sysm.n_electrons
        self.frags = build_fragments(self.n_grid, cfg.num_fragment, cfg.num_rgrid_buffer)
        self.vloc = local_potential(sysm, self.n_grid)
        keep = set(range(len(self.frags)) if fragments is None else (int(a) for a in fragments))
        self.subset = None if fragments is None else sorted(keep)
        self.m = [int(v) for v in cfg.nstate_frag]
        # fragment eigensolves on a pool of fresh interpreter processes ("spawn":
        # nothing of the caller's process, such as an initialised GPU runtime, is
        # inherited), kept until close(); with a pool the per-fragment set-up
        # (restricted projectors, initial orbitals) runs there too
        self.workers = workers
        self.blas_threads = blas_threads
        self._pool = None
        self.fproj = [None] * len(self.frags)
        self.psi = [None] * len(self.frags)
        todo = [f for f in self.frags if f.alpha in keep]
        if workers > 1 and len(todo) > 1:
            self._start_pool()
            jobs = [(f, self.n_global, cfg.seed, self.m[f.alpha], self.dv) for f in todo]
            for f, (proj, psi) in zip(todo, self._pool.map(_setup_fragment, jobs)):
                self.fproj[f.alpha], self.psi[f.alpha] = proj, psi
        else:
            projectors = kb_projectors(sysm, self.n_grid)
            for f in todo:
                self.fproj[f.alpha] = fragment_projectors(projectors, f, self.n_global)
                raw = initial_orbitals(cfg.seed, f.alpha, self.m[f.alpha], f.shape).reshape(
                    self.m[f.alpha], -1)
                self.psi[f.alpha] = cholesky_orthonormalize(raw, self.dv)[0]
        omega = float(np.prod(sysm.cell))
        self.rho_in = np.full(self.n_grid[::-1], self.ne / omega)
        self.rho_frag_in = [np.full(f.n, self.ne / omega) for f in self.frags]
        self.rho_out = None
        self.rho_frag_out = None
        self.eps = None
        self.w = None
        self.mu = None
        self.iteration = 0
        self.veff_last = {}         # V_eff of each fragment in the last eigensolve
        self.fixed_density = False
        self.template_xi = 0.0      # xi of V^alpha (Eq. (5)); 0: no template potential
        self.mixer = None           # None: linear mixing with cfg.mixing

    def set_mixer(self, kind: str, alpha: float = 0.3, q0: float = 0.8, history: int = 8):
        """kind "linear" (cfg.mixing, the default) or "pulay" (Pulay mixing with
        step alpha, Kerker wave number q0 (bohr^-1; 0: no preconditioner) and up to
        `history` pairs); a new Pulay mixer starts with an empty history."""
        if kind == "linear":
            self.mixer = None
        elif kind == "pulay":
            self.mixer = PulayKerkerMixer(self.n_grid, self.h, alpha, q0, history)
        else:
            raise ValueError(f"unknown mixer {kind}")

    def set_density(self, rho_tot, rho_frag=None):
        """Replace rho_tot^in; every rho_alpha^in becomes rho_frag[alpha] or, when
        rho_frag is None, rho_tot^in on the fragment box (periodic images)."""
        self.rho_in = np.array(rho_tot, dtype=np.float64).reshape(self.n_grid[::-1])
        flat = self.rho_in.ravel()
        if rho_frag is None:
            self.rho_frag_in = [flat[f.global_index].copy() for f in self.frags]
        else:
            self.rho_frag_in = [np.array(r, dtype=np.float64).ravel() for r in rho_frag]

    def _start_pool(self):
        if self._pool is None:
            import multiprocessing as mp
            self._pool = mp.get_context("spawn").Pool(
                self.workers, _worker_init, (self.blas_threads, self.cfg.system, self.n_grid))

    def close(self):
        """End the worker pool (if one was started)."""
        if self._pool is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def veff(self, alpha: int, v_h: np.ndarray) -> np.ndarray:
        f = self.frags[alpha]
        _, vxc = lda_pz81(self.rho_frag_in[alpha])
        v = self.vloc.ravel()[f.global_index] + v_h.ravel()[f.global_index] + vxc
        if self.template_xi > 0.0:
            # density-template potential (Eq. (5)) of the input densities
            v = v + (self.rho_frag_in[alpha] - self.rho_in.ravel()[f.global_index]) / self.template_xi
        return v

    def solve_fragments(self, v_h: np.ndarray, alphas=None):
        alphas = range(len(self.frags)) if alphas is None else alphas
        jobs = []
        for a in alphas:
            f = self.frags[a]
            veff = self.veff(a, v_h)
            self.veff_last[a] = veff
            jobs.append((self.psi[a], veff.reshape(f.shape), self.fproj[a], self.h,
                         self.dv, self.cfg.cg_sweeps, f.shape))
        if self.workers > 1 and len(jobs) > 1:
            self._start_pool()
            res = self._pool.map(_solve_fragment, jobs)
        else:
            res = [_solve_fragment(j) for j in jobs]
        return dict(zip(alphas, res))

    def step(self) -> dict:
        if self.subset is not None:
            raise RuntimeError("this oracle holds a subset of the fragments; step() needs all")
        cfg = self.cfg
        dv = self.dv
        v_h = poisson_fd(self.rho_in, self.h)
        res = self.solve_fragments(v_h)
        self.eps, self.w = [], []
        for a, f in enumerate(self.frags):
            psi, eps = res[a]
            self.psi[a] = psi
            self.eps.append(eps)
            self.w.append(core_weights(psi, f.core_mask, dv))
        eps_all = np.concatenate(self.eps)
        w_all = np.concatenate(self.w)
        mu = fermi_level(eps_all, w_all, self.ne, cfg.smearing)
        self.mu = mu
        rho_out = np.zeros(self.n_global)
        self.rho_frag_out = []
        occ_all = []
        for a, f in enumerate(self.frags):
            occ = fermi_occupation((self.eps[a] - mu) / cfg.smearing)
            occ_all.append(occ)
            rf = fragment_density(self.psi[a], occ)
            self.rho_frag_out.append(rf)
            rho_out[f.global_index[f.core_mask]] = rf[f.core_mask]
        rho_out = rho_out.reshape(self.rho_in.shape)
        self.rho_out = rho_out
        occ_all = np.concatenate(occ_all)
        e_band = float(np.sum(2.0 * occ_all * eps_all * w_all))
        ent = entropy_term(occ_all, w_all)
        e_tot = total_energy(e_band, self.rho_in, v_h, dv, cfg.smearing, ent)
        r_out_in = dv * float(np.sum(np.abs(rho_out - self.rho_in))) / self.ne
        charge = dv * float(np.sum(rho_out))
        if self.fixed_density:
            rho_new, frag_new = self.rho_in, self.rho_frag_in
        elif self.mixer is None:
            a_mix = cfg.mixing
            rho_new = self.rho_in + a_mix * (rho_out - self.rho_in)
            frag_new = [ri + a_mix * (ro - ri)
                        for ri, ro in zip(self.rho_frag_in, self.rho_frag_out)]
        else:
            # fragment densities as the gathered total density plus a deviation
            fin, fout = self.rho_in.ravel(), rho_out.ravel()
            d_in = [self.rho_frag_in[a] - fin[f.global_index] for a, f in enumerate(self.frags)]
            d_out = [self.rho_frag_out[a] - fout[f.global_index] for a, f in enumerate(self.frags)]
            rho_new, d_new = self.mixer.mix(self.rho_in, rho_out, d_in, d_out)
            fnew = rho_new.ravel()
            frag_new = [fnew[f.global_index] + d_new[a] for a, f in enumerate(self.frags)]
        r_paper = dv * float(np.sum(np.abs(rho_new - self.rho_in))) / self.ne
        self.rho_in = rho_new
        self.rho_frag_in = frag_new
        self.iteration += 1
        self.v_h = v_h
        return dict(iter=self.iteration, mu=mu, e_total=e_tot, e_band=e_band,
                    residual_paper=r_paper, residual_out_in=r_out_in, charge=charge,
                    entropy=ent)
