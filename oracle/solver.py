"""Fragment Kohn-Sham solve, occupations and density (test infrastructure only).

Eq. (1): each fragment alpha solves H^alpha phi = eps phi on its own periodic
box.  The paper does not name its eigensolver; the reading adopted here is a
per-band conjugate-gradient trace minimisation with Cholesky
re-orthonormalisation and a closing Rayleigh-Ritz rotation, steps (a)-(l)
written out in ``cg_eigensolver``.  Eqs. (2)-(4): fragment densities with a
globally determined chemical potential, projected onto the cores.

All arrays are FP64.  Orbital blocks are (m, nz, ny, nx); the functions work
on their (m, n) flattening.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .grid import laplacian_periodic


class NotSPDError(RuntimeError):
    pass


class CapacityError(RuntimeError):
    pass


def kb_project(psi_flat: np.ndarray, proj, dv: float) -> np.ndarray:
    """c[a, i] = dV sum_l beta_a(l) psi_i(l), shape (A, m)."""
    if proj.matrix.shape[0] == 0:
        return np.zeros((0, psi_flat.shape[0]))
    return dv * (proj.matrix @ psi_flat.T)


def apply_h_local(psi: np.ndarray, veff: np.ndarray, h) -> np.ndarray:
    """(-1/2 Laplacian_FD + V_eff) psi on the periodic fragment box (Eq. (5),
    kinetic and local terms)."""
    return -0.5 * laplacian_periodic(psi, h) + veff[None] * psi


def apply_h(psi: np.ndarray, veff: np.ndarray, proj, h, dv: float) -> np.ndarray:
    """Full fragment Hamiltonian of Eq. (5) with V^alpha = 0:
    kinetic + V_eff + sum_a E_a |beta_a><beta_a|.  psi is (m, nz, ny, nx)."""
    out = apply_h_local(psi, veff, h)
    if proj.matrix.shape[0]:
        m = psi.shape[0]
        flat = psi.reshape(m, -1)
        c = kb_project(flat, proj, dv)                      # (A, m)
        nl = (proj.matrix.T @ (proj.energy[:, None] * c)).T  # (m, n)
        out = out + nl.reshape(psi.shape)
    return out


def _sym(a: np.ndarray) -> np.ndarray:
    return 0.5 * (a + a.T)


def cholesky_orthonormalize(psi_flat: np.ndarray, dv: float, *others):
    """S = sym(dV Psi Psi^T) = L L^T; Psi <- L^-1 Psi (and the same for others)."""
    s = _sym(dv * (psi_flat @ psi_flat.T))
    try:
        l = np.linalg.cholesky(s)
    except np.linalg.LinAlgError as exc:
        raise NotSPDError(str(exc)) from exc
    out = [scipy.linalg.solve_triangular(l, psi_flat, lower=True)]
    for o in others:
        out.append(scipy.linalg.solve_triangular(l, o, lower=True))
    return out


def canonical_signs(u: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry (lowest index on
    ties) is positive."""
    idx = np.argmax(np.abs(u), axis=0)
    s = np.sign(u[idx, np.arange(u.shape[1])])
    s[s == 0] = 1.0
    return u * s[None, :]


def cg_eigensolver(psi: np.ndarray, hop, n_sweeps: int, dv: float):
    """Band-by-band CG on span(Psi) followed by Rayleigh-Ritz.

    psi: (m, n) orthonormal rows (dV inner product).  hop(X) applies H^alpha to
    rows of X.  Returns (psi, eps, w) with eps ascending and w = H psi rows
    *before* the Rayleigh-Ritz rotation is not returned (only psi, eps).

    Per sweep s (f = 1 for every band):
      (a) Hs = sym(<Psi, W>)            (b) G = W - Hs Psi
      (c) gamma_i = <g_i, g_i>; beta_i = gamma_i / gamma_prev_i (Fletcher-Reeves,
          0 on the first sweep or when gamma_prev_i = 0)
      (d) P = -G + beta P_prev          (e) P <- P - <Psi, P>^T Psi
      (f) nu_i = <p_i, p_i>; p_hat = p / sqrt(nu) (theta_i = 0 if nu_i <= 1e-300)
      (g) Q = H p_hat                   (h) a = <psi,w>, b = <p_hat,w>, c = <p_hat,q>
      (i) theta = atan2(-2b, c - a) / 2  (exact minimiser of the 2x2 Rayleigh quotient)
      (j) psi <- cos psi + sin p_hat,  w <- cos w + sin q
      (k) P_prev <- P (after (e)), gamma_prev <- gamma
      (l) S = sym(<Psi, Psi>) = L L^T; Psi <- L^-1 Psi, W <- L^-1 W
    then Rayleigh-Ritz: sym(<Psi, W>) = U diag(eps) U^T, Psi <- U^T Psi.
    """
    m = psi.shape[0]
    w = hop(psi)
    p_prev = np.zeros_like(psi)
    gamma_prev = np.zeros(m)
    for s in range(n_sweeps):
        hs_full = dv * (psi @ w.T)                  # <psi_i, w_j>
        hs = _sym(hs_full)
        g = w - hs @ psi
        gamma = dv * np.einsum("ij,ij->i", g, g)
        if s == 0:
            beta = np.zeros(m)
        else:
            beta = np.where(gamma_prev > 0.0, gamma / np.where(gamma_prev > 0.0, gamma_prev, 1.0), 0.0)
        p = -g + beta[:, None] * p_prev
        x = dv * (psi @ p.T)                        # <psi_i, p_j>
        p = p - x.T @ psi
        nu = dv * np.einsum("ij,ij->i", p, p)
        live = nu > 1e-300
        inv = np.where(live, 1.0 / np.sqrt(np.where(live, nu, 1.0)), 0.0)
        p_hat = p * inv[:, None]
        q = hop(p_hat)
        a = np.diag(hs_full).copy()
        b = dv * np.einsum("ij,ij->i", p_hat, w)
        c = dv * np.einsum("ij,ij->i", p_hat, q)
        theta = np.where(live, 0.5 * np.arctan2(-2.0 * b, c - a), 0.0)
        cs, sn = np.cos(theta), np.sin(theta)
        psi = cs[:, None] * psi + sn[:, None] * p_hat
        w = cs[:, None] * w + sn[:, None] * q
        p_prev = p
        gamma_prev = gamma
        psi, w = cholesky_orthonormalize(psi, dv, w)
    hs = _sym(dv * (psi @ w.T))
    eps, u = np.linalg.eigh(hs)
    u = canonical_signs(u)
    psi = u.T @ psi
    return psi, eps


def core_weights(psi_flat: np.ndarray, core_mask: np.ndarray, dv: float) -> np.ndarray:
    """w_i = dV sum_{l in core} psi_i(l)^2: the weight of orbital i inside the
    core, so that the core-projected density of Eq. (3) integrates to
    sum_i 2 f_i w_i."""
    pc = psi_flat[:, core_mask]
    return dv * np.einsum("ij,ij->i", pc, pc)


def fermi_occupation(x: np.ndarray) -> np.ndarray:
    """f(x) = 1 / (1 + e^x), evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    pos = x >= 0
    t = np.exp(-x[pos])
    out[pos] = t / (1.0 + t)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def electron_count(mu: float, eps: np.ndarray, w: np.ndarray, sigma: float) -> float:
    return float(np.sum(2.0 * fermi_occupation((eps - mu) / sigma) * w))


def fermi_level(eps: np.ndarray, w: np.ndarray, n_electrons: float, sigma: float) -> float:
    """Global chemical potential (Sec. 2.2): the mu with
    N(mu) = sum_alpha sum_i 2 f((eps_i^alpha - mu) / sigma) w_i^alpha = N_e,
    by bisection on [min eps - 50 sigma, max eps + 50 sigma] until the midpoint
    equals an end point or 200 halvings.  N is strictly increasing, so mu is
    unique.  Raises CapacityError when sum 2 w < N_e (1 - 1e-12)."""
    eps = np.asarray(eps, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cap = float(np.sum(2.0 * w))
    if cap < n_electrons * (1.0 - 1e-12):
        raise CapacityError(f"fragment states hold {cap:.6f} < {n_electrons} electrons")
    lo = float(eps.min()) - 50.0 * sigma
    hi = float(eps.max()) + 50.0 * sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if electron_count(mid, eps, w, sigma) < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def fragment_density(psi_flat: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """rho_alpha(l) = sum_i 2 f_i psi_i(l)^2 (Eq. (4), spin-unpolarised)."""
    return np.einsum("i,ij->j", 2.0 * occ, psi_flat * psi_flat)
