"""DC-LCFO basis and Hamiltonian matrix of the whole system (Sec. 2.3, Eqs. (6)-(9)).
Test infrastructure only: a plain FP64 statement of the post-processing that
follows a converged DC-DFT run; the diagonalisation of the global matrix is not
part of it.

Per fragment alpha:
  1. select the fragment orbitals with eps_i < eps_cut;
  2. project them on the core, phibar_i = phi_i on core points, 0 elsewhere (the
     same projection as Eq. (3));
  3. overlap S_ij = <phibar_i|phibar_j> (Eq. (6), inner products with dV);
  4. eigenpairs S v_l = sigma_l v_l; the eigenvectors with sigma_l > lambda_cut
     define the basis lambda_l = sum_j phibar_j v_jl / sqrt(sigma_l), orthonormal
     within the core and therefore over the whole system (Eq. (7)); basis
     functions are ordered by ascending sigma.
Global matrix (Eq. (9)), H^alpha the fragment Hamiltonian applied on the fragment
box with its own V_eff:
  same fragment:      <lambda_i^a|H^a lambda_j^a>
  different fragments: 1/2 [<H^a lambda_i^a|lambda_j^b> + <lambda_i^a|H^b lambda_j^b>]
with every inner product taken on the global grid (each function placed at its
fragment box's global points, zero elsewhere).

Pins (tests/test_oracle_lcfo.py): one unbuffered fragment gives the Ritz
spectrum of the selected orbitals; buffers wider than the stencil and two
projector radii give Lambda^T H Lambda with an independently built dense global
Hamiltonian; narrow buffers give a symmetric matrix; the basis is orthonormal and
its size matches the singular values of the projected orbitals.
"""
from __future__ import annotations

from typing import List

import numpy as np

from .solver import apply_h


def lcfo_basis(psi: np.ndarray, eps: np.ndarray, core_mask: np.ndarray, dv: float,
               eps_cut: float, lambda_cut: float) -> np.ndarray:
    """Basis functions of one fragment on its box, shape (n_basis, n)."""
    phibar = psi[eps < eps_cut] * core_mask[None, :]
    s = dv * (phibar @ phibar.T)
    sigma, v = np.linalg.eigh(s)
    keep = sigma > lambda_cut
    return (v[:, keep] / np.sqrt(sigma[keep])[None, :]).T @ phibar


def lcfo_hamiltonian(o, basis: List[np.ndarray], veffs: List[np.ndarray]) -> np.ndarray:
    """The global matrix of Eq. (9) for the bases of every fragment of the oracle
    state o (an OracleSCF), H^alpha taking V_eff = veffs[alpha] (fragment box
    points, the potential the orbitals were computed in: OracleSCF.veff_last).
    Rows and columns: fragments in order, each fragment's basis in its own order."""
    ng = o.n_global
    lam_g, hlam_g = [], []
    for a, f in enumerate(o.frags):
        lam = basis[a]
        nb = lam.shape[0]
        veff = np.asarray(veffs[a]).reshape(f.shape)
        hl = apply_h(lam.reshape((nb,) + f.shape), veff, o.fproj[a], o.h, o.dv).reshape(nb, -1)
        lg = np.zeros((nb, ng))
        hg = np.zeros((nb, ng))
        lg[:, f.global_index] = lam
        hg[:, f.global_index] = hl
        lam_g.append(lg)
        hlam_g.append(hg)
    sizes = [b.shape[0] for b in basis]
    off = np.concatenate([[0], np.cumsum(sizes)])
    h = np.zeros((off[-1], off[-1]))
    for a in range(len(basis)):
        for b in range(len(basis)):
            if a == b:
                blk = o.dv * (lam_g[a] @ hlam_g[a].T)
            else:
                blk = 0.5 * o.dv * (hlam_g[a] @ lam_g[b].T + lam_g[a] @ hlam_g[b].T)
            h[off[a]:off[a + 1], off[b]:off[b + 1]] = blk
    return h
