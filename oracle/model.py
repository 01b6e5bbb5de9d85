"""Model potentials of the synthetic workloads (test infrastructure only).

The paper's fragment Hamiltonian (Eq. (5)) contains a local pseudopotential,
a non-local pseudopotential defined within the fragment, the Hartree
potential of the total density and the LDA exchange-correlation potential of
the fragment density (Perdew-Zunger 1981 parametrisation, Sec. 2.2).  The
synthetic workloads use:

* a Gaussian local well per atom, V_loc(r) = sum_a D exp(-|r - R_a|^2 / (2 s^2)),
  minimum-image distance, each term included where |r - R_a| <= 10 s
  (the neglected tail is below 1e-21 of D);
* one s-type Kleinman-Bylander projector per atom,
  beta_a = b_a / ||b_a||, b_a(r) = exp(-|r - R_a|^2 / (2 r_c^2)) for
  |r - R_a| <= R_cut and 0 beyond, normalised on the global grid
  (||b||^2 = dV sum b^2); V_NL = sum_a E_a |beta_a><beta_a|.
  Inside a fragment the projector is the restriction of the global one to the
  fragment box (no renormalisation, no wrap across the fragment seam).

Pins: V_loc and beta against direct O(N * n_atoms) evaluation on small grids,
normalisation, LDA exchange closed form, V_xc = d(rho eps_xc)/d rho by central
differences, continuity of the two correlation branches at r_s = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np
import scipy.sparse as sp

VLOC_CUTOFF_SIGMAS = 10.0


def grid_spacing(cell, n_grid) -> np.ndarray:
    return np.asarray(cell, dtype=np.float64) / np.asarray(n_grid, dtype=np.float64)


def _axis_candidates(center: float, radius: float, h: float, n: int, length: float):
    """Wrapped grid indices within radius of center along one axis and their
    minimum-image displacements."""
    lo = math.floor((center - radius) / h) - 1
    hi = math.ceil((center + radius) / h) + 1
    idx = np.unique(np.mod(np.arange(lo, hi + 1), n))
    d = idx * h - center
    d = d - length * np.round(d / length)
    keep = np.abs(d) <= radius
    return idx[keep], d[keep]


def _ball(center, radius, h, n_grid, cell):
    """Global flat indices and squared min-image distances of grid points with
    |r - center| <= radius."""
    ix, dx = _axis_candidates(center[0], radius, h[0], n_grid[0], cell[0])
    iy, dy = _axis_candidates(center[1], radius, h[1], n_grid[1], cell[1])
    iz, dz = _axis_candidates(center[2], radius, h[2], n_grid[2], cell[2])
    r2 = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
    g = (ix[None, None, :] + n_grid[0] * (iy[None, :, None] + n_grid[1] * iz[:, None, None]))
    keep = r2 <= radius * radius
    return g[keep], r2[keep]


def local_potential(system, n_grid) -> np.ndarray:
    """V_loc on the global grid, shape (Nz, Ny, Nx)."""
    n_grid = tuple(int(v) for v in n_grid)
    h = grid_spacing(system.cell, n_grid)
    v = np.zeros(int(np.prod(n_grid)))
    for a in range(system.n_atoms):
        s = system.species[system.species_index[a]]
        g, r2 = _ball(system.positions[a], VLOC_CUTOFF_SIGMAS * s.vloc_sigma, h, n_grid,
                      system.cell)
        np.add.at(v, g, s.vloc_depth * np.exp(-r2 / (2.0 * s.vloc_sigma ** 2)))
    return v.reshape(n_grid[2], n_grid[1], n_grid[0])


@dataclasses.dataclass
class Projector:
    atom: int
    energy: float
    index: np.ndarray   # global flat indices of the support
    value: np.ndarray   # normalised beta values there


def kb_projectors(system, n_grid) -> List[Projector]:
    n_grid = tuple(int(v) for v in n_grid)
    h = grid_spacing(system.cell, n_grid)
    dv = float(np.prod(h))
    out = []
    for a in range(system.n_atoms):
        s = system.species[system.species_index[a]]
        g, r2 = _ball(system.positions[a], s.kb_rcut, h, n_grid, system.cell)
        b = np.exp(-r2 / (2.0 * s.kb_sigma ** 2))
        b = b / math.sqrt(dv * float(np.sum(b * b)))
        out.append(Projector(a, s.kb_energy, g, b))
    return out


@dataclasses.dataclass
class FragmentProjectors:
    atoms: np.ndarray       # atom ids with a non-zero restriction
    energy: np.ndarray      # E_a for those atoms
    matrix: sp.csr_matrix   # (A, n) restricted beta values


def fragment_projectors(projectors: List[Projector], frag, n_global: int) -> FragmentProjectors:
    loc = np.full(n_global, -1, dtype=np.int64)
    loc[frag.global_index] = np.arange(frag.n)
    rows, cols, vals, atoms, energies = [], [], [], [], []
    for p in projectors:
        l = loc[p.index]
        keep = l >= 0
        if not np.any(keep):
            continue
        r = len(atoms)
        atoms.append(p.atom)
        energies.append(p.energy)
        rows.append(np.full(int(keep.sum()), r))
        cols.append(l[keep])
        vals.append(p.value[keep])
    if atoms:
        mat = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                            shape=(len(atoms), frag.n))
    else:
        mat = sp.csr_matrix((0, frag.n))
    return FragmentProjectors(np.array(atoms, dtype=np.int64), np.array(energies), mat)


# Perdew-Zunger 1981, unpolarised Ceperley-Alder fit (constants of that paper)
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
RHO_FLOOR = 1e-20


def lda_pz81(rho: np.ndarray):
    """(eps_xc, v_xc) per point for the unpolarised LDA; zero where rho < 1e-20."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    vxc = np.zeros_like(rho)
    ok = rho >= RHO_FLOOR
    r = rho[ok]
    rs = (3.0 / (4.0 * math.pi * r)) ** (1.0 / 3.0)
    # exchange: eps_x = -(3/4) (3/pi)^(1/3) rho^(1/3) = -(3/(4 pi)) (9 pi / 4)^(1/3) / r_s
    cx = (3.0 / (4.0 * math.pi)) * (9.0 * math.pi / 4.0) ** (1.0 / 3.0)
    ex = -cx / rs
    vx = 4.0 / 3.0 * ex
    ec = np.empty_like(rs)
    vc = np.empty_like(rs)
    hi = rs >= 1.0
    sq = np.sqrt(rs[hi])
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * rs[hi]
    ec[hi] = PZ_GAMMA / den
    vc[hi] = ec[hi] * (1.0 + 7.0 / 6.0 * PZ_BETA1 * sq + 4.0 / 3.0 * PZ_BETA2 * rs[hi]) / den
    lo = ~hi
    rl = rs[lo]
    ln = np.log(rl)
    ec[lo] = PZ_A * ln + PZ_B + PZ_C * rl * ln + PZ_D * rl
    vc[lo] = PZ_A * ln + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * rl * ln \
        + (2.0 * PZ_D - PZ_C) / 3.0 * rl
    eps[ok] = ex + ec
    vxc[ok] = vx + vc
    return eps, vxc
