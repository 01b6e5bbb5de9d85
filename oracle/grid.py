"""Real-space grid, finite-difference kinetic operator and fragment geometry
(test infrastructure only).

Kinetic operator (Eq. (5), first term): -1/2 times the nine-point-per-axis
central second derivative, periodic on the box it acts on.  The coefficients
are the unique symmetric half-width-4 stencil exact for polynomials up to
degree 9; they are derived here in exact rational arithmetic.  Pinned by the
published Fornberg (1988) table, by the exact second derivative of x^2 .. x^8
and by the O(h^8) error of a smooth periodic function.

Fragments (Sec. 2.2 and Fig. 1): the periodic cell is cut into a regular
F_x x F_y x F_z grid of non-overlapping core boxes of n_core = N / F points
per axis; each fragment is its core extended by b buffer points on both sides
of every axis, n = n_core + 2 b points, with periodic boundary conditions on the
fragment box itself.  Local index l_d maps to global g_d = (a_d n_core_d - b_d +
l_d) mod N_d.  Pinned by the partition-of-unity of the core indicators.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import List

import numpy as np

HALF_WIDTH = 4


def fd_second_derivative_coefficients(half_width: int = HALF_WIDTH) -> List[Fraction]:
    """c_0..c_M of the symmetric stencil sum_k c_|k| f(x + k h) / h^2 ~ f''(x).

    Conditions: exactness on x^(2p), p = 0..M, at x = 0:
      p = 0: c_0 + 2 sum_j c_j = 0;  p = 1: 2 sum_j j^2 c_j = 2;
      p >= 2: sum_j j^(2p) c_j = 0.
    Solved by Gaussian elimination over the rationals."""
    m = half_width
    rows = []
    rhs = []
    # p = 0 row uses c_0
    rows.append([Fraction(1)] + [Fraction(2)] * m)
    rhs.append(Fraction(0))
    for p in range(1, m + 1):
        rows.append([Fraction(0)] + [Fraction(2 * j ** (2 * p)) for j in range(1, m + 1)])
        rhs.append(Fraction(2) if p == 1 else Fraction(0))
    n = m + 1
    a = [r[:] + [b] for r, b in zip(rows, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col] / a[col][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [a[i][n] / a[i][i] for i in range(n)]


FD_COEFFS = np.array([float(c) for c in fd_second_derivative_coefficients()])


def laplacian_periodic(u: np.ndarray, h, axes=(-1, -2, -3)) -> np.ndarray:
    """FD Laplacian of ``u`` over its last three axes (x is the last), periodic.

    ``h`` = (h_x, h_y, h_z)."""
    out = np.zeros_like(u)
    for d, ax in enumerate(axes):
        acc = FD_COEFFS[0] * u
        for k in range(1, HALF_WIDTH + 1):
            acc = acc + FD_COEFFS[k] * (np.roll(u, k, axis=ax) + np.roll(u, -k, axis=ax))
        out += acc / (h[d] * h[d])
    return out


@dataclasses.dataclass
class FragmentMap:
    """Geometry of one fragment alpha."""
    alpha: int
    origin: np.ndarray          # (3,) a_d * n_core_d - b_d  (global index of local 0)
    shape: tuple                # (nz, ny, nx)
    global_index: np.ndarray    # (n,) flattened global index of each local point
    core_mask: np.ndarray       # (n,) bool, local point lies in the core box

    @property
    def n(self) -> int:
        return int(self.global_index.size)


def build_fragments(n_grid, num_fragment, buffer) -> List[FragmentMap]:
    n_grid = np.array(n_grid)
    nf = np.array(num_fragment)
    b = np.array(buffer)
    if np.any(n_grid % nf):
        raise ValueError("grid not divisible by the fragment count")
    ncore = n_grid // nf
    nloc = ncore + 2 * b
    if np.any(nloc > n_grid):
        raise ValueError("fragment box larger than the cell")
    frags = []
    for az in range(nf[2]):
        for ay in range(nf[1]):
            for ax in range(nf[0]):
                a = np.array([ax, ay, az])
                origin = a * ncore - b
                lx = np.arange(nloc[0])
                ly = np.arange(nloc[1])
                lz = np.arange(nloc[2])
                gx = (origin[0] + lx) % n_grid[0]
                gy = (origin[1] + ly) % n_grid[1]
                gz = (origin[2] + lz) % n_grid[2]
                gidx = (gx[None, None, :] + n_grid[0] * (gy[None, :, None]
                                                         + n_grid[1] * gz[:, None, None]))
                cx = (lx >= b[0]) & (lx < b[0] + ncore[0])
                cy = (ly >= b[1]) & (ly < b[1] + ncore[1])
                cz = (lz >= b[2]) & (lz < b[2] + ncore[2])
                core = cz[:, None, None] & cy[None, :, None] & cx[None, None, :]
                alpha = ax + nf[0] * (ay + nf[1] * az)
                frags.append(FragmentMap(alpha, origin, (nloc[2], nloc[1], nloc[0]),
                                         gidx.ravel(), core.ravel()))
    return frags
