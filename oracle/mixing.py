"""Density mixing of the SCF loop (test infrastructure only).

The paper iterates the total density "by the same procedure as conventional
DFT" (Sec. 2.2) and names no mixing scheme.  Two readings are implemented:

* linear mixing, rho <- rho + a (rho_out - rho), for rho_tot and every fragment
  density (the workloads' stated scheme);
* Pulay (DIIS) mixing with a Kerker preconditioner, the usual scheme of
  conventional grid and plane-wave codes: from the last M pairs
  (rho_in^(j), R^(j) = rho_out^(j) - rho_in^(j)) the weights c minimise
  |sum_j c_j R^(j)|^2 subject to sum_j c_j = 1, and
      rho_new = sum_j c_j rho_in^(j) + a K[ sum_j c_j R^(j) ],
  K(q) = q^2 / (q^2 + q0^2) on the Fourier modes of the periodic grid, with q^2
  the symbol of minus the same nine-point Laplacian the Poisson solve uses
  (K(0) = 0).

Fragment densities.  Each rho_alpha is split into the total density gathered
on the fragment box and a deviation, rho_alpha = rho_tot(g(l)) + delta_alpha(l).
On core points delta_alpha^out = 0 (Eq. (3)), and delta_alpha^in stays 0 there.
The deviations are mixed with the same weights c and step a, without the
preconditioner (they live on the fragment boxes, not the periodic cell):
      delta_new = sum_j c_j delta_in^(j) + a sum_j c_j (delta_out^(j) - delta_in^(j)).
With linear mixing this split changes nothing: rho_alpha <- rho_alpha + a
(rho_alpha^out - rho_alpha).

Weights.  The bordered system [[A, 1], [1^T, 0]] [c; lambda] = [0; 1], A_ij =
sum_g R^(i)(g) R^(j)(g), is solved by Gaussian elimination with partial
pivoting, oldest history entry first.  When a pivot falls to 1e-12 of the
largest |A_ij| or below (dependent residuals), the history is cut to the newest
entry, whose weight is then 1.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .grid import FD_COEFFS, HALF_WIDTH


def minus_laplacian_symbol(n_grid, h) -> np.ndarray:
    """q^2(k) = -(eigenvalue of the periodic nine-point FD Laplacian) on the
    Fourier modes, shape (Nz, Ny, Nx); zero for the constant mode."""
    lam = []
    for d in range(3):
        k = np.arange(n_grid[d])
        s = FD_COEFFS[0] + 2.0 * sum(FD_COEFFS[j] * np.cos(2.0 * np.pi * j * k / n_grid[d])
                                     for j in range(1, HALF_WIDTH + 1))
        lam.append(s / (h[d] * h[d]))
    return -(lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :])


def kerker_filter(r: np.ndarray, n_grid, h, q0: float) -> np.ndarray:
    """K r with K(q) = q^2 / (q^2 + q0^2) mode by mode (FFT of the periodic grid),
    K = 0 on the constant mode.  r has shape (Nz, Ny, Nx)."""
    q2 = minus_laplacian_symbol(n_grid, h)
    k = q2 / (q2 + q0 * q0)
    k[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(np.fft.fftn(r) * k))


def pulay_weights(a: np.ndarray):
    """Weights c (sum 1) minimising c^T A c, by Gaussian elimination with partial
    pivoting on the bordered system.  Returns (c, ok); ok is False when a pivot
    is at most 1e-12 max|A| (then c is None)."""
    k = a.shape[0]
    m = np.zeros((k + 1, k + 2))
    m[:k, :k] = a
    m[:k, k] = 1.0
    m[k, :k] = 1.0
    m[k, k + 1] = 1.0
    tiny = 1e-12 * float(np.abs(a).max())
    for col in range(k + 1):
        piv = col + int(np.argmax(np.abs(m[col:, col])))
        if abs(m[piv, col]) <= tiny:
            return None, False
        if piv != col:
            m[[col, piv]] = m[[piv, col]]
        for r in range(col + 1, k + 1):
            f = m[r, col] / m[col, col]
            m[r, col:] -= f * m[col, col:]
    x = np.zeros(k + 1)
    for r in range(k, -1, -1):
        x[r] = (m[r, k + 1] - float(np.dot(m[r, r + 1:k + 1], x[r + 1:]))) / m[r, r]
    return x[:k], True


class PulayKerkerMixer:
    """Pulay mixing with a Kerker preconditioner of rho_tot, and the same
    weights for the fragment deviations (see the module text)."""

    def __init__(self, n_grid, h, alpha: float, q0: float, history: int):
        if not (alpha > 0.0) or q0 < 0.0 or history < 1:
            raise ValueError("alpha > 0, q0 >= 0, history >= 1")
        self.n_grid = tuple(int(v) for v in n_grid)
        self.h = np.asarray(h, dtype=np.float64)
        self.alpha = float(alpha)
        self.q0 = float(q0)
        self.history = int(history)
        self.rho: List[np.ndarray] = []      # rho_in^(j)
        self.res: List[np.ndarray] = []      # R^(j)
        self.d_in: List[List[np.ndarray]] = []
        self.d_res: List[List[np.ndarray]] = []

    def mix(self, rho_in: np.ndarray, rho_out: np.ndarray, d_in: Sequence[np.ndarray],
            d_out: Sequence[np.ndarray]):
        """One mixing step.  rho_in, rho_out: (Nz, Ny, Nx); d_in, d_out: the
        fragment deviations.  Returns (rho_new, [delta_new per fragment])."""
        self.rho.append(np.array(rho_in, dtype=np.float64))
        self.res.append(np.asarray(rho_out, dtype=np.float64) - rho_in)
        self.d_in.append([np.array(x, dtype=np.float64) for x in d_in])
        self.d_res.append([np.asarray(o, dtype=np.float64) - i for i, o in zip(d_in, d_out)])
        if len(self.rho) > self.history:
            for lst in (self.rho, self.res, self.d_in, self.d_res):
                lst.pop(0)
        k = len(self.res)
        flat = [r.ravel() for r in self.res]
        a = np.array([[float(np.dot(flat[i], flat[j])) for j in range(k)] for i in range(k)])
        c, ok = pulay_weights(a)
        if not ok:
            for lst in (self.rho, self.res, self.d_in, self.d_res):
                del lst[:-1]
            c = np.ones(1)
        rho_bar = sum(cj * r for cj, r in zip(c, self.rho))
        res_bar = sum(cj * r for cj, r in zip(c, self.res))
        rho_new = rho_bar + self.alpha * (kerker_filter(res_bar, self.n_grid, self.h, self.q0)
                                          if self.q0 > 0.0 else res_bar)
        d_new = []
        for f in range(len(d_in)):
            di = sum(cj * e[f] for cj, e in zip(c, self.d_in))
            dr = sum(cj * e[f] for cj, e in zip(c, self.d_res))
            d_new.append(di + self.alpha * dr)
        return rho_new, d_new
