"""Band-energy functional and its gradient (test infrastructure only).

E(Psi, V) = sum_i f_i <psi_i | H[V] | psi_i>, with fixed weights f (not
differentiated through mu).  With <x, y> = dV sum x y and a symmetric H:
  dE/dpsi_i(l) = 2 f_i dV (H psi_i)(l),
  dE/dV(l)     = dV sum_i f_i psi_i(l)^2,
the second being dV times the fragment density of Eq. (4) when f_i carries
the spin factor and the Fermi occupation.  Pins: exact central differences
(E is quadratic in psi and linear in V), Euler identities
sum psi . dE/dpsi = 2 E and sum V . dE/dV = sum f <psi|V|psi>.
"""
import numpy as np

from .solver import apply_h


def band_energy(psi, veff, proj, h, dv, f) -> float:
    hp = apply_h(psi, veff, proj, h, dv)
    m = psi.shape[0]
    return float(dv * np.sum(f[:, None] * (psi.reshape(m, -1) * hp.reshape(m, -1))))


def band_energy_grad(psi, veff, proj, h, dv, f):
    hp = apply_h(psi, veff, proj, h, dv)
    g_psi = 2.0 * dv * f.reshape((-1,) + (1,) * (psi.ndim - 1)) * hp
    g_v = dv * np.einsum("i,i...->...", f, psi * psi)
    return g_psi, g_v
