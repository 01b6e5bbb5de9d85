"""Independent constructions used to pin the oracle (dense matrices, brute force)."""
import math

import numpy as np
import scipy.linalg

from workloads.systems import RunConfig, small_system


def dense_second_derivative_1d(n: int, h: float, coeffs) -> np.ndarray:
    col = np.zeros(n)
    col[0] += coeffs[0]
    for j in range(1, len(coeffs)):
        col[j % n] += coeffs[j]
        col[(-j) % n] += coeffs[j]
    return scipy.linalg.circulant(col) / (h * h)


def dense_kinetic(shape_zyx, h_xyz, coeffs) -> np.ndarray:
    """-1/2 Laplacian as a dense matrix on a periodic box, x fastest."""
    nz, ny, nx = shape_zyx
    dx = dense_second_derivative_1d(nx, h_xyz[0], coeffs)
    dy = dense_second_derivative_1d(ny, h_xyz[1], coeffs)
    dz = dense_second_derivative_1d(nz, h_xyz[2], coeffs)
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    lap = (np.kron(iz, np.kron(iy, dx)) + np.kron(iz, np.kron(dy, ix))
           + np.kron(dz, np.kron(iy, ix)))
    return -0.5 * lap


def brute_gaussian_on_grid(system, n_grid, radius_of, value_of):
    """Sum over atoms of value_of(species, r2) over every grid point (no ball
    enumeration), min-image distances, zero beyond radius_of(species)."""
    nx, ny, nz = n_grid
    h = system.cell / np.array(n_grid)
    gx, gy, gz = np.meshgrid(np.arange(nx) * h[0], np.arange(ny) * h[1], np.arange(nz) * h[2],
                             indexing="ij")
    out = []
    for a in range(system.n_atoms):
        s = system.species[system.species_index[a]]
        d = [gx - system.positions[a, 0], gy - system.positions[a, 1], gz - system.positions[a, 2]]
        d = [di - system.cell[k] * np.round(di / system.cell[k]) for k, di in enumerate(d)]
        r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        v = np.where(r2 <= radius_of(s) ** 2, value_of(s, r2), 0.0)
        out.append(np.transpose(v, (2, 1, 0)))  # -> (z, y, x)
    return out


def tiny_config(n_grid=(10, 10, 10), cell=(6.0, 6.0, 6.0), n_atoms=2, nstate=6,
                num_fragment=(1, 1, 1), buffer=(0, 0, 0), seed=11, valence=2.0,
                sweeps=4, smearing=0.05, mixing=0.3, kb_rcut=2.4):
    sysm = small_system(n_grid, cell, n_atoms, seed, valence=valence, kb_rcut=kb_rcut)
    nf = int(np.prod(num_fragment))
    return RunConfig("tiny", sysm, tuple(n_grid), tuple(num_fragment), tuple(buffer),
                     np.full(nf, nstate, dtype=np.int32), smearing=smearing, mixing=mixing,
                     cg_sweeps=sweeps, scf_iterations=10, seed=seed)
