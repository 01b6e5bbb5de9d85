"""Synthetic structures and run configurations.

The paper's a-Si coordinates and liquid-water snapshot are not available, so
the workloads are seeded stand-ins with the same cell sizes, grid densities and
fragment shapes (Sec. 3.1-3.3 give the paper's own systems).  Every array here
is generated from ``numpy.random.default_rng(seed)``.

Units are Hartree atomic units (bohr, Ha).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Species:
    """Model pseudopotential of one species.

    The paper uses norm-conserving Troullier-Martins pseudopotentials
    (Sec. 2.2); the synthetic workloads replace them with a Gaussian local well
    and one s-type Kleinman-Bylander projector, parameters below.
    """
    name: str
    valence: float
    vloc_depth: float      # D in V(r) = D exp(-r^2 / (2 sigma^2))  (Ha)
    vloc_sigma: float      # sigma of the local well (bohr)
    kb_energy: float       # E_a of the projector (Ha)
    kb_sigma: float        # r_c of the Gaussian projector (bohr)
    kb_rcut: float         # hard support radius of the projector (bohr)


SI = Species("Si", 4.0, -3.0, 1.0, 1.0, 1.5, 4.5)
O = Species("O", 6.0, -3.0, 1.0, 1.0, 1.5, 4.5)
H = Species("H", 1.0, -3.0, 1.0, 1.0, 1.5, 4.5)


@dataclasses.dataclass
class System:
    cell: np.ndarray            # (3,) periodic box lengths (bohr)
    positions: np.ndarray       # (n_atoms, 3) bohr, wrapped into [0, L)
    species_index: np.ndarray   # (n_atoms,) int32 index into ``species``
    species: List[Species]

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_electrons(self) -> float:
        val = np.array([s.valence for s in self.species])
        return float(val[self.species_index].sum())


@dataclasses.dataclass
class RunConfig:
    """Grid, fragment decomposition and solver settings of one workload.

    ``num_fragment``, ``nstate_frag`` and ``num_rgrid_buffer`` are the
    fragment keywords of the paper's input table (Table 1).
    """
    name: str
    system: System
    n_grid: tuple
    num_fragment: tuple
    num_rgrid_buffer: tuple
    nstate_frag: np.ndarray     # (F,) int32, orbitals per fragment
    smearing: float = 0.01      # kT (Ha)
    mixing: float = 0.3
    cg_sweeps: int = 4
    scf_iterations: int = 20
    seed: int = 1

    @property
    def n_fragments(self) -> int:
        f = self.num_fragment
        return int(f[0] * f[1] * f[2])

    @property
    def fragment_shape(self) -> tuple:
        return tuple(self.n_grid[d] // self.num_fragment[d] + 2 * self.num_rgrid_buffer[d]
                     for d in range(3))


def diamond_si(cells: Sequence[int], a: float, jitter: float, seed: int) -> System:
    """Diamond-structure Si supercell of ``cells`` conventional cubes of edge ``a``,
    each coordinate displaced by N(0, jitter^2)."""
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0],
                      [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75],
                      [0.75, 0.75, 0.25]])
    cx, cy, cz = cells
    cell = np.array([cx * a, cy * a, cz * a], dtype=np.float64)
    pos = []
    for k in range(cz):
        for j in range(cy):
            for i in range(cx):
                pos.append((basis + np.array([i, j, k])) * a)
    pos = np.concatenate(pos, axis=0)
    rng = np.random.default_rng(seed)
    pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    pos = np.mod(pos, cell)
    return System(cell, pos, np.zeros(pos.shape[0], dtype=np.int32), [SI])


def _random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_box(n_mol: int, edge: float, d_oh: float, angle_deg: float,
              min_oo: float, seed: int) -> System:
    """Random liquid-water-like box: O atoms by random sequential addition with a
    minimum periodic O-O distance, each molecule with a uniformly random
    orientation."""
    rng = np.random.default_rng(seed)
    cell = np.array([edge, edge, edge], dtype=np.float64)
    ox = np.empty((0, 3))
    # spatial hashing keeps the rejection test O(1) per trial
    nb = max(1, int(edge // min_oo))
    bw = edge / nb
    buckets: Dict[tuple, List[int]] = {}
    placed = []
    tries = 0
    while len(placed) < n_mol:
        tries += 1
        if tries > 200 * n_mol:
            raise RuntimeError("water_box: random sequential addition did not finish")
        p = rng.uniform(0.0, edge, size=3)
        b = tuple((p // bw).astype(int) % nb)
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((b[0] + dx) % nb, (b[1] + dy) % nb, (b[2] + dz) % nb)
                    for idx in buckets.get(key, ()):
                        d = p - placed[idx]
                        d -= edge * np.round(d / edge)
                        if d @ d < min_oo * min_oo:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            buckets.setdefault(b, []).append(len(placed))
            placed.append(p)
    ox = np.array(placed)
    half = math.radians(angle_deg) / 2.0
    h1 = np.array([d_oh * math.sin(half), 0.0, d_oh * math.cos(half)])
    h2 = np.array([-d_oh * math.sin(half), 0.0, d_oh * math.cos(half)])
    pos = []
    spc = []
    for p in ox:
        r = _random_rotation(rng)
        pos.extend([p, p + r @ h1, p + r @ h2])
        spc.extend([0, 1, 1])
    pos = np.mod(np.array(pos), cell)
    return System(cell, pos, np.array(spc, dtype=np.int32), [O, H])


def fragment_valence_counts(system: System, n_grid, num_fragment, buffer) -> np.ndarray:
    """Valence electrons of the atoms whose position lies inside each fragment box
    (core plus buffer, periodic).  Used only to size uneven orbital counts."""
    cell = system.cell
    h = cell / np.array(n_grid)
    nf = np.array(num_fragment)
    ncore = np.array(n_grid) // nf
    b = np.array(buffer)
    val = np.array([s.valence for s in system.species])[system.species_index]
    counts = np.zeros(int(nf.prod()))
    for fz in range(nf[2]):
        for fy in range(nf[1]):
            for fx in range(nf[0]):
                a = np.array([fx, fy, fz])
                lo = (a * ncore - b) * h          # box start (may be negative)
                ext = (ncore + 2 * b) * h
                rel = np.mod(system.positions - lo, cell)
                inside = np.all(rel < ext, axis=1)
                counts[fx + nf[0] * (fy + nf[1] * fz)] = val[inside].sum()
    return counts


def superposed_density(system: System, n_grid, width: float = 1.2,
                       background: float = 0.25) -> np.ndarray:
    """Input density of the fixed-density mode, a stand-in for a density read from
    a file: a fraction 1 - background of every atom's valence charge in a Gaussian
    of the given width (bohr) centred on the atom (periodic images, cut at 5
    widths), the rest spread uniformly, then scaled so that dV * sum = N_e on the
    grid.  Returns (Nz, Ny, Nx), x fastest."""
    n = np.array(n_grid, dtype=np.int64)
    h = system.cell / n
    val = np.array([s.valence for s in system.species])[system.species_index]
    rho = np.zeros((n[2], n[1], n[0]))
    for a in range(system.n_atoms):
        idx, fac = [], []
        for d in range(3):
            half = min(int(math.ceil(5.0 * width / h[d])), int((n[d] - 1) // 2))
            c = int(math.floor(system.positions[a, d] / h[d]))
            k = np.arange(c - half, c + half + 1)
            r = k * h[d] - system.positions[a, d]
            idx.append(np.mod(k, n[d]))
            fac.append(np.exp(-r * r / (2.0 * width * width)))
        g = fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
        rho[np.ix_(idx[2], idx[1], idx[0])] += val[a] * g / g.sum()
    rho = (1.0 - background) * rho + background * val.sum() / float(n.prod())
    return rho * (system.n_electrons / (float(np.prod(h)) * rho.sum()))


CONFIG_NAMES = {
    1: "si64_fp64",
    2: "asi512",
    3: "water4134",
    4: "si64_grad",
    5: "si4096",
}


def config(k: int, nstate: Optional[int] = None) -> RunConfig:
    """The five synthetic workloads (seeded with the config number).

    1: 64-atom diamond Si, 32^3 grid, 2x2x2 fragments of 24^3.
    2: 512-atom a-Si-like cell, 64^3 grid, 4x4x4 fragments of 24^3, 64 orbitals.
    3: 1378 H2O in a 65.2 bohr cube, 160^3 grid, 8x8x8 fragments of 32^3,
       uneven orbital counts ceil(1.2 * N_loc / 2).
    4: same system as 1 (used for the band-energy gradient checks).
    5: 4096-atom diamond Si, 128^3 grid, 8x8x8 fragments of 24^3, 68 orbitals.
    """
    if k in (1, 4):
        sysm = diamond_si((2, 2, 2), 10.26, 0.05, seed=k)
        # 48 states per 24^3 fragment cannot hold the 32 electrons a core needs
        # (core weight ~ (16/24)^3), so the default is 64, the count used for
        # the identical fragment geometry of the 512-atom cell.
        m = 64 if nstate is None else nstate
        return RunConfig(CONFIG_NAMES[k], sysm, (32, 32, 32), (2, 2, 2), (4, 4, 4),
                         np.full(8, m, dtype=np.int32), scf_iterations=20, seed=k)
    if k == 2:
        sysm = diamond_si((4, 4, 4), 10.26, 0.3, seed=2)
        m = 64 if nstate is None else nstate
        return RunConfig(CONFIG_NAMES[2], sysm, (64, 64, 64), (4, 4, 4), (4, 4, 4),
                         np.full(64, m, dtype=np.int32), scf_iterations=20, seed=2)
    if k == 3:
        sysm = water_box(1378, 65.2, 1.81, 104.5, 4.7, seed=3)
        counts = fragment_valence_counts(sysm, (160, 160, 160), (8, 8, 8), (6, 6, 6))
        m = np.ceil(1.2 * counts / 2.0).astype(np.int32)
        if nstate is not None:
            m = np.full(512, nstate, dtype=np.int32)
        return RunConfig(CONFIG_NAMES[3], sysm, (160, 160, 160), (8, 8, 8), (6, 6, 6),
                         m, scf_iterations=20, seed=3)
    if k == 5:
        sysm = diamond_si((8, 8, 8), 10.26, 0.05, seed=5)
        m = 68 if nstate is None else nstate
        return RunConfig(CONFIG_NAMES[5], sysm, (128, 128, 128), (8, 8, 8), (4, 4, 4),
                         np.full(512, m, dtype=np.int32), scf_iterations=300, seed=5)
    raise ValueError(f"unknown config {k}")


def si_cells_config(cells: Sequence[int], num_fragment: Sequence[int] = (1, 1, 1),
                    buffer: Sequence[int] = (0, 0, 0), points_per_cell: int = 16,
                    seed: int = 7, nstate: Optional[int] = None) -> RunConfig:
    """Diamond Si supercell of ``cells`` cubes (a = 10.26 bohr, jitter 0.05 bohr) on
    points_per_cell grid points per cube edge (h = 0.641 bohr, the grid density of
    the other Si workloads).  With one fragment and no buffer this is the
    conventional calculation of the same cell, with ceil(1.2 N_e / 2) orbitals;
    with fragments, every fragment gets ceil(1.2 N_loc / 2) orbitals from the
    valence inside its box (unless nstate is given)."""
    sysm = diamond_si(cells, 10.26, 0.05, seed=seed)
    n_grid = tuple(int(points_per_cell * c) for c in cells)
    nf = int(np.prod(num_fragment))
    if nstate is not None:
        m = np.full(nf, nstate, dtype=np.int32)
    elif nf == 1 and not any(buffer):
        m = np.array([int(math.ceil(1.2 * sysm.n_electrons / 2.0))], dtype=np.int32)
    else:
        counts = fragment_valence_counts(sysm, n_grid, num_fragment, buffer)
        m = np.ceil(1.2 * counts / 2.0).astype(np.int32)
    name = f"si{sysm.n_atoms}_{'x'.join(map(str, num_fragment))}"
    return RunConfig(name, sysm, n_grid, tuple(num_fragment), tuple(buffer), m,
                     scf_iterations=20, seed=seed)


def small_system(n_grid=(12, 12, 12), cell=(7.2, 7.2, 7.2), n_atoms=2, seed=11,
                 depth=-3.0, sigma=1.0, kb_e=1.0, kb_sigma=1.0, kb_rcut=2.4,
                 valence=2.0) -> System:
    """A few atoms at random positions in a small box (for brute-force tests)."""
    rng = np.random.default_rng(seed)
    cellv = np.array(cell, dtype=np.float64)
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * cellv
    sp = Species("X", valence, depth, sigma, kb_e, kb_sigma, kb_rcut)
    return System(cellv, pos, np.zeros(n_atoms, dtype=np.int32), [sp])
