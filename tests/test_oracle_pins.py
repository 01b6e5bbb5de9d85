"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, brute force, invariants).  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import grid as og
from oracle import model as om
from oracle import rng as orng
from oracle import scf as oscf
from oracle import solver as osol
from tests.helpers import brute_gaussian_on_grid, dense_kinetic, tiny_config
from workloads.systems import small_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --- finite-difference operator (Eq. (5), kinetic term) -------------------------------

def test_fd_coefficients_match_fornberg_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fornberg_d2_halfwidth4.txt"))
            if not l.startswith("#")]
    table = [Fraction(int(r[1]), int(r[2])) for r in rows]
    assert og.fd_second_derivative_coefficients(4) == table


def test_fd_stencil_exact_on_polynomials():
    c = og.FD_COEFFS
    h = 0.37
    for p in range(0, 10):
        f = lambda x: x ** p
        x0 = 0.3
        approx = (c[0] * f(x0) + sum(c[k] * (f(x0 + k * h) + f(x0 - k * h)) for k in range(1, 5))) / h ** 2
        exact = p * (p - 1) * x0 ** (p - 2) if p >= 2 else 0.0
        assert abs(approx - exact) <= 1e-8 * max(1.0, abs(exact)), p


def test_laplacian_is_eighth_order_on_smooth_periodic_field():
    errs = []
    for n in (16, 32):
        length = 7.0
        h = length / n
        x = np.arange(n) * h
        k = 2 * math.pi / length
        f = np.sin(k * x)[None, None, :] * np.ones((n, n, 1)) + np.cos(2 * k * x)[:, None, None]
        lap = og.laplacian_periodic(f, (h, h, h))
        exact = -k * k * np.sin(k * x)[None, None, :] * np.ones((n, n, 1)) \
            - 4 * k * k * np.cos(2 * k * x)[:, None, None]
        errs.append(np.abs(lap - exact).max())
    rate = math.log2(errs[0] / errs[1])
    assert 7.5 < rate < 8.6, (errs, rate)


def test_free_electron_spectrum_closed_form():
    """V = 0, no projectors: the CG solver reaches the closed-form FD spectrum
    eps(k) = sum_d (1/(2 h_d^2)) (-c0 - 2 sum_j c_j cos(2 pi j k_d / n_d))."""
    n = (10, 10, 10)
    h = (0.5, 0.5, 0.5)
    dv = 0.125
    c = og.FD_COEFFS
    lam1 = [np.array([(-c[0] - 2 * sum(c[j] * math.cos(2 * math.pi * j * k / n[d]) for j in range(1, 5)))
                      / (2 * h[d] ** 2) for k in range(n[d])]) for d in range(3)]
    spec = np.sort((lam1[2][:, None, None] + lam1[1][None, :, None] + lam1[0][None, None, :]).ravel())
    m = 7   # k = 0 and the six |k| = 1 modes: a closed shell
    proj = om.FragmentProjectors(np.zeros(0, int), np.zeros(0), __import__("scipy").sparse.csr_matrix((0, 1000)))
    veff = np.zeros((10, 10, 10))
    hop = lambda x: osol.apply_h(x.reshape((x.shape[0], 10, 10, 10)), veff, proj, h, dv).reshape(x.shape[0], -1)
    psi = orng.initial_orbitals(5, 0, m, (10, 10, 10)).reshape(m, -1)
    psi = osol.cholesky_orthonormalize(psi, dv)[0]
    for _ in range(40):
        psi, eps = osol.cg_eigensolver(psi, hop, 6, dv)
    np.testing.assert_allclose(eps, spec[:m], rtol=0, atol=1e-12)


# --- model potentials -----------------------------------------------------------------

def test_local_potential_and_projectors_against_brute_force():
    sysm = small_system((12, 10, 14), (7.2, 6.4, 8.1), n_atoms=3, seed=3, kb_rcut=2.2)
    n_grid = (12, 10, 14)
    v = om.local_potential(sysm, n_grid)
    brute = brute_gaussian_on_grid(sysm, n_grid, lambda s: om.VLOC_CUTOFF_SIGMAS * s.vloc_sigma,
                                   lambda s, r2: s.vloc_depth * np.exp(-r2 / (2 * s.vloc_sigma ** 2)))
    np.testing.assert_allclose(v, sum(brute), rtol=1e-13, atol=1e-14)
    projs = om.kb_projectors(sysm, n_grid)
    dv = float(np.prod(sysm.cell / np.array(n_grid)))
    raw = brute_gaussian_on_grid(sysm, n_grid, lambda s: s.kb_rcut,
                                 lambda s, r2: np.exp(-r2 / (2 * s.kb_sigma ** 2)))
    for p, r in zip(projs, raw):
        dense = np.zeros(r.size)
        dense[p.index] = p.value
        ref = r.ravel() / math.sqrt(dv * float(np.sum(r * r)))
        np.testing.assert_allclose(dense, ref, rtol=1e-13, atol=1e-15)
        assert abs(dv * np.sum(p.value ** 2) - 1.0) < 1e-13


def _tiny_fragment_operator(n=(8, 9, 10), n_atoms=2, seed=4):
    sysm = small_system((n[0], n[1], n[2]), (4.8, 5.4, 6.0), n_atoms=n_atoms, seed=seed, kb_rcut=2.0)
    n_grid = n
    h = sysm.cell / np.array(n_grid)
    dv = float(np.prod(h))
    frags = og.build_fragments(n_grid, (1, 1, 1), (0, 0, 0))
    projs = om.kb_projectors(sysm, n_grid)
    fp = om.fragment_projectors(projs, frags[0], int(np.prod(n_grid)))
    rng = np.random.default_rng(seed)
    veff = rng.normal(size=(n[2], n[1], n[0])) * 0.3
    dense = dense_kinetic((n[2], n[1], n[0]), h, og.FD_COEFFS) + np.diag(veff.ravel())
    bm = fp.matrix.toarray()
    dense = dense + dv * bm.T @ np.diag(fp.energy) @ bm
    return sysm, h, dv, veff, fp, dense


def test_apply_h_matches_independent_dense_matrix_and_is_symmetric():
    sysm, h, dv, veff, fp, dense = _tiny_fragment_operator()
    shape = veff.shape
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3,) + shape)
    hx = osol.apply_h(x, veff, fp, h, dv)
    ref = (dense @ x.reshape(3, -1).T).T.reshape(hx.shape)
    np.testing.assert_allclose(hx, ref, rtol=1e-12, atol=1e-11)
    assert np.abs(dense - dense.T).max() < 1e-12
    y = rng.normal(size=(1,) + shape)
    hy = osol.apply_h(y, veff, fp, h, dv)
    lhs = dv * np.sum(x[:1] * hy)
    rhs = dv * np.sum(hx[:1] * y)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_cg_solver_reaches_dense_lowest_eigenvalues():
    sysm, h, dv, veff, fp, dense = _tiny_fragment_operator()
    evals = np.linalg.eigvalsh(dense)
    m = 6
    while abs(evals[m] - evals[m - 1]) < 1e-3:   # keep a gap at the subspace edge
        m += 1
    shape = veff.shape
    hop = lambda x: osol.apply_h(x.reshape((x.shape[0],) + shape), veff, fp, h, dv).reshape(x.shape[0], -1)
    psi = orng.initial_orbitals(9, 0, m, shape).reshape(m, -1)
    psi = osol.cholesky_orthonormalize(psi, dv)[0]
    traces = []
    for _ in range(60):
        psi, eps = osol.cg_eigensolver(psi, hop, 4, dv)
        traces.append(eps.sum())
    # the dense matrix is the operator on the dV-orthonormal grid basis up to a scale:
    # H psi = eps psi with psi normalised by dV - the eigenvalues are the same.
    np.testing.assert_allclose(eps, evals[:m], rtol=0, atol=1e-10)
    assert all(b <= a + 1e-12 for a, b in zip(traces, traces[1:]))


# --- fragments (Sec. 2.2, Eqs. (2)-(3)) -----------------------------------------------

@pytest.mark.parametrize("n_grid,nf,b", [((32, 32, 32), (2, 2, 2), (4, 4, 4)),
                                         ((64, 64, 64), (4, 4, 4), (4, 4, 4)),
                                         ((24, 30, 12), (3, 5, 1), (2, 3, 0)),
                                         ((160, 160, 160), (8, 8, 8), (6, 6, 6))])
def test_core_indicators_partition_the_cell(n_grid, nf, b):
    frags = og.build_fragments(n_grid, nf, b)
    count = np.zeros(int(np.prod(n_grid)), dtype=np.int64)
    for f in frags:
        np.add.at(count, f.global_index[f.core_mask], 1)
        assert len(np.unique(f.global_index)) == f.n   # no point twice in a fragment
    assert np.all(count == 1)


# --- occupations and the global chemical potential ------------------------------------

def test_fermi_level_properties():
    rng = np.random.default_rng(1)
    eps = np.sort(rng.normal(size=200))
    w = rng.uniform(0.2, 1.0, size=200)
    ne = 0.9 * float(np.sum(2 * w))
    sigma = 0.01
    mu = osol.fermi_level(eps, w, ne, sigma)
    n = osol.electron_count(mu, eps, w, sigma)
    assert abs(n - ne) <= 1e-10 * ne
    grid = np.linspace(eps.min() - 1, eps.max() + 1, 400)
    counts = [osol.electron_count(x, eps, w, sigma) for x in grid]
    assert all(b >= a for a, b in zip(counts, counts[1:]))
    # symmetric two-level system with unit weights holds two electrons at the midpoint
    mu2 = osol.fermi_level(np.array([-0.3, 0.5]), np.array([1.0, 1.0]), 2.0, 0.05)
    assert abs(mu2 - 0.1) < 1e-14
    # f(x) + f(-x) = 1 and no overflow at large |x|
    x = np.array([-800.0, -3.0, 0.0, 2.5, 800.0])
    f = osol.fermi_occupation(x)
    np.testing.assert_allclose(f + osol.fermi_occupation(-x), 1.0, rtol=0, atol=1e-15)
    assert np.all(np.isfinite(f))
    with pytest.raises(osol.CapacityError):
        osol.fermi_level(eps, w, 2.1 * float(np.sum(w)), sigma)


# --- Hartree potential -----------------------------------------------------------------

def test_poisson_closed_form_and_cg_agreement():
    n_grid = (16, 12, 20)
    cell = np.array([6.0, 5.0, 7.5])
    h = cell / np.array(n_grid)
    x = np.arange(n_grid[0]) * h[0]
    k = 3
    rho = np.cos(2 * math.pi * k * x / cell[0])[None, None, :] * np.ones((n_grid[2], n_grid[1], 1))
    v = oscf.poisson_fd(rho, h)
    c = og.FD_COEFFS
    lam = (c[0] + 2 * sum(c[j] * math.cos(2 * math.pi * j * k / n_grid[0]) for j in range(1, 5))) / h[0] ** 2
    np.testing.assert_allclose(v, -4 * math.pi * rho / lam, rtol=0, atol=1e-12)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0, 1, size=(n_grid[2], n_grid[1], n_grid[0]))
    v = oscf.poisson_fd(rho, h)
    resid = og.laplacian_periodic(v, h) + 4 * math.pi * (rho - rho.mean())
    assert np.abs(resid).max() < 1e-10
    assert abs(v.mean()) < 1e-13
    v_cg = oscf.poisson_fd_cg(rho, h, tol=1e-14)
    assert np.abs(v - v_cg).max() < 1e-11


# --- exchange-correlation ------------------------------------------------------------

def test_lda_pz81_closed_forms_and_derivative():
    rho = np.array([1e-4, 1e-3, 0.01, 0.05, 0.2, 1.0, 3.0])
    eps, v = om.lda_pz81(rho)
    # exchange alone: eps_x = -(3/4)(3/pi)^(1/3) rho^(1/3)
    rs = (3 / (4 * math.pi * rho)) ** (1 / 3)
    ex = -0.75 * (3 / math.pi) ** (1 / 3) * rho ** (1 / 3)
    ec = eps - ex
    assert np.all(ec < 0) and np.all(ec > -0.2)
    # v_xc = d(rho eps_xc)/d rho by central differences
    for r in rho:
        t = 1e-6 * r
        ep, _ = om.lda_pz81(np.array([r + t]))
        em, _ = om.lda_pz81(np.array([r - t]))
        fd = ((r + t) * ep[0] - (r - t) * em[0]) / (2 * t)
        _, vv = om.lda_pz81(np.array([r]))
        assert abs(fd - vv[0]) < 1e-7 * max(1.0, abs(vv[0])), r
    # the two correlation branches meet at r_s = 1 (to the precision of the fit)
    rho1 = 3 / (4 * math.pi)
    e_hi, _ = om.lda_pz81(np.array([rho1 * (1 - 1e-9)]))
    e_lo, _ = om.lda_pz81(np.array([rho1 * (1 + 1e-9)]))
    assert abs(e_hi[0] - e_lo[0]) < 1e-4
    # floor
    e0, v0 = om.lda_pz81(np.array([0.0, 1e-21]))
    assert np.all(e0 == 0) and np.all(v0 == 0)


# --- generator of the initial orbitals --------------------------------------------------

def _unmix(z):
    """Inverse of the SplitMix64 finaliser (undo xor-shifts and odd multiplies)."""
    z = np.uint64(z)
    def unxorshift(x, s):
        y = x
        for _ in range(64 // s + 1):
            y = x ^ (y >> np.uint64(s))
        return y
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    with np.errstate(over="ignore"):
        z = unxorshift(z, 31)
        z = np.uint64((int(z) * inv2) % (1 << 64))
        z = unxorshift(z, 27)
        z = np.uint64((int(z) * inv1) % (1 << 64))
        z = unxorshift(z, 30)
    return z


def test_splitmix64_is_the_sequential_stream_and_uniform():
    seed = 12345
    # sequential definition: state += golden; output = mix(state)
    state = seed
    seq = []
    for _ in range(5):
        state = (state + 0x9E3779B97F4A7C15) % (1 << 64)
        seq.append(state)
    outs = orng.splitmix64_outputs(seed, np.arange(1, 6, dtype=np.uint64))
    for s, o in zip(seq, outs):
        assert int(_unmix(o)) == s
    u = orng.splitmix64_uniform(7, np.arange(1, 200001, dtype=np.uint64))
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    assert u.min() >= 0 and u.max() < 1
    hist, _ = np.histogram(u, bins=20, range=(0, 1))
    assert np.all(np.abs(hist - 10000) < 500)


# --- band-energy gradient --------------------------------------------------------------

def test_band_energy_gradient_exact_central_differences_and_euler():
    sysm, h, dv, veff, fp, dense = _tiny_fragment_operator()
    shape = veff.shape
    rng = np.random.default_rng(8)
    m = 4
    psi = rng.normal(size=(m,) + shape) * 0.1
    f = rng.uniform(0.1, 2.0, size=m)
    e = oracle.band_energy(psi, veff, fp, h, dv, f)
    gp, gv = oracle.band_energy_grad(psi, veff, fp, h, dv, f)
    for _ in range(4):
        d = rng.normal(size=psi.shape)
        t = 1e-3
        fd = (oracle.band_energy(psi + t * d, veff, fp, h, dv, f)
              - oracle.band_energy(psi - t * d, veff, fp, h, dv, f)) / (2 * t)
        assert abs(fd - np.sum(gp * d)) < 1e-9 * max(1.0, abs(fd))
        dvv = rng.normal(size=veff.shape)
        fdv = (oracle.band_energy(psi, veff + t * dvv, fp, h, dv, f)
               - oracle.band_energy(psi, veff - t * dvv, fp, h, dv, f)) / (2 * t)
        assert abs(fdv - np.sum(gv * dvv)) < 1e-9 * max(1.0, abs(fdv))
    assert abs(np.sum(psi * gp) - 2 * e) < 1e-10 * abs(e)
    pot = float(np.sum(f[:, None] * dv * (psi.reshape(m, -1) ** 2 * veff.ravel()[None])))
    assert abs(np.sum(veff * gv) - pot) < 1e-12 * max(1.0, abs(pot))
