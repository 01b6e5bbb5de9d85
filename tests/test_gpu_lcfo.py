"""DC-LCFO basis and global Hamiltonian (Sec. 2.3, Eqs. (6)-(9)) on the GPU against
the FP64 oracle, after a few SCF steps taken by both (same orbitals to ~1e-12).

The basis of a fragment is fixed only up to rotations inside degenerate overlap
eigenvalues, so the comparison uses what is unique: the basis count of every
fragment (exact), the span of every fragment's basis (projector distance), the
spectrum of the whole matrix, the eigenvalues of every same-fragment block and the
singular values of every neighbour block.  Cut-offs are placed away from the
eigenvalues they separate, so that both sides select the same functions."""
import math

import numpy as np
import pytest

import oracle
from oracle.lcfo import lcfo_basis, lcfo_hamiltonian
from tests.gpu_common import require_gpu
from tests.test_gpu_parity import _ragged_tiny
import workloads

pytestmark = pytest.mark.gpu

HARTREE_EV = 27.211386


def _gpu(cfg, **kw):
    from paper_2606_21125_amd import DCDFT
    return DCDFT.from_config(cfg, **kw)


def _eps_cut(o):
    """mu + 0.1 eV (the paper's choice), moved to the middle of the gap it falls in
    if an eigenvalue lies within 1e-6 Ha of it."""
    cut = o.mu + 0.1 / HARTREE_EV
    allv = np.sort(np.concatenate(o.eps))
    if np.min(np.abs(allv - cut)) < 1e-6:
        k = int(np.searchsorted(allv, cut))
        cut = 0.5 * (allv[k - 1] + allv[k])
    return cut


def _lambda_cut(o, eps_cut, target=1e-7):
    """target unless an overlap eigenvalue lies within a factor 10 of it; then the
    geometric middle of the widest gap between 1e-10 and 1e-4."""
    sig = []
    for a, f in enumerate(o.frags):
        phibar = o.psi[a][o.eps[a] < eps_cut] * f.core_mask[None, :]
        sig.extend(np.linalg.eigvalsh(o.dv * phibar @ phibar.T))
    sig = np.sort(np.array(sig))
    if not np.any((sig > target / 10) & (sig < target * 10)):
        return target
    grid = sig[(sig > 1e-10) & (sig < 1e-4)]
    pts = np.concatenate([[1e-10], grid, [1e-4]])
    k = int(np.argmax(np.log(pts[1:]) - np.log(pts[:-1])))
    return float(np.sqrt(pts[k] * pts[k + 1]))


def _subspace_distance(a, b, dv):
    if a.shape[0] == 0 and b.shape[0] == 0:
        return 0.0
    r = b - (dv * (b @ a.T)) @ a
    return math.sqrt(2.0 * dv * float(np.sum(r * r)))


def _compare(o, d, cfg, basis_ref, h_ref, tol_h, tol_span):
    nb = [b.shape[0] for b in basis_ref]
    off = np.concatenate([[0], np.cumsum(nb)])
    h = d.dcdft_lcfo_hamiltonian()
    assert h.shape == h_ref.shape
    for a in range(cfg.n_fragments):
        lam = d.dcdft_lcfo_basis(a)
        assert lam.shape[0] == nb[a], a
        np.testing.assert_allclose(o.dv * lam @ lam.T, np.eye(nb[a]), rtol=0, atol=1e-11)
        assert _subspace_distance(lam, basis_ref[a], o.dv) < tol_span, a
    ev = np.linalg.eigvalsh(0.5 * (h + h.T))
    ev_ref = np.linalg.eigvalsh(0.5 * (h_ref + h_ref.T))
    print("global spectrum max diff", np.abs(ev - ev_ref).max())
    np.testing.assert_allclose(ev, ev_ref, rtol=0, atol=tol_h)
    for a in range(cfg.n_fragments):
        sa = slice(off[a], off[a + 1])
        np.testing.assert_allclose(np.linalg.eigvalsh(0.5 * (h[sa, sa] + h[sa, sa].T)),
                                   np.linalg.eigvalsh(0.5 * (h_ref[sa, sa] + h_ref[sa, sa].T)),
                                   rtol=0, atol=tol_h)
        for b in range(cfg.n_fragments):
            if b == a:
                continue
            sb = slice(off[b], off[b + 1])
            # neighbour blocks are assembled symmetric
            assert np.array_equal(h[sa, sb], h[sb, sa].T)
            np.testing.assert_allclose(np.linalg.svd(h[sa, sb], compute_uv=False),
                                       np.linalg.svd(h_ref[sa, sb], compute_uv=False),
                                       rtol=0, atol=tol_h)


def _wide_dc():
    """Two fragments with 40 x 36 x 12 boxes (planes past 1024 points: the tiled
    stencil applies H^alpha to the basis) and 12 and 21 orbitals."""
    from tests.test_gpu_wide_plane import _wide
    cfg = _wide(12, num_fragment=(1, 1, 2), buffer=(0, 0, 2), n_grid=(40, 36, 16))
    cfg.nstate_frag = np.array([12, 21], dtype=np.int32)
    return cfg


@pytest.mark.parametrize("which", ["ragged", "config1", "wide"])
def test_lcfo_matches_oracle(which):
    require_gpu()
    cfg = {"config1": lambda: workloads.config(1), "ragged": _ragged_tiny,
           "wide": _wide_dc}[which]()
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg) as d:
        for _ in range(3):
            o.step()
            d.dcdft_scf_step()
        ecut = _eps_cut(o)
        lcut = _lambda_cut(o, ecut)
        basis = [lcfo_basis(o.psi[a], o.eps[a], f.core_mask.astype(float), o.dv, ecut, lcut)
                 for a, f in enumerate(o.frags)]
        h_ref = lcfo_hamiltonian(o, basis, [o.veff_last[a] for a in range(len(o.frags))])
        info = d.dcdft_lcfo_build(ecut, lcut)
        print(which, info, "eps_cut", ecut, "lambda_cut", lcut)
        assert info["n_basis"] == sum(b.shape[0] for b in basis)
        _compare(o, d, cfg, basis, h_ref, 1e-9, 1e-8)
        # every block accessed alone equals its slice of the dense matrix
        h = d.dcdft_lcfo_hamiltonian()
        nb = [b.shape[0] for b in basis]
        off = np.concatenate([[0], np.cumsum(nb)])
        for a in range(cfg.n_fragments):
            for b in range(cfg.n_fragments):
                assert np.array_equal(d.dcdft_lcfo_block(a, b),
                                      h[off[a]:off[a + 1], off[b]:off[b + 1]]), (a, b)
        # a second build with a lower cut-off selects fewer functions
        d.dcdft_lcfo_build(ecut - 0.05, lcut)
        assert d.dcdft_lcfo_hamiltonian().shape[0] < h_ref.shape[0]


def test_lcfo_from_mixed_precision_orbitals():
    require_gpu()
    cfg = _ragged_tiny()
    o = oracle.OracleSCF(cfg)
    with _gpu(cfg, precision=1) as d:
        for _ in range(3):
            o.step()
            d.dcdft_scf_step()
        ecut = _eps_cut(o)
        lcut = _lambda_cut(o, ecut)
        basis = [lcfo_basis(o.psi[a], o.eps[a], f.core_mask.astype(float), o.dv, ecut, lcut)
                 for a, f in enumerate(o.frags)]
        h_ref = lcfo_hamiltonian(o, basis, [o.veff_last[a] for a in range(len(o.frags))])
        d.dcdft_lcfo_build(ecut, lcut)
        _compare(o, d, cfg, basis, h_ref, 1e-5, 1e-4)


def test_lcfo_errors():
    require_gpu()
    from paper_2606_21125_amd.binding import DcdftError
    cfg = _ragged_tiny()
    with _gpu(cfg) as d:
        with pytest.raises(DcdftError):
            d.dcdft_lcfo_build(0.0, 1e-7)            # no step taken yet
        d.dcdft_scf_step()
        with pytest.raises(DcdftError):
            d.dcdft_lcfo_hamiltonian()               # nothing built
        with pytest.raises(DcdftError):
            d.dcdft_lcfo_build(0.0, 0.0)             # lambda_cut must be > 0
        with pytest.raises(DcdftError):
            d.dcdft_lcfo_build(float("nan"), 1e-7)
