"""The boundary's convention for caller-allocated outputs: a buffer one element
too small gives DCDFT_ERR_ARG with the required size in the error message and
leaves the buffer untouched; the exact size succeeds.  Checked through the raw C
entry points on the 64-atom system after one step, for every call that fills a
caller buffer (host and device copies of the density, eigenvalues, global and
fragment fields, orbitals, the DC-LCFO basis and global matrix)."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import require_gpu
import workloads

pytestmark = pytest.mark.gpu

PD = ctypes.POINTER(ctypes.c_double)


def _check_small_then_exact(lib, ctx, call, need):
    """call(buf_pointer, size) -> status; need: the required element count."""
    from paper_2606_21125_amd import binding as B
    small = np.full(max(1, need), 7.0)
    st = call(small.ctypes.data_as(PD), need - 1)
    msg = B.dcdft_last_error(ctx)
    assert st == -1, (st, msg)
    assert str(need) in msg, (need, msg)
    assert np.all(small == 7.0)
    exact = np.zeros(need)
    assert call(exact.ctypes.data_as(PD), need) == 0, B.dcdft_last_error(ctx)
    return exact


def test_every_output_buffer_too_small_by_one():
    require_gpu()
    import torch
    from paper_2606_21125_amd import DCDFT
    from paper_2606_21125_amd import binding as B
    cfg = workloads.config(1)
    ng = int(np.prod(cfg.n_grid))
    with DCDFT.from_config(cfg) as d:
        info = d.dcdft_scf_step()
        lib, ctx = d._lib, d.ctx
        n = d.n
        m0 = int(cfg.nstate_frag[0])
        rho = _check_small_then_exact(lib, ctx, lambda p, k: lib.dcdft_density(ctx, p, k), ng)
        assert np.array_equal(rho, d.dcdft_density().ravel())
        for which in (B.FIELD_RHO_IN,):
            _check_small_then_exact(lib, ctx,
                                    lambda p, k: lib.dcdft_get_field(ctx, which, p, k), ng)
        _check_small_then_exact(lib, ctx,
                                lambda p, k: lib.dcdft_get_fragment_field(ctx, 0, B.FFIELD_RHO_IN,
                                                                          p, k), n)
        _check_small_then_exact(lib, ctx, lambda p, k: lib.dcdft_get_orbitals(ctx, 1, p, k),
                                m0 * n)
        # eigenvalues: capacity one short of m
        eps = np.full(m0, 7.0)
        mm = ctypes.c_int32()
        st = lib.dcdft_eigenvalues(ctx, 0, eps.ctypes.data_as(PD), None, m0 - 1,
                                   ctypes.byref(mm))
        assert st == -1 and str(m0) in B.dcdft_last_error(ctx) and np.all(eps == 7.0)
        assert lib.dcdft_eigenvalues(ctx, 0, eps.ctypes.data_as(PD), None, m0,
                                     ctypes.byref(mm)) == 0 and mm.value == m0
        # device copy of the density
        dev = torch.full((ng,), 7.0, device="cuda", dtype=torch.float64)
        assert lib.dcdft_density_device(ctx, ctypes.c_void_p(dev.data_ptr()), ng - 1) == -1
        assert str(ng) in B.dcdft_last_error(ctx)
        assert bool((dev == 7.0).all())
        assert lib.dcdft_density_device(ctx, ctypes.c_void_p(dev.data_ptr()), ng) == 0
        assert np.array_equal(dev.cpu().numpy(), rho)
        # DC-LCFO basis and global matrix
        li = d.dcdft_lcfo_build(info["mu"] + 0.1 / 27.211386, 1e-7)
        nb = ctypes.c_int32()
        fb = 0
        for fb in range(cfg.n_fragments):   # a fragment with a nonempty basis
            assert lib.dcdft_lcfo_basis(ctx, fb, None, 0, ctypes.byref(nb)) == 0
            if nb.value > 0:
                break
        assert nb.value > 0
        _check_small_then_exact(lib, ctx,
                                lambda p, k: lib.dcdft_lcfo_basis(ctx, fb, p, k, ctypes.byref(nb)),
                                nb.value * n)
        nt = li["n_basis"]
        _check_small_then_exact(lib, ctx,
                                lambda p, k: lib.dcdft_lcfo_hamiltonian(ctx, p, k,
                                                                        ctypes.byref(nb)),
                                nt * nt)
