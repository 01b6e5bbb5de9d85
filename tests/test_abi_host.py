"""C-ABI checks that need no GPU: the library loads, exports every function
that include/dcdft.h declares, and its host-side validation reports each error
with a status code and a message (validation runs before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_21125_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcdft.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2606_21125_amd import build
        build.build()
    return B.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dcdft_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(B.EXPORTED) == set(names)


def test_status_strings(lib):
    for code in range(0, -10, -1):
        s = lib.dcdft_status_string(code)
        assert s and len(s) > 1
    assert lib.dcdft_status_string(-42) == b"unknown status"


def _params(**over):
    from workloads.systems import small_system
    sysm = small_system((12, 12, 12), (7.2, 7.2, 7.2), n_atoms=2, seed=1)
    keep = {}
    pos = np.ascontiguousarray(sysm.positions)
    spi = np.ascontiguousarray(sysm.species_index)
    sp = (B.DcdftSpecies * 1)()
    s = sysm.species[0]
    sp[0] = B.DcdftSpecies(s.valence, s.vloc_depth, s.vloc_sigma, s.kb_energy, s.kb_sigma, s.kb_rcut)
    p = B.DcdftParams()
    p.n_grid[:] = [12, 12, 12]
    p.cell[:] = [7.2, 7.2, 7.2]
    p.num_fragment[:] = [2, 2, 1]
    p.num_rgrid_buffer[:] = [2, 2, 0]
    p.n_atoms = 2
    p.atom_pos = pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.atom_species = spi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    p.n_species = 1
    p.species = ctypes.cast(sp, ctypes.POINTER(B.DcdftSpecies))
    p.nstate_frag = None
    p.nstate_frag_uniform = 8
    p.n_electrons = 4.0
    p.smearing = 0.05
    p.mixing = 0.3
    p.cg_sweeps = 4
    p.precision = 0
    p.batched = 1
    p.seed = 1
    keep.update(pos=pos, spi=spi, sp=sp)
    for k, v in over.items():
        if k in ("n_grid", "num_fragment", "num_rgrid_buffer", "cell"):
            getattr(p, k)[:] = v
        else:
            setattr(p, k, v)
    return p, keep


def _setup_status(lib, p):
    ctx = ctypes.c_void_p()
    st = lib.dcdft_setup(ctypes.byref(p) if p is not None else None, ctypes.byref(ctx))
    msg = B.dcdft_last_error(None)
    if st == 0:
        lib.dcdft_destroy(ctx)
    return st, msg


@pytest.mark.parametrize("over,code,needle", [
    (dict(n_grid=[12, 13, 12]), -2, "not divisible"),
    (dict(num_rgrid_buffer=[4, 2, 0]), -2, "exceeds"),
    (dict(smearing=0.0), -1, "smearing"),
    (dict(mixing=1.5), -1, "mixing"),
    (dict(cg_sweeps=0), -1, "cg_sweeps"),
    (dict(nstate_frag_uniform=81), -1, "range 1..80"),
    # one fragment (the conventional calculation) takes the large-orbital path
    (dict(num_fragment=[1, 1, 1], num_rgrid_buffer=[0, 0, 0], nstate_frag_uniform=4097), -1,
     "range 1..4096"),
    (dict(n_electrons=-1.0), -1, "n_electrons"),
    (dict(precision=7), -1, "PREC"),
    (dict(n_species=0), -1, "species"),
])
def test_setup_validation_errors(lib, over, code, needle):
    p, keep = _params(**over)
    st, msg = _setup_status(lib, p)
    assert st == code, (st, msg)
    assert needle.lower() in msg.lower()


def test_setup_rejects_nonfinite_positions_and_null(lib):
    p, keep = _params()
    keep["pos"][0, 1] = np.nan
    st, msg = _setup_status(lib, p)
    assert st == -6 and "not finite" in msg
    st, msg = _setup_status(lib, None)
    assert st == -1
    ctx = ctypes.c_void_p()
    assert lib.dcdft_setup(None, None) == -1


def test_null_safe_calls(lib):
    lib.dcdft_destroy(None)
    assert lib.dcdft_scf_step(None, None) == -1
    buf = ctypes.create_string_buffer(8)
    assert lib.dcdft_last_error(None, buf, 0) == -1
    assert lib.dcdft_kernel_timing(None, 1) == -1
    assert lib.dcdft_fix_density(None, 1) == -1
    assert lib.dcdft_set_template(None, 1.0) == -1
    assert lib.dcdft_lcfo_build(None, 0.0, 1e-7, None) == -1
    assert lib.dcdft_lcfo_hamiltonian(None, None, 0, None) == -1
    assert lib.dcdft_lcfo_basis(None, 0, None, 0, None) == -1
    assert lib.dcdft_lcfo_block(None, 0, 0, None, 0, None, None) == -1
    assert lib.dcdft_autotune(None, None, None) == -1
    assert lib.dcdft_get_launch(None, None, None, None, None, None) == -1
    assert lib.dcdft_set_launch(None, 1, 4, 1, 2) == -1


@pytest.mark.parametrize("over", [
    dict(),
    # 200 orbitals in one fragment pass validation (large-orbital path)
    dict(num_fragment=[1, 1, 1], num_rgrid_buffer=[0, 0, 0], nstate_frag_uniform=200),
])
def test_valid_setup_without_gpu_reports_hip_error(lib, over):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible; the GPU tests cover a successful setup")
    p, keep = _params(**over)
    st, msg = _setup_status(lib, p)
    assert st == -7 and "device" in msg.lower()
