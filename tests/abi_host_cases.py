"""Host-side ABI cases for a library built under AddressSanitizer and
UndefinedBehaviorSanitizer, run in a process of its own with the sanitizer
runtime preloaded (tests/test_abi_sanitized.py starts it).  No GPU is needed:
every call either fails its argument checks or stops at the missing device.

The cases: status strings; every entry point with a NULL context; setup with
each documented validation error; and a seeded sweep over parameter sets with
extreme values (negative, zero, huge and non-finite sizes, spacings, counts and
species parameters), each set self-consistent in its array lengths (the caller's
side of the contract), every call expected to return a nonzero status with a
message.  Usage: python abi_host_cases.py <library path>."""
import ctypes
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2606_21125_amd import binding as B  # noqa: E402

INT_MAX = 2 ** 31 - 1


def null_ctx_calls(lib):
    lib.dcdft_destroy(None)
    skip = {"dcdft_setup", "dcdft_destroy", "dcdft_status_string", "dcdft_last_error"}
    for name in B.EXPORTED:
        if name in skip:
            continue
        fn = getattr(lib, name)
        args = []
        for t in fn.argtypes:
            if t in (ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int):
                args.append(0)
            elif t is ctypes.c_double:
                args.append(0.0)
            else:
                args.append(None)
        st = fn(*args)
        assert st == -1, (name, st)
    buf = ctypes.create_string_buffer(64)
    assert lib.dcdft_last_error(None, buf, 64) in (0, -1)


def make_params(rng, over=None):
    """A parameter set with consistent array lengths; 'over' fixes fields."""
    over = dict(over or {})
    keep = {}
    p = B.DcdftParams()
    # each field takes its first (valid) value with probability 0.8, so that some
    # sets pass validation and reach the device check
    pick = lambda vals: vals[0] if rng.random() < 0.8 else vals[int(rng.integers(len(vals)))]
    p.n_grid[:] = over.pop("n_grid", [pick([12, -1, 0, 1, 7, 64, 1 << 20, INT_MAX])
                                      for _ in range(3)])
    p.num_fragment[:] = over.pop("num_fragment", [pick([2, -1, 0, 1, 3, 1000, INT_MAX])
                                                  for _ in range(3)])
    p.num_rgrid_buffer[:] = over.pop("num_rgrid_buffer",
                                     [pick([2, -5, 0, 1000, 1 << 30, INT_MAX]) for _ in range(3)])
    p.cell[:] = over.pop("cell", [pick([7.2, -1.0, 0.0, np.nan, np.inf, 1e300])
                                  for _ in range(3)])
    n_species = over.pop("n_species", pick([1, 0, 2]))
    sp = (B.DcdftSpecies * max(1, n_species))()
    for s in range(n_species):
        sp[s] = B.DcdftSpecies(pick([4.0, -1.0]), pick([-3.0, np.nan]), pick([1.0, 0.0, -1.0]),
                               pick([1.0, np.inf]), pick([1.5, 0.0]), pick([2.0, -1.0, 0.0]))
    n_atoms = over.pop("n_atoms", pick([2, 0, 5]))
    pos = np.ascontiguousarray(rng.uniform(0, 7.2, size=(max(1, n_atoms), 3)))
    if n_atoms and rng.random() < 0.2:
        pos[0, 2] = pick([np.nan, np.inf])
    spi = np.ascontiguousarray(rng.integers(-1, max(1, n_species) + 1, size=max(1, n_atoms)),
                               dtype=np.int32)
    if rng.random() < 0.8:
        spi[:] = 0
    p.n_atoms = n_atoms
    p.atom_pos = pos.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if n_atoms else None
    p.atom_species = spi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if n_atoms else None
    p.n_species = n_species
    p.species = ctypes.cast(sp, ctypes.POINTER(B.DcdftSpecies)) if n_species else None
    nf = int(np.prod([max(0, v) for v in p.num_fragment], dtype=np.int64))
    if 0 < nf <= 4096 and rng.random() < 0.5:
        ns = np.ascontiguousarray(rng.choice([8, 80, -1, 0, 81, INT_MAX], size=nf,
                                             p=[0.45, 0.45, 0.025, 0.025, 0.025, 0.025]),
                                  dtype=np.int32)
        keep["ns"] = ns
        p.nstate_frag = ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    else:
        p.nstate_frag = None
    p.nstate_frag_uniform = over.pop("nstate_frag_uniform", pick([8, -1, 0, 81, INT_MAX]))
    p.n_electrons = pick([4.0, np.nan, -1.0])
    p.smearing = pick([0.05, 0.0, np.nan])
    p.mixing = pick([0.3, 0.0, 1.0, 1.5, np.nan])
    p.cg_sweeps = pick([4, 0, INT_MAX])
    p.precision = pick([0, 1, 7])
    p.batched = pick([1, 0, 2])
    p.seed = 1
    for k, v in over.items():
        setattr(p, k, v)
    keep.update(pos=pos, spi=spi, sp=sp)
    return p, keep


def setup_status(lib, p):
    ctx = ctypes.c_void_p()
    st = lib.dcdft_setup(ctypes.byref(p), ctypes.byref(ctx))
    msg = B.dcdft_last_error(None)
    if st == 0:
        lib.dcdft_destroy(ctx)
    return st, msg


def main(path):
    lib = B.load_library(path)
    for code in range(0, -10, -1):
        assert lib.dcdft_status_string(code)
    assert lib.dcdft_status_string(-42) == b"unknown status"
    null_ctx_calls(lib)
    ctx = ctypes.c_void_p()
    assert lib.dcdft_setup(None, ctypes.byref(ctx)) == -1
    assert lib.dcdft_setup(None, None) == -1
    rng = np.random.default_rng(2024)
    seen = set()
    for _ in range(3000):
        p, keep = make_params(rng)
        st, msg = setup_status(lib, p)
        assert st != 0 and msg, (st, msg)
        seen.add(st)
    # sizes at the edge of 32-bit arithmetic with everything else valid
    for ng, nfr, buf in (([INT_MAX] * 3, [1, 1, 1], [0, 0, 0]),
                         ([1 << 30] * 3, [1 << 10] * 3, [1 << 28] * 3),
                         ([64, 64, 64], [64, 64, 64], [INT_MAX // 2] * 3),
                         ([1 << 16] * 3, [1 << 14] * 3, [1, 1, 1])):
        p, keep = make_params(rng, dict(n_grid=ng, num_fragment=nfr, num_rgrid_buffer=buf,
                                        cell=[7.2] * 3, n_species=1, n_atoms=0,
                                        nstate_frag_uniform=8, n_electrons=4.0,
                                        smearing=0.05, mixing=0.3, cg_sweeps=4, precision=0,
                                        batched=1))
        st, msg = setup_status(lib, p)
        assert st != 0 and msg, (ng, nfr, buf, st, msg)
    print("statuses seen:", sorted(seen), flush=True)
    # the sweep reaches every check: argument and shape errors, non-finite
    # positions, and (with every value valid) the missing device
    assert {-1, -2, -6, -7} <= seen, seen


if __name__ == "__main__":
    main(sys.argv[1])
