"""ctypes binding of ``libdcdft.so`` (argument marshalling only).

Every function here forwards to the C entry point of the same name declared
in ``include/dcdft.h``; all computation happens in the HIP library.  When the
library is missing the binding raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdcdft.so")

DCDFT_OK = 0
STATUS_NAMES = {
    0: "DCDFT_OK", -1: "DCDFT_ERR_ARG", -2: "DCDFT_ERR_SHAPE", -3: "DCDFT_ERR_CAPACITY",
    -4: "DCDFT_ERR_NOT_SPD", -5: "DCDFT_ERR_EIG", -6: "DCDFT_ERR_NAN", -7: "DCDFT_ERR_HIP",
    -8: "DCDFT_ERR_OOM", -9: "DCDFT_ERR_NOT_CONVERGED",
}
PREC_FP64, PREC_MIXED = 0, 1
FIELD_VLOC, FIELD_VH, FIELD_RHO_IN, FIELD_RHO_OUT = 0, 1, 2, 3
FFIELD_VEFF, FFIELD_RHO_IN, FFIELD_RHO_OUT = 0, 1, 2

EXPORTED = [
    "dcdft_setup", "dcdft_scf_step", "dcdft_density", "dcdft_density_device",
    "dcdft_eigenvalues", "dcdft_fragment_info", "dcdft_get_field", "dcdft_get_fragment_field",
    "dcdft_get_orbitals", "dcdft_set_orbitals", "dcdft_set_density", "dcdft_fix_density",
    "dcdft_set_template", "dcdft_set_mixer", "dcdft_lcfo_build", "dcdft_lcfo_basis", "dcdft_lcfo_hamiltonian",
    "dcdft_lcfo_block",
    "dcdft_apply_h",
    "dcdft_band_energy", "dcdft_band_energy_bwd", "dcdft_band_energy_all",
    "dcdft_band_energy_noalloc",
    "dcdft_kernel_timing", "dcdft_kernel_time", "dcdft_autotune",
    "dcdft_get_launch", "dcdft_set_launch",
    "dcdft_destroy",
    "dcdft_status_string", "dcdft_last_error",
]
KERNEL_HLOC, KERNEL_GRAM, KERNEL_ROTATE, KERNEL_GRAM_FUSED, KERNEL_KB = 0, 1, 2, 3, 4
MIX_LINEAR, MIX_PULAY = 0, 1
HLOC_VARIANTS = ("plane", "halo_pd2", "halo_pd3", "halo_pd4", "halo_pd2_ends", "vec",
                 "vec_wide", "vec_z2", "vec_z3", "vec8", "vec8_wide")


class DcdftSpecies(ctypes.Structure):
    _fields_ = [("valence", ctypes.c_double), ("vloc_depth", ctypes.c_double),
                ("vloc_sigma", ctypes.c_double), ("kb_energy", ctypes.c_double),
                ("kb_sigma", ctypes.c_double), ("kb_rcut", ctypes.c_double)]


class DcdftParams(ctypes.Structure):
    _fields_ = [
        ("n_grid", ctypes.c_int32 * 3), ("cell", ctypes.c_double * 3),
        ("num_fragment", ctypes.c_int32 * 3), ("num_rgrid_buffer", ctypes.c_int32 * 3),
        ("n_atoms", ctypes.c_int32), ("atom_pos", ctypes.POINTER(ctypes.c_double)),
        ("atom_species", ctypes.POINTER(ctypes.c_int32)), ("n_species", ctypes.c_int32),
        ("species", ctypes.POINTER(DcdftSpecies)),
        ("nstate_frag", ctypes.POINTER(ctypes.c_int32)), ("nstate_frag_uniform", ctypes.c_int32),
        ("n_electrons", ctypes.c_double), ("smearing", ctypes.c_double),
        ("mixing", ctypes.c_double), ("cg_sweeps", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("batched", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
    ]


class DcdftScfInfo(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("mu", ctypes.c_double), ("e_total", ctypes.c_double),
                ("e_band", ctypes.c_double), ("entropy", ctypes.c_double),
                ("residual_paper", ctypes.c_double), ("residual_out_in", ctypes.c_double),
                ("charge", ctypes.c_double), ("ms_step", ctypes.c_float),
                ("ms_poisson", ctypes.c_float), ("ms_fragments", ctypes.c_float),
                ("ms_fermi_density", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class DcdftTuneInfo(ctypes.Structure):
    _fields_ = [("hloc_variant", ctypes.c_int32), ("rot_tiles", ctypes.c_int32),
                ("gram_chunks", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ms_hloc", ctypes.c_double * 11), ("ms_rot", ctypes.c_double * 3),
                ("gram_candidates", ctypes.c_int32 * 4), ("ms_gram", ctypes.c_double * 4)]

    def as_dict(self) -> dict:
        return {"hloc_variant": HLOC_VARIANTS[self.hloc_variant], "rot_tiles": self.rot_tiles,
                "gram_chunks": self.gram_chunks, "from_cache": bool(self.from_cache),
                "ms_hloc": dict(zip(HLOC_VARIANTS, (round(v, 4) for v in self.ms_hloc))),
                "ms_rot": dict(zip((2, 4, 8), (round(v, 4) for v in self.ms_rot))),
                "ms_gram": {int(c): round(v, 4) for c, v in zip(self.gram_candidates,
                                                                 self.ms_gram) if v >= 0}}


class DcdftLcfoInfo(ctypes.Structure):
    _fields_ = [("n_basis", ctypes.c_int32), ("n_pairs", ctypes.c_int32), ("ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class DcdftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None):
    """Load the HIP library (built by ``paper_2606_21125_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with paper_2606_21125_amd.build.build()")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "dcdft_setup": ([ctypes.POINTER(DcdftParams), ctypes.POINTER(vp)], ctypes.c_int),
        "dcdft_scf_step": ([vp, ctypes.POINTER(DcdftScfInfo)], ctypes.c_int),
        "dcdft_density": ([vp, pd, ctypes.c_size_t], ctypes.c_int),
        "dcdft_density_device": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "dcdft_eigenvalues": ([vp, ctypes.c_int32, pd, pd, ctypes.c_int32, pi], ctypes.c_int),
        "dcdft_fragment_info": ([vp, ctypes.c_int32, pi, pi, pi, pi], ctypes.c_int),
        "dcdft_get_field": ([vp, ctypes.c_int32, pd, ctypes.c_size_t], ctypes.c_int),
        "dcdft_get_fragment_field": ([vp, ctypes.c_int32, ctypes.c_int32, pd, ctypes.c_size_t],
                                     ctypes.c_int),
        "dcdft_get_orbitals": ([vp, ctypes.c_int32, pd, ctypes.c_size_t], ctypes.c_int),
        "dcdft_set_orbitals": ([vp, ctypes.c_int32, pd, ctypes.c_size_t], ctypes.c_int),
        "dcdft_set_density": ([vp, pd, pd], ctypes.c_int),
        "dcdft_fix_density": ([vp, ctypes.c_int32], ctypes.c_int),
        "dcdft_set_template": ([vp, ctypes.c_double], ctypes.c_int),
        "dcdft_set_mixer": ([vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int32], ctypes.c_int),
        "dcdft_lcfo_build": ([vp, ctypes.c_double, ctypes.c_double,
                              ctypes.POINTER(DcdftLcfoInfo)], ctypes.c_int),
        "dcdft_lcfo_basis": ([vp, ctypes.c_int32, pd, ctypes.c_size_t, pi], ctypes.c_int),
        "dcdft_lcfo_hamiltonian": ([vp, pd, ctypes.c_size_t, pi], ctypes.c_int),
        "dcdft_lcfo_block": ([vp, ctypes.c_int32, ctypes.c_int32, pd, ctypes.c_size_t, pi, pi],
                             ctypes.c_int),
        "dcdft_apply_h": ([vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32],
                          ctypes.c_int),
        "dcdft_band_energy": ([vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32, vp,
                               vp, vp, vp], ctypes.c_int),
        "dcdft_band_energy_noalloc": ([vp, ctypes.c_int32, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                       vp, vp, vp, vp], ctypes.c_int),
        "dcdft_band_energy_all": ([vp, vp, vp, ctypes.c_int32, vp, vp, vp], ctypes.c_int),
        "dcdft_band_energy_bwd": ([vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32,
                                   ctypes.c_int32], ctypes.c_int),
        "dcdft_kernel_timing": ([vp, ctypes.c_int32], ctypes.c_int),
        "dcdft_kernel_time": ([vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), pd, pd, pd],
                              ctypes.c_int),
        "dcdft_autotune": ([vp, ctypes.c_char_p, ctypes.POINTER(DcdftTuneInfo)], ctypes.c_int),
        "dcdft_get_launch": ([vp, pi, pi, pi, pi, pi], ctypes.c_int),
        "dcdft_set_launch": ([vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                             ctypes.c_int),
        "dcdft_destroy": ([vp], None),
        "dcdft_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "dcdft_last_error": ([vp, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def dcdft_last_error(ctx) -> str:
    lib = load_library()
    buf = ctypes.create_string_buffer(1024)
    lib.dcdft_last_error(ctx, buf, 1024)
    return buf.value.decode(errors="replace")


def _check(status: int, ctx=None):
    if status != DCDFT_OK:
        raise DcdftError(status, dcdft_last_error(ctx))


def _device_inputs_ready(t) -> None:
    """The library works on its own stream and does not wait for work queued on
    torch's streams: finish what torch's current stream has queued (which
    produced the tensors handed over) before the call."""
    import torch
    torch.cuda.current_stream(t.device).synchronize()


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ipt(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def dcdft_setup(params: DcdftParams):
    lib = load_library()
    ctx = ctypes.c_void_p()
    _check(lib.dcdft_setup(ctypes.byref(params), ctypes.byref(ctx)), None)
    return ctx


def dcdft_scf_step(ctx) -> dict:
    info = DcdftScfInfo()
    _check(load_library().dcdft_scf_step(ctx, ctypes.byref(info)), ctx)
    return info.as_dict()


def dcdft_destroy(ctx) -> None:
    load_library().dcdft_destroy(ctx)


class DCDFT:
    """One DC-DFT SCF context on the GPU (owns the C context)."""

    def __init__(self, n_grid: Sequence[int], cell: Sequence[float], num_fragment: Sequence[int],
                 num_rgrid_buffer: Sequence[int], positions: np.ndarray,
                 species_index: np.ndarray, species: Sequence, nstate_frag, n_electrons: float,
                 smearing: float = 0.01, mixing: float = 0.3, cg_sweeps: int = 4,
                 precision: int = PREC_FP64, batched: int = 1, seed: int = 1,
                 hip_stream: Optional[int] = None):
        self._lib = load_library()
        self._pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 3)
        self._spi = np.ascontiguousarray(species_index, dtype=np.int32)
        sp = (DcdftSpecies * len(species))()
        for i, s in enumerate(species):
            sp[i] = DcdftSpecies(s.valence, s.vloc_depth, s.vloc_sigma, s.kb_energy, s.kb_sigma,
                                 s.kb_rcut)
        self._sp = sp
        nf = int(np.prod(num_fragment))
        ns = np.asarray(nstate_frag, dtype=np.int32)
        if ns.ndim == 0:
            ns = np.full(nf, int(ns), dtype=np.int32)
        self._ns = np.ascontiguousarray(ns)
        p = DcdftParams()
        p.n_grid[:] = [int(v) for v in n_grid]
        p.cell[:] = [float(v) for v in cell]
        p.num_fragment[:] = [int(v) for v in num_fragment]
        p.num_rgrid_buffer[:] = [int(v) for v in num_rgrid_buffer]
        p.n_atoms = self._pos.shape[0]
        p.atom_pos = _dptr(self._pos)
        p.atom_species = _ipt(self._spi)
        p.n_species = len(species)
        p.species = ctypes.cast(sp, ctypes.POINTER(DcdftSpecies))
        p.nstate_frag = _ipt(self._ns)
        p.nstate_frag_uniform = int(self._ns[0]) if self._ns.size else 0
        p.n_electrons = float(n_electrons)
        p.smearing = float(smearing)
        p.mixing = float(mixing)
        p.cg_sweeps = int(cg_sweeps)
        p.precision = int(precision)
        p.batched = int(batched)
        p.seed = int(seed)
        p.hip_stream = hip_stream
        self.params = p
        self.n_grid = tuple(int(v) for v in n_grid)
        self.n_fragments = nf
        self.nstate = self._ns
        self.ctx = dcdft_setup(p)
        shape = (ctypes.c_int32 * 3)()
        self.frag_shape = None
        _check(self._lib.dcdft_fragment_info(self.ctx, 0, shape, None, None, None), self.ctx)
        self.frag_shape = (shape[0], shape[1], shape[2])
        self.n = int(np.prod(self.frag_shape))

    @classmethod
    def from_config(cls, cfg, **kw):
        s = cfg.system
        args = dict(smearing=cfg.smearing, mixing=cfg.mixing, cg_sweeps=cfg.cg_sweeps,
                    seed=cfg.seed)
        args.update(kw)
        return cls(cfg.n_grid, s.cell, cfg.num_fragment, cfg.num_rgrid_buffer, s.positions,
                   s.species_index, s.species, cfg.nstate_frag, s.n_electrons, **args)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self._lib.dcdft_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls -------------------------------------------------------------------------
    def dcdft_scf_step(self) -> dict:
        return dcdft_scf_step(self.ctx)

    def dcdft_density(self) -> np.ndarray:
        n = int(np.prod(self.n_grid))
        out = np.empty(n)
        _check(self._lib.dcdft_density(self.ctx, _dptr(out), n), self.ctx)
        return out.reshape(self.n_grid[::-1])

    def dcdft_density_device(self, tensor) -> None:
        _check(self._lib.dcdft_density_device(self.ctx, ctypes.c_void_p(tensor.data_ptr()),
                                              tensor.numel()), self.ctx)

    def dcdft_eigenvalues(self, frag: int):
        cap = int(self.nstate[frag])
        eps = np.empty(cap)
        w = np.empty(cap)
        m = ctypes.c_int32()
        _check(self._lib.dcdft_eigenvalues(self.ctx, frag, _dptr(eps), _dptr(w), cap,
                                           ctypes.byref(m)), self.ctx)
        return eps[:m.value], w[:m.value]

    def dcdft_fragment_info(self, frag: int) -> dict:
        shape = (ctypes.c_int32 * 3)()
        origin = (ctypes.c_int32 * 3)()
        m = ctypes.c_int32()
        na = ctypes.c_int32()
        _check(self._lib.dcdft_fragment_info(self.ctx, frag, shape, origin, ctypes.byref(m),
                                             ctypes.byref(na)), self.ctx)
        return dict(shape=tuple(shape), origin=tuple(origin), m=m.value, n_proj=na.value)

    def dcdft_get_field(self, which: int) -> np.ndarray:
        n = int(np.prod(self.n_grid))
        out = np.empty(n)
        _check(self._lib.dcdft_get_field(self.ctx, which, _dptr(out), n), self.ctx)
        return out.reshape(self.n_grid[::-1])

    def dcdft_get_fragment_field(self, frag: int, which: int) -> np.ndarray:
        out = np.empty(self.n)
        _check(self._lib.dcdft_get_fragment_field(self.ctx, frag, which, _dptr(out), self.n),
               self.ctx)
        return out

    def dcdft_get_orbitals(self, frag: int) -> np.ndarray:
        m = int(self.nstate[frag])
        out = np.empty((m, self.n))
        _check(self._lib.dcdft_get_orbitals(self.ctx, frag, _dptr(out), out.size), self.ctx)
        return out

    def dcdft_set_orbitals(self, frag: int, psi: np.ndarray) -> None:
        a = np.ascontiguousarray(psi, dtype=np.float64)
        _check(self._lib.dcdft_set_orbitals(self.ctx, frag, _dptr(a), a.size), self.ctx)

    def dcdft_set_density(self, rho_tot: np.ndarray, rho_frag: Optional[np.ndarray] = None):
        a = np.ascontiguousarray(rho_tot, dtype=np.float64)
        b = None if rho_frag is None else np.ascontiguousarray(rho_frag, dtype=np.float64)
        _check(self._lib.dcdft_set_density(self.ctx, _dptr(a), None if b is None else _dptr(b)),
               self.ctx)

    def save_state(self, path: str) -> None:
        """Checkpoint of the SCF state: rho_tot^in, every rho_alpha^in and every
        fragment's orbitals (FP64), written with numpy.savez (no pickled objects),
        with the geometry and precision they belong to.  The CG history is rebuilt
        in every step, so these arrays are the whole state a later step reads."""
        p = self.params
        arrays = {"n_grid": np.array(self.n_grid), "nstate": np.array(self.nstate),
                  "frag_shape": np.array(self.frag_shape),
                  "num_fragment": np.array(list(p.num_fragment)),
                  "num_rgrid_buffer": np.array(list(p.num_rgrid_buffer)),
                  "precision": np.array(p.precision),
                  "rho_in": self.dcdft_get_field(FIELD_RHO_IN),
                  "rho_frag_in": np.stack([self.dcdft_get_fragment_field(f, FFIELD_RHO_IN)
                                           for f in range(len(self.nstate))])}
        for f in range(len(self.nstate)):
            arrays[f"psi_{f}"] = self.dcdft_get_orbitals(f)
        np.savez(path, **arrays)

    def load_state(self, path: str) -> None:
        """Restore a checkpoint written by save_state for the same grid, fragment
        decomposition, buffer, orbital counts and precision; every array's shape
        is checked before anything is handed to the library."""
        p = self.params
        with np.load(path, allow_pickle=False) as z:
            want = {"n_grid": tuple(self.n_grid), "nstate": tuple(int(v) for v in self.nstate),
                    "frag_shape": tuple(self.frag_shape),
                    "num_fragment": tuple(p.num_fragment),
                    "num_rgrid_buffer": tuple(p.num_rgrid_buffer)}
            for key, val in want.items():
                if key not in z or tuple(int(v) for v in np.atleast_1d(z[key])) != val:
                    raise ValueError(f"checkpoint {key} does not match this context ({val})")
            if "precision" not in z or int(z["precision"]) != int(p.precision):
                raise ValueError("checkpoint precision does not match this context")
            nf = len(self.nstate)
            if z["rho_in"].size != int(np.prod(self.n_grid)):
                raise ValueError("checkpoint rho_in has the wrong size")
            if z["rho_frag_in"].shape != (nf, self.n):
                raise ValueError(f"checkpoint rho_frag_in is {z['rho_frag_in'].shape}, "
                                 f"expected {(nf, self.n)}")
            for f in range(nf):
                if z[f"psi_{f}"].shape != (int(self.nstate[f]), self.n):
                    raise ValueError(f"checkpoint psi_{f} is {z[f'psi_{f}'].shape}, expected "
                                     f"{(int(self.nstate[f]), self.n)}")
            for f in range(nf):
                self.dcdft_set_orbitals(f, z[f"psi_{f}"])
            self.dcdft_set_density(z["rho_in"], z["rho_frag_in"])

    def dcdft_fix_density(self, fixed: bool = True) -> None:
        _check(self._lib.dcdft_fix_density(self.ctx, int(bool(fixed))), self.ctx)

    def dcdft_set_template(self, xi: float) -> None:
        _check(self._lib.dcdft_set_template(self.ctx, float(xi)), self.ctx)

    def dcdft_set_mixer(self, kind, alpha: float = 0.3, q0: float = 0.8,
                        history: int = 8) -> None:
        """kind: MIX_LINEAR / MIX_PULAY (or "linear" / "pulay")."""
        k = {"linear": MIX_LINEAR, "pulay": MIX_PULAY}.get(kind, kind)
        _check(self._lib.dcdft_set_mixer(self.ctx, int(k), float(alpha), float(q0),
                                         int(history)), self.ctx)

    def dcdft_lcfo_build(self, eps_cut: float, lambda_cut: float = 1e-7) -> dict:
        info = DcdftLcfoInfo()
        _check(self._lib.dcdft_lcfo_build(self.ctx, float(eps_cut), float(lambda_cut),
                                          ctypes.byref(info)), self.ctx)
        return info.as_dict()

    def dcdft_lcfo_basis(self, frag: int) -> np.ndarray:
        nb = ctypes.c_int32(0)
        _check(self._lib.dcdft_lcfo_basis(self.ctx, frag, None, 0, ctypes.byref(nb)), self.ctx)
        out = np.empty((nb.value, self.n))
        _check(self._lib.dcdft_lcfo_basis(self.ctx, frag, _dptr(out), out.size, None), self.ctx)
        return out

    def dcdft_lcfo_hamiltonian(self) -> np.ndarray:
        nb = ctypes.c_int32(0)
        _check(self._lib.dcdft_lcfo_hamiltonian(self.ctx, None, 0, ctypes.byref(nb)), self.ctx)
        out = np.empty((nb.value, nb.value))
        _check(self._lib.dcdft_lcfo_hamiltonian(self.ctx, _dptr(out), out.size, None), self.ctx)
        return out

    def dcdft_lcfo_block(self, a: int, b: int) -> np.ndarray:
        rows, cols = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self._lib.dcdft_lcfo_block(self.ctx, a, b, None, 0, ctypes.byref(rows),
                                          ctypes.byref(cols)), self.ctx)
        out = np.empty((rows.value, cols.value))
        _check(self._lib.dcdft_lcfo_block(self.ctx, a, b, _dptr(out), out.size, None, None),
               self.ctx)
        return out

    def dcdft_apply_h(self, frag: int, psi, hpsi, prec: int = PREC_FP64) -> None:
        """psi, hpsi: contiguous device tensors of shape (m, n)."""
        m = psi.shape[0]
        _device_inputs_ready(psi)
        _check(self._lib.dcdft_apply_h(self.ctx, frag, ctypes.c_void_p(psi.data_ptr()),
                                       ctypes.c_void_p(hpsi.data_ptr()), m, prec), self.ctx)

    def dcdft_kernel_timing(self, enable: bool) -> None:
        _check(self._lib.dcdft_kernel_timing(self.ctx, int(bool(enable))), self.ctx)

    def dcdft_kernel_time(self, kernel: int) -> dict:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        fl = ctypes.c_double()
        _check(self._lib.dcdft_kernel_time(self.ctx, kernel, ctypes.byref(n), ctypes.byref(ms),
                                           ctypes.byref(by), ctypes.byref(fl)), self.ctx)
        return dict(launches=n.value, ms=ms.value, bytes=by.value, flops=fl.value)

    def dcdft_autotune(self, cache_path: Optional[str] = None) -> dict:
        info = DcdftTuneInfo()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(self._lib.dcdft_autotune(self.ctx, path, ctypes.byref(info)), self.ctx)
        return info.as_dict()

    def dcdft_get_launch(self) -> dict:
        v = [ctypes.c_int32() for _ in range(5)]
        _check(self._lib.dcdft_get_launch(self.ctx, *[ctypes.byref(x) for x in v]), self.ctx)
        return dict(hloc_variant=v[0].value, rot_tiles=v[1].value, gram_chunks=v[2].value,
                    gram_chunks_max=v[3].value, streams=v[4].value)

    def dcdft_set_launch(self, hloc_variant: int, rot_tiles: int, gram_chunks: int,
                         streams: Optional[int] = None) -> None:
        if streams is None:
            streams = self.dcdft_get_launch()["streams"]
        _check(self._lib.dcdft_set_launch(self.ctx, hloc_variant, rot_tiles, gram_chunks,
                                          streams), self.ctx)

    def dcdft_band_energy(self, frag: int, psi, f, veff=None, energy=None, grad_psi=None,
                          grad_v=None, prec: int = PREC_FP64) -> None:
        """psi: device (m, n) double/float; f: device (m,) double; veff: device (n,)
        double or None; outputs are device tensors (energy (1,), grad_psi like psi,
        grad_v (n,) double)."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _device_inputs_ready(psi)
        _check(self._lib.dcdft_band_energy(self.ctx, frag, ctypes.c_void_p(psi.data_ptr()),
                                           ctypes.c_void_p(f.data_ptr()), psi.shape[0], prec,
                                           ptr(veff), ptr(energy), ptr(grad_psi), ptr(grad_v)),
               self.ctx)

    def dcdft_band_energy_bwd(self, frag: int, psi, f, grad_psi=None, grad_v=None,
                              prec: int = PREC_FP64) -> None:
        """The backward in the boundary's original argument order (the fragment's
        V_eff of the last step, no energy)."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _device_inputs_ready(psi)
        _check(self._lib.dcdft_band_energy_bwd(self.ctx, frag, ctypes.c_void_p(psi.data_ptr()),
                                               ctypes.c_void_p(f.data_ptr()), ptr(grad_psi),
                                               ptr(grad_v), psi.shape[0], prec), self.ctx)

    def dcdft_band_energy_all(self, psi, f, energy=None, grad_psi=None, grad_v=None,
                              prec: int = PREC_FP64) -> None:
        """psi: device (M_tot, n) double/float, every fragment's vectors in fragment
        order; f: device (M_tot,) double; outputs are device tensors (energy (1,),
        grad_psi like psi, grad_v (Nz, Ny, Nx) or (N,) double on the global grid)."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _device_inputs_ready(psi)
        _check(self._lib.dcdft_band_energy_all(self.ctx, ctypes.c_void_p(psi.data_ptr()),
                                               ctypes.c_void_p(f.data_ptr()), prec, ptr(energy),
                                               ptr(grad_psi), ptr(grad_v)), self.ctx)

    def dcdft_band_energy_noalloc(self, frag: int, psi, f, veff=None, energy=None,
                                  grad_psi=None, grad_v=None, prec: int = PREC_FP64) -> None:
        """As dcdft_band_energy, through the entry point that allocates nothing
        (its scratch is the library's static device array)."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _device_inputs_ready(psi)
        _check(self._lib.dcdft_band_energy_noalloc(
            self.ctx, frag, ctypes.c_void_p(psi.data_ptr()), ctypes.c_void_p(f.data_ptr()),
            psi.shape[0], prec, ptr(veff), ptr(energy), ptr(grad_psi), ptr(grad_v)), self.ctx)
