#!/usr/bin/env python3
"""Throughput of the DC-DFT fragment SCF step on one MI355X.

One step = one SCF iteration over all fragments (Hartree potential, fragment
potentials, CG sweeps + Rayleigh-Ritz on every fragment, core weights, global
chemical potential, density assembly, energy, residuals, mixing).  The
default workload is the largest single-GPU configuration, the liquid-water-like
cell (1378 H2O = 4134 atoms, 160^3 grid, 8x8x8 fragments of 32^3 points, 27-80
orbitals per fragment) with synthetic, seeded atom positions, in mixed precision;
--config 2 (512-atom a-Si-like cell) and --config 5 (4096-atom Si cell) are the
other timed workloads.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fragment H·ψ GB/s + SCF iters/sec (all fragments), mixed+batched vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3


def workload_config(k: int):
    import workloads
    return workloads.config(k)


def cpu_baseline(cfg, max_workers: int = 16, min_seconds: float = 10.0) -> dict:
    """The FP64 oracle as it stands on host cores, one BLAS thread per worker
    process.  Up to 64 fragments: whole SCF iterations of the same workload,
    repeated until at least min_seconds of wall time.  More fragments: a bounded
    sample of one iteration -- the global Poisson solve, and the fragment
    eigensolves (with their V_eff, core weights and densities) of two fragments per
    worker spread evenly over the cell -- scaled to all fragments."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle.solver import core_weights, fermi_level, fermi_occupation, fragment_density

    workers = max(1, min(max_workers, os.cpu_count() or 1, cfg.n_fragments))
    if cfg.n_fragments <= 64:
        # worker processes are spawned (fresh interpreters with one BLAS thread each),
        # once, by the untimed first iteration
        o = oracle.OracleSCF(cfg, workers=workers, blas_threads=1)
        steps = 0
        with threadpool_limits(limits=1):
            o.step()
            t0 = time.perf_counter()
            while True:
                o.step()
                steps += 1
                elapsed = time.perf_counter() - t0
                if elapsed >= min_seconds:
                    break
        o.close()
        return {"value": steps / elapsed, "unit": "SCF iter/s", "cores": workers,
                "kind": "oracle",
                "sample": (f"{steps} whole SCF iterations of the same workload after one "
                           f"untimed iteration (all {cfg.n_fragments} fragment eigensolves on "
                           f"{workers} processes, 1 BLAS thread each), {elapsed:.1f} s wall")}
    nf = cfg.n_fragments
    sample = sorted(set(int(round(v)) for v in np.linspace(0, nf - 1, 3 * workers)))
    warm, timed = sample[:workers], sample[workers:]
    o = oracle.OracleSCF(cfg, workers=workers, blas_threads=1, fragments=sample)
    with threadpool_limits(limits=1):
        v_h = oracle.poisson_fd(o.rho_in, o.h)
        o.solve_fragments(v_h, alphas=warm)          # starts the worker pool (untimed)
        t0 = time.perf_counter()
        v_h = oracle.poisson_fd(o.rho_in, o.h)
        t1 = time.perf_counter()
        res = o.solve_fragments(v_h, alphas=timed)
        eps, w = [], []
        for a in timed:
            psi, e = res[a]
            eps.append(e)
            w.append(core_weights(psi, o.frags[a].core_mask, o.dv))
        # the chemical potential of the sample (N_e scaled to its share of the cell)
        ne = o.ne * len(timed) / nf
        mu = fermi_level(np.concatenate(eps), np.concatenate(w), ne, cfg.smearing)
        for a, e in zip(timed, eps):
            fragment_density(res[a][0], fermi_occupation((e - mu) / cfg.smearing))
        t2 = time.perf_counter()
    o.close()
    per_iter = (t1 - t0) + (t2 - t1) * nf / len(timed)
    return {"value": 1.0 / per_iter, "unit": "SCF iter/s", "cores": workers, "kind": "oracle",
            "sample": (f"one SCF iteration estimated from a sample: the global Poisson solve "
                       f"({t1 - t0:.2f} s) plus the eigensolves, core weights and densities "
                       f"of {len(timed)} of the {nf} fragments spread over the cell "
                       f"({t2 - t1:.1f} s on {workers} processes, 1 BLAS thread each) scaled "
                       f"by {nf}/{len(timed)}; {per_iter:.1f} s per iteration")}


def crossover(args, prec) -> dict:
    """Per-step time of the conventional calculation (one fragment, no buffer,
    ceil(1.2 N_e / 2) orbitals) and of DC-DFT (cores of one Si cube, buffers of 4
    points, ceil(1.2 N_loc / 2) orbitals) on Si supercells, same kernels, same
    precision.  Past 80 orbitals the conventional side runs the large-orbital
    path (BLAS products, FP64 factorisations in the solver library); its Gram
    products are reported as achieved TFLOP/s against the dense matrix-core peak
    of the orbital precision, from one more step with per-launch timing."""
    import torch
    import workloads
    from paper_2606_21125_amd import DCDFT
    from paper_2606_21125_amd.binding import DcdftError

    def timed(cfg):
        try:
            d = DCDFT.from_config(cfg, precision=prec)
        except DcdftError as e:
            return {"config": cfg.name, "error": str(e).split(":")[0],
                    "orbitals": int(cfg.nstate_frag.max())}
        if not args.no_autotune:
            d.dcdft_autotune(args.tune_cache)
        for _ in range(args.warmup):
            d.dcdft_scf_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            d.dcdft_scf_step()
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / args.steps
        out = {"config": cfg.name, "ms_per_step": round(ms, 3),
               "orbitals": int(cfg.nstate_frag.sum()), "fragments": cfg.n_fragments}
        if cfg.n_fragments == 1 and int(cfg.nstate_frag[0]) > 80:
            from paper_2606_21125_amd.binding import KERNEL_GRAM
            d.dcdft_kernel_timing(True)
            d.dcdft_scf_step()
            kt = d.dcdft_kernel_time(KERNEL_GRAM)
            d.dcdft_kernel_timing(False)
            if kt["ms"] > 0:
                tf = kt["flops"] / (kt["ms"] * 1e-3) / 1e12
                peak = 157.3 if prec != 0 else 78.6
                out["gram"] = {"launches": kt["launches"], "ms": round(kt["ms"], 3),
                               "tflops": round(tf, 2), "peak_tflops": peak,
                               "frac": round(tf / peak, 3)}
        d.close()
        return out

    rows = []
    for cells in ((1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2), (3, 3, 3), (4, 4, 4)):
        n_atoms = 8 * cells[0] * cells[1] * cells[2]
        print(f"[bench] crossover: {n_atoms} atoms", file=sys.stderr, flush=True)
        row = {"atoms": n_atoms, "grid": [16 * c for c in cells]}
        row["conventional"] = timed(workloads.si_cells_config(cells))
        if cells[0] >= 2:     # a buffered box must fit the cell (n_core + 2 b <= N)
            nf = tuple(cells)
            b = tuple(4 if c >= 2 else 0 for c in cells)
            row["dc"] = timed(workloads.si_cells_config(cells, nf, b))
        rows.append(row)
    return {"metric": "SCF step time, conventional vs DC, Si cells", "unit": "ms/step",
            "dtype": "f32/f64" if prec != 0 else "f64", "steps": args.steps,
            "warmup": args.warmup, "data": "synthetic", "rows": rows}


def converge(args) -> dict:
    """Whole SCF runs to the paper's convergence measure (Sec. 3.3: dV sum |rho_k^in -
    rho_(k-1)^in| / N_e) below args.converge, from the initial state, for the
    workload and for the 64-atom cell (per-atom time, linearity), in mixed and FP64
    precision, with Pulay-Kerker mixing and the density-template potential as
    given.  Reports the first iteration that meets the tolerance, the time to it,
    the time per iteration and per atom, and the spread of both residuals over the
    last 50 of up to args.max_iter iterations."""
    import torch
    import workloads
    from paper_2606_21125_amd import DCDFT, PREC_FP64, PREC_MIXED
    from paper_2606_21125_amd.binding import DcdftError

    rows = []
    for role, k in (("workload", args.config), ("si64", 1)):
        for prec in (PREC_MIXED, PREC_FP64):
            cfg = workloads.config(k)
            name = "mixed" if prec == PREC_MIXED else "fp64"
            print(f"[bench] converge {cfg.name} {name}", file=sys.stderr, flush=True)
            d = DCDFT.from_config(cfg, precision=prec)
            if not args.no_autotune:
                d.dcdft_autotune(args.tune_cache)
            d.dcdft_set_mixer(args.mixer, args.mix_alpha, args.kerker_q0, args.mix_history)
            if args.template_xi > 0.0:
                d.dcdft_set_template(args.template_xi)
            rp, ro, first, t_first, err = [], [], None, None, None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                for it in range(args.max_iter):
                    info = d.dcdft_scf_step()
                    rp.append(info["residual_paper"])
                    ro.append(info["residual_out_in"])
                    if first is None and it > 0 and rp[-1] < args.converge:
                        first = it + 1
                        t_first = time.perf_counter() - t0
            except DcdftError as e:
                err = str(e).split(":")[0]
            wall = time.perf_counter() - t0
            d.close()
            n = len(rp)
            tail = slice(max(0, n - 50), n)
            rows.append({"role": role, "workload": cfg.name, "atoms": cfg.system.n_atoms,
                         "precision": name,
                         "iterations_run": n, "error": err,
                         "first_iteration_below_tol": first,
                         "seconds_to_tol": None if t_first is None else round(t_first, 3),
                         "ms_per_iteration": round(1000.0 * wall / max(1, n), 3),
                         "us_per_atom_iteration": round(1e6 * wall / max(1, n)
                                                        / cfg.system.n_atoms, 4),
                         "residual_paper_last50": [min(rp[tail]), max(rp[tail])] if n else None,
                         "residual_out_in_last50": [min(ro[tail]), max(ro[tail])] if n else None})
            print(f"[bench] {json.dumps(rows[-1])}", file=sys.stderr, flush=True)
    lin = {}
    for name in ("mixed", "fp64"):
        big = next(r for r in rows if r["precision"] == name and r["role"] == "workload")
        small = next(r for r in rows if r["precision"] == name and r["role"] == "si64")
        lin[name] = round(big["us_per_atom_iteration"] / small["us_per_atom_iteration"], 3)
    return {"metric": "SCF iterations and time to the paper's density residual",
            "tolerance": args.converge, "max_iter": args.max_iter,
            "mixer": {"kind": args.mixer, "alpha": args.mix_alpha, "kerker_q0": args.kerker_q0,
                      "history": args.mix_history}, "template_xi": args.template_xi,
            "data": "synthetic", "rows": rows,
            "per_atom_time_ratio_to_si64": lin}


HLOC_KERNEL = {"plane": "k_hloc<{t}>", "halo_pd2": "k_hloc_halo<{t}, {nx}, 2, false>",
               "halo_pd3": "k_hloc_halo<{t}, {nx}, 3, false>",
               "halo_pd4": "k_hloc_halo<{t}, {nx}, 4, false>",
               "halo_pd2_ends": "k_hloc_halo<{t}, {nx}, 2, true>"}


def hloc_kernel_name(variant: str, prec_mixed: bool, box) -> str:
    """Kernel the library launches for a stencil variant on this machine shape."""
    t = "float" if prec_mixed else "double"
    nx, ny, nz = box
    halo = nx >= 4 and ny >= 4 and nz >= 8
    if variant.startswith("vec"):
        vb = 8 if variant.startswith("vec8") else 16
        rx = vb // (4 if prec_mixed else 8)
        if halo and nx % rx == 0:
            return f"k_hloc_vec<{t}, 1, {vb}>"
        variant = "halo_pd2"
    if variant != "plane" and not halo:
        variant = "plane"
    return HLOC_KERNEL[variant].format(t=t, nx=nx if nx in (24, 32) else 0)


def _orbital_source_sha() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2606_21125_amd", "csrc", "k_orbital.hip")
    with open(src, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _traffic_records(tag: str):
    """(fields, file) of every '<tag>: a | b | ...' line of the committed counter
    summaries."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md"))):
        with open(path) as fh:
            for line in fh:
                if line.startswith(tag + ":"):
                    yield ([p.strip() for p in line[len(tag) + 1:].split("|")],
                           os.path.relpath(path, ROOT))


def recorded_traffic(variant: str, kernel: str, workload: str):
    """HBM bytes per stencil launch from the committed counter summaries, if they
    were taken on the current kernel source for this launch shape (variant and
    kernel) and workload."""
    sha = _orbital_source_sha()
    for parts, path in _traffic_records("traffic"):
        if len(parts) == 5 and parts[0] == variant and parts[1] == kernel and \
                parts[2] == workload and parts[4] == sha:
            return float(parts[3]), path
    return None, None


def recorded_projector_traffic(workload: str):
    """HBM bytes of the projector kernels (projection, reduction, application)
    per H psi application, under the same conditions."""
    sha = _orbital_source_sha()
    for parts, path in _traffic_records("traffic_kb"):
        if len(parts) == 3 and parts[0] == workload and parts[2] == sha:
            return float(parts[1]), path
    return None, None


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3,
                    help="workload number (default 3: the water-like cell)")
    ap.add_argument("--batched", type=int, default=1)
    ap.add_argument("--precision", choices=("mixed", "fp64"), default="mixed",
                    help="mixed: FP32 orbital arrays/stencil/matrix cores with FP64 "
                         "reductions, Cholesky, eigensolve and Fermi level")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of timing the candidates")
    ap.add_argument("--tune-cache", default=None,
                    help="text file of earlier autotuner choices (read, then appended)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain per-fragment FP64 comparison run")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="run one plain device-to-device copy of this many MB first (a "
                         "reference kernel for scaling HBM counters)")
    ap.add_argument("--fixed-density", action="store_true",
                    help="fixed-density DC: freeze rho_tot at a superposition of atomic "
                         "Gaussians and time the iterations without Poisson, V_eff or "
                         "mixing updates (no comparison runs, no CPU baseline)")
    ap.add_argument("--crossover", action="store_true",
                    help="instead of the benchmark line: time conventional (one fragment, "
                         "no buffer) and DC steps on Si cells of 8 to 512 atoms and print "
                         "that table as one JSON line")
    ap.add_argument("--lcfo", action="store_true",
                    help="after the timed steps, build the DC-LCFO basis and global matrix "
                         "(eps_cut = mu + 0.1 eV, lambda_cut = 1e-7) and report its time")
    ap.add_argument("--template-xi", type=float, default=0.0,
                    help="xi of the density-template potential V^alpha (0: off, the default; "
                         "--converge uses 1.0 unless given)")
    ap.add_argument("--converge", type=float, default=0.0,
                    help="instead of the benchmark line: run whole SCFs (the workload, default "
                         "5, and the 64-atom cell) until the paper's residual is below this "
                         "tolerance and print that table as one JSON line")
    ap.add_argument("--max-iter", type=int, default=300)
    ap.add_argument("--mixer", choices=("linear", "pulay"), default=None,
                    help="density mixing (default: linear for the benchmark, pulay for "
                         "--converge)")
    ap.add_argument("--mix-alpha", type=float, default=0.3)
    ap.add_argument("--kerker-q0", type=float, default=0.8)
    ap.add_argument("--mix-history", type=int, default=8)
    args = ap.parse_args()
    if args.converge > 0.0:
        if args.mixer is None:
            args.mixer = "pulay"
        if "--template-xi" not in sys.argv:
            args.template_xi = 1.0
        if "--config" not in sys.argv:
            args.config = 5
    elif args.mixer is None:
        args.mixer = "linear"
    if args.fixed_density:
        args.no_compare = True
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(json.dumps({"error": "the SCF step runs on one GPU per process (no multi-GPU path); --gpus must be 1"}))
        return 2

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    from paper_2606_21125_amd import (DCDFT, HLOC_VARIANTS, KERNEL_GRAM, KERNEL_GRAM_FUSED,
                                      KERNEL_HLOC, KERNEL_KB, KERNEL_ROTATE, PREC_FP64,
                                      PREC_MIXED)
    prec = PREC_MIXED if args.precision == "mixed" else PREC_FP64

    if args.copy_probe_mb > 0:
        # one elementwise kernel that reads and writes n * 8 bytes (y = 1.0 * x)
        n = int(args.copy_probe_mb * 1e6) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {n * 8} bytes read, {n * 8} bytes written",
              file=sys.stderr, flush=True)
        del src, dst
    if args.crossover:
        print(json.dumps(crossover(args, prec)), flush=True)
        return 0
    if args.converge > 0.0:
        print(json.dumps(converge(args)), flush=True)
        return 0
    cfg = workload_config(args.config)
    print(f"[bench] setup {cfg.name}: {cfg.system.n_atoms} atoms, grid {cfg.n_grid}, "
          f"{cfg.n_fragments} fragments of {cfg.fragment_shape}", file=sys.stderr, flush=True)
    def configure(dd):
        """The run's template potential, mixer and fixed density (every context the
        line reports on, comparison runs included, takes the same settings)."""
        if args.template_xi > 0.0:
            dd.dcdft_set_template(args.template_xi)
        if args.mixer == "pulay":
            dd.dcdft_set_mixer("pulay", args.mix_alpha, args.kerker_q0, args.mix_history)
        if args.fixed_density:
            from workloads import superposed_density
            dd.dcdft_set_density(superposed_density(cfg.system, cfg.n_grid))
            dd.dcdft_fix_density(True)

    d = DCDFT.from_config(cfg, batched=args.batched, precision=prec)
    configure(d)
    launch0 = d.dcdft_get_launch()
    tune = None
    if not args.no_autotune:
        tune = d.dcdft_autotune(args.tune_cache)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        d.dcdft_scf_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = None
    for _ in range(args.steps):
        info = d.dcdft_scf_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel device times: the same steps run eagerly with every launch of the
    # stencil, Gram and rotation families bracketed by HIP events on the
    # library's stream (event records cannot be captured into the step graph)
    d.dcdft_kernel_timing(True)
    n_timed = max(2, min(args.steps, 4))
    for _ in range(n_timed):
        d.dcdft_scf_step()
    kt = {name: d.dcdft_kernel_time(k) for name, k in
          (("hloc", KERNEL_HLOC), ("gram", KERNEL_GRAM), ("rotate", KERNEL_ROTATE),
           ("gram_fused", KERNEL_GRAM_FUSED), ("kb", KERNEL_KB))}
    d.dcdft_kernel_timing(False)
    lcfo = None
    if args.lcfo:
        eps_cut = info["mu"] + 0.1 / 27.211386
        builds = []
        for _ in range(3):       # the first build allocates its arrays
            t0b = time.perf_counter()
            li = d.dcdft_lcfo_build(eps_cut, 1e-7)
            builds.append((li, 1000.0 * (time.perf_counter() - t0b)))
        li, wall = builds[-1]
        lcfo = {"n_basis": li["n_basis"], "n_pairs": li["n_pairs"],
                "ms_device": round(li["ms"], 3), "ms_wall": round(wall, 3),
                "eps_cut": eps_cut, "lambda_cut": 1e-7,
                "note": "device time from the core projection to the neighbour products; "
                        "wall time adds the copies of the blocks to the host"}
    d.close()
    elapsed = t1 - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = args.steps / elapsed

    mfma_peak = FP32_MFMA_PEAK_TFLOPS if prec != PREC_FP64 else FP64_MFMA_PEAK_TFLOPS
    h = kt["hloc"]
    h_gbs = h["bytes"] / (h["ms"] * 1e-3) / 1e9 if h["ms"] > 0 else 0.0
    g = kt["gram"]
    g_tf = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    r = kt["rotate"]
    r_gbs = r["bytes"] / (r["ms"] * 1e-3) / 1e9 if r["ms"] > 0 else 0.0
    gf = kt["gram_fused"]
    gf_gbs = gf["bytes"] / (gf["ms"] * 1e-3) / 1e9 if gf["ms"] > 0 else 0.0
    kb = kt["kb"]
    kb_gbs = kb["bytes"] / (kb["ms"] * 1e-3) / 1e9 if kb["ms"] > 0 else 0.0
    variant = tune["hloc_variant"] if tune else HLOC_VARIANTS[launch0["hloc_variant"]]
    kname = hloc_kernel_name(variant, prec != PREC_FP64, cfg.fragment_shape)
    traffic, traffic_src = recorded_traffic(variant, kname, cfg.name)
    kb_traffic, kb_src = recorded_projector_traffic(cfg.name)
    n_app = max(1, h["launches"])            # H psi applications (one stencil launch each)
    stencil = {"bound": "hbm", "achieved": round(h_gbs, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(h_gbs / HBM_PEAK_GBS, 4),
               "traffic": None if traffic is None else round(traffic),
               "traffic_source": traffic_src, "kernel": kname,
               "avg_launch_ms": round(h["ms"] / n_app, 4),
               "bytes_per_launch": h["bytes"] / n_app}
    # the whole H psi unit: stencil + projection (with its reduction) + application,
    # the same algorithmic bytes (read psi, write H psi, V_eff once per fragment)
    hpsi_ms = (h["ms"] + kb["ms"]) / n_app
    hpsi_gbs = (h["bytes"] / n_app) / (hpsi_ms * 1e-3) / 1e9 if hpsi_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(hpsi_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hpsi_gbs / HBM_PEAK_GBS, 4),
                "traffic": (None if traffic is None or kb_traffic is None
                            else round(traffic + kb_traffic)),
                "traffic_source": None if kb_src is None or traffic_src is None else kb_src,
                "kernel": f"H psi = {kname} + k_kb_project + k_kb_reduce + "
                                            f"k_kb_apply",
                "avg_launch_ms": round(hpsi_ms, 4),
                "bytes_per_launch": h["bytes"] / n_app,
                "measured": f"HIP events around every launch over {n_timed} eager steps "
                            f"following the timed region; one H psi application = one "
                            f"stencil launch plus the projector launches of the same "
                            f"orbitals", "stencil": stencil}
    extra = {
        "hpsi_gbs": round(hpsi_gbs, 1),
        "gram": {"bound": "mfma", "achieved": round(g_tf, 2), "peak": mfma_peak,
                 "unit": "TFLOP/s", "frac": round(g_tf / mfma_peak, 4),
                 "avg_launch_ms": round(g["ms"] / max(1, g["launches"]), 4)},
        "rotate": {"bound": "hbm", "achieved": round(r_gbs, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(r_gbs / HBM_PEAK_GBS, 4),
                   "avg_launch_ms": round(r["ms"] / max(1, r["launches"]), 4)},
        "gram_fused": {"bound": "hbm", "achieved": round(gf_gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(gf_gbs / HBM_PEAK_GBS, 4),
                       "avg_launch_ms": round(gf["ms"] / max(1, gf["launches"]), 4)},
        "projectors": {"bound": "hbm", "achieved": round(kb_gbs, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(kb_gbs / HBM_PEAK_GBS, 4),
                       "avg_launch_ms": round(kb["ms"] / max(1, kb["launches"]), 4)},
        "kernel_ms_per_step": {k: round(v["ms"] / n_timed, 3) for k, v in kt.items()},
        "launch_shapes": tune,
        "last_step": {k: info[k] for k in ("mu", "e_total", "residual_out_in", "charge")},
        "phase_ms": {k: round(info[k], 3) for k in ("ms_poisson", "ms_fragments",
                                                    "ms_fermi_density", "ms_step")},
    }
    # comparison paths on the same workload: batched FP64 (graph) and plain FP64
    # (one launch sequence per fragment, no graph)
    comparisons = {}
    if args.batched and not args.no_compare:
        variants = [("plain_fp64_per_fragment", 0, PREC_FP64, 2)]
        if prec != PREC_FP64:
            variants.insert(0, ("batched_fp64", 1, PREC_FP64, max(3, args.steps // 2)))
        for name, batched, pr, k in variants:
            print(f"[bench] comparison {name}", file=sys.stderr, flush=True)
            d2 = DCDFT.from_config(cfg, batched=batched, precision=pr)
            configure(d2)
            if batched and not args.no_autotune:
                d2.dcdft_autotune(args.tune_cache)
            d2.dcdft_scf_step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                d2.dcdft_scf_step()
            torch.cuda.synchronize()
            tk = (time.perf_counter() - t0) / k
            d2.close()
            comparisons[name] = {"value": round(1.0 / tk, 3), "unit": "SCF iter/s",
                                 "ms_per_step": round(1000.0 * tk, 3), "steps": k,
                                 "speedup_of_value": round(value * tk, 3)}
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg)
    kind = ("water-like cell" if cfg.name.startswith("water") else
            "a-Si-like cell" if cfg.name.startswith("asi") else "diamond Si cell")
    ms = [int(v) for v in cfg.nstate_frag]
    orbitals = (f"{ms[0]} orbitals each" if min(ms) == max(ms)
                else f"{min(ms)}-{max(ms)} orbitals per fragment")
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "SCF iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32/f64" if prec != PREC_FP64 else "f64",
        "data": "synthetic",
        "config": {"workload": (f"{cfg.name}: {cfg.system.n_atoms}-atom {kind}, grid "
                                f"{'x'.join(map(str, cfg.n_grid))}, "
                                f"{'x'.join(map(str, cfg.num_fragment))} fragments of "
                                f"{'x'.join(map(str, cfg.fragment_shape))} points, "
                                f"{orbitals}, "
                                f"{cfg.cg_sweeps} CG sweeps per SCF iteration"),
                   "n_fragments": cfg.n_fragments, "batched": bool(args.batched),
                   "precision": args.precision,
                   "mode": "fixed-density" if args.fixed_density else "scf",
                   "template_xi": args.template_xi, "mixer": args.mixer},
        "roofline": roofline, "cpu_baseline": cpu, "comparisons": comparisons, **extra,
        **({"lcfo": lcfo} if lcfo else {}),
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
