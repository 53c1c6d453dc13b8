"""Benchmark: Chebyshev-filtered subspace iteration steps on one MI355X.

One step = Lanczos spectrum bound (k = 10) -> Chebyshev filter of degree m on
N vectors -> Cholesky-QR -> Rayleigh-Ritz, all through the C ABI of
libchebfilter.so.  The workload is the 30-atom Si cluster on 24^3 degree-4
cells (n = 857,645 DOFs incl. 270 enrichment DOFs, N = 260, m = 40), built
by the seeded synthetic generator; the start block is the atomic-orbital
(enrichment-pencil) subspace.

Prints one JSON line.  value = n * N * m / (seconds per step): DOF-vectors
per second per Chebyshev degree over the whole step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12          # MI355X dense FP64 matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12         # MI355X dense FP32 matrix, FLOP/s
PEAK_BF16_MFMA = 2.5e15           # MI355X dense BF16 matrix, FLOP/s
PEAK_HBM = 8.0e12                 # MI355X HBM3E, B/s
CELL_KERNEL = {"fp64": ("cell_gemm", "k_cell_gemm", PEAK_FP64_MFMA),
               "fp32": ("cell_gemm_fp32", "k_cell_gemm_lp<fp32>", PEAK_FP32_MFMA),
               "bf16": ("cell_gemm_bf16", "k_cell_gemm_lp<bf16>", PEAK_BF16_MFMA)}
PROFILED = ("cell_gemm", "cell_gemv", "cell_gemm_fp32", "cell_gemm_bf16", "enr_part", "enr_reduce",
            "enr_q", "enr_gemm", "epilogue", "gram", "rotate")

WORKLOADS = {
    # name: (generator, N, m, wanted)
    "si30-24c": ("config2", 260, 40, 210),
    "hydrogen-8c": ("config1", 16, 20, 14),
    # the same Si cluster and mesh with classical elements only (n_e = 0)
    "si30-classical": ("config2_classical", 260, 40, 210),
    # 256 independent Si clusters of 1-40 atoms (N 16-350 each), batched form
    "si-batch256": ("batch_workload", None, 40, None),
    # the 280-atom cluster (48^3 cells, n = 6,970,391, n_e = 2520): the whole
    # 2200-vector block (1960 wanted), m = 50, precision forms against an FP64 run
    "si280-48c": ("config3", 2200, 50, 1960),
}


def cell_kernel_source_hash() -> str:
    """sha256 of the k_cell_gemm kernel's source text (the counters in the
    committed profile are valid only for that text)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_1610_02121_amd", "csrc", "cf_ops.hip")).read()
    i = src.index("void k_cell_gemm(")
    j = src.index("hipError_t launch_cell_gemm(", i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()


def measured_traffic():
    """HBM bytes per k_cell_gemm launch from the committed counter profile, if
    it was taken on the current kernel source; else None."""
    import re
    path = os.path.join(ROOT, "profiles", "k_cell_gemm-si30-24c.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"pmc-traffic: kernel=k_cell_gemm bytes_per_launch=(\d+) source_sha256=([0-9a-f]+)",
                  open(path).read())
    if not m or m.group(2) != cell_kernel_source_hash():
        return None
    return int(m.group(1))


GOLDEN_FIXED_POINT = {"si30-24c": "si30_24c_ritz.txt"}


def oracle_fixed_point_errors(name, seed, theta, wanted):
    """Ritz and band-energy error of the wanted Ritz values against the fixed
    point the oracle's own CPU iteration reached (a committed text file of
    its Ritz values), where one exists for the workload."""
    import numpy as np
    fn = GOLDEN_FIXED_POINT.get(name)
    path = os.path.join(ROOT, "tests", "golden", fn) if fn else None
    if seed != 0 or not path or not os.path.exists(path):
        return {}
    ref = np.loadtxt(path)[:, 1]
    d = np.asarray(theta[:wanted]) - ref[:wanted]
    return {"ritz_err_vs_oracle_Ha": float(np.abs(d).max()),
            "energy_err_vs_oracle_Ha": float(2.0 * abs(d.sum())),
            "oracle_reference": f"tests/golden/{fn}"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_problem(name, seed):
    from synth import configs
    gen = getattr(configs, WORKLOADS[name][0])
    return gen(seed=seed) if name.startswith("si") else gen()


def host_cpu():
    """(logical CPUs this process may use, CPU model name)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def cpu_baseline(prob, N_total, m, seed, budget_s=20.0):
    """The FP64 oracle's Chebyshev recurrence (cell-by-cell elemental
    products and block-wise M^-1, torch CPU on all host threads) on the
    workload's whole N-column block, timed for whole filter degrees until
    ~budget_s, scaled to DOF-vectors-degree/s."""
    import numpy as np
    import torch
    from oracle.cellwise import CellOperators
    nproc, model = host_cpu()
    threads = min(nproc, int(os.environ.get("OMP_NUM_THREADS", nproc)))
    t0 = time.time()
    ops = CellOperators(prob, threads=threads)
    ops.schur()                              # factor S outside the timing
    t_setup = time.time() - t0
    X = torch.from_numpy(np.random.default_rng(seed).standard_normal((ops.n, N_total)))
    e, c = 2.0 / 1000.0, 0.0
    deg = 0
    t0 = time.time()
    Yp, Y = X, X
    while True:
        Z = 2.0 * (e * ops.apply_Htilde(Y) - c * Y) - Yp
        Yp, Y = Y, Z
        deg += 1
        if time.time() - t0 > budget_s or deg >= m:
            break
    dt = time.time() - t0
    return {"value": ops.n * N_total * deg / dt, "unit": "DOF*vectors*degree/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "host": {"nproc": nproc, "cpu_model": model},
            "sample": f"{deg} degree(s) of the oracle's recurrence (cell-by-cell elemental "
                      f"products, block-wise M^-1; torch CPU FP64, {torch.get_num_threads()} "
                      f"threads) on the whole {N_total}-column block; setup {t_setup:.1f}s "
                      f"untimed"}


def assembly_timing(ctx, prob, reps=5):
    """H_cc_e = K + B^T diag(w V_e) B on the device for every cell without
    enrichment functions (the per-step operator update of a self-consistent
    iteration), V = the workload's potential at the cells' Gauss points.
    Kernel time from HIP events; the reduced copies' refresh is timed apart."""
    import numpy as np
    import torch
    from synth.assemble import plain_points, plain_tables
    B, w, K, _ = plain_tables(prob)
    ep = np.asarray(prob.enr_ptr)
    cells = np.nonzero(ep[1:] == ep[:-1])[0].astype(np.int32)
    pts = plain_points(prob, cells)
    V = torch.tensor(prob.meta["potential"](pts.reshape(-1, 3)).reshape(len(cells), -1),
                     dtype=torch.float64, device=ctx.device)
    ctx.assembly_tables(B, w, K)
    ctx.assemble_cells(cells, V)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.assemble_cells(cells, V)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    launches, ms, flops = ctx.profile_query("assemble")
    ctx.profile(False)
    kern = ms / max(launches, 1)
    return {"cells": int(len(cells)), "quadrature_points": int(len(w)),
            "kernel_ms": kern, "with_reduced_copies_ms": 1e3 * wall,
            "tflops": flops / max(launches, 1) / (kern / 1e3) / 1e12,
            "flops_credited": "2*36*256*nq per cell (the 36 upper 16x16 tiles)",
            "peak_tflops_fp64_mfma": PEAK_FP64_MFMA / 1e12,
            "hbm_write_gb": len(cells) * 128 * 128 * 8 / 1e9}


def enriched_assembly_timing(ctx, prob, reps=3):
    """The blocks of the cells with an adaptive rule (every enriched cell) on
    the device: H^cc_e, H^ec and H^ee from the potential at the generator's
    leaf-box grid (Sec. IV.C), then the rebuilt H^ee - M^ec D^-1 H^ec^T.
    Kernel times from HIP events; compared with the generator's host time
    for the same cells (numpy on its worker processes)."""
    import numpy as np
    import torch
    from synth.basis import gll_rule
    from synth.assemble import plain_tables
    qb, mesh, enr = prob.meta["quad_boxes"], prob.meta["mesh"], prob.meta["enr"]
    bp = np.asarray(qb["box_ptr"])
    cells = np.nonzero(bp[1:] > bp[:-1])[0].astype(np.int32)
    x, w = np.polynomial.legendre.leggauss(qb["ng"])
    gx, gw = 0.5 * (x + 1.0), 0.5 * w
    B, wq, K, _ = plain_tables(prob)
    ctx.assembly_tables(B, wq, K)
    ctx.enriched_tables(cells=cells, cell_lo=mesh.cell_lo()[cells], h=mesh.h,
                        nodes=0.5 * (gll_rule(mesh.p)[0] + 1.0), gauss_x=gx, gauss_w=gw,
                        box_ptr=np.concatenate([bp[cells], [bp[-1]]]), box_lo=qb["box_lo"],
                        box_size=qb["box_size"], centers=enr.centers, shells=enr.shell_terms(),
                        r0=enr.r0, t=enr.t)
    ng3 = len(gx) ** 3
    lo, sz = np.asarray(qb["box_lo"]), np.asarray(qb["box_size"])
    zz, yy, xx = np.meshgrid(gx, gx, gx, indexing="ij")
    ref = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    V = np.empty(lo.shape[0] * ng3)
    for s in range(0, lo.shape[0], 20000):          # points box by box, bounded temporaries
        pts = lo[s:s + 20000, None, :] + sz[s:s + 20000, None, None] * ref[None]
        V[s * ng3:(s + pts.shape[0]) * ng3] = prob.meta["potential"](pts.reshape(-1, 3))
    Vd = torch.tensor(V, dtype=torch.float64, device=ctx.device)
    ctx.assemble_enriched(Vd)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.assemble_enriched(Vd)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    la, ms_a, _ = ctx.profile_query("assemble_adaptive")
    lh, ms_h, _ = ctx.profile_query("rebuild_hmod")
    ctx.profile(False)
    ep = np.asarray(prob.enr_ptr)
    nq = np.diff(np.concatenate([bp[cells], [bp[-1]]])) * ng3
    na = ep[cells + 1] - ep[cells]
    nte = (na + 15) // 16
    # MFMA tile products: 36 upper 16 x 16 tiles of H^cc_e (one product per
    # point), 8 nte + nte (nte + 1) / 2 enrichment-row tiles (four per point)
    flops = float(np.sum(2.0 * 256 * nq * (36 + 4 * (8 * nte + nte * (nte + 1) // 2))))
    kern = (ms_a / max(la, 1))
    quad = prob.meta.get("quad", {})
    return {"cells": int(len(cells)), "enriched_cells": int((na > 0).sum()), "points": int(V.size),
            "boxes": int(lo.shape[0]), "blocks_ms": kern,
            "rebuild_hmod_ms": ms_h / max(lh, 1), "total_ms": 1e3 * wall,
            "tflops_blocks": flops / (kern / 1e3) / 1e12,
            "flops_credited": "2*256*nq per 16x16 tile and point term (36 H^cc tiles; "
                              "4 terms for each H^ec / upper H^ee tile)",
            "host_generator_s": quad.get("t_enriched"),
            "host_generator_workers": "forked numpy workers, one per host core (<= 16)"}


def run_si280(args):
    """The 280-atom precision-form workload at its full shape on one GPU: the
    whole operator (the plain cells' potential term assembled on the device),
    the whole N = 2200 block (122.7 GB in FP64) filtered and projected in
    place, work blocks of --col-chunk columns, m = 50, from the atomic-orbital
    start.  Forms (--forms): fp64 runs until the wanted Ritz values settle
    (the reference, saved with --ref-out); fp32 / bf16 run --reduced-steps
    steps in that filter arithmetic, then FP64 cleanup steps until the wanted
    Ritz values are within 1e-6 Ha of the reference (--ref-in)."""
    import numpy as np
    import scipy.linalg as sla
    import torch

    from paper_1610_02121_amd import Context, empty_block
    from synth import configs
    from synth.assemble import plain_points, plain_tables, potential_at_points
    _, N, m, wanted = WORKLOADS["si280-48c"]
    forms = [f for f in args.forms.split(",") if f]
    t0 = time.time()
    if args.problem_cache and os.path.exists(args.problem_cache):
        from synth.problem import Problem
        prob = Problem.load(args.problem_cache)
        prob.meta["quad"] = {"enriched_cells": int((np.diff(prob.enr_ptr) > 0).sum())}
        prob.meta.update(configs.config3_meta(seed=args.seed))
    else:
        log("generating the 280-atom cluster (enriched cells on the host)")
        prob = configs.config3(seed=args.seed, progress=log)
        if args.problem_cache:
            prob.save(args.problem_cache)
    if args.gen_only:
        log(f"generated and cached in {args.problem_cache}")
        return
    log(f"generated n={prob.n} n_e={prob.n_e} cells={prob.n_cells} enriched cells="
        f"{prob.meta['quad']['enriched_cells']} coupling rows={len(prob.enr_idx)} in "
        f"{time.time() - t0:.0f}s")
    # potential at the plain cells' Gauss points, on the host before the GPU is touched
    B, w, K, _ = plain_tables(prob)
    ep = np.asarray(prob.enr_ptr)
    cells = np.nonzero(ep[1:] == ep[:-1])[0].astype(np.int32)
    t1 = time.time()
    Vq = potential_at_points(prob.meta["potential"], plain_points(prob, cells).reshape(-1, 3))
    log(f"potential at {Vq.size} Gauss points of {len(cells)} plain cells ({time.time() - t1:.0f}s)")
    _, Vee = sla.eigh(prob.H_ee, prob.M_ee)
    v0h = np.random.default_rng(args.seed + 1).standard_normal(prob.n)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t1 = time.time()
    ctx = Context(prob, max_cols=N, col_chunk=args.col_chunk)
    log(f"context ready ({time.time() - t1:.0f}s), work blocks of {args.col_chunk} columns")
    Vd = torch.tensor(Vq.reshape(len(cells), -1), dtype=torch.float64, device=dev)
    del Vq
    ctx.assembly_tables(B, w, K)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    ctx.assemble_cells(cells, Vd)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - ta
    del Vd
    H_keep = prob.H_cc
    prob.H_cc = None                                     # the host copy is no longer needed
    del H_keep
    Vee_d = torch.tensor(Vee[:, :N], dtype=torch.float64, device=dev)
    v0 = torch.tensor(v0h, dtype=torch.float64, device=dev)
    Y = empty_block(prob.n, N, dev).zero_()   # the 2200-vector block (ld padded to 16)
    free, total = torch.cuda.mem_get_info()
    log(f"device memory in use {(total - free) / 2**30:.1f} GiB of {total / 2**30:.1f} GiB")
    ref = None
    if args.ref_in:
        ref = np.asarray(json.load(open(args.ref_in))["theta"])

    def start():
        Y.zero_()
        Y[prob.n_h:, :] = Vee_d
        return ctx.rayleigh_ritz(Y)

    runs = {}
    for form in forms:
        theta = start()
        rec = {"steps": [], "theta": None}
        b = None
        for st in range(args.max_steps):
            reduced = form != "fp64" and st < args.reduced_steps
            prec = form if reduced else "fp64"
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, b = ctx.lanczos_bounds(v0, 10)
            s1 = time.perf_counter()
            ctx.filter(Y, m, float(theta[-1]), b, Y=Y, prec=prec)
            torch.cuda.synchronize()
            s2 = time.perf_counter()
            th = ctx.rayleigh_ritz(Y)
            s3 = time.perf_counter()
            d = float(np.abs(th[:wanted] - theta[:wanted]).max())
            theta = th
            step = {"prec": prec, "t_bounds": s1 - s0, "t_filter": s2 - s1, "t_rr": s3 - s2,
                    "dtheta": d, "theta_1": float(th[0]), "theta_w": float(th[wanted - 1])}
            if ref is not None:
                step["ritz_err_vs_ref"] = float(np.abs(th[:wanted] - ref[:wanted]).max())
                step["energy_err_vs_ref"] = float(2 * abs(np.sum(th[:wanted] - ref[:wanted])))
            rec["steps"].append(step)
            log(f"{form} step {st + 1} ({prec}): bounds {s1 - s0:.2f}s filter {s2 - s1:.2f}s "
                f"rr {s3 - s2:.2f}s dtheta {d:.3e} theta_1 {th[0]:.8f} theta_{wanted} "
                f"{th[wanted - 1]:.8f}" + (f" err_vs_ref {step['ritz_err_vs_ref']:.3e}"
                                          if ref is not None else ""))
            if form == "fp64" and d < args.settle:
                break
            if form != "fp64" and not reduced and ref is not None and \
                    step["ritz_err_vs_ref"] <= 1e-6:
                break
        rec["theta"] = theta
        rec["b"] = b
        rec["res_max_wanted"] = float(np.max(ctx.residual_norms(Y, theta)[:wanted]))
        runs[form] = rec
        if form == "fp64" and args.ref_out:
            with open(args.ref_out, "w") as f:
                json.dump({"workload": "si280-48c", "N": N, "m": m, "wanted": wanted,
                           "steps": len(rec["steps"]), "settle": args.settle,
                           "theta": [float(x) for x in theta]}, f)
    work = prob.n * N * m
    out = {
        "metric": "Chebyshev-filter DOF*vectors/s (per degree, whole SCF step) and SCF-step time, "
                  "FP64 vs mixed, Ritz error against the FP64 run",
        "unit": "DOF*vectors*degree/s", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "data": "synthetic",
        "config": {"workload": "si280-48c", "n_dof": prob.n, "n_enrich": prob.n_e,
                   "cells": prob.n_cells, "enriched_cells": prob.meta["quad"]["enriched_cells"],
                   "degree_p": prob.p, "vectors": N, "wanted": wanted, "cheb_degree": m,
                   "col_chunk": args.col_chunk},
        "plain_cell_assembly_ms": 1e3 * t_asm,
        "device_memory_gib": (total - free) / 2 ** 30,
        "forms": {},
    }
    for form, rec in runs.items():
        stp = rec["steps"]
        tot = [s["t_bounds"] + s["t_filter"] + s["t_rr"] for s in stp]
        f = {"steps": len(stp), "seconds_total": float(sum(tot)),
             "precs": [s["prec"] for s in stp],
             "step_s": tot, "filter_s": [s["t_filter"] for s in stp],
             "rr_s": [s["t_rr"] for s in stp], "bounds_s": [s["t_bounds"] for s in stp],
             "dtheta": [s["dtheta"] for s in stp],
             "max_residual_Minv_wanted": rec["res_max_wanted"],
             "theta_1": float(rec["theta"][0]), "theta_wanted_max": float(rec["theta"][wanted - 1]),
             "theta_N": float(rec["theta"][-1]), "b": rec["b"]}
        if ref is not None:
            f["ritz_err_vs_ref"] = [s["ritz_err_vs_ref"] for s in stp]
            f["energy_err_vs_ref"] = [s["energy_err_vs_ref"] for s in stp]
        fp64_steps = [s for s in stp if s["prec"] == "fp64"]
        red_steps = [s for s in stp if s["prec"] != "fp64"]
        if fp64_steps:
            t = np.mean([s["t_bounds"] + s["t_filter"] + s["t_rr"] for s in fp64_steps])
            f["fp64_step_s"] = float(t)
            f["fp64_dof_vec_deg_per_s"] = work / t
            f["fp64_filter_dof_vec_deg_per_s"] = work / np.mean([s["t_filter"] for s in fp64_steps])
        if red_steps:
            t = np.mean([s["t_bounds"] + s["t_filter"] + s["t_rr"] for s in red_steps])
            f["reduced_step_s"] = float(t)
            f["reduced_filter_dof_vec_deg_per_s"] = work / np.mean([s["t_filter"] for s in red_steps])
        out["forms"][form] = f
    first = out["forms"][forms[0]]
    out["value"] = first.get("fp64_dof_vec_deg_per_s", first.get("reduced_filter_dof_vec_deg_per_s"))
    out["ms_per_step"] = 1e3 * first["seconds_total"] / first["steps"]
    out["steps"] = first["steps"]
    out["warmup"] = 0
    out["dtype"] = "f64" if forms[0] == "fp64" else forms[0].replace("fp", "f")
    print(json.dumps(out), flush=True)
    ctx.close()


def precision_forms(ctx, X, Y, m, a, b, reps=3):
    """Filter-only time of each precision form on the same block and interval,
    with the cell-product kernel's event-timed launches."""
    import torch
    n, N = X.shape
    res = {}
    tiles = {}
    for prec in ("fp64", "fp32", "bf16"):
        ctx.filter(X, m, a, b, Y=Y, prec=prec)          # first use builds the reduced copies
        if prec != "fp64":
            # tile shape of the reduced cell product, chosen by the library's autotuner
            tiles[prec] = ctx.autotune(X, m, a, b, prec=prec, reps=2, Y=Y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.filter(X, m, a, b, Y=Y, prec=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ctx.profile(True)
        ctx.filter(X, m, a, b, Y=Y, prec=prec)
        key, kname, peak = CELL_KERNEL[prec]
        launches, ms, flops = ctx.profile_query(key)
        ctx.profile(False)
        res[prec] = {"filter_ms": 1e3 * dt, "dof_vec_deg_per_s": n * N * m / dt,
                     "cell_kernel": kname, "cell_avg_launch_ms": ms / max(launches, 1),
                     "cell_tflops": flops / (ms / 1e3) / 1e12 if ms > 0 else None,
                     "cell_peak_tflops": peak / 1e12,
                     "cell_frac": flops / (ms / 1e3) / peak if ms > 0 else None}
    for prec in ("fp32", "bf16"):
        res[prec]["speedup_vs_fp64"] = res["fp64"]["filter_ms"] / res[prec]["filter_ms"]
        res[prec]["cell_tile_blocks_autotuned"] = tiles[prec]
    return res


def mixed_study(ctx, prob, N, m, wanted, seed, m_lp, max_passes=30):
    """Time to tolerance from the atomic-orbital start (seconds of device work
    per form, counted over whole passes: bounds + filter + Rayleigh-Ritz).
    Reference eigenvalues: an FP64 run continued until the wanted Ritz values
    change by < 1e-12 Ha between passes.  FP64 form: passes until the Ritz
    error <= 1e-8 Ha.  Mixed forms: reduced-precision passes of degree m_lp
    until the wanted Ritz values stop improving (change between passes no
    longer shrinks by 2x, or < 1e-7 Ha), then FP64 cleanup passes of degree m
    until the Ritz error <= 1e-6 Ha."""
    import numpy as np
    import torch

    from paper_1610_02121_amd import empty_block
    from synth import configs
    dev = torch.device("cuda", 0)
    v0 = torch.tensor(np.random.default_rng(seed + 1).standard_normal(prob.n),
                      dtype=torch.float64, device=dev)

    def run(schedule):
        X = empty_block(prob.n, N, dev)
        X.copy_(torch.from_numpy(configs.initial_block(prob, N, seed=seed)))
        Y = empty_block(prob.n, N, dev)
        th = ctx.rayleigh_ritz(X)
        hist = []
        t = 0.0
        phase = "reduced"
        for it in range(max_passes):
            prec, deg, phase, stop = schedule(it, hist, phase)
            if stop:
                break
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, b = ctx.lanczos_bounds(v0, 10)
            a = float(th[-1])
            try:
                ctx.filter(X, deg, a, b, Y=Y, prec=prec)
                th_new = ctx.rayleigh_ritz(Y)
            except Exception as exc:                     # reported, not hidden
                log(f"study pass {it}: {prec} m={deg} a={a:.6f} b={b:.6f} failed: {exc}")
                hist.append({"prec": prec, "degree": deg, "t": t, "failed": str(exc)})
                break
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            X, Y = Y, X
            d = float(np.abs(th_new[:wanted] - th[:wanted]).max())
            th = th_new
            hist.append({"prec": prec, "degree": deg, "t": t, "dtheta": d, "theta": th.copy()})
            log(f"study pass {it}: {prec} m={deg} a={a:.6f} b={b:.6f} dtheta={d:.3e} t={t:.3f}s")
        return hist

    # reference: FP64 passes until the wanted Ritz values settle at the FP64
    # noise level (change < 1e-8 Ha on three passes in a row), at most max_passes
    def settled(h):
        return len(h) >= 3 and all(x.get("dtheta", 1.0) < 1e-8 for x in h[-3:])
    ref = run(lambda it, h, ph: ("fp64", m, ph, settled(h)))
    if "failed" in ref[-1]:
        return {"failed": "reference run: " + ref[-1]["failed"]}
    lam = ref[-1]["theta"][:wanted]

    def err(h):
        return float(np.abs(h["theta"][:wanted] - lam).max()) if "theta" in h else None

    out = {"reference_passes": len(ref), "m": m, "m_reduced": m_lp}
    hit = next((h for h in ref if err(h) <= 1e-8), None)
    out["fp64"] = {"passes": ref.index(hit) + 1 if hit else None, "seconds": hit["t"] if hit else None,
                   "tolerance": 1e-8, "errors": [err(h) for h in ref]}
    for prec in ("fp32", "bf16"):
        def sched(it, h, ph, prec=prec):
            if h and h[-1]["prec"] == "fp64" and "theta" in h[-1] and err(h[-1]) <= 1e-6:
                return None, None, ph, True
            if ph == "reduced" and len(h) >= 3:
                d1, d0 = h[-1]["dtheta"], h[-2]["dtheta"]
                if d1 < 1e-7 or d1 > 0.5 * d0:
                    ph = "cleanup"
            return (prec, m_lp, ph, False) if ph == "reduced" else ("fp64", m, ph, False)
        hist = run(sched)
        last = hist[-1]
        ok = last["prec"] == "fp64" and "theta" in last and err(last) <= 1e-6
        out[prec] = {"passes": len(hist), "reduced_passes": sum(h["prec"] == prec for h in hist),
                     "seconds": last["t"] if ok else None, "tolerance": 1e-6,
                     "errors": [err(h) for h in hist], "reached": ok}
        if "failed" in last:
            out[prec]["failed"] = last["failed"]
        if ok and out["fp64"]["seconds"]:
            out[prec]["speedup_vs_fp64_time_to_tolerance"] = out["fp64"]["seconds"] / last["t"]
    return out


def batch_groups(pool, atoms, Ns, budget_gib=130.0, max_rows=12_000_000):
    """Entries (sorted by atom count) packed into groups that fit the device:
    per entry the FP64 blocks X, Y and the FP32 recurrence blocks
    (~28 n N bytes), per distinct problem of a group its operator (cell
    matrices FP64 + FP32, coupling blocks) and four n x N_max FP64 work
    blocks; at most max_rows block rows per group (launch sizes)."""
    order = sorted(range(len(atoms)), key=lambda i: (atoms[i], i))
    groups, cur = [], []

    def cost(g):
        maxc = max(Ns[i] for i in g)
        probs = {atoms[i] for i in g}
        ent = sum(28.0 * pool[atoms[i]].n * Ns[i] for i in g)
        ops = sum(12.0 * pool[a].n_cells * 128 * 128 + 32.0 * pool[a].n * maxc
                  + 48.0 * len(pool[a].enr_idx) * (128 + maxc) for a in probs)
        rows = sum(pool[atoms[i]].n for i in g)
        return (ent + ops) / 2 ** 30, rows

    for i in order:
        gib, rows = cost(cur + [i])
        if cur and (gib > budget_gib or rows > max_rows):
            groups.append(cur)
            cur = []
        cur.append(i)
    if cur:
        groups.append(cur)
    return groups


def run_batch(args):
    """The batched form at its specified sizes: 256 independent Si clusters
    of 1-40 atoms (seeded, uniform in atoms; each in its own cube with 8^3 to
    20^3 degree-4 cells; 16-350 vectors), FP32 filter (m = 40) and FP64
    Rayleigh-Ritz.  The entries are packed into groups that fit the device
    (batch_groups); one SCF step = for every group: the grouped Lanczos
    bounds, the batched filter (one launch per kernel family and step for all
    the group's entries, replayed from a HIP graph), the batched projection.
    Also times the filter alone batched and entry by entry through the
    single-problem entry point, and checks that both give the same bits."""
    import numpy as np
    import torch

    from paper_1610_02121_amd import Batch, Context
    from synth import configs
    m = WORKLOADS["si-batch256"][2]
    prec = "fp32" if args.prec == "fp64" else args.prec
    t0 = time.time()
    log("generating the batch pool (Si clusters of 1-40 atoms)")
    pool, atoms, Ns = configs.batch_workload(256, seed=args.seed, progress=log)
    log(f"pool of {len(pool)} problems (n = {min(p.n for p in pool.values())} .. "
        f"{max(p.n for p in pool.values())}) in {time.time() - t0:.0f}s; 256 entries, "
        f"sum n*N = {sum(pool[a].n * N for a, N in zip(atoms, Ns))}")
    groups = batch_groups(pool, atoms, Ns)
    # the group with the most work first: the autotuner runs on it, the other
    # groups take its coupling map
    groups.sort(key=lambda g: -sum(pool[atoms[i]].n * Ns[i] for i in g))
    log(f"{len(groups)} groups of {[len(g) for g in groups]} entries")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    work = sum(pool[a].n * N for a, N in zip(atoms, Ns)) * m
    tot = {"bounds": 0.0, "filter": 0.0, "rr": 0.0, "graph": 0.0, "nograph": 0.0, "seq": 0.0}
    tiles, same_all, checked = [], True, 0
    for gi, g in enumerate(groups):
        probs = [pool[atoms[i]] for i in g]
        gN = [Ns[i] for i in g]
        maxc = max(gN)
        batch = Batch(probs, max_cols=maxc)
        X = [torch.tensor(configs.initial_block(p, N, seed=args.seed + i), dtype=torch.float64,
                          device=dev) for i, p, N in zip(g, probs, gN)]
        Y = [torch.empty_like(x) for x in X]
        v0 = [torch.tensor(np.random.default_rng(args.seed + 1 + i).standard_normal(p.n),
                           dtype=torch.float64, device=dev) for i, p in zip(g, probs)]
        theta = batch.rayleigh_ritz(X)
        _, b0 = batch.lanczos_bounds(v0, 10)
        if gi == 0:
            tiles.append(batch.autotune(X, m, [float(th[-1]) for th in theta], b0, prec=prec,
                                        reps=1, Y=Y))
            cmap = batch.tuning()["coupling_map"]
            log(f"autotuned on group 1: {tiles[-1]} column block(s) per tile, coupling map "
                f"{cmap:08b}")
        else:
            batch.tuning(cmap)
        st = {"X": X, "Y": Y, "theta": theta}

        def step(timed):
            s0 = time.perf_counter()
            _, b = batch.lanczos_bounds(v0, 10)
            s1 = time.perf_counter()
            a = [float(th[-1]) for th in st["theta"]]
            batch.filter(st["X"], m, a, b, Y=st["Y"], prec=prec, use_graph=True)
            torch.cuda.synchronize()
            s2 = time.perf_counter()
            th = batch.rayleigh_ritz(st["Y"])
            s3 = time.perf_counter()
            st["X"], st["Y"], st["theta"], st["a"], st["b"] = st["Y"], st["X"], th, a, b
            if timed:
                tot["bounds"] += (s1 - s0) / args.steps
                tot["filter"] += (s2 - s1) / args.steps
                tot["rr"] += (s3 - s2) / args.steps

        for _ in range(args.warmup):
            step(False)
        for _ in range(args.steps):
            step(True)

        def time_filter(fn, reps=2):
            fn()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t1) / reps

        a, b = st["a"], st["b"]
        tot["graph"] += time_filter(lambda: batch.filter(st["X"], m, a, b, Y=st["Y"], prec=prec,
                                                         use_graph=True))
        tot["nograph"] += time_filter(lambda: batch.filter(st["X"], m, a, b, Y=st["Y"], prec=prec,
                                                           use_graph=False))
        # a few entries' batched outputs kept to compare with the single-problem path
        keep = list(range(0, len(g), max(1, len(g) // 4)))
        Yb = {k: st["Y"][k].clone() for k in keep}
        batch.close()
        del batch
        torch.cuda.empty_cache()
        singles = {}
        for i, N in zip(g, gN):
            singles[atoms[i]] = max(singles.get(atoms[i], 0), N)
        singles = {k: Context(pool[k], max_cols=c) for k, c in singles.items()}

        def sequential():
            for k, i in enumerate(g):
                singles[atoms[i]].filter(st["X"][k], m, a[k], b[k], Y=st["Y"][k], prec=prec)
        tot["seq"] += time_filter(sequential)
        torch.cuda.synchronize()
        for k, y in Yb.items():
            same_all &= bool(torch.equal(y, st["Y"][k]))
            checked += 1
        for c in singles.values():
            c.close()
        del X, Y, st, Yb, singles
        torch.cuda.empty_cache()
        log(f"group {gi + 1}/{len(groups)}: {len(g)} entries (atoms {atoms[g[0]]}-{atoms[g[-1]]}, "
            f"N <= {maxc}) done; running totals {', '.join(f'{k} {v:.2f}s' for k, v in tot.items())}")
    step_s = tot["bounds"] + tot["filter"] + tot["rr"]
    out = {
        "metric": "batched Chebyshev-filter DOF*vectors/s (per degree, whole SCF step), "
                  "256 independent problems",
        "value": work / step_s,
        "unit": "DOF*vectors*degree/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * step_s,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16"}[prec], "data": "synthetic",
        "config": {"workload": "si-batch256", "entries": 256, "distinct_problems": len(pool),
                   "atoms_per_entry": "U{1..40}", "cells_per_axis": "8-20",
                   "vectors": f"{min(Ns)}-{max(Ns)}", "cheb_degree": m,
                   "sum_n_times_N": work // m, "groups": [len(g) for g in groups],
                   "precision": f"{prec} filter, fp64 Schur solve and Rayleigh-Ritz",
                   "cell_tile_blocks_autotuned": tiles[0], "coupling_map_autotuned": cmap},
        "phases_ms": {"bounds": 1e3 * tot["bounds"], "filter": 1e3 * tot["filter"],
                      "cholqr_rr": 1e3 * tot["rr"]},
        "filter_only_ms": {"batched_graph": 1e3 * tot["graph"],
                           "batched_no_graph": 1e3 * tot["nograph"],
                           "entry_by_entry": 1e3 * tot["seq"]},
        "filter_dof_vec_deg_per_s": work / tot["graph"],
        "speedup_batched_vs_entry_by_entry": tot["seq"] / tot["graph"],
        "batched_equals_entry_by_entry": bool(same_all), "entries_compared_bitwise": checked,
    }
    print(json.dumps(out), flush=True)


def run_scf(args):
    """Kohn-Sham self-consistent steps on the 30-atom workload (Sec. II, V):
    per step the effective potential from the input density (LDA, Hartree
    Poisson solve), the Hamiltonian blocks of every cell from it (device
    assembly), --scf-filter Chebyshev-filtered subspace steps (filter of
    degree m, Rayleigh-Ritz), occupations and Fermi level, the output
    density and Anderson mixing.  The synthetic Si nuclei (Z = 14, softened)
    give 14 electrons per atom: 420 electrons, 210 occupied states, N = 260.
    Reports each phase's time per step and the density residual."""
    import numpy as np
    import torch

    from paper_1610_02121_amd import Context, empty_block, fermi_level
    from synth import configs
    from synth.assemble import plain_tables
    from synth.basis import gll_rule
    name = "si30-24c"
    _, N, m, wanted = WORKLOADS[name]
    t0 = time.time()
    log("generating the 30-atom workload (with its adaptive grid)")
    prob = configs.config2(seed=args.seed)
    log(f"generated in {time.time() - t0:.0f}s")
    mesh, qb, enr = prob.meta["mesh"], prob.meta["quad_boxes"], prob.meta["enr"]
    n_el = 14.0 * enr.n_atoms
    kT = args.scf_kt
    dev_ = torch.device("cuda", 0)
    torch.cuda.set_device(dev_)
    ctx = Context(prob, max_cols=N)
    B, wq, K, ref = plain_tables(prob)
    ctx.assembly_tables(B, wq, K)
    bp = np.asarray(qb["box_ptr"])
    cells = np.nonzero(bp[1:] > bp[:-1])[0].astype(np.int32)
    x, w = np.polynomial.legendre.leggauss(qb["ng"])
    ctx.enriched_tables(cells=cells, cell_lo=mesh.cell_lo()[cells], h=mesh.h,
                        nodes=0.5 * (gll_rule(mesh.p)[0] + 1.0), gauss_x=0.5 * (x + 1.0),
                        gauss_w=0.5 * w, box_ptr=np.concatenate([bp[cells], [bp[-1]]]),
                        box_lo=qb["box_lo"], box_size=qb["box_size"], centers=enr.centers,
                        shells=enr.shell_terms(), r0=enr.r0, t=enr.t)
    center = np.asarray(enr.centers).mean(axis=0)
    ctx.scf_setup(mesh.cell_lo(), ref, center, args.scf_width, cg_max_iter=20000,
                  cg_tol=1e-10, mix_depth=4, mix_beta=0.5)
    xyz, _ = ctx.scf_geometry()
    vext = torch.tensor(prob.meta["potential"](xyz), dtype=torch.float64, device=dev_)
    del xyz
    log(f"{ctx.scf_points} points ({ctx.scf_plain_points} on plain cells)")
    X = empty_block(prob.n, N, dev_)
    X.copy_(torch.from_numpy(configs.initial_block(prob, N, seed=args.seed)))
    theta = ctx.rayleigh_ritz(X)
    v0 = torch.tensor(np.random.default_rng(args.seed + 1).standard_normal(prob.n),
                      dtype=torch.float64, device=dev_)
    state = {"X": X, "Y": empty_block(prob.n, N, dev_), "theta": theta}

    def chefsi(steps):
        _, b = ctx.lanczos_bounds(v0, 10)
        for _ in range(steps):
            ctx.filter(state["X"], m, float(state["theta"][-1]), b, Y=state["Y"])
            state["theta"] = ctx.rayleigh_ritz(state["Y"])
            state["X"], state["Y"] = state["Y"], state["X"]

    def sync():
        torch.cuda.synchronize()
        return time.perf_counter()

    chefsi(args.scf_init_steps)
    f, mu = fermi_level(state["theta"], n_el, kT)
    rho_in = ctx.scf_density(state["X"], f)
    steps = []
    for it in range(args.scf_steps):
        s0 = sync()
        veff, terms, cg = ctx.scf_potential(rho_in, vext)
        s1 = sync()
        ctx.scf_assemble(veff)
        s2 = sync()
        chefsi(args.scf_filter)
        s3 = sync()
        f, mu = fermi_level(state["theta"], n_el, kT)
        rho_out = ctx.scf_density(state["X"], f)
        s4 = sync()
        rho_in, res = ctx.scf_mix(rho_in, rho_out)
        s5 = sync()
        th = state["theta"]
        e_tot = 2 * float(f @ th) + terms["E_xc"] - terms["int_rho_vxc"] - terms["half_int_rho_vh"]
        rec = {"step": it + 1, "density_residual": res, "potential_s": s1 - s0, "cg_iters": cg,
               "assembly_s": s2 - s1, "chefsi_s": s3 - s2, "density_s": s4 - s3, "mix_s": s5 - s4,
               "step_s": s5 - s0, "mu": mu, "eps_1": float(th[0]), "eps_homo": float(th[wanted - 1]),
               "energy_terms_Ha": e_tot, "charge": terms["charge"]}
        steps.append(rec)
        log(f"SCF step {it + 1}: residual {res:.3e}, step {s5 - s0:.3f}s (potential {s1 - s0:.3f}, "
            f"assembly {s2 - s1:.3f}, ChFSI {s3 - s2:.3f}, density {s4 - s3:.3f}, mix {s5 - s4:.3f}), "
            f"CG {cg}, mu {mu:.6f}, charge {terms['charge']:.6f}")
    mean = {k: float(np.mean([r[k] for r in steps])) for k in
            ("potential_s", "assembly_s", "chefsi_s", "density_s", "mix_s", "step_s")}
    out = {"metric": "Kohn-Sham SCF step time (potential, assembly, ChFSI, density, mixing)",
           "value": mean["step_s"], "unit": "s/SCF step", "n_gpus": 1, "steps": args.scf_steps,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "n_dof": prob.n, "n_enrich": prob.n_e, "vectors": N,
                      "cheb_degree": m, "filter_steps_per_scf_step": args.scf_filter,
                      "electrons": n_el, "kT_Ha": kT, "points": ctx.scf_points,
                      "mixing": "Anderson, 4 stages, beta 0.5"},
           "mean_phase_s": mean, "steps_detail": steps}
    print(json.dumps(out), flush=True)
    ctx.close()


def classical_study(args):
    """The paper's DOF x degree argument (Sec. VI.B.1: enriched degree 80
    against classical 1500, lambda_max 1e3 against 1e6) on the hydrogen
    workload: the enriched 8^3-cell discretization against classical
    (enrichment-free) uniform meshes of degree-4 cells on the same 20 Bohr
    box.  Each runs the subspace iteration (N = 16, 14 wanted) from its own
    start (atomic orbitals where there are enrichments, else N(0,1)) with the
    10-step Lanczos bound and one degree rule for all (per step, the smallest
    m that damps the top wanted Ritz value against theta_N by 100:
    m = ln(100) / acosh|t(theta_Nw)|), until the wanted Ritz values move
    less than 1e-10 Ha.  Reported: DOFs, b, degrees, steps, time, and the
    ground-state error against -1/2 Ha.  Meshes are uniform here (the paper
    refines classical meshes towards the nuclei)."""
    import numpy as np
    import torch

    from paper_1610_02121_amd import Context
    from synth import configs
    N, wanted = 16, 14
    cases = [("enriched", 8)] + [("classical", int(k)) for k in args.classical_meshes.split(",")]
    probs = {}
    for kind, nc in cases:           # generate before the GPU is touched
        t0 = time.time()
        probs[(kind, nc)] = configs.hydrogen(nc=nc, length=20.0, p=4, r_c=6.0,
                                             enrich=kind == "enriched")
        log(f"{kind} {nc}^3: n={probs[(kind, nc)].n} generated in {time.time() - t0:.0f}s")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    res = []
    for kind, nc in cases:
        prob = probs.pop((kind, nc))
        ctx = Context(prob, max_cols=N)
        X = torch.tensor(configs.initial_block(prob, N, seed=args.seed), dtype=torch.float64,
                         device=dev)
        v0 = torch.tensor(np.random.default_rng(args.seed + 1).standard_normal(prob.n),
                          dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = ctx.rayleigh_ritz(X)
        _, b = ctx.lanczos_bounds(v0, 10)
        degs = []
        for step in range(args.max_steps):
            a = float(th[-1])
            t = abs((2.0 * th[wanted - 1] - a - b) / (b - a))
            m = int(min(4000, max(8, np.ceil(np.log(100.0) / np.arccosh(max(t, 1.0 + 1e-12))))))
            degs.append(m)
            Y = ctx.filter(X, m, a, b)
            th_new = ctx.rayleigh_ritz(Y)
            d = float(np.abs(th_new[:wanted] - th[:wanted]).max())
            X, th = Y, th_new
            if d < 1e-10:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"kind": kind, "cells_per_axis": nc, "n_dof": prob.n, "n_enrich": prob.n_e,
               "b": b, "degrees": degs, "steps": len(degs), "seconds": dt,
               "dof_times_degree_sum": float(prob.n * sum(degs)),
               "lambda_1": float(th[0]), "ground_state_err_Ha": float(th[0] + 0.5),
               "n2_levels": [float(x) for x in th[1:5]]}
        res.append(rec)
        log(f"{kind} {nc}^3: n={prob.n} b={b:.1f} degrees {degs[0]}..{degs[-1]} steps {len(degs)} "
            f"{dt:.2f}s lambda_1 {th[0]:.8f} (err {th[0] + 0.5:.2e})")
        ctx.close()
        del prob
    enr = res[0]
    match = [r for r in res[1:] if abs(r["ground_state_err_Ha"]) <= abs(enr["ground_state_err_Ha"])]
    out = {"study": "classical (enrichment-free) against enriched finite elements, hydrogen, "
                    "DOF x Chebyshev degree to the same ground-state accuracy",
           "vectors": N, "wanted": wanted, "cases": res,
           "classical_matching_accuracy": match[0]["cells_per_axis"] if match else None}
    if match:
        c = match[0]
        out["ratios_classical_over_enriched"] = {
            "dof": c["n_dof"] / enr["n_dof"], "b": c["b"] / enr["b"],
            "mean_degree": float(np.mean(c["degrees"]) / np.mean(enr["degrees"])),
            "time": c["seconds"] / enr["seconds"]}
    print(json.dumps(out), flush=True)


def learned_study(args):
    """Learned bounds (the network with the guard) against the Lanczos bound on
    a self-consistent-step sequence.  Training corpus: three perturbation
    sequences of 40 steps on each Si cluster of 1-6 atoms (labels: theta_N, a
    40-step Lanczos bound and the degree rule), 2000 Adam steps on batches of
    64 with a cosine step-size decay.  Evaluation: 30 steps on the 8-atom
    cluster with a new perturbation sequence, each step's Ritz values against
    a reference from FP64 passes (Lanczos bound, degree rule) continued until
    they settle."""
    import numpy as np
    import torch

    from paper_1610_02121_amd import Context, Mlp
    from paper_1610_02121_amd import learned as L
    from synth import configs
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    inputs, targets = [], []
    for nat in (1, 2, 3, 4, 5, 6):
        prob = configs.learned_cluster(nat, seed=args.seed)
        N = 16 + round(48 * (nat - 1) / 7)
        wanted = N - 8
        ctx = Context(prob, max_cols=N)
        v0 = torch.tensor(np.random.default_rng(args.seed + nat).standard_normal(prob.n),
                          dtype=torch.float64, device=dev)
        for sq in range(3):
            recs, _ = L.run_sequence(ctx, prob, N, wanted, 40, seed=100 * nat + sq,
                                     chooser=L.lanczos_chooser(ctx, v0, wanted), v0=v0, label_k=40)
            inputs += [r["input"] for r in recs]
            targets += [r["target"] for r in recs]
        ctx.close()
        log(f"corpus: {nat}-atom cluster done ({len(inputs)} samples, {time.time() - t0:.0f}s)")
    inputs, targets = np.array(inputs), np.array(targets)
    net = Mlp(L.N_IN, L.WIDTH, L.DEPTH, L.N_OUT, max_batch=64)
    net.set_params(L.init_params(seed=args.seed))
    t1 = time.time()
    losses = L.train(net, inputs, targets, steps=2000, batch=64, lr=1e-3, seed=args.seed, log=log,
                     lr_end=1e-5)
    t_train = time.time() - t1
    # the corpus's labels and the trained network's outputs on it, against the
    # guard's acceptance window for beta
    pred = net.predict(inputs)
    diag = {"label_beta_mean": float(targets[:, 1].mean()),
            "label_beta_p10_p50_p90": [float(x) for x in np.percentile(targets[:, 1], [10, 50, 90])],
            "label_beta_below_guard": float(np.mean(targets[:, 1] < 0.98)),
            "pred_beta_below_guard": float(np.mean(pred[:, 1] < 0.98)),
            "pred_abs_err_beta_median": float(np.median(np.abs(pred[:, 1] - targets[:, 1]))),
            "pred_abs_err_m_median": float(np.median(np.abs(pred[:, 2] - targets[:, 2])))}
    log(f"labels vs guard: {diag}")
    # evaluation
    prob = configs.learned_cluster(8, seed=args.seed)
    N, wanted, steps = 64, 56, 30
    ctx = Context(prob, max_cols=N)
    v0 = torch.tensor(np.random.default_rng(args.seed + 99).standard_normal(prob.n),
                      dtype=torch.float64, device=dev)
    runs = {}
    for name, chooser in (("lanczos", L.lanczos_chooser(ctx, v0, wanted)),
                          ("learned", L.mlp_chooser(ctx, net, v0))):
        recs, _ = L.run_sequence(ctx, prob, N, wanted, steps, seed=777, chooser=chooser, v0=v0,
                                 log=None, lanczos_fallback=L.lanczos_chooser(ctx, v0, wanted))
        runs[name] = recs
        log(f"{name}: done")
    # reference per step: the same operator sequence, FP64 passes until settled
    from synth import perturb
    X = torch.tensor(configs.initial_block(prob, N, seed=777), dtype=torch.float64, device=dev)
    Y = torch.empty_like(X)
    ref = []
    for s, Hs in enumerate(perturb.sequence(prob, steps, seed=777)):
        ctx.update_H_cc(Hs)
        th = ctx.rayleigh_ritz(X)
        for it in range(40):
            _, b = ctx.lanczos_bounds(v0, 10)
            mref = L.degree_rule(float(th[0]), float(th[wanted - 1]), float(th[-1]), b)
            ctx.filter(X, mref, float(th[-1]), b, Y=Y)
            thn = ctx.rayleigh_ritz(Y)
            X, Y = Y, X
            d = float(np.abs(thn[:wanted] - th[:wanted]).max())
            th = thn
            if d < 1e-10 and it >= 2:
                break
        ref.append(th[:wanted].copy())
    ctx.close()
    out = {"study": "learned filter bounds vs Lanczos bound", "corpus_samples": int(len(inputs)),
           "train_steps": 2000, "train_seconds": t_train, "train_loss_first": float(losses[:20].mean()),
           "train_loss_last": float(losses[-20:].mean()), "corpus_vs_guard": diag,
           "eval": {"workload": "8-atom Si cluster, 12^3 cells, n = %d, N = %d, wanted %d, %d steps"
                                % (prob.n, N, wanted, steps)}}
    for name, recs in runs.items():
        errs = [float(np.abs(r["theta"][:wanted] - ref[i]).max()) for i, r in enumerate(recs)]
        out["eval"][name] = {
            "ritz_err_last10_max": max(errs[-10:]), "ritz_err_median": float(np.median(errs)),
            "ritz_err_per_step": errs,
            "bounds_ms_mean": 1e3 * float(np.mean([r["t_bounds"] for r in recs])),
            "pass_ms_mean": 1e3 * float(np.mean([r["t_pass"] for r in recs])),
            "degree_mean": float(np.mean([r["m"] for r in recs])),
            "lanczos_fallbacks": int(sum(r["fallback"] for r in recs)) if name == "learned" else None,
            "rescued_steps": int(sum(r["rescued"] for r in recs)),
        }
    bl = [r["b"] for r in runs["lanczos"]]
    bm = [r["b"] for r in runs["learned"]]
    out["eval"]["b_learned_over_lanczos"] = [float(x / y) for x, y in zip(bm, bl)]
    print(json.dumps(out), flush=True)
    net.close()


LEARNED_CORPUS_ATOMS = (10, 20, 30, 40, 50, 60)


def learned_vectors(n_atoms: int) -> tuple[int, int]:
    """Block width and wanted count of a learned-bounds corpus cluster: 16 + 4
    vectors per atom (16 .. 256 for 10 .. 60 atoms), the top eighth a guard."""
    N = 16 + 4 * n_atoms
    return N, N - max(8, N // 8)


def learned_corpus(args):
    """Training corpus of the learned bounds at its stated scale: 2000 filter
    steps on seeded Si clusters of 10, 20, .., 60 atoms on the 30-atom
    workload's mesh (48 Bohr cube, 24^3 degree-4 cells, r_c = 8), 50
    sequences of 40 self-consistent steps (a fresh seeded smooth field on the
    plain cells' potential each step, rebuilt on the device; labels from a
    40-step Lanczos run and the degree rule), then 2000 Adam steps of the
    network.  Writes the parameters and the corpus (for the normalisation) to
    --learned-out and prints one JSON line."""
    import numpy as np

    from synth import configs, perturb
    from synth.assemble import plain_points, potential_at_points
    t0 = time.time()
    probs = {}
    for k in LEARNED_CORPUS_ATOMS:
        # generated on the host before anything touches the GPU (forked workers)
        prob = configs.si_cluster(n_atoms=k, length=48.0, nc=24, p=4, r_c=8.0,
                                  seed=args.seed + 100 + k, plain_blocks=False)
        plain, far = perturb.plain_cell_sets(prob)
        V0 = potential_at_points(prob.meta["potential"], plain_points(prob, plain).reshape(-1, 3))
        probs[k] = (prob, plain, far, V0)
        log(f"corpus cluster {k} atoms: n = {prob.n}, {len(plain)} plain cells ({len(far)} far), "
            f"{time.time() - t0:.0f}s")
    import torch

    from paper_1610_02121_amd import Context, Mlp
    from paper_1610_02121_amd import learned as L
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    inputs, targets, per = [], [], {}
    nseq = [9, 9, 8, 8, 8, 8]                    # 50 sequences of 40 steps: 2000 samples
    for (k, (prob, plain, far, V0)), ns in zip(probs.items(), nseq):
        N, wanted = learned_vectors(k)
        ctx = Context(prob, max_cols=N)
        steps = L.DeviceSteps(ctx, prob, plain, far, V0)
        v0 = torch.tensor(np.random.default_rng(args.seed + 7 * k).standard_normal(prob.n),
                          dtype=torch.float64, device=dev)
        t1 = time.time()
        for sq in range(ns):
            seed = 1000 * k + sq
            recs, _ = L.run_sequence(ctx, prob, N, wanted, 40, seed=seed,
                                     chooser=L.lanczos_chooser(ctx, v0, wanted), v0=v0, label_k=40,
                                     apply_step=steps.start(seed))
            inputs += [r["input"] for r in recs]
            targets += [r["target"] for r in recs]
        per[k] = {"n": prob.n, "N": N, "wanted": wanted, "sequences": ns,
                  "seconds": time.time() - t1}
        log(f"corpus: {k}-atom cluster done ({len(inputs)} samples, {time.time() - t1:.0f}s)")
        ctx.close()
        del steps
    inputs, targets = np.array(inputs), np.array(targets)
    net = Mlp(L.N_IN, L.WIDTH, L.DEPTH, L.N_OUT, max_batch=64)
    net.set_params(L.init_params(seed=args.seed))
    t1 = time.time()
    losses = L.train(net, inputs, targets, steps=2000, batch=64, lr=1e-3, seed=args.seed, log=log,
                     lr_end=1e-5)
    t_train = time.time() - t1
    pred = net.predict(inputs)
    np.savez(args.learned_out, params=net.get_params(), inputs=inputs, targets=targets)
    out = {"study": "learned-bounds corpus", "corpus_samples": int(len(inputs)),
           "clusters": per, "train_steps": 2000, "train_seconds": t_train,
           "train_loss_first": float(losses[:20].mean()), "train_loss_last": float(losses[-20:].mean()),
           "label_beta_below_guard": float(np.mean(targets[:, 1] < 0.98)),
           "pred_beta_below_guard": float(np.mean(pred[:, 1] < 0.98)),
           "pred_abs_err_beta_median": float(np.median(np.abs(pred[:, 1] - targets[:, 1]))),
           "pred_abs_err_m_median": float(np.median(np.abs(pred[:, 2] - targets[:, 2]))),
           "seconds": time.time() - t0}
    print(json.dumps(out), flush=True)
    net.close()


def learned_eval280(args):
    """The trained network (--learned-in) against the Lanczos bound on the
    280-atom cluster: 30 self-consistent steps (a fresh seeded smooth field on
    the far plain cells' potential each step, rebuilt on the device), both
    paths in lockstep on one context from the atomic-orbital start, N = 600
    vectors (560 wanted: the 1s and 2s bands), 256-column work blocks.  Accuracy:
    references at steps 10, 20 and 30 from the Lanczos path's block (FP64
    passes until the wanted Ritz values settle), and every step's largest
    residual norm of the wanted pairs."""
    import numpy as np

    from synth import configs, perturb
    from synth.assemble import plain_points, potential_at_points
    N, wanted, steps = 600, 560, 30
    t0 = time.time()
    prob = configs.config3(progress=log)
    plain, far = perturb.plain_cell_sets(prob)
    V0 = potential_at_points(prob.meta["potential"], plain_points(prob, plain).reshape(-1, 3))
    log(f"280-atom cluster: n = {prob.n}, {len(plain)} plain cells ({len(far)} far), "
        f"{time.time() - t0:.0f}s")
    import torch

    from paper_1610_02121_amd import Context, Mlp
    from paper_1610_02121_amd import learned as L
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = Context(prob, max_cols=N, col_chunk=256)
    H_keep = prob.H_cc
    prob.H_cc = None                                     # the host copy is no longer needed
    del H_keep
    dsteps = L.DeviceSteps(ctx, prob, plain, far, V0)
    del V0
    d = np.load(args.learned_in)
    net = Mlp(L.N_IN, L.WIDTH, L.DEPTH, L.N_OUT, max_batch=64)
    net.set_params(d["params"])
    net.fit_normalization(d["inputs"], d["targets"])
    v0 = torch.tensor(np.random.default_rng(args.seed + 280).standard_normal(prob.n),
                      dtype=torch.float64, device=dev)
    choosers = {"lanczos": L.lanczos_chooser(ctx, v0, wanted), "learned": L.mlp_chooser(ctx, net, v0)}
    t1 = time.time()
    recs, refs = L.run_paths(ctx, prob, N, wanted, steps, seed=args.seed + 777, choosers=choosers,
                             v0=v0, apply_step=dsteps.start(args.seed + 777), ref_steps=(10, 20, 30),
                             log=log, lanczos_fallback=L.lanczos_chooser(ctx, v0, wanted))
    out = {"study": "learned filter bounds vs Lanczos bound, 280-atom cluster",
           "workload": "si280-48c: n = %d, N = %d, wanted %d, %d steps" % (prob.n, N, wanted, steps),
           "corpus_samples": int(len(d["inputs"])), "seconds": time.time() - t1}
    for name, rr in recs.items():
        errs = {str(st): float(np.abs(rr[st - 1]["theta"][:wanted] - ref).max())
                for st, ref in refs.items()}
        eerr = {str(st): float(2.0 * abs(rr[st - 1]["theta"][:wanted].sum() - ref.sum()))
                for st, ref in refs.items()}
        out[name] = {"ritz_err_at": errs, "band_energy_err_at": eerr,
                     "res_max_per_step": [r["res_max"] for r in rr],
                     "degree_per_step": [int(r["m"]) for r in rr],
                     "b_per_step": [float(r["b"]) for r in rr],
                     "degree_sum": int(sum(r["m"] for r in rr)),
                     "pass_s_mean": float(np.mean([r["t_pass"] for r in rr])),
                     "bounds_s_mean": float(np.mean([r["t_bounds"] for r in rr])),
                     "lanczos_fallbacks": int(sum(r["fallback"] for r in rr)),
                     "rescued_steps": int(sum(r["rescued"] for r in rr))}
    print(json.dumps(out), flush=True)
    net.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="si30-24c", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-assembly", action="store_true",
                    help="skip the timing of the device assembly of the plain cells")
    ap.add_argument("--passes", type=int, default=1,
                    help="filter passes per step (each of degree m, Rayleigh-Ritz between them)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="arithmetic of the filter in the timed steps (Rayleigh-Ritz stays FP64)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the filter-only timing of the three precision forms")
    ap.add_argument("--mixed-study", action="store_true",
                    help="run the time-to-tolerance study of the precision forms instead")
    ap.add_argument("--problem-cache", default=None,
                    help="load the generated workload from this .npz if it exists, else "
                         "generate it and save it there (profiling runs avoid the generator's "
                         "worker processes this way)")
    ap.add_argument("--gen-only", action="store_true",
                    help="generate the workload into --problem-cache and exit (no GPU work)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy an n x N FP64 block 5 times with the library's copy kernel "
                         "(a kernel of known traffic, to calibrate the HBM byte counters)")
    ap.add_argument("--learned-corpus", action="store_true",
                    help="learned bounds: corpus of 2000 steps on 10-60-atom clusters + training "
                         "(writes --learned-out)")
    ap.add_argument("--learned-eval280", action="store_true",
                    help="learned bounds: 30 steps on the 280-atom cluster against the Lanczos "
                         "bound (reads --learned-in)")
    ap.add_argument("--learned-out", default="learned_net.npz")
    ap.add_argument("--learned-in", default="learned_net.npz")
    ap.add_argument("--learned-study", action="store_true",
                    help="train the bounds network and compare it with the Lanczos bound")
    ap.add_argument("--m-reduced", type=int, default=20,
                    help="filter degree of the reduced-precision passes in the study")
    ap.add_argument("--scf", action="store_true",
                    help="Kohn-Sham SCF steps on the 30-atom workload: potential, device "
                         "assembly, ChFSI, density, Anderson mixing")
    ap.add_argument("--scf-steps", type=int, default=8)
    ap.add_argument("--scf-filter", type=int, default=1,
                    help="Chebyshev-filtered subspace steps per SCF step")
    ap.add_argument("--scf-init-steps", type=int, default=4,
                    help="subspace steps on the starting Hamiltonian before the first density")
    ap.add_argument("--scf-kt", type=float, default=0.005, help="Fermi-Dirac smearing (Ha)")
    ap.add_argument("--scf-width", type=float, default=4.0,
                    help="width of the neutralising Gaussian (Bohr)")
    ap.add_argument("--classical-study", action="store_true",
                    help="enriched against classical (enrichment-free) hydrogen meshes at the "
                         "same ground-state accuracy: DOFs, bounds, degrees, time")
    ap.add_argument("--classical-meshes", default="8,16,24,32",
                    help="cells per axis of the classical meshes in the classical study")
    ap.add_argument("--col-chunk", type=int, default=256,
                    help="si280-48c: columns of the library's work blocks")
    ap.add_argument("--forms", default="fp64",
                    help="si280-48c: comma list of fp64, fp32, bf16 runs from the same start")
    ap.add_argument("--max-steps", type=int, default=20, help="si280-48c: steps per form at most")
    ap.add_argument("--reduced-steps", type=int, default=6,
                    help="si280-48c: steps in the reduced arithmetic before the FP64 cleanup")
    ap.add_argument("--settle", type=float, default=1e-9,
                    help="si280-48c: the FP64 run stops once the wanted Ritz values move less")
    ap.add_argument("--ref-in", default=None, help="si280-48c: FP64 reference Ritz values (json)")
    ap.add_argument("--ref-out", default=None, help="si280-48c: write the FP64 run's Ritz values")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1610_02121_amd import Context, empty_block
    from synth import configs

    name = args.workload
    if args.classical_study:
        classical_study(args)
        return
    if args.learned_study:
        learned_study(args)
        return
    if args.learned_corpus:
        learned_corpus(args)
        return
    if args.learned_eval280:
        learned_eval280(args)
        return
    if args.scf:
        run_scf(args)
        return
    if name == "si-batch256":
        run_batch(args)
        return
    if name == "si280-48c":
        run_si280(args)
        return
    _, N, m, wanted = WORKLOADS[name]
    t0 = time.time()
    if args.problem_cache and os.path.exists(args.problem_cache):
        from synth.problem import Problem
        log(f"loading {name} from {args.problem_cache}")
        prob = Problem.load(args.problem_cache)
    else:
        log(f"generating {name} (seed {args.seed})")
        prob = make_problem(name, args.seed)
        if args.problem_cache:
            prob.save(args.problem_cache)
    if args.gen_only:
        return
    log(f"generated n={prob.n} n_h={prob.n_h} n_e={prob.n_e} cells={prob.n_cells} in "
        f"{time.time() - t0:.1f}s")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # the study checks every filter output for non-finite values
    ctx = Context(prob, max_cols=N, check_finite=args.mixed_study)
    log(f"context ready ({time.time() - t0:.1f}s)")
    if args.copy_probe:
        # filter of degree 0 = k_copy of the n x N block: 8 n N bytes read and written
        Xc = torch.randn(prob.n, N, dtype=torch.float64, device=dev)
        Yc = torch.empty_like(Xc)
        for _ in range(5):
            ctx.filter(Xc, 0, 0.0, 1.0, Y=Yc)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe": "k_copy", "bytes_read": 8 * prob.n * N,
                          "bytes_written": 8 * prob.n * N, "calls": 5}), flush=True)
        ctx.close()
        return
    X0 = configs.initial_block(prob, N, seed=args.seed)
    # blocks with a leading dimension padded to 16 doubles (aligned row segments)
    X = empty_block(prob.n, N, dev)
    X.copy_(torch.from_numpy(X0))
    Y = empty_block(prob.n, N, dev)
    v0 = torch.tensor(np.random.default_rng(args.seed + 1).standard_normal(prob.n),
                      dtype=torch.float64, device=dev)
    if args.mixed_study:
        study = mixed_study(ctx, prob, N, m, wanted, args.seed, args.m_reduced)
        print(json.dumps({"study": "time to tolerance by precision form", "workload": name,
                          "n_dof": prob.n, "vectors": N, "wanted": wanted, **study}), flush=True)
        ctx.close()
        return
    theta = ctx.rayleigh_ritz(X)
    log(f"initial Rayleigh-Ritz: theta[0]={theta[0]:.6f} theta[N-1]={theta[-1]:.6f}")

    state = {"X": X, "Y": Y, "theta": theta, "b": None, "t_bounds": 0.0, "t_filter": 0.0,
             "t_rr": 0.0}

    def step(timed):
        s0 = time.perf_counter()
        lo, b = ctx.lanczos_bounds(v0, 10)          # synchronises
        s1 = time.perf_counter()
        a = float(state["theta"][-1])
        if args.passes > 1:
            ctx.filter_multipass(state["X"], m, args.passes, a, b, Y=state["Y"], prec=args.prec)
        else:
            ctx.filter(state["X"], m, a, b, Y=state["Y"], prec=args.prec)
        torch.cuda.synchronize()
        s2 = time.perf_counter()
        th = ctx.rayleigh_ritz(state["Y"])          # synchronises
        s3 = time.perf_counter()
        state["X"], state["Y"] = state["Y"], state["X"]
        state["prev_theta"], state["theta"], state["b"] = state["theta"], th, b
        if timed:
            state["t_bounds"] += s1 - s0
            state["t_filter"] += s2 - s1
            state["t_rr"] += s3 - s2

    for i in range(args.warmup):
        step(False)
        log(f"warmup step {i + 1}/{args.warmup}: theta[0]={state['theta'][0]:.8f} "
            f"theta[{wanted - 1}]={state['theta'][wanted - 1]:.8f} b={state['b']:.3f}")
    if not args.no_profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(True)
        log(f"step {i + 1}/{args.steps}: theta[0]={state['theta'][0]:.8f} "
            f"theta[{wanted - 1}]={state['theta'][wanted - 1]:.8f}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps

    # kernel timing over the timed region (HIP events on the library's stream)
    prof = {}
    if not args.no_profile:
        for k in PROFILED:
            prof[k] = ctx.profile_query(k)
        ctx.profile(False)

    # convergence of the wanted set: change of Ritz values over the last step and
    # residual norms ||H z - theta M z||_{M^-1} of the Ritz vectors
    dtheta = float(np.abs(state["theta"][:wanted] - state["prev_theta"][:wanted]).max())
    Z = state["X"]
    HZ = ctx.apply_H(Z)
    MZ = ctx.apply_M(Z)
    th = torch.tensor(state["theta"], dtype=torch.float64, device=dev)
    Rz = HZ - MZ * th[None, :]
    MinvR = ctx.apply_Sinv(Rz)
    res = torch.sqrt(torch.clamp((Rz * MinvR).sum(dim=0), min=0.0)).cpu().numpy()
    res_max = float(res[:wanted].max())

    n = prob.n
    value = n * N * m * args.passes / (ms_per_step / 1e3)
    out = {
        "metric": "Chebyshev-filter DOF*vectors/s (per degree, whole SCF step) and SCF-step time",
        "value": value,
        "unit": "DOF*vectors*degree/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.prec], "data": "synthetic",
        "config": {"workload": name, "n_dof": n, "n_enrich": prob.n_e, "cells": prob.n_cells,
                   "degree_p": prob.p, "vectors": N, "cheb_degree": m, "filter_passes": args.passes,
                "wanted": wanted,
                   "precision": args.prec if args.prec == "fp64" else
                   f"{args.prec} filter, fp64 Schur solve and Rayleigh-Ritz"},
        "phases_ms": {"bounds": 1e3 * state["t_bounds"] / args.steps,
                      "filter": 1e3 * state["t_filter"] / args.steps,
                      "cholqr_rr": 1e3 * state["t_rr"] / args.steps},
        "filter_dof_vec_deg_per_s": n * N * m * args.passes / (state["t_filter"] / args.steps),
        "convergence": {"max_dtheta_wanted": dtheta, "max_residual_Minv_wanted": res_max,
                        "theta_min": float(state["theta"][0]),
                        "theta_wanted_max": float(state["theta"][wanted - 1]),
                        **oracle_fixed_point_errors(name, args.seed, state["theta"], wanted)},
    }
    key, kname, peak = CELL_KERNEL[args.prec]
    if prof and prof[key][0] > 0:
        # every launch of the MFMA cell kernel in the timed region (the filter's and
        # the Rayleigh-Ritz products; single-vector Lanczos products run k_cell_gemv),
        # credited 2 npc^2 N flops per cell
        launches, ms, flops = prof[key]
        achieved = flops / (ms / 1e3)
        out["roofline"] = {"kernel": kname, "bound": "mfma", "achieved": achieved / 1e12,
                           "peak": peak / 1e12, "unit": "TFLOP/s",
                           "frac": achieved / peak,
                           "traffic": measured_traffic() if args.prec == "fp64" else None,
                           "launches": launches, "avg_launch_ms": ms / launches,
                           "flops_per_launch": flops / launches}
        out["kernel_ms_per_step"] = {k: v[1] / args.steps for k, v in prof.items() if v[0] > 0}
    if not args.no_forms:
        log("timing the filter alone in the three precision forms")
        out["precision_forms"] = precision_forms(ctx, state["X"], state["Y"], m,
                                                 float(state["theta"][-1]), state["b"])
    if not args.no_assembly and "potential" in prob.meta and "mesh" in prob.meta:
        log("timing the device assembly of the plain cells' blocks")
        out["plain_cell_assembly"] = assembly_timing(ctx, prob)
        if "quad_boxes" in prob.meta and prob.n_e:
            log("timing the device assembly of the enriched cells' blocks")
            out["enriched_cell_assembly"] = enriched_assembly_timing(ctx, prob)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(prob, N, m, args.seed)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
