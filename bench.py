"""Benchmark: FP64 Schwarz-preconditioned CG on the 3-D finite cell
elasticity workload (32^3 cells, p = 3, 64 seeded spherical voids,
alpha = 1e-8, clamped bottom face, traction on the top face; 2,738,019
unknowns), solved to a relative residual of 1e-8 on one MI355X.

One step = one pass of the whole hot path: build the preconditioner
(extract the 32,768 element blocks, their FP64 local inverses, the
diagonal fallback) and run PCG to ||b - A x|| / ||b|| <= 1e-8.  The
problem (assembled matrix and load) is resident in HBM before the timed
region starts.

Prints one JSON line.  The kernel-level roofline is measured live: the
solver brackets every SpMV and Schwarz block-product launch with HIP events
on its own stream during the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch on the 32^3 elasticity workload from two rocprofv3
# counter passes (FETCH_SIZE, WRITE_SIZE), scaled by what the same counters
# read for a plain 4 GiB copy (profiles/pcg_fp64_elastic32_p3_hbm_counters.md, full
# copies; profiles/pcg_fp64_elastic32_p3_shared_hbm_counters.md, shared copies one
# at a time; profiles/pcg_fp64_elastic32_p3_grouped_hbm_counters.md, grouped);
# to be re-measured whenever one of these kernels changes.
TRAFFIC = {"spmv": 8.3640e9, "spmv_shared": 9.2376e8, "spmv_grouped": 1.1796e9,
           "schwarz": 4.6881e9,
           "schwarz_shared": 1.3893e9, "schwarz_grouped": 1.3664e9}
METRIC = "DOF·iter/s and time-to-1e-8 residual: mixed/learned vs plain FP64 PCG"


def workload(small: bool, name: str = "elastic32"):
    import fcgen
    if small:
        return fcgen.porous_elasticity_3d(seed=0, n=8), "3D elasticity 8^3 cells (reduced check)"
    if name == "poisson64":
        return (fcgen.porous_poisson_3d(100, n=64, p=2),
                "3D finite cell Poisson, 64^3 cells, p=2, 64 spherical voids, alpha=1e-10")
    return (fcgen.porous_elasticity_3d(seed=0),
            "3D finite cell linear elasticity, 32^3 cells, p=3, 64 spherical voids, alpha=1e-8")


def algorithmic_bytes(info, m, n_blocks, nn, distinct_blocks=0):
    """Bytes each streaming kernel must move per launch (FP64 layout).
    Shared rows and shared local inverses count once per distinct copy."""
    n = info["n_dofs"]
    bd = info["bsr_dim"]
    nnzb = info["nnzb"]
    # values (and column indices unless the columns follow from the
    # lattice), row pointers, x and q once
    col_bytes = 0 if info.get("lattice_columns") else 4
    if info.get("shared_values"):
        # bitwise-equal rows stored once: the kept values once, one 8-byte
        # value offset per block row
        spmv = (info["shared_values"] * 8 + nnzb * col_bytes + (n // bd) * 8
                + (n // bd + 1) * 4 + 2 * n * 8)
    else:
        spmv = nnzb * (bd * bd * 8 + col_bytes) + (n // bd + 1) * 4 + 2 * n * 8
    # stored half of each symmetric P_B once ((m/2+1)*m wrapped diagonals),
    # element node lists, gathered r and q once, y_B written
    stored = distinct_blocks if distinct_blocks else n_blocks
    schwarz = stored * (m // 2 + 1) * m * 8 + n_blocks * nn * 4 + 2 * n * 8 + n_blocks * m * 8
    if distinct_blocks:
        schwarz += n_blocks * 8     # one 8-byte offset per block
    return spmv, schwarz


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(seconds=10.0):
    """The FP64 oracle's PCG on a bounded sample of the same workload family
    (4^3 cells of the same generator, seed 0), timed on the host."""
    import numpy as np
    import fcgen
    from oracle import assemble, pcg, schwarz
    d = fcgen.porous_elasticity_3d(seed=0, n=4)
    log("cpu baseline: oracle assembly of the 4^3-cell sample")
    s = assemble.assemble(d)
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], 1.0)
    S, _ = schwarz.compute_preconditioner(s["A"], blocks)
    n = s["A"].shape[0]
    t0 = time.perf_counter()
    total = 0
    runs = 0
    while True:
        _, info = pcg.pcg(s["A"], s["b"], S, tol=1e-8, stop="residual")
        total += info["iters"]
        runs += 1
        log(f"cpu baseline: oracle solve {runs} done ({info['iters']} iterations)")
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        blas = None
    return {
        "value": n * total / dt, "unit": "DOF·iter/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle PCG (scipy CSR products with A and with the assembled S) to "
                   f"1e-8 residual on the 4^3-cell instance of the same generator "
                   f"({n} DOFs, {info['iters']} iterations), {runs} solves in {dt:.1f} s; "
                   f"single-threaded sparse products (BLAS threads available: {blas}); "
                   f"the small instance is cache-resident, so this overstates the "
                   f"oracle's rate at full size"),
        "host_cpus": os.cpu_count(), "cpu_model": platform.processor() or platform.machine(),
    }


def forms(fc, pb, b, tol, t_f64, it_f64):
    """Time-to-tolerance of the mixed-precision forms against plain FP64 on
    the same problem: build (FP64 inverses plus the low-precision copy the
    form uses) + solve to ||b - A x|| / ||b|| <= tol."""
    import torch
    x64 = torch.zeros_like(b)
    res = {"fp64": {"time_to_tol_ms": t_f64, "iters": it_f64}}
    pc = fc.Precond(pb)
    fc.pcg_solve(pb, pc, b, x64, tol=tol, stop="residual")
    del pc
    for store, modes in ((fc.STORE_F64 | fc.STORE_F32, ("s_f32", "ir_f32")),
                         (fc.STORE_F64 | fc.STORE_BF16, ("s_bf16", "ir_bf16"))):
        for mode in modes:
            torch.cuda.synchronize()
            tb = time.perf_counter()
            pc = fc.Precond(pb, store=store)
            torch.cuda.synchronize()
            build = (time.perf_counter() - tb) * 1e3
            x = torch.zeros_like(b)
            # inner tolerance of the refinement: 1e-4 with the FP32 inverses
            # (two outer steps to 1e-8; 1e-2 takes four and 6 % more inner
            # iterations), 1e-2 with the weaker BF16 ones
            inner = 1e-4 if mode == "ir_f32" else 1e-2
            r = fc.pcg_solve(pb, pc, b, x, tol=tol, stop="residual", mode=mode, inner_tol=inner,
                             maxit=60000)
            diff = float((x - x64).norm() / x64.norm())
            res[mode] = {"time_to_tol_ms": build + r["ms_solve"], "solve_ms": r["ms_solve"],
                         "build_ms": build, "iters": r["iters"], "outer": r["outer_iters"],
                         "inner_tol": inner if mode.startswith("ir") else None,
                         "fallbacks": r["fallbacks"], "status": r["status"],
                         "rel_res_true": r["rel_res_true"], "rel_diff_vs_fp64": diff,
                         "speedup_vs_fp64": t_f64 / (build + r["ms_solve"])}
            if mode.endswith("f32"):
                info = pc.info()
                res[mode]["f32_blocks"] = info["n_f32_blocks"]
                res[mode]["f32_blocks_from_f64"] = info["n_f32_from_f64"]
            log(f"form {mode}: build {build:.0f} ms, {r['iters']} iterations, "
                f"{r['ms_solve']:.0f} ms, {r['status']}")
            del pc
    best = max((k for k in res if k != "fp64"), key=lambda k: res[k]["speedup_vs_fp64"])
    res["best"] = {"form": best, "speedup_vs_fp64": res[best]["speedup_vs_fp64"],
                   "time_to_tol_ms": res[best]["time_to_tol_ms"]}
    return res


COPY_BYTES = 4 << 30


def copy_calibration(torch):
    """Three device-to-device copies of COPY_BYTES by torch's elementwise copy
    kernel: it reads and writes exactly COPY_BYTES, so a byte counter's
    reading for it gives the factor from counter units to HBM bytes."""
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {COPY_BYTES} bytes")
    del a, b


def learned_bench(fc, args):
    """Learned coarse correction: a U-Net trained on solver-generated pairs
    from 48^3-cell, p=2 porous Poisson cubes, evaluated inside flexible CG
    on a 64^3-cell, p=2 cube (2.1M unknowns), against plain FP64 PCG, both
    to ||r||/||b|| <= 1e-8; then plain PCG judges whether the network is kept."""
    import torch
    import fcgen
    from paper_1809_00828_amd import learned as LR
    ch = (8, 16, 32, 32)
    m = args.learned_fcg_m
    t0 = time.perf_counter()
    descs = [fcgen.porous_poisson_3d(1000 + i, n=48, p=2) for i in range(args.learned_train)]
    xin, t, G = LR.training_set(descs, args.learned_pairs // args.learned_train,
                                kind=args.learned_target, log=log)
    t_data = time.perf_counter() - t0
    model = fc.Model(fcgen.unet_init(ch, 2, seed=0), ch)
    t0 = time.perf_counter()
    hist = LR.train(model, xin, t, G, epochs=args.learned_epochs, batch=8, lr=args.learned_lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"learned: {xin.shape[0]} pairs in {t_data:.0f} s, {args.learned_epochs} epochs in "
        f"{t_train:.0f} s, loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    del xin, t
    desc = fcgen.porous_poisson_3d(100, n=64, p=2)
    hs = fc.HostSystem(desc)
    pb = hs.upload()
    del hs
    pc = fc.Precond(pb)
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    runs = {}
    for name, mode in (("plain", "f64"), ("learned", "learned")):
        if mode == "learned":
            pc.attach(model)
        fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", mode=mode, fcg_m=m)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", mode=mode, fcg_m=m)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        runs[name] = {"iters": info["iters"], "time_to_tol_ms": wall,
                      "ms_per_iter": wall / max(1, info["iters"]), "status": info["status"],
                      "rel_res_true": info["rel_res_true"]}
        log(f"learned: {name} {info['iters']} iterations, {wall:.0f} ms")
    st = pc.learned_stats()
    use, ip, il = pc.validate(b, tol=args.tol, fcg_m=m)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", mode="learned", fcg_m=m)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    log(f"learned: validated solve ({'network kept' if use else 'plain fallback'}) "
        f"{info['iters']} iterations, {wall:.0f} ms")
    return {
        "workload": "3D finite cell Poisson, 64^3 cells, p=2, 64 spherical voids, alpha=1e-10 "
                    "(2.1M unknowns); network trained on 48^3-cell cubes",
        "n_dofs": pb.n, "coarse_grid": pc.coarse_grid(), "train_coarse_grid": G,
        "fcg_directions": m,
        "params": model.n_params,
        "train": {"problems": len(descs), "pairs": int(args.learned_pairs // args.learned_train)
                  * len(descs), "target": args.learned_target, "epochs": args.learned_epochs,
                  "lr": args.learned_lr,
                  "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                  "data_s": t_data, "train_s": t_train},
        "plain": runs["plain"], "learned": runs["learned"],
        "corrections": st,
        "speedup_vs_plain": runs["plain"]["time_to_tol_ms"] / runs["learned"]["time_to_tol_ms"],
        "iteration_ratio": runs["learned"]["iters"] / max(1, runs["plain"]["iters"]),
        "validated": {"network_kept": use, "iters": info["iters"], "time_to_tol_ms": wall,
                      "fallbacks": info["fallbacks"],
                      "speedup_vs_plain": runs["plain"]["time_to_tol_ms"] / wall},
    }


def _solve_record(fc, pb, pc, b, x, **kw):
    import torch
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = fc.pcg_solve(pb, pc, b, x, **kw)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    return {"iters": info["iters"], "status": info["status"], "solve_ms": wall,
            "ms_per_iter": wall / max(1, info["iters"]),
            "rel_res_true": info["rel_res_true"], "rel_res_prec": info["rel_res_prec"]}


def eta_sweep_bench(fc, args):
    """Blocks only for elements with eta_T <= eta_bar, diagonal scaling for
    the unknowns no block covers (the paper's study of the threshold):
    iterations, time and preconditioner size on the 32^3-cell, p = 3
    elasticity workload; eta_bar < 0 leaves only the diagonal scaling."""
    import torch
    import fcgen
    desc = fcgen.porous_elasticity_3d(seed=0)
    pb = fc.HostSystem(desc).upload()
    info = pb.info()
    m = info["m"]
    b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    rows = []
    for eb in args.eta_values:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = fc.Precond(pb, eta_bar=eb)
        torch.cuda.synchronize()
        build = (time.perf_counter() - t0) * 1e3
        pi = pc.info()
        rec = _solve_record(fc, pb, pc, b, x, tol=args.tol, maxit=args.maxit, stop="residual")
        rec.update({"eta_bar": eb, "blocks": pi["n_blocks"], "diag_unknowns": pi["n_fallback"],
                    "inverse_bytes": pi["n_blocks"] * (m // 2 + 1) * m * 8, "build_ms": build,
                    "time_to_tol_ms": build + rec["solve_ms"]})
        log(f"eta sweep: eta_bar {eb}: {pi['n_blocks']} blocks, {rec['iters']} iterations "
            f"{rec['status']}, {rec['solve_ms']:.0f} ms ({rec['ms_per_iter']:.3f} ms/iter)")
        rows.append(rec)
        del pc
    return {"metric": "time-to-1e-8 residual vs the block threshold eta_bar",
            "workload": "3D finite cell elasticity, 32^3 cells, p=3, 64 spherical voids, "
                        "alpha=1e-8 (2,738,019 unknowns)",
            "n_dofs": pb.n, "maxit": args.maxit, "sweep": rows}


def compare_bench(fc, args):
    """Preconditioners compared on the elasticity geometry at fictitious
    stiffnesses down to zero (the paper's CT examples use about 1e-12),
    optionally after removing the functions of cells without material:
    diagonal scaling (DA), Schwarz with plain local inverses (S*) and with
    the stabilised pseudo-inverses (S), stopped by the relative
    preconditioned residual ||z|| / ||z_0|| <= 1e-10 (Eq. 12) or at maxit."""
    import torch
    import fcgen
    rows = []
    n = 0
    for alpha in args.compare_alpha:
        desc = fcgen.porous_elasticity_3d(seed=0, alpha=alpha,
                                          discard_fictitious=args.discard_fictitious)
        pb = fc.HostSystem(desc).upload()
        n = pb.n
        b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        pb.rhs(b)
        x = torch.zeros_like(b)
        for name, kw in (("DA", {"eta_bar": -1.0}), ("S*", {"stabilize": False}), ("S", {})):
            pc = fc.Precond(pb, **kw)
            pi = pc.info()
            rec = _solve_record(fc, pb, pc, b, x, tol=1e-10, maxit=args.maxit, stop="precond")
            rec.update({"alpha": alpha, "preconditioner": name,
                        "discard_fictitious": bool(args.discard_fictitious),
                        "dropped_eigenvalues": pi["n_dropped"]})
            log(f"compare: alpha {alpha:g} {name}: {rec['iters']} iterations {rec['status']}, "
                f"||z||/||z0|| {rec['rel_res_prec']:.2e}, ||r||/||b|| {rec['rel_res_true']:.2e}, "
                f"{pi['n_dropped']} eigenvalues dropped")
            rows.append(rec)
            del pc
        del pb
    return {"metric": "PCG with DA, S* and S to ||z||/||z_0|| <= 1e-10",
            "workload": "3D finite cell elasticity, 32^3 cells, p=3, 64 spherical voids "
                        "(2,738,019 unknowns), fictitious stiffness alpha as listed",
            "n_dofs": n, "maxit": args.maxit, "runs": rows}


def batch_bench(fc, args):
    """Uneven batch of 2-D/3-D Poisson problems (grids 8^2..128^2 and
    8^3..24^3, p = 1..4, elliptical inclusions or voids, alpha = 1e-10,
    50k-200k DOFs each) solved together to ||r||/||b|| <= 1e-8."""
    import torch
    import fcgen
    descs = fcgen.batch_poisson(seed=0, count=args.batch)
    pbs, pcs = [], []
    t0 = time.perf_counter()
    for k, d in enumerate(descs):
        hs = fc.HostSystem(d)
        pbs.append(hs.upload())
        del hs
        pcs.append(fc.Precond(pbs[-1]))
        if k % 16 == 15 or k == len(descs) - 1:
            log(f"batch: {k + 1}/{len(descs)} problems assembled and preconditioned "
                f"({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    tb = time.perf_counter()
    batch = fc.Batch(pbs, pcs, autotune=True)
    t_tune = time.perf_counter() - tb
    info = batch.info()
    log("batch: autotuned\n" + info["report"])
    bs, xs = [], []
    for p in pbs:
        b = torch.empty(p.n, dtype=torch.float64, device="cuda")
        p.rhs(b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    # the library reports converged members every 64 chunks of 32 steps
    os.environ.setdefault("FC_BATCH_PROGRESS", "64")
    for _ in range(args.warmup):
        batch.solve(bs, xs, tol=args.tol, stop="residual", check_every=32)
        log("batch: warmup solve done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        res = batch.solve(bs, xs, tol=args.tol, stop="residual", check_every=32)
        log(f"batch: timed solve {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    dof_iters = sum(p.n * r["iters"] for p, r in zip(pbs, res))
    return {
        "metric": METRIC + " (batched form)", "value": dof_iters / wall, "unit": "DOF·iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(descs)} uneven 2D/3D finite cell Poisson problems, "
                               f"p=1..4, alpha=1e-10, one batch",
                   "total_dofs": info["total_dofs"], "tol": args.tol},
        "converged": sum(r["status"] == "OK" for r in res),
        "iters_min": min(r["iters"] for r in res), "iters_max": max(r["iters"] for r in res),
        "setup_s": t_setup, "batch_create_autotune_s": t_tune,
        "classes": {"spmv": info["spmv_classes"], "schwarz": info["schwarz_classes"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--small", action="store_true", help="8^3-cell check run")
    ap.add_argument("--workload", default="elastic32", choices=["elastic32", "poisson64"],
                    help="the FP64 PCG workload: 32^3-cell p=3 elasticity (the benchmark) or "
                         "64^3-cell p=2 Poisson (the learned form's problem)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision forms comparison")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned coarse-correction comparison")
    ap.add_argument("--learned-train", type=int, default=8, help="training problems (48^3)")
    ap.add_argument("--learned-pairs", type=int, default=2000, help="training pairs in total")
    ap.add_argument("--learned-epochs", type=int, default=20)
    ap.add_argument("--learned-lr", type=float, default=1e-3)
    ap.add_argument("--learned-target", default="coarse", choices=["coarse", "e-Sr", "e"],
                    help="training target: the coarse Galerkin projection of the error, the "
                         "error left by the Schwarz apply, or the error")
    ap.add_argument("--learned-fcg-m", type=int, default=64,
                    help="directions kept by the learned flexible CG")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 4 GiB three times with a plain copy kernel, the reference "
                         "for scaling hardware byte counters")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead: solve this many problems of the uneven batch "
                         "generator together (512 = the full batch)")
    ap.add_argument("--eta-sweep", action="store_true",
                    help="instead: sweep the block threshold eta_bar on the elasticity workload")
    ap.add_argument("--eta-values", type=float, nargs="+",
                    default=[1.0, 0.9, 0.8, 0.7, 0.6, 0.4, 0.2, 0.0, -1.0])
    ap.add_argument("--learned-only", action="store_true",
                    help="instead: only the learned coarse-correction comparison")
    ap.add_argument("--compare", action="store_true",
                    help="instead: DA, S* and S on the elasticity geometry at small alpha")
    ap.add_argument("--compare-alpha", type=float, nargs="+", default=[1e-12, 1e-16, 0.0])
    ap.add_argument("--discard-fictitious", action="store_true",
                    help="compare: first remove the functions of cells without material")
    ap.add_argument("--maxit", type=int, default=20000,
                    help="iteration cap of the sweep and comparison runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1809_00828_amd as fc

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
    if args.batch:
        print(json.dumps(batch_bench(fc, args)), flush=True)
        return
    if args.learned_only:
        print(json.dumps(learned_bench(fc, args)), flush=True)
        return
    if args.eta_sweep:
        print(json.dumps(eta_sweep_bench(fc, args)), flush=True)
        return
    if args.compare:
        print(json.dumps(compare_bench(fc, args)), flush=True)
        return
    desc, wl = workload(args.small, args.workload)
    t0 = time.perf_counter()
    hs = fc.HostSystem(desc)
    t_asm = time.perf_counter() - t0
    log(f"host assembly {t_asm:.1f} s")
    pb = hs.upload()
    del hs
    info = pb.info()
    n = info["n_dofs"]
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    pb.rhs(b)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()

    def step():
        tb = time.perf_counter()
        pc = fc.Precond(pb)
        torch.cuda.synchronize()
        build = time.perf_counter() - tb
        r = fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", check_every=16,
                         timing=True)
        pinfo = pc.info()
        del pc
        log(f"step: build {build * 1e3:.1f} ms, solve {r['ms_solve']:.1f} ms, "
            f"{r['iters']} iterations, {r['status']}")
        return build, r, pinfo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    iters = [r[1]["iters"] for r in res]
    status = [r[1]["status"] for r in res]
    builds = [r[0] * 1e3 for r in res]
    solves = [r[1]["ms_solve"] for r in res]
    pinfo = res[-1][2]
    m = info["m"]
    nn = m // info["bsr_dim"]
    dblk = pinfo.get("shared_distinct_blocks", 0)
    spmv_b, schw_b = algorithmic_bytes(info, m, pinfo["n_blocks"], nn, dblk)
    ms_spmv = sum(r[1]["ms_spmv"] for r in res) / max(1, sum(r[1]["n_timed"] for r in res))
    ms_schw = sum(r[1]["ms_schwarz"] for r in res) / max(1, sum(r[1]["n_timed"] for r in res))
    gbs_schw = schw_b / (ms_schw * 1e-3) / 1e9
    gbs_spmv = spmv_b / (ms_spmv * 1e-3) / 1e9
    total_dof_iters = n * sum(iters)
    # the counter traffic was taken on the elasticity workload
    on_bench_workload = not args.small and args.workload == "elastic32"
    shared = bool(info.get("shared_values"))
    grouped = bool(info.get("row_groups"))
    spmv_name = (f"k_spmv_bsr{'_grp' if grouped else ''}<{info['bsr_dim']},{info['spmv_group']},double,"
                 f"{'lattice' if info.get('lattice_columns') else 'columns'}"
                 f"{',shared' if shared else ''}> (SpMV q = A p)")
    k_spmv = {"bound": "hbm", "kernel": spmv_name,
              "achieved": gbs_spmv, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": gbs_spmv / HBM_PEAK_GBS,
              "traffic": (TRAFFIC["spmv_grouped" if grouped else
                                  "spmv_shared" if shared else "spmv"]
                          if on_bench_workload else None),
              "bytes_per_launch": spmv_b, "avg_ms": ms_spmv,
              # values the lanes load per launch when every row is counted
              # (repeats of shared rows come from the caches)
              "loaded_bytes_per_launch": algorithmic_bytes(
                  {**info, "shared_values": 0}, m, pinfo["n_blocks"], nn)[0]}
    bgrp = bool(pinfo.get("block_groups"))
    schw_name = (("k_schwarz_sym_grp<double,4>" if bgrp else
                  f"k_schwarz_sym_staged<double{',shared' if dblk else ''}>") if m > 64
                 else "k_schwarz_small<double,sym>")
    k_schw = {"bound": "hbm", "kernel": schw_name + " (block products)",
              "achieved": gbs_schw, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": gbs_schw / HBM_PEAK_GBS,
              "traffic": (TRAFFIC["schwarz_grouped" if bgrp else
                                  "schwarz_shared" if dblk else "schwarz"]
                          if on_bench_workload else None),
              "bytes_per_launch": schw_b, "avg_ms": ms_schw,
              "loaded_bytes_per_launch": algorithmic_bytes(info, m, pinfo["n_blocks"], nn)[1]}
    dominant, other = (k_spmv, k_schw) if ms_spmv >= ms_schw else (k_schw, k_spmv)
    out = {
        "metric": METRIC,
        "value": total_dof_iters / wall,
        "unit": "DOF·iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": wl, "n_dofs": n, "nnz_blocks": info["nnzb"],
                   "blocks": pinfo["n_blocks"], "block_size": m, "tol": args.tol,
                   "stop": "relative residual ||b-Ax||/||b||", "form": "fp64",
                   "shared_rows": info.get("shared_rows", 0),
                   "shared_values": info.get("shared_values", 0),
                   "row_groups": info.get("row_groups", 0),
                   "shared_distinct_blocks": dblk,
                   "block_groups": pinfo.get("block_groups", 0)},
        "roofline": dominant,
        "roofline_other": other,
        "iters": iters, "status": status,
        "time_to_tol_ms": [bd + sv for bd, sv in zip(builds, solves)],
        "build_ms": builds, "solve_ms": solves,
        "solve_dof_iter_per_s": n * iters[-1] / (solves[-1] * 1e-3),
        "ms_per_iter": solves[-1] / max(1, iters[-1]),
        "rel_res_true": res[-1][1]["rel_res_true"],
        "precond": pinfo, "host_assembly_s": t_asm,
    }
    if not args.no_forms:
        out["forms"] = forms(fc, pb, b, args.tol, out["time_to_tol_ms"][-1], iters[-1])
    if not args.no_learned and not args.small:
        out["learned"] = learned_bench(fc, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
