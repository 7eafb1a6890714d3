"""Benchmark: FP64 Schwarz-preconditioned CG on the 3-D finite cell
elasticity workload (32^3 cells, p = 3, 64 seeded spherical voids,
alpha = 1e-8, clamped bottom face, traction on the top face; 2,738,019
unknowns), solved to a relative residual of 1e-8 on one MI355X.

One step = one pass of the whole hot path: build the preconditioner
(extract the 32,768 element blocks, their FP64 local inverses, the
diagonal fallback) and run PCG to ||b - A x|| / ||b|| <= 1e-8.  The
problem (assembled matrix and load) is resident in HBM before the timed
region starts.  Every block row and every local inverse is read from its
own stored copy.  The timed steps run the production launch mode (each
chunk of PCG steps replayed from a captured hipGraph).

Prints one JSON line.  The kernel-level roofline comes from one more solve
after the timed steps, in the library's timing mode: the same kernels with
the same launch shapes, launched directly with HIP events around every SpMV
and every Schwarz block-product launch on the solver's own stream.
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
# read for a plain 4 GiB copy (profiles/pcg_fp64_elastic32_p3_hbm_counters.md);
# to be re-measured whenever one of these kernels changes.
TRAFFIC = {"spmv": 8.5163e9, "schwarz": 4.9990e9}
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


def algorithmic_bytes(info, m, n_blocks, nn):
    """Bytes each streaming kernel must move per launch in the implemented
    FP64 layout: the matrix once (values, plus 4-byte block columns unless
    the columns follow from the lattice), row pointers, x and y once; the
    stored half of every symmetric local inverse once ((m/2+1)*m wrapped
    diagonals), the element node lists, the gathered r and q once and the
    block outputs y_B written."""
    n = info["n_dofs"]
    bd = info["bsr_dim"]
    nnzb = info["nnzb"]
    col_bytes = 0 if info.get("lattice_columns") else 4
    spmv = nnzb * (bd * bd * 8 + col_bytes) + (n // bd + 1) * 4 + 2 * n * 8
    schwarz = n_blocks * (m // 2 + 1) * m * 8 + n_blocks * nn * 4 + 2 * n * 8 + n_blocks * m * 8
    return spmv, schwarz


def iteration_bytes(info, m, n_blocks, nn):
    """Bytes of one whole PCG iteration: both streaming kernels, plus the
    vector passes of the CG updates (p and q read for (p, A p); the pull
    reads y_B, the inverse map, x, r, p, q and writes x, r, z; p = z + beta p
    reads z, p and writes p)."""
    spmv, schwarz = algorithmic_bytes(info, m, n_blocks, nn)
    n = info["n_dofs"]
    n_entries = n_blocks * nn
    pull = n_blocks * m * 8 + n_entries * 4 + (n // info["bsr_dim"] + 1) * 4 + 7 * n * 8
    return spmv + schwarz + 2 * n * 8 + pull + 3 * n * 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(full_desc, gpu_iters, cpu_iters=50):
    """The FP64 oracle timed on the host, in two parts.

    Full size (the reported value): cpu_iters oracle PCG iterations on the
    benchmark problem itself, with the element-by-element forms of A and S
    (oracle/ebe.py; a sparse S of the 32^3-cell problem would not be
    smaller).  The element matrices are the oracle's own for the cells of a
    4^3-cell instance of the same generator, placed cyclically on the full
    lattice: the cost of an iteration depends on the sizes, not on the
    values.  One BLAS thread (the stacked element products and scipy's
    vector operations are single-threaded either way).  The time to
    tolerance is that time per iteration times the GPU's iteration count,
    labelled extrapolated.

    Sample: the 4^3-cell instance solved to 1e-8 with the assembled oracle
    (assembly once, then Algorithm 1 and PCG with every BLAS thread and with
    one), with the assembly, preconditioner and solve times apart."""
    import numpy as np
    import fcgen
    from oracle import assemble, ebe, pcg, schwarz
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except Exception:  # noqa: BLE001
        threadpool_info = threadpool_limits = None
    blas = (max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
            if threadpool_info else None)
    if full_desc["pde"] == "elasticity":
        d = fcgen.porous_elasticity_3d(seed=0, n=4, p=full_desc["p"])
    else:
        d = fcgen.porous_poisson_3d(seed=0, n=4, p=full_desc["p"])
    log("cpu baseline: oracle assembly of the 4^3-cell sample")
    t0 = time.perf_counter()
    s = assemble.assemble(d, keep_elements=True)
    t_asm = time.perf_counter() - t0
    A, b = s["A"], s["b"]
    n = A.shape[0]
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], 1.0)
    runs = {}
    for label, limit in (("all_threads", None), ("one_thread", 1)):
        ctx = threadpool_limits(limits=limit) if (threadpool_limits and limit) else None
        if ctx is not None:
            ctx.__enter__()
        try:
            t0 = time.perf_counter()
            S, _ = schwarz.compute_preconditioner(A, blocks)
            t_pre = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, info = pcg.pcg(A, b, S, tol=1e-8, stop="residual")
            t_sol = time.perf_counter() - t0
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)
        runs[label] = {"blas_threads": limit or blas, "precond_s": t_pre, "solve_s": t_sol,
                       "iters": info["iters"], "ms_per_iter": t_sol / max(1, info["iters"]) * 1e3,
                       "dof_iter_per_s": n * info["iters"] / t_sol}
        log(f"cpu baseline ({label}): precond {t_pre:.2f} s, solve {t_sol:.2f} s, "
            f"{info['iters']} iterations")
    # full size, element by element
    log("cpu baseline: element-by-element operators of the full problem")
    t0 = time.perf_counter()
    cells = list(assemble.cells(full_desc))
    dofs = np.array([assemble.element_dofs(full_desc, c) for c in cells])
    n_full = assemble.n_dofs(full_desc)
    Pb = np.array([schwarz.pseudo_inverse(schwarz.extract_submatrix(A, B)) for B in blocks])
    pick = np.arange(len(cells)) % len(s["cells"])
    Aop = ebe.ElementOperator(dofs, s["Ke"][pick], n_full,
                              clamped=assemble.clamped_dofs(full_desc))
    Sop = ebe.ElementOperator(dofs, Pb[pick], n_full)
    t_build = time.perf_counter() - t0
    rhs = np.random.default_rng(0).standard_normal(n_full)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    if ctx is not None:
        ctx.__enter__()
    try:
        t0 = time.perf_counter()
        _, finfo = pcg.pcg(Aop, rhs, Sop, tol=0.0, maxit=cpu_iters, stop="residual")
        t_it = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    its = max(1, finfo["iters"])
    per_iter = t_it / its
    log(f"cpu baseline (full size): {its} iterations in {t_it:.1f} s "
        f"({per_iter * 1e3:.0f} ms per iteration)")
    gib = (Aop.mats.nbytes + Sop.mats.nbytes) / 2**30
    del Aop, Sop
    return {
        "value": n_full / per_iter, "unit": "DOF·iter/s", "cores": 1, "kind": "oracle",
        "sample": (f"{its} oracle PCG iterations (python/numpy/scipy, FP64, one thread) on the "
                   f"full problem ({n_full} DOFs, {len(cells)} cells) with element-by-element "
                   f"A and S ({gib:.1f} GiB of element matrices, those of the 4^3-cell "
                   f"instance's cells placed cyclically)"),
        "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "blas_threads": blas,
        "full": {"iters": its, "seconds": t_it, "ms_per_iter": per_iter * 1e3,
                 "build_s": t_build, "status": finfo["status"]},
        "extrapolated_full": {
            "label": "extrapolated",
            "time_to_tol_s": per_iter * gpu_iters,
            "how": f"{per_iter * 1e3:.0f} ms per full-size iteration x {gpu_iters} iterations "
                   f"(the GPU's count)"},
        "sample_4cube": {"n_dofs": n, "assembly_s": t_asm, "runs": runs},
    }


def _energy(fc, pb, v, work):
    """sqrt(v . A v) with the library's FP64 product."""
    pb.apply_A(v, work)
    return float(max((v * work).sum().item(), 0.0)) ** 0.5


def forms(fc, pb, b, tol, t_f64, it_f64):
    """Time-to-tolerance of the mixed-precision forms against plain FP64 on
    the same problem: build (FP64 inverses plus the low-precision copy the
    form uses) + solve to ||b - A x|| / ||b|| <= tol.  Each result's error
    is stated in the energy norm (Eq. 13) against an FP64 reference solved
    to ||b - A x|| / ||b|| <= 1e-12 (at this size the oracle's own solve
    would take hours; its parity with the oracle is checked at smaller
    sizes), for the plain FP64 result too."""
    import torch
    x64 = torch.zeros_like(b)
    xref = torch.zeros_like(b)
    work = torch.empty_like(b)
    pc = fc.Precond(pb)
    fc.pcg_solve(pb, pc, b, x64, tol=tol, stop="residual")
    ref = fc.pcg_solve(pb, pc, b, xref, tol=1e-12, stop="residual")
    del pc
    eref = _energy(fc, pb, xref, work)
    e64 = _energy(fc, pb, x64 - xref, work) / eref
    res = {"fp64": {"time_to_tol_ms": t_f64, "iters": it_f64, "energy_error_vs_ref": e64},
           "reference": {"tol": 1e-12, "iters": ref["iters"], "status": ref["status"],
                         "rel_res_true": ref["rel_res_true"]}}
    log(f"forms: FP64 reference to 1e-12 in {ref['iters']} iterations; FP64 energy error "
        f"{e64:.2e}")
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
            # (two outer steps to 1e-8), 1e-2 with the weaker BF16 ones
            inner = 1e-4 if mode == "ir_f32" else 1e-2
            r = fc.pcg_solve(pb, pc, b, x, tol=tol, stop="residual", mode=mode, inner_tol=inner,
                             maxit=60000)
            diff = float((x - x64).norm() / x64.norm())
            err = _energy(fc, pb, x - xref, work) / eref
            res[mode] = {"time_to_tol_ms": build + r["ms_solve"], "solve_ms": r["ms_solve"],
                         "build_ms": build, "iters": r["iters"], "outer": r["outer_iters"],
                         "inner_tol": inner if mode.startswith("ir") else None,
                         "fallbacks": r["fallbacks"], "status": r["status"],
                         "rel_res_true": r["rel_res_true"], "rel_diff_vs_fp64": diff,
                         "energy_error_vs_ref": err,
                         "iteration_overhead": r["iters"] / max(1, it_f64),
                         "speedup_vs_fp64": t_f64 / (build + r["ms_solve"])}
            if mode.endswith("f32"):
                info = pc.info()
                res[mode]["f32_blocks"] = info["n_f32_blocks"]
                res[mode]["f32_blocks_from_f64"] = info["n_f32_from_f64"]
            log(f"form {mode}: build {build:.0f} ms, {r['iters']} iterations, "
                f"{r['ms_solve']:.0f} ms, {r['status']}, energy error {err:.2e}")
            del pc
    best = max((k for k in res if k not in ("fp64", "reference")),
               key=lambda k: res[k]["speedup_vs_fp64"])
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


def net_timing(fc, reps=200):
    """Network kernels alone: the forward pass the solver runs per iteration
    (batch 1 on the 33^3 coarse grid of the 64^3-cell problem) and one
    training step's loss and gradient (batch 8 on the 25^3 coarse grid of
    the 48^3-cell training problems), widths (8, 16, 32, 32), random
    weights.  Mean wall time per call over reps calls after a warm-up."""
    import torch
    import fcgen
    ch = (8, 16, 32, 32)
    model = fc.Model(fcgen.unet_init(ch, 2, seed=1), ch)
    gen = torch.Generator(device="cuda").manual_seed(5)
    out = {"widths": list(ch)}
    for key, B, g in (("forward_b1_33", 1, 33), ("train_b8_25", 8, 25)):
        x = torch.randn((B, 2, g, g, g), device="cuda", generator=gen)
        y = torch.empty((B, 1, g, g, g), device="cuda")
        t = torch.randn((B, 1, g, g, g), device="cuda", generator=gen)
        n = reps if key.startswith("forward") else reps // 4

        def call():
            if key.startswith("forward"):
                model.forward(x, y)
            else:
                model.loss_grad(x, t)
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            call()
        torch.cuda.synchronize()
        out[key + "_ms"] = (time.perf_counter() - t0) / n * 1e3
    return out


def learned_bench(fc, args):
    """Learned coarse correction: a U-Net trained on solver-generated pairs
    from 48^3-cell, p=2 porous Poisson cubes, evaluated inside flexible CG
    on a 64^3-cell, p=2 cube (2.1M unknowns), against plain FP64 PCG, both
    to ||r||/||b|| <= 1e-8; then plain PCG judges whether the network is kept."""
    import torch
    import fcgen
    from paper_1809_00828_amd import learned as LR
    ch = (8, 16, 32, 32)
    ms = args.learned_fcg_m
    m = ms[0]
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
    sweep = []
    for mm in ms[1:]:
        fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", mode="learned", fcg_m=mm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", mode="learned", fcg_m=mm)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        sweep.append({"fcg_directions": mm, "iters": info["iters"], "time_to_tol_ms": wall,
                      "ms_per_iter": wall / max(1, info["iters"]), "status": info["status"]})
        log(f"learned: FCG({mm}) {info['iters']} iterations, {wall:.0f} ms")
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
        "fcg_sweep": sweep,
        "network": net_timing(fc),
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


def small_bench(fc, seeds=range(10), reps=5):
    """Config 1 (2-D disk Poisson, 16^2 cells, p = 2, about 1k unknowns) with
    vertex-patch and element blocks, and config 3 (its precision forms), to
    ||b - Ax|| / ||b|| <= 1e-10: latency-bound, so the record is microseconds
    per iteration, from hipGraph-captured chunks and from direct launches
    (the timing mode, with events), medians over the seeds."""
    import statistics
    import torch
    import fcgen
    rows = {}
    for seed in seeds:
        d = fcgen.disk_poisson_2d(seed)
        pb = fc.Problem.setup(d)
        b = torch.empty(pb.n, dtype=torch.float64, device="cuda")
        pb.rhs(b)
        x = torch.zeros_like(b)
        runs = [("vertex_patch", "f64", False), ("vertex_patch", "f64", True),
                ("element", "f64", False), ("element", "f64", True),
                ("element", "ir_f32", False), ("element", "s_f32", False)]
        pcs = {}
        for kind, mode, timing in runs:
            if kind not in pcs:
                pcs[kind] = fc.Precond(pb, block_kind=kind,
                                       store=fc.STORE_F64 | fc.STORE_F32 if kind == "element"
                                       else fc.STORE_F64)
            pc = pcs[kind]
            best = None
            for _ in range(reps + 1):
                x.zero_()
                info = fc.pcg_solve(pb, pc, b, x, tol=1e-10, stop="residual", mode=mode,
                                    timing=timing)
                us = info["ms_solve"] * 1e3 / max(1, info["iters"])
                if best is None or us < best[0]:
                    best = (us, info["iters"], info["status"])
            key = f"{kind}/{mode}/{'direct' if timing else 'graph'}"
            rows.setdefault(key, []).append(best)
        del pcs, pb
    out = {"workload": "2D finite cell Poisson, disk r=0.37 on 16^2 cells, p=2, alpha=1e-10 "
                       "(1,089 unknowns), seeds 0-9, tol 1e-10",
           "runs": {}}
    for key, v in rows.items():
        out["runs"][key] = {"us_per_iter_median": statistics.median(r[0] for r in v),
                            "iters_median": statistics.median(r[1] for r in v),
                            "all_ok": all(r[2] == "OK" for r in v)}
    return out


def eta_pair(fc, pb, b, args, t_f64, it_f64):
    """The paper's study of preconditioning only cut cells, at one point:
    blocks only for elements with eta_T <= 0.8 and diagonal scaling for
    every unknown they leave uncovered, against blocks for every element
    (the timed steps), both to ||b - A x|| / ||b|| <= tol; the time counts
    the preconditioner build."""
    import torch
    x = torch.zeros_like(b)
    rec = {}
    for eb in (0.8,):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc = fc.Precond(pb, eta_bar=eb)
        torch.cuda.synchronize()
        build = (time.perf_counter() - t0) * 1e3
        pi = pc.info()
        r = _solve_record(fc, pb, pc, b, x, tol=args.tol, maxit=args.maxit, stop="residual")
        rec = {"eta_bar": eb, "blocks": pi["n_blocks"], "diag_unknowns": pi["n_fallback"],
               "iters": r["iters"], "status": r["status"], "build_ms": build,
               "solve_ms": r["solve_ms"], "time_to_tol_ms": build + r["solve_ms"],
               "ms_per_iter": r["ms_per_iter"]}
        del pc
        log(f"eta_bar {eb}: {pi['n_blocks']} blocks, {r['iters']} iterations, "
            f"{build + r['solve_ms']:.0f} ms to tol")
    return {"all_blocks": {"eta_bar": 1.0, "iters": it_f64, "time_to_tol_ms": t_f64},
            "threshold": rec, "speedup": t_f64 / rec["time_to_tol_ms"]}


def compare_bench(fc, args, alphas=None, maxit=None):
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
    maxit = maxit or args.maxit
    for alpha in (alphas if alphas is not None else args.compare_alpha):
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
            rec = _solve_record(fc, pb, pc, b, x, tol=1e-10, maxit=maxit, stop="precond")
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
            "n_dofs": n, "maxit": maxit, "runs": rows}


def batch_bench(fc, args, count=None, line=True):
    """Uneven batch of 2-D/3-D Poisson problems (grids 8^2..128^2 and
    8^3..24^3, p = 1..4, elliptical inclusions or voids, alpha = 1e-10,
    50k-200k DOFs each) solved together to ||r||/||b|| <= 1e-8."""
    import torch
    import fcgen
    count = count or args.batch
    descs = fcgen.batch_poisson(seed=0, count=count)
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
    steps, warmup = (args.steps, args.warmup) if line else (1, 1)
    for _ in range(warmup):
        batch.solve(bs, xs, tol=args.tol, stop="residual", check_every=32)
        log("batch: warmup solve done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        res = batch.solve(bs, xs, tol=args.tol, stop="residual", check_every=32)
        log(f"batch: timed solve {k + 1}/{steps} done")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    dof_iters = sum(p.n * r["iters"] for p, r in zip(pbs, res))
    # HBM fraction against the summed algorithmic bytes: every member's
    # iterations times the bytes of one of its iterations (the batch reads
    # its block columns; symmetric storage of the local inverses)
    moved = 0
    for p, c, r in zip(pbs, pcs, res):
        inf = dict(p.info(), lattice_columns=False)
        moved += r["iters"] * iteration_bytes(inf, c.m, c.info()["n_blocks"],
                                              c.m // inf["bsr_dim"])
    gbs = moved / wall / 1e9
    return {
        "metric": METRIC + " (batched form)", "value": dof_iters / wall, "unit": "DOF·iter/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(descs)} uneven 2D/3D finite cell Poisson problems, "
                               f"p=1..4, alpha=1e-10, one batch",
                   "total_dofs": info["total_dofs"], "tol": args.tol},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "bytes_per_solve": moved,
                     "basis": "sum over members of iterations x bytes of one PCG iteration "
                              "(matrix with block columns, symmetric local inverses, vectors)"},
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
    ap.add_argument("--cpu-iters", type=int, default=50,
                    help="full-size oracle PCG iterations of the CPU baseline")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the mixed-precision forms comparison")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned coarse-correction comparison")
    ap.add_argument("--small-configs", action="store_true",
                    help="only the 2-D disk (configs 1 and 3) microseconds-per-iteration record")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the block-threshold, DA/S*/S and 32-member batch extras")
    ap.add_argument("--learned-train", type=int, default=8, help="training problems (48^3)")
    ap.add_argument("--learned-pairs", type=int, default=2000, help="training pairs in total")
    ap.add_argument("--learned-epochs", type=int, default=20)
    ap.add_argument("--learned-lr", type=float, default=1e-3)
    ap.add_argument("--learned-target", default="coarse", choices=["coarse", "e-Sr", "e"],
                    help="training target: the coarse Galerkin projection of the error, the "
                         "error left by the Schwarz apply, or the error")
    ap.add_argument("--learned-fcg-m", type=int, nargs="+", default=[32],
                    help="directions kept by the learned flexible CG (the first is the "
                         "reported run; further values are solved too)")
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
    ap.add_argument("--net-only", action="store_true",
                    help="instead: only the network kernels (forward and training step)")
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
    if args.net_only:
        print(json.dumps(net_timing(fc)), flush=True)
        return
    if args.small_configs:
        print(json.dumps(small_bench(fc)), flush=True)
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

    def step(timing=0):
        tb = time.perf_counter()
        pc = fc.Precond(pb)
        torch.cuda.synchronize()
        build = time.perf_counter() - tb
        r = fc.pcg_solve(pb, pc, b, x, tol=args.tol, stop="residual", check_every=16,
                         timing=timing)
        pinfo = pc.info()
        del pc
        log(f"step{' (kernel timing)' if timing else ''}: build {build * 1e3:.1f} ms, "
            f"solve {r['ms_solve']:.1f} ms, {r['iters']} iterations, {r['status']}")
        return build, r, pinfo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel durations: one more solve with events around every SpMV
    # and block-product launch (direct launches, same kernels and shapes)
    kt = step(timing=1)[1]

    iters = [r[1]["iters"] for r in res]
    status = [r[1]["status"] for r in res]
    builds = [r[0] * 1e3 for r in res]
    solves = [r[1]["ms_solve"] for r in res]
    pinfo = res[-1][2]
    m = info["m"]
    nn = m // info["bsr_dim"]
    spmv_b, schw_b = algorithmic_bytes(info, m, pinfo["n_blocks"], nn)
    it_b = iteration_bytes(info, m, pinfo["n_blocks"], nn)
    ms_spmv = kt["ms_spmv"] / max(1, kt["n_timed"])
    ms_schw = kt["ms_schwarz"] / max(1, kt["n_timed"])
    gbs_schw = schw_b / (ms_schw * 1e-3) / 1e9
    gbs_spmv = spmv_b / (ms_spmv * 1e-3) / 1e9
    total_dof_iters = n * sum(iters)
    # the counter traffic was taken on the elasticity workload
    on_bench_workload = not args.small and args.workload == "elastic32"
    if info.get("sliced"):
        spmv_name = ("k_spmv_sell (SpMV q = A p: sliced scalar rows, then the boundary vertex "
                     "rows with k_spmv_bsr)")
    else:
        spmv_name = (f"k_spmv_bsr<{info['bsr_dim']},{info['spmv_group']},double,"
                     f"{'lattice' if info.get('lattice_columns') else 'columns'}> (SpMV q = A p)")
    k_spmv = {"bound": "hbm", "kernel": spmv_name,
              "achieved": gbs_spmv, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": gbs_spmv / HBM_PEAK_GBS,
              "traffic": TRAFFIC["spmv"] if on_bench_workload else None,
              "bytes_per_launch": spmv_b, "avg_ms": ms_spmv, "launches_timed": kt["n_timed"]}
    if info.get("lattice_columns"):
        # the same product with the 4-byte block columns read from memory
        k_spmv["bytes_per_launch_with_columns"] = spmv_b + info["nnzb"] * 4
    schw_name = ("k_schwarz_sym_staged<double,%s>" % ("true" if m > 128 else "false")
                 if m > 64 else "k_schwarz_small<double,sym>")
    k_schw = {"bound": "hbm", "kernel": schw_name + " (block products)",
              "achieved": gbs_schw, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": gbs_schw / HBM_PEAK_GBS,
              "traffic": TRAFFIC["schwarz"] if on_bench_workload else None,
              "bytes_per_launch": schw_b, "avg_ms": ms_schw, "launches_timed": kt["n_timed"]}
    dominant, other = (k_spmv, k_schw) if ms_spmv >= ms_schw else (k_schw, k_spmv)
    ms_iter = sum(solves) / max(1, sum(iters))
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
                   "launch": "hipGraph-captured chunks of 16 PCG steps",
                   "spmv_lanes_per_row": info["spmv_group"]},
        "roofline": dominant,
        "roofline_other": other,
        "iteration_roofline": {
            "bytes_per_iter": it_b, "ms_per_iter": ms_iter,
            "achieved": it_b / (ms_iter * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": it_b / (ms_iter * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "iters": iters, "status": status,
        "time_to_tol_ms": [bd + sv for bd, sv in zip(builds, solves)],
        "build_ms": builds, "solve_ms": solves,
        "solve_dof_iter_per_s": n * sum(iters) / (sum(solves) * 1e-3),
        "ms_per_iter": ms_iter,
        "kernel_timing_solve": {"iters": kt["iters"], "ms_solve": kt["ms_solve"],
                                "ms_per_iter": kt["ms_solve"] / max(1, kt["iters"])},
        "rel_res_true": res[-1][1]["rel_res_true"],
        "precond": pinfo, "host_assembly_s": t_asm,
    }
    on_full = not args.small and args.workload == "elastic32"
    if not args.no_forms:
        out["forms"] = forms(fc, pb, b, args.tol, out["time_to_tol_ms"][-1], iters[-1])
    if not args.no_extras and on_full:
        out["eta_bar"] = eta_pair(fc, pb, b, args, out["time_to_tol_ms"][-1], iters[-1])
        del pb
        out["compare"] = compare_bench(fc, args, alphas=[0.0], maxit=1500)
        out["batch"] = batch_bench(fc, args, count=32, line=False)
        out["small"] = small_bench(fc)
    if not args.no_learned and not args.small:
        out["learned"] = learned_bench(fc, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc, iters[-1], args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
