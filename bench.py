#!/usr/bin/env python
"""Benchmark of the hot path on one MI355X.

Headline workload (C2): H(grad) Q_7 on a uniform 32^3 hexahedral mesh of the unit
cube (225^3 = 11,390,625 lattice DoFs), cellwise-constant alpha, beta log-uniform
in [1e-2, 1e2) (SplitMix64 seeds 1, 2), U[-1,1) right-hand side (seed 0),
homogeneous Dirichlet boundary.

One step = one PCG solve from x = 0 to a true relative residual of 1e-8 with the
p-multigrid V(1,1) preconditioner (statically condensed vertex-star relaxation
with IC patch factors, p=1 coarse solve), all vectors resident in HBM; setup is
done once before the timed region and reported separately.  The timed solves run
without per-kernel events; a second pass of the same solves with the events on
gives the per-kernel breakdown and the launch times of the rooflines.

Printed: one JSON line with the FP64 solve throughput as `value`, the mixed and
defect-correction protocols, the operator applies with their rooflines, the
workloads C1 (Q_4 on 4^3), C3 (NCE_6 on 16^3, solved), C5 (Q_8 on a perturbed
24^3 mesh) and the batched workload (64 problems of all three spaces), and the
CPU oracle timed on a bounded sample with the errors of GPU solutions against it.

`--only NAME` runs one piece alone (for profiling): c2, c2-apply, c3, c3-apply,
c5-apply.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
# HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0; factors from a plain 1 GiB copy in the same run), valid for the kernel
# version they were taken on (profiles/pmc_patch_solve_hgrad_q7_n32.md)
# HBM traffic per launch from FETCH_SIZE / WRITE_SIZE (calibrated against a plain copy), at
# the standard sizes only: C2 (Q_7, 32^3) and C3 (NCE_6, 16^3); apply = both of its kernels
MEASURED_TRAFFIC = {"patch": 2.281e9, "apply_c2_f64": 341.8e6, "apply_c2_f32": 179.0e6,
                    "apply_c3_f64": 156.6e6, "apply_c3_f32": 107.7e6}
METRIC = "GDoF/s sum-factorized apply; PCG time-to-1e-8, FP64 vs mixed, H(grad) p=7"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(n, p):
    import synth
    nc = n ** 3
    alpha = synth.cell_coefficients(nc, 1)
    beta = synth.cell_coefficients(nc, 2)
    ndofs = (n * p + 1) ** 3
    b = synth.rhs_values(ndofs, 0)
    return alpha, beta, b


def time_solves(torch, pb, bt, x, steps, warmup):
    """Wall time per solve over `steps` solves with the per-kernel events off; then
    the same number of solves with them on, for the per-kernel breakdown only."""
    for _ in range(warmup):
        pb.solve(bt, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [pb.solve(bt, x) for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pb.timing(True)
    pb.timing_read()
    for _ in range(steps):
        pb.solve(bt, x)
    kt = pb.timing_read()
    pb.timing(False)
    return (t1 - t0) * 1e3 / steps, infos, kt


def time_graph(torch, pb, bt, x, steps, warmup=2):
    """Wall time per solve with the CG iterations run from captured HIP graphs
    (captured during the warm-up solves), and the capture/replay counts."""
    pb.set_graph(True)
    for _ in range(warmup):
        pb.solve(bt, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [pb.solve(bt, x) for _ in range(steps)]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stats = pb.graph_stats()
    pb.set_graph(False)
    return ms, infos, {"captures": stats[0], "iterations_replayed": stats[1], "segments": stats[2]}


def time_apply(torch, pb, dtype_t, code, reps=50, warm=10):
    """Median device time (ms) of one apply, HIP events on the library's stream."""
    x = torch.rand(pb.ndofs, dtype=dtype_t, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(warm):
        pb.apply(x, y, code)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record(s)
        pb.apply(x, y, code)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def hbm_roof(bytes_, ms, kernel, note):
    ach = bytes_ / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": kernel, "avg_launch_ms": round(ms, 4),
            "algorithmic_bytes_per_launch": int(bytes_), "bytes": note}


def alu_roof(flops, ms, peak, kernel, note):
    ach = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "kernel": kernel, "avg_launch_ms": round(ms, 4),
            "algorithmic_flops_per_launch": int(flops), "flops": note}


# ---------------------------------------------------------------------------------------
def bench_c2(torch, rz, ctx, args, out):
    alpha, beta, b = workload(args.n, args.p)
    log(f"C2 setup FP64 n={args.n} p={args.p}")
    t0 = time.perf_counter()
    pb = rz.Problem(ctx, args.n, args.p, alpha, beta, precision=rz.PREC_F64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup done in {setup_s:.2f} s; timing {args.steps} FP64 solves")
    bt = torch.as_tensor(b, device="cuda:0")
    x = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    ms, infos, kt = time_solves(torch, pb, bt, x, args.steps, args.warmup)
    log("FP64 solves from captured HIP graphs")
    mg, ig, gs = time_graph(torch, pb, bt, x, args.steps)
    st = pb.stats()
    nd = pb.ndofs
    # the patch solve, the dominant kernel: its own bytes per launch as the scope
    # table states them (two sweeps over the factor of every non-empty patch, the
    # patch vectors in and out), and the single-read minimum beside them
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    two_sweeps = (2 * st["factor_nnz"] + 2 * st["patch_rows"]) * 8
    one_read = (st["factor_nnz"] + 2 * st["patch_rows"]) * 8
    roof = hbm_roof(two_sweeps, per_launch["patch"], "patch",
                    "2 sweeps x factor nnz of all non-empty vertex patches + patch vectors in/out, FP64")
    roof["frac_single_read"] = round(one_read / (per_launch["patch"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    roof["bytes_single_read"] = int(one_read)
    roof["traffic"] = MEASURED_TRAFFIC["patch"] if (args.p == 7 and args.n == 32) else None
    dom = max(kt, key=lambda k: kt[k][0])
    log(f"FP64 solve {ms:.3f} ms, {infos[-1].iters} iterations; timing the apply")
    a64 = time_apply(torch, pb, torch.float64, rz.F64)
    a32 = time_apply(torch, pb, torch.float32, rz.F32)
    nc = pb.ncells
    bf = bf16_apply_report(torch, rz, pb, 0, "k_apply_pencil+k_apply_faces (BF16 vectors)")
    bf.pop("roofline")
    bf["roofline"] = hbm_roof(2 * nd * 2 + 6 * nc * 4, bf["apply_ms"], "k_apply_pencil+k_apply_faces",
                              "x in, y out (BF16), 6 FP32 weights per cell")
    out.update({
        "value": round(nd / (ms * 1e-3) / 1e9, 5), "ms_per_step": round(ms, 4),
        "config": {"workload": f"C2: H(grad) Q_{args.p} on {args.n}^3 uniform hex mesh, cellwise log-uniform "
                               f"alpha,beta in [1e-2,1e2), U[-1,1) RHS; PCG to true rel. residual 1e-8",
                   "ndofs": nd, "nfree": pb.nfree, "cells": nc, "p": args.p},
        "pcg_ms_f64": round(ms, 4), "iters_f64": infos[-1].iters, "rel_res_f64": max(i.rel_res for i in infos),
        "iters_natural_f64": infos[-1].iters_natural,
        "pcg_ms_f64_graph": round(mg, 4), "iters_f64_graph": ig[-1].iters, "graph": gs,
        "setup_s_f64": round(setup_s, 3), "omega": pb.omega(),
        "apply_ms_f64": round(a64, 4), "apply_ms_f32": round(a32, 4), "apply_bf16": bf,
        "apply_gdofs_f64": round(nd / (a64 * 1e-3) / 1e9, 2), "apply_gdofs_f32": round(nd / (a32 * 1e-3) / 1e9, 2),
        "kernel_ms_per_step_f64": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "kernel_launches_per_step_f64": {k: v[1] / args.steps for k, v in kt.items()},
        "dominant_kernel": dom,
        "roofline": roof,
    })
    out["rooflines"] = {
        "patch_f64": roof,
        "apply_c2_f64": hbm_roof(2 * nd * 8 + 6 * nc * 8, a64, "k_apply_pencil+k_apply_faces",
                                 "x in, y out, 6 weights per cell (FP64)"),
        "apply_c2_f32": hbm_roof(2 * nd * 4 + 6 * nc * 4, a32, "k_apply_pencil+k_apply_faces",
                                 "x in, y out, 6 weights per cell (FP32)"),
    }
    std = args.p == 7 and args.n == 32
    out["rooflines"]["apply_c2_f64"]["traffic"] = MEASURED_TRAFFIC["apply_c2_f64"] if std else None
    out["rooflines"]["apply_c2_f32"]["traffic"] = MEASURED_TRAFFIC["apply_c2_f32"] if std else None
    if args.nrhs > 1:
        out["multi_rhs_f64"] = bench_multi_rhs(torch, rz, pb, args.nrhs, per_launch["patch"], ms, infos[-1].iters)
    pb.close()
    if not args.no_mixed:
        for prec, name in ((rz.PREC_MIXED, "mixed"), (rz.PREC_DEFECT, "defect")):
            log(f"C2 setup ({name})")
            t0 = time.perf_counter()
            pm = rz.Problem(ctx, args.n, args.p, alpha, beta, precision=prec)
            torch.cuda.synchronize()
            out[f"setup_s_{name}"] = round(time.perf_counter() - t0, 3)
            msm, infm, ktm = time_solves(torch, pm, bt, x, args.steps, args.warmup)
            out[f"pcg_ms_{name}"] = round(msm, 4)
            out[f"iters_{name}"] = infm[-1].iters
            out[f"rel_res_{name}"] = max(i.rel_res for i in infm)
            out[f"kernel_ms_per_step_{name}"] = {k: round(v[0] / args.steps, 4) for k, v in ktm.items()}
            out[f"speedup_{name}_vs_f64"] = round(ms / msm, 3)
            pm.close()


def bench_multi_rhs(torch, rz, pb, nrhs, patch_ms_1, solve_ms_1, iters_1, reps=3):
    """One rz_solve on nrhs right-hand sides (seeds 0..nrhs-1, interleaved (ndofs,
    nrhs)) against nrhs single solves: wall time, and the patch solve's time per
    launch (each slot's factor read once for two vectors)."""
    import synth
    log(f"C2 multi-RHS: {nrhs} right-hand sides in one solve")
    B = torch.as_tensor(np.ascontiguousarray(np.stack([synth.rhs_values(pb.ndofs, r) for r in range(nrhs)], axis=1)),
                        device="cuda:0")
    X = torch.empty_like(B)
    pb.solve(B, X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        infos = pb.solve(B, X)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    pb.timing(True)
    pb.timing_read()
    pb.solve(B, X)
    kt = pb.timing_read()
    pb.timing(False)
    patch_launch = kt["patch"][0] / max(kt["patch"][1], 1)
    return {"nrhs": nrhs, "ms_per_call": round(ms, 3), "ms_per_rhs": round(ms / nrhs, 3),
            "single_rhs_ms": round(solve_ms_1, 3), "speedup_per_rhs_vs_single": round(solve_ms_1 * nrhs / ms, 3),
            "iters": [i.iters for i in infos], "single_rhs_iters": iters_1,
            "max_rel_res": max(i.rel_res for i in infos),
            "patch_ms_per_launch": round(patch_launch, 4), "patch_ms_per_launch_single": round(patch_ms_1, 4),
            "patch_vectors_per_launch": min(nrhs, 2),
            "kernel_ms_per_call": {k: round(v[0], 3) for k, v in kt.items()}}


def bench_hmg(torch, rz, ctx, steps=3, warmup=1):
    """The p = 1 solve of the p-multigrid cycle by geometric h-multigrid (one V(1,1)
    cycle, point Jacobi, Hiptmair relaxation on the vector spaces, coarsest level
    dense) against the exact solve: iterations, time per PCG solve and the coarse
    solver's share.  H(grad): the C2 workload (Q_7 on 32^3, log-uniform cell
    coefficients), the same mesh with alpha = beta = 1, and a 64^3 mesh (Q_3, alpha =
    beta = 1; 4 levels) where the exact solver's dense plane blocks would take about
    24 GB and minutes of setup, so only h-MG runs.  H(curl)/H(div): NCE_6 and NCF_6 on
    16^3 (the C3 layout, alpha = beta = 1), and NCE_3 on 32^3, where the dense NCE_1
    inverse would take 68 GB, so only h-MG runs."""
    import synth
    res = {}
    cases = [("c2_q7_n32_loguniform", "grad", 32, 7, True, (rz.COARSE_DIRECT, rz.COARSE_HMG)),
             ("q7_n32_const", "grad", 32, 7, False, (rz.COARSE_DIRECT, rz.COARSE_HMG)),
             ("q3_n64_const", "grad", 64, 3, False, (rz.COARSE_HMG,)),
             ("c3_nce6_n16", "curl", 16, 6, False, (rz.COARSE_DIRECT, rz.COARSE_HMG)),
             ("ncf6_n16", "div", 16, 6, False, (rz.COARSE_DIRECT, rz.COARSE_HMG)),
             ("nce3_n32", "curl", 32, 3, False, (rz.COARSE_HMG,))]
    for name, space, n, p, logu, coarses in cases:
        al, be = (synth.cell_coefficients(n ** 3, 1), synth.cell_coefficients(n ** 3, 2)) if logu else (1.0, 1.0)
        row = {}
        bt = x = None
        for co in coarses:
            key = "hmg" if co == rz.COARSE_HMG else "direct"
            log(f"h-MG study: {name} {key}")
            t0 = time.perf_counter()
            pb = rz.Problem(ctx, n, p, al, be, space=space, coarse=co)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            if bt is None:
                bt = torch.as_tensor(synth.rhs_values(pb.ndofs, 0), device="cuda:0")
                x = torch.zeros_like(bt)
                row["ndofs"] = pb.ndofs
            ms, infos, kt = time_solves(torch, pb, bt, x, steps, warmup)
            r = {"setup_s": round(setup, 3), "pcg_ms": round(ms, 3), "iters": infos[-1].iters,
                 "rel_res": max(i.rel_res for i in infos),
                 "coarse_ms_per_step": round(kt["coarse"][0] / steps, 4),
                 "coarse_ms_per_call": round(kt["coarse"][0] / max(kt["coarse"][1], 1), 4)}
            if co == rz.COARSE_HMG:
                r["levels"] = pb.hmg_levels()
                gms, ginf, gst = time_graph(torch, pb, bt, x, steps)
                r["pcg_ms_graph"] = round(gms, 3)
                r["graph_segments"] = gst["segments"]
            row[key] = r
            pb.close()
        res[name] = row
    return res


def bench_c1(torch, rz, ctx, steps=20):
    """C1: Q_4 on 4^3, alpha = beta = 1; apply latency and PCG time (FP64)."""
    import synth
    pb = rz.Problem(ctx, 4, 4, 1.0, 1.0)
    b = torch.as_tensor(synth.rhs_values(pb.ndofs, 0), device="cuda:0")
    x = torch.empty_like(b)
    ms, infos, _ = time_solves(torch, pb, b, x, steps, 2)
    mg, ig, gs = time_graph(torch, pb, b, x, steps)
    a = time_apply(torch, pb, torch.float64, rz.F64)
    out = {"workload": "C1: H(grad) Q_4 on 4^3, alpha=beta=1", "ndofs": pb.ndofs, "nfree": pb.nfree,
           "apply_us_f64": round(a * 1e3, 2), "pcg_ms_f64": round(ms, 4), "iters_f64": infos[-1].iters,
           "rel_res_f64": infos[-1].rel_res, "pcg_ms_f64_graph": round(mg, 4), "iters_f64_graph": ig[-1].iters,
           "graph": gs, "speedup_graph": round(ms / mg, 3)}
    sol = x.cpu().numpy()
    pb.close()
    return out, sol


# Tables hcurl-iter and hdiv-iter, Cartesian meshes, PAFW column as the paper prints it
PAPER_PAFW_ITER = {("curl", 1, 0): 2, ("curl", 3, 0): 14, ("div", 1, 0): 2, ("div", 3, 0): 9}
# Tables hcurl-iter and hdiv-iter, Cartesian meshes, SC-PAFW column as the paper prints it
PAPER_SCPAFW_ITER = {("curl", 3, 0): 11, ("curl", 3, 1): 12, ("div", 3, 0): 8, ("div", 3, 1): 8}
# the PH column (without static condensation)
PAPER_PH_ITER = {("curl", 3, 0): 20, ("curl", 3, 1): 22, ("div", 3, 0): 15, ("div", 3, 1): 16}
# Tables hcurl-iter and hdiv-iter, Cartesian meshes, SC-PH column as the paper prints it
PAPER_SCPH_ITER = {("curl", 3, 0): 14, ("curl", 3, 1): 16, ("curl", 7, 0): 15, ("curl", 7, 1): 16,
                   ("div", 3, 0): 11, ("div", 3, 1): 13, ("div", 7, 0): 13, ("div", 7, 1): 13}
# Table hgrad-iter, Cartesian meshes, as the paper prints them: (chol, SC-chol, ICC, SC-ICC)
PAPER_HGRAD_ITER = {(3, 0): (14, 11, 14, 11), (3, 1): (15, 11, 15, 11), (7, 0): (12, 9, 13, 10),
                    (7, 1): (12, 9, 13, 10)}


def bench_table_hgrad_iter(torch, rz, ctx):
    """The paper's H(grad) iteration study on Cartesian meshes (Table hgrad-iter, SC
    and full-star columns): alpha = 1, beta = 1e-8, homogeneous Dirichlet, the right-hand side the
    Riesz representative of a random w (b = (M + K) w, w from U[-1,1) seed 7), CG to a
    1e-8 reduction of the natural P^{-1}-norm; vertex stars without (RZ_DECOMP_FULL) and
    with static condensation, each with exact Cholesky and with IC on the pattern.  The paper's coarse Cartesian mesh has six cells in the vertical (the
    horizontal layout is in a figure): l = 0 is taken as 6^3 cells, l = 1 as 12^3."""
    import synth
    out = {"workload": "Tables hgrad-iter (four columns), hcurl-iter and hdiv-iter (SC-PH), Cartesian: alpha=1, "
                       "beta=1e-8, b = (M+K) w, natural-norm criterion",
           "rows": []}
    for p, l in ((3, 0), (3, 1), (7, 0), (7, 1)):
        n = 6 * 2 ** l
        riesz = rz.Problem(ctx, n, p, 1.0, 1.0)
        w = torch.as_tensor(synth.rhs_values(riesz.ndofs, 7), device="cuda:0")
        b = torch.empty_like(w)
        riesz.apply(w, b)
        riesz.close()
        row = {"p": p, "l": l, "cells": n ** 3}
        for name, dc, ps in (("chol", rz.DECOMP_FULL, rz.PATCH_CHOLESKY), ("sc_chol", rz.DECOMP_SC, rz.PATCH_CHOLESKY),
                             ("icc", rz.DECOMP_FULL, rz.PATCH_IC), ("sc_icc", rz.DECOMP_SC, rz.PATCH_IC)):
            if (dc == rz.DECOMP_FULL and p > 3) or (name == "sc_chol" and (p, l) == (7, 1)):
                # dense factors of the full stars (2,197 rows at p = 7), or 2,197 dense 469-row
                # condensed factors: host setup of minutes, skipped
                row[name] = None
                continue
            pb = rz.Problem(ctx, n, p, 1.0, 1e-8, patch_solver=ps, decomposition=dc, norm=rz.NORM_NATURAL)
            x = torch.empty_like(b)
            info = pb.solve(b, x)
            row[name] = {"iters_natural": info.iters_natural, "rel_res_2norm_at_exit": info.rel_res}
            pb.close()
        row["paper_chol_scchol_icc_scicc"] = list(PAPER_HGRAD_ITER[(p, l)])
        out["rows"].append(row)
        log(f"table hgrad-iter p={p} l={l}: {row}")
    # H(curl) and H(div): the PAFW column (vertex stars, no static condensation) where
    # the dense star factors stay small
    out["pafw"] = []
    for space in ("curl", "div"):
        # (p = 1 at l >= 1 is left out: the p = 1 coarse level is then the fine level itself,
        # while the paper's hierarchy coarsens in h there)
        for p, l in ((1, 0), (3, 0)):
            n = 6 * 2 ** l
            riesz = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, omega=0.3)
            w = torch.as_tensor(synth.rhs_values(riesz.ndofs, 7), device="cuda:0")
            b = torch.empty_like(w)
            riesz.apply(w, b)
            riesz.close()
            pb = rz.Problem(ctx, n, p, 1.0, 1e-8, space=space, norm=rz.NORM_NATURAL, decomposition=rz.DECOMP_FULL,
                            patch_solver=rz.PATCH_CHOLESKY)
            x = torch.empty_like(b)
            info = pb.solve(b, x)
            pb.close()
            row = {"space": space, "p": p, "l": l, "cells": n ** 3, "iters_natural": info.iters_natural,
                   "paper_pafw": PAPER_PAFW_ITER[(space, p, l)]}
            out["pafw"].append(row)
            log(f"table {space}-iter PAFW p={p} l={l}: {row}")
    # SC-PAFW (the vertex stars on the condensed interface, exact solves)
    out["sc_pafw"] = []
    for space in ("curl", "div"):
        for p, l in ((3, 0), (3, 1)):
            n = 6 * 2 ** l
            riesz = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, omega=0.3)
            w = torch.as_tensor(synth.rhs_values(riesz.ndofs, 7), device="cuda:0")
            b = torch.empty_like(w)
            riesz.apply(w, b)
            riesz.close()
            # 40 Lanczos steps: with 10 the damping exceeds 2 / lambda_max at beta = 1e-8
            # and the cycle is indefinite (CG breakdown)
            pb = rz.Problem(ctx, n, p, 1.0, 1e-8, space=space, norm=rz.NORM_NATURAL,
                            decomposition=rz.DECOMP_SC_VERTEX, patch_solver=rz.PATCH_CHOLESKY, lanczos_steps=40)
            x = torch.empty_like(b)
            info = pb.solve(b, x, check=False)
            pb.close()
            row = {"space": space, "p": p, "l": l, "cells": n ** 3, "iters_natural": info.iters_natural,
                   "status": info.status, "lanczos_steps": 40, "paper_sc_pafw": PAPER_SCPAFW_ITER[(space, p, l)]}
            out["sc_pafw"].append(row)
            log(f"table {space}-iter SC-PAFW p={p} l={l}: {row}")
    # PH without static condensation (edge / face stars with every DoF of their cells)
    out["ph"] = []
    for space in ("curl", "div"):
        for p, l in ((3, 0), (3, 1)):
            n = 6 * 2 ** l
            riesz = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, omega=0.3)
            w = torch.as_tensor(synth.rhs_values(riesz.ndofs, 7), device="cuda:0")
            b = torch.empty_like(w)
            riesz.apply(w, b)
            riesz.close()
            pb = rz.Problem(ctx, n, p, 1.0, 1e-8, space=space, norm=rz.NORM_NATURAL,
                            decomposition=rz.DECOMP_FULL_PH, patch_solver=rz.PATCH_CHOLESKY)
            x = torch.empty_like(b)
            info = pb.solve(b, x, check=False)
            pb.close()
            row = {"space": space, "p": p, "l": l, "cells": n ** 3, "iters_natural": info.iters_natural,
                   "status": info.status, "paper_ph": PAPER_PH_ITER[(space, p, l)]}
            out["ph"].append(row)
            log(f"table {space}-iter PH p={p} l={l}: {row}")
    # H(curl) and H(div): the SC-PH column (the library's relaxation for these spaces)
    out["sc_ph"] = []
    for space in ("curl", "div"):
        for p, l in ((3, 0), (3, 1), (7, 0), (7, 1)):
            n = 6 * 2 ** l
            riesz = rz.Problem(ctx, n, p, 1.0, 1.0, space=space, omega=0.3)
            w = torch.as_tensor(synth.rhs_values(riesz.ndofs, 7), device="cuda:0")
            b = torch.empty_like(w)
            riesz.apply(w, b)
            riesz.close()
            pb = rz.Problem(ctx, n, p, 1.0, 1e-8, space=space, norm=rz.NORM_NATURAL)
            x = torch.empty_like(b)
            info = pb.solve(b, x)
            pb.close()
            row = {"space": space, "p": p, "l": l, "cells": n ** 3, "iters_natural": info.iters_natural,
                   "rel_res_2norm_at_exit": info.rel_res, "paper_sc_ph": PAPER_SCPH_ITER[(space, p, l)]}
            out["sc_ph"].append(row)
            log(f"table {space}-iter SC-PH p={p} l={l}: {row}")
    return out


# Table hodge-iter, Cartesian columns: (p, l) -> MINRES iterations for k = 1, 2, 3
PAPER_HODGE_ITER = {(3, 0): (9, 8, 8), (3, 1): (9, 7, 8), (3, 2): (9, 7, 8), (7, 0): (9, 8, 8), (7, 1): (9, 8, 8),
                    (7, 2): (8, 6, 8)}
HODGE_CASES = ((3, 0, "direct"), (3, 1, "direct"), (7, 0, "direct"), (7, 1, "direct"))
# l = 2 (24^3 cells): the dense NCE_1 / NCF_1 inverse would not fit, so the p = 1 problems
# are solved by the h-multigrid; l = 1 repeated with it for comparison
HODGE_CASES_HMG = ((3, 1, "hmg"), (3, 2, "hmg"), (7, 2, "hmg"))


def bench_hodge(torch, rz, ctx, cases=HODGE_CASES):
    """Mixed Hodge Laplacians (Sec. 5.3, Table hodge-iter, Cartesian columns): no
    essential boundary, right-hand side [0; A_k w] (the Riesz representative of a
    random w in V^k, w from U[-1,1) seed 7; for k = 3 A_3 = M_3 = 8 n^3 I on the unit
    cube), MINRES with 4 Chebyshev steps per block preconditioned by each Riesz map's
    V-cycle (alpha = beta = 1), natural-norm reduction 1e-8.  l = 0 is 6^3 cells, l = 1
    12^3 (as for the other iteration tables).  Setup (two Riesz-map problems and the
    Chebyshev intervals) is outside the timed solve."""
    import synth
    sp_ = ["grad", "curl", "div"]
    out = {"workload": "Table hodge-iter (Cartesian): MINRES, blockdiag Riesz-map preconditioner, "
                       "4 Chebyshev steps per block, natural-norm 1e-8", "rows": []}
    for p, l, coarse in cases:
        n = 6 * 2 ** l
        co = rz.COARSE_HMG if coarse == "hmg" else rz.COARSE_DIRECT
        row = {"p": p, "l": l, "cells": n ** 3, "coarse": coarse}
        for k in (1, 2, 3):
            t0 = time.time()
            lo = rz.Problem(ctx, n, p, 1.0, 1.0, space=sp_[k - 1], dirichlet=0, coarse=co)
            hi = rz.Problem(ctx, n, p, 1.0, 1.0, space=sp_[k], dirichlet=0, coarse=co) if k < 3 else None
            hg = rz.Hodge(k, lo, hi, 4)
            setup_s = time.time() - t0
            w = torch.as_tensor(synth.uniform_pm1(7, hg.n_hi), device="cuda:0")
            b = torch.zeros(hg.n_lo + hg.n_hi, dtype=torch.float64, device="cuda:0")
            if hi is not None:
                hi.apply(w, b[hg.n_lo:])
            else:
                b[hg.n_lo:] = 8.0 * n ** 3 * w
            x = torch.empty_like(b)
            hg.solve(b, x)
            info = hg.solve(b, x)
            row[f"k{k}"] = {"ndofs": hg.n_lo + hg.n_hi, "iters": info.iters, "solve_ms": round(info.t_solve_ms, 3),
                            "rel_res_2norm": info.rel_res, "setup_s": round(setup_s, 2),
                            "ritz_lo_hi": [round(e, 4) for e in hg.eig]}
            hg.close()
            lo.close()
            if hi is not None:
                hi.close()
            # the mixed protocol: FP32 relaxation inside the V-cycles, FP64 MINRES
            lo = rz.Problem(ctx, n, p, 1.0, 1.0, space=sp_[k - 1], dirichlet=0, precision=1, coarse=co)
            hi = rz.Problem(ctx, n, p, 1.0, 1.0, space=sp_[k], dirichlet=0, precision=1, coarse=co) if k < 3 else None
            hg = rz.Hodge(k, lo, hi, 4)
            hg.solve(b, x, check=False)
            info = hg.solve(b, x, check=False)
            row[f"k{k}_mixed"] = {"iters": info.iters, "solve_ms": round(info.t_solve_ms, 3), "status": info.status,
                                  "rel_res_2norm": info.rel_res,
                                  "speedup_vs_f64": round(row[f"k{k}"]["solve_ms"] / info.t_solve_ms, 3)}
            hg.close()
            lo.close()
            if hi is not None:
                hi.close()
        row["paper_k1_k2_k3"] = list(PAPER_HODGE_ITER[(p, l)])
        out["rows"].append(row)
        log(f"table hodge-iter p={p} l={l} coarse={coarse}: {row}")
    return out


def bench_c3(torch, rz, ctx, steps, warmup, n=16, p=6):
    """C3: H(curl) NCE_6 on a uniform 16^3 mesh, alpha = beta = 1: applies and PCG in
    the three precision protocols (FP64, FP32 relaxation, FP32 operator)."""
    import synth
    out = {"workload": f"C3: H(curl) NCE_{p} on {n}^3 uniform hex mesh, alpha=beta=1, tangential Dirichlet, "
                       f"SC-PH relaxation, NCE_1 coarse"}
    b = None
    for prec, name in ((rz.PREC_F64, "f64"), (rz.PREC_MIXED, "mixed"), (rz.PREC_DEFECT, "defect")):
        log(f"C3 setup ({name})")
        t0 = time.perf_counter()
        pb = rz.Problem(ctx, n, p, 1.0, 1.0, space="curl", precision=prec)
        torch.cuda.synchronize()
        out[f"setup_s_{name}"] = round(time.perf_counter() - t0, 3)
        if b is None:
            # entries on Dirichlet rows are read as zero by the solver
            b = torch.as_tensor(synth.rhs_values(pb.ndofs, 0), device="cuda:0")
            x = torch.empty_like(b)
            out["ndofs"], out["nfree"] = pb.ndofs, pb.nfree
        ms, infos, kt = time_solves(torch, pb, b, x, steps, warmup)
        out[f"pcg_ms_{name}"] = round(ms, 4)
        out[f"iters_{name}"] = infos[-1].iters
        out[f"rel_res_{name}"] = max(i.rel_res for i in infos)
        out[f"kernel_ms_per_step_{name}"] = {k: round(v[0] / steps, 4) for k, v in kt.items()}
        if prec == rz.PREC_F64:
            out["gdofs_f64"] = round(pb.ndofs / (ms * 1e-3) / 1e9, 5)
            mg, ig, gs = time_graph(torch, pb, b, x, steps)
            out["pcg_ms_f64_graph"], out["iters_f64_graph"], out["graph"] = round(mg, 4), ig[-1].iters, gs
            for nm, dt, code, sz in (("f64", torch.float64, rz.F64, 8), ("f32", torch.float32, rz.F32, 4)):
                a = time_apply(torch, pb, dt, code)
                out[f"apply_ms_{nm}"] = round(a, 4)
                out[f"apply_gdofs_{nm}"] = round(pb.ndofs / (a * 1e-3) / 1e9, 2)
                out[f"roofline_apply_{nm}"] = hbm_roof(2 * pb.ndofs * sz + 6 * pb.ncells * sz, a,
                                                       "k_apply_vec_p+k_apply_vec_gather",
                                                       "x in, y out, 6 weights per cell")
                out[f"roofline_apply_{nm}"]["traffic"] = MEASURED_TRAFFIC[f"apply_c3_{nm}"] if (n, p) == (16, 6) \
                    else None
        pb.close()
    out["speedup_mixed_vs_f64"] = round(out["pcg_ms_f64"] / out["pcg_ms_mixed"], 3)
    out["speedup_defect_vs_f64"] = round(out["pcg_ms_f64"] / out["pcg_ms_defect"], 3)
    return out


def c5_aux_variants(torch, rz, ctx, pb, b, x, n, p, train_seeds=(10, 11, 12, 13)):
    """FP64 PCG on the C5 problem with three separable auxiliaries: cell averages
    (default), the least-squares fit to the broken diagonals, and an MLP trained on
    meshes with other perturbation seeds (features -> log(fit / average)); and with
    the paper's auxiliary itself (the broken diagonals per DoF)."""
    import synth
    res = {}
    t_fit, feats, base = pb.aux_data()

    def run(coef, name):
        pb.set_aux(coef)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = pb.solve(b, x)
        torch.cuda.synchronize()
        res[name] = {"iters": info.iters, "pcg_ms": round((time.perf_counter() - t0) * 1e3, 3),
                     "rel_res": info.rel_res, "omega": pb.omega()}

    run(base, "cell_average")
    run(t_fit, "lsq_fit")
    log("C5: MLP training data from meshes with seeds " + str(list(train_seeds)))
    t0 = time.perf_counter()
    Xs, Ys = [], []
    for s in train_seeds:
        v = synth.perturbed_vertices(n, s)
        hctx = rz.Context(-1)
        hp = rz.Problem(hctx, n, p, synth.c5_coefficient_samples(v, n), 1.0, vertices=v)
        t, f, bs = hp.aux_data()
        hp.close()
        hctx.close()
        Xs.append(f.astype(np.float32))
        Ys.append(np.log(t / bs).astype(np.float32))
    X = torch.as_tensor(np.concatenate(Xs), device="cuda:0")
    Y = torch.as_tensor(np.concatenate(Ys), device="cuda:0")
    t_data = time.perf_counter() - t0
    mlp = rz.MLP(ctx, 51, 64, 6, seed=1)
    t0 = time.perf_counter()
    loss = mlp.train(X, Y, epochs=20, batch=512, lr=2e-3, seed=11)
    t_train = time.perf_counter() - t0
    Xt = torch.as_tensor(feats.astype(np.float32), device="cuda:0")
    out = torch.empty((pb.ncells, 6), dtype=torch.float32, device="cuda:0")
    mlp.predict(Xt, out)
    pred = out.cpu().numpy().astype(np.float64)
    mlp.close()
    res["mlp_rms_log_error"] = float(np.sqrt(np.mean((pred - np.log(t_fit / base)) ** 2)))
    res["cell_average_rms_log_error"] = float(np.sqrt(np.mean(np.log(t_fit / base) ** 2)))
    run(base * np.exp(pred), "mlp")
    res["mlp_train"] = {"cells": int(X.shape[0]), "data_s": round(t_data, 2), "train_s": round(t_train, 2),
                        "final_loss": loss}
    pb.set_aux(base)
    # the paper's own auxiliary: per-DoF broken diagonals (not separable), its own
    # problem (setup includes the diagonals of every cell)
    log("C5: the paper's auxiliary (broken diagonals)")
    v = synth.perturbed_vertices(n, 3)
    t0 = time.perf_counter()
    pp = rz.Problem(ctx, n, p, synth.c5_coefficient_samples(v, n), 1.0, vertices=v, aux=rz.AUX_PAPER_DIAG)
    torch.cuda.synchronize()
    setup_pd = time.perf_counter() - t0
    pp.solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = pp.solve(b, x)
    torch.cuda.synchronize()
    res["paper_diagonals"] = {"iters": info.iters, "pcg_ms": round((time.perf_counter() - t0) * 1e3, 3),
                              "rel_res": info.rel_res, "omega": pp.omega(), "setup_s": round(setup_pd, 2)}
    pp.close()
    return res


def c5_flops_per_cell(p, q):
    """Algorithmic flops of one trilinear cell of the quadrature apply: the
    contractions 2[4q(p+1)^3 + 6q^2(p+1)^2 + 8q^3(p+1)] plus about 150 per
    quadrature point for J, the adjugate, det J, the coefficient and the pullback."""
    n1 = p + 1
    return 2 * (4 * q * n1 ** 3 + 6 * q * q * n1 ** 2 + 8 * q ** 3 * n1) + 150 * q ** 3


def bench_c5(torch, rz, ctx, steps, warmup, n=24, p=8, aux=True):
    """Q_8 on a 24^3 mesh with interior vertices perturbed by up to 0.15 h (seed 3),
    alpha = exp(0.5 sin 2pi x sin 2pi y sin 2pi z) sampled at 27 reference points per
    cell, beta = 1, U[-1,1) RHS (seed 0): PCG with the cell-averaged separable
    auxiliary in the relaxation, FP64 and mixed."""
    import synth
    v = synth.perturbed_vertices(n, 3)
    a = synth.c5_coefficient_samples(v, n)
    out = {"workload": f"C5: H(grad) Q_{p} on a perturbed {n}^3 mesh (trilinear cells, interior vertices "
                       f"+-0.15h), alpha=exp(0.5 sin sin sin) sampled 27/cell, beta=1; "
                       f"cell-averaged separable auxiliary"}
    q = int(np.ceil(3 * (p + 1) / 2))
    for prec, name in ((rz.PREC_F64, "f64"), (rz.PREC_MIXED, "mixed")):
        log(f"C5 setup ({name})")
        t0 = time.perf_counter()
        pb = rz.Problem(ctx, n, p, a, 1.0, vertices=v, precision=prec)
        torch.cuda.synchronize()
        out[f"setup_s_{name}"] = round(time.perf_counter() - t0, 3)
        b = torch.as_tensor(synth.rhs_values(pb.ndofs, 0), device="cuda:0")
        x = torch.empty_like(b)
        ms, infos, kt = time_solves(torch, pb, b, x, steps, warmup)
        out["ndofs"] = pb.ndofs
        out[f"pcg_ms_{name}"] = round(ms, 4)
        out[f"iters_{name}"] = infos[-1].iters
        out[f"rel_res_{name}"] = max(i.rel_res for i in infos)
        out[f"kernel_ms_per_step_{name}"] = {k: round(v_[0] / steps, 4) for k, v_ in kt.items()}
        if prec == rz.PREC_F64:
            if aux:
                out["aux"] = c5_aux_variants(torch, rz, ctx, pb, b, x, n, p)
            out["gdofs_f64"] = round(pb.ndofs / (ms * 1e-3) / 1e9, 5)
            fl = c5_flops_per_cell(p, q) * pb.ncells
            for nm, dt, code, peak in (("f64", torch.float64, rz.F64, FP64_PEAK_TFLOPS),
                                       ("f32", torch.float32, rz.F32, FP32_PEAK_TFLOPS)):
                am = time_apply(torch, pb, dt, code)
                out[f"apply_ms_{nm}"] = round(am, 4)
                out[f"apply_gdofs_{nm}"] = round(pb.ndofs / (am * 1e-3) / 1e9, 2)
                out[f"roofline_apply_{nm}"] = alu_roof(fl, am, peak, "k_apply_quad+k_apply_gather",
                                                       f"sum factorization at q={q} + ~150 flops per point")
            out["apply_bf16"] = bf16_apply_report(torch, rz, pb, fl, "k_apply_quad_mfma+k_apply_gather")
        pb.close()
    return out


def bf16_apply_report(torch, rz, pb, flops, kernel):
    """BF16 apply: median time, its rate against the FP32 vector peak (the pointwise
    pullback in FP32 sets its floor; the contractions run on the matrix cores), and
    its error against the library's FP64 apply of the same BF16 input (the FP64 apply
    equals the oracle to 1e-12)."""
    am = time_apply(torch, pb, torch.bfloat16, rz.BF16)
    x = (torch.rand(pb.ndofs, dtype=torch.float64, device="cuda:0") * 2 - 1).to(torch.bfloat16)
    y = torch.empty_like(x)
    pb.apply(x, y, rz.BF16)
    x64 = x.to(torch.float64)
    y64 = torch.empty_like(x64)
    pb.apply(x64, y64, rz.F64)
    torch.cuda.synchronize()
    d = y.to(torch.float64) - y64
    return {"apply_ms": round(am, 4), "apply_gdofs": round(pb.ndofs / (am * 1e-3) / 1e9, 2),
            "rel_err_2norm_vs_f64": float(d.norm() / y64.norm()),
            "rel_err_max_vs_f64": float(d.abs().max() / y64.abs().max()),
            "roofline": alu_roof(flops, am, FP32_PEAK_TFLOPS, kernel,
                                 "the FP32 apply's flop count (contractions + pointwise), FP32 vector peak")}


def bench_batched(torch, rz, nrhs=4, nctx=2, count=64):
    """The batched workload: 64 problems with (space, n, p) drawn per problem
    (space in grad/curl/div, n in 4..16, p in 3..9, streams 1000+i), 4 right-hand
    sides each (seeds 4i..4i+3), alpha = beta = 1.  Sequential single-vector
    rz_solve calls vs one rz_solve_batched over `nctx` contexts (streams), each
    problem's right-hand sides in lockstep as one multi-vector."""
    import synth
    streams = [torch.cuda.Stream() for _ in range(nctx)]
    ctxs = [rz.Context(0, s) for s in streams]
    log(f"batched: setting up {count} problems")
    t0 = time.perf_counter()
    probs, bs, xs, spec, bcols, xcols = [], [], [], [], [], []
    for i in range(count):
        space, n, p = synth.batch_spec(i)
        pb = rz.Problem(ctxs[i % nctx], n, p, 1.0, 1.0, space=space)
        probs.append(pb)
        spec.append((space, n, p))
        cols = [synth.rhs_values(pb.ndofs, 4 * i + r) for r in range(nrhs)]
        bs.append(torch.as_tensor(np.ascontiguousarray(np.stack(cols, axis=1)), device="cuda:0"))
        xs.append(torch.zeros((pb.ndofs, nrhs), dtype=torch.float64, device="cuda:0"))
        bcols.append([torch.as_tensor(c, device="cuda:0") for c in cols])
        xcols.append([torch.zeros(pb.ndofs, dtype=torch.float64, device="cuda:0") for _ in range(nrhs)])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    dofs_rhs = sum(pb.ndofs for pb in probs) * nrhs
    log("batched: sequential solves")

    def sequential():
        for pb, b, x in zip(probs, bcols, xcols):
            for r in range(nrhs):
                pb.solve(b[r], x[r])
        torch.cuda.synchronize()

    sequential()   # warm-up
    rz.solve_batched(probs, bs, xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    t_seq = time.perf_counter() - t0
    log("batched: concurrent solves")
    t0 = time.perf_counter()
    con = rz.solve_batched(probs, bs, xs)
    torch.cuda.synchronize()
    t_con = time.perf_counter() - t0
    iters = [inf.iters for row in con for inf in row]
    log("batched: the same with the CG iterations from captured HIP graphs")
    for pb in probs:
        pb.set_graph(True)
    rz.solve_batched(probs, bs, xs)   # captures
    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sequential()
    t_seq_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    cong = rz.solve_batched(probs, bs, xs)
    torch.cuda.synchronize()
    t_con_g = time.perf_counter() - t0
    same_iters = [inf.iters for row in cong for inf in row] == iters
    for pb in probs:
        pb.set_graph(False)
    out = {"workload": f"C4: {count} Riesz maps, space in grad/curl/div, n in 4..16, p in 3..9 (drawn per "
                       f"problem), {nrhs} RHS each, alpha=beta=1, FP64",
           "problems": count, "rhs_per_problem": nrhs, "total_dofs_x_rhs": dofs_rhs,
           "spaces": {s: sum(1 for q in spec if q[0] == s) for s in ("grad", "curl", "div")},
           "setup_s": round(setup_s, 2), "sequential_s": round(t_seq, 4), "batched_s": round(t_con, 4),
           "contexts": nctx, "gdofs_rhs_per_s_sequential": round(dofs_rhs / t_seq / 1e9, 4),
           "gdofs_rhs_per_s_batched": round(dofs_rhs / t_con / 1e9, 4),
           "speedup": round(t_seq / t_con, 3), "iters_min_max": [min(iters), max(iters)],
           "sequential_graph_s": round(t_seq_g, 4), "batched_graph_s": round(t_con_g, 4),
           "gdofs_rhs_per_s_batched_graph": round(dofs_rhs / t_con_g / 1e9, 4),
           "speedup_graph_vs_sequential": round(t_seq / t_con_g, 3), "graph_iters_equal": same_iters,
           "max_rel_res": max(inf.rel_res for row in con for inf in row)}
    for pb in probs:
        pb.close()
    for c in ctxs:
        c.close()
    return out


def gpu_small_solutions(torch, rz, ctx):
    """GPU solutions of small instances of the workloads, for the error against the
    oracle computed in the CPU leg: C2's recipe at n = 4 (Q_7), C3's at n = 3 (NCE_6),
    and the H(div) Riesz map NCF_4 on 3^3."""
    import synth
    sols = {}
    al, be = synth.cell_coefficients(64, 1), synth.cell_coefficients(64, 2)
    for name, (space, n, p, a, bcoef) in {"c2_n4": ("grad", 4, 7, al, be), "c3_n3": ("curl", 3, 6, 1.0, 1.0),
                                          "div_n3": ("div", 3, 4, 1.0, 1.0)}.items():
        pb = rz.Problem(ctx, n, p, a, bcoef, space=space)
        b = torch.as_tensor(synth.rhs_values(pb.ndofs, 0), device="cuda:0")
        x = torch.empty_like(b)
        info = pb.solve(b, x)
        sols[name] = {"x": x.cpu().numpy(), "iters": info.iters, "rel_res": info.rel_res}
        pb.close()
    return sols


def cpu_baseline(gpu, min_s=10.0):
    """The oracle (plain NumPy/SciPy FP64, as it stands) on the host's cores, on
    bounded samples of the workloads, and the error of GPU solutions against it."""
    from threadpoolctl import threadpool_limits
    import scipy.sparse.linalg as spla
    import synth
    from oracle.lattice import Mesh, Lattice
    from oracle import assemble as asm, auxop, schwarz, pmg, matfree, hiptmair as hp
    from oracle import quadrature as oq
    cores = len(os.sched_getaffinity(0))
    res = {}
    with threadpool_limits(limits=cores):
        # PCG time-to-1e-8 on the C2 recipe at n = 6 (Q_7, 79,507 DoFs), setup excluded
        n, p = 6, 7
        al, be = synth.cell_coefficients(n ** 3, 1), synth.cell_coefficients(n ** 3, 2)
        m = Mesh(n, n, n)
        lat, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
        A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
        R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, auxop.cartesian_coefficient_array(lat, al, be)))
        Pr = pmg.prolongation(lat, latc)
        cs = pmg.CoarseSolver(latc, asm.with_dirichlet(latc, asm.cartesian_operator(latc, al, be)))
        mask = lat.dirichlet_mask()
        v0 = np.where(mask, 0.0, synth.uniform_pm1(99, lat.ndofs))
        lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
        V = pmg.VCycle(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
        b = np.where(mask, 0.0, synth.rhs_values(lat.ndofs, 0))
        reps, t = 0, 0.0
        while t < min_s:
            t0 = time.perf_counter()
            _, it, _ = pmg.pcg(A, b, V)
            t += time.perf_counter() - t0
            reps += 1
        t /= reps
        pcg_value = lat.ndofs / t / 1e9
        res["pcg_sample"] = (f"oracle FP64 PCG to 1e-8 (same V(1,1)/IC/p-MG method, C2 coefficient recipe), "
                             f"Q_{p} on {n}^3 cells = {lat.ndofs} DoFs, {it} iterations, setup excluded, "
                             f"{t:.3f} s per solve, mean of {reps}")
        # O6 matrix-free apply on the C2 recipe at n = 16 (1/8 of C2's cells)
        n16 = 16
        al16, be16 = synth.cell_coefficients(n16 ** 3, 1), synth.cell_coefficients(n16 ** 3, 2)
        lat16 = Lattice(Mesh(n16, n16, n16), "grad", 7)
        x16 = synth.uniform_pm1(5, lat16.ndofs)
        t0 = time.perf_counter()
        matfree.apply(lat16, x16, al16, be16)
        ta = time.perf_counter() - t0
        res["apply_gdofs"] = lat16.ndofs / ta / 1e9
        res["apply_sample"] = (f"oracle sum-factorized einsum apply (FP64), Q_7 on 16^3 = {lat16.ndofs} DoFs "
                               f"with the C2 coefficient recipe, {ta:.2f} s")
        # errors of GPU solutions against the oracle's direct solves
        errs = {}

        def a_err(A_, xs_, xg):
            e = xg - xs_
            return float(np.sqrt(e @ (A_ @ e) / (xs_ @ (A_ @ xs_))))
        if "c1" in gpu:
            lat1 = Lattice(Mesh(4, 4, 4), "grad", 4)
            A1 = asm.with_dirichlet(lat1, asm.cartesian_operator(lat1, 1.0, 1.0))
            b1 = np.where(lat1.dirichlet_mask(), 0.0, synth.rhs_values(lat1.ndofs, 0))
            errs["c1"] = a_err(A1, spla.spsolve(A1.tocsc(), b1), np.where(lat1.dirichlet_mask(), 0.0, gpu["c1"]))
        small = gpu.get("small", {})
        for name, (space, n_, p_, a_, b_) in {"c2_n4": ("grad", 4, 7, True, True),
                                              "c3_n3": ("curl", 3, 6, False, False),
                                              "div_n3": ("div", 3, 4, False, False)}.items():
            if name not in small:
                continue
            la = Lattice(Mesh(n_, n_, n_), space, p_)
            aa = synth.cell_coefficients(n_ ** 3, 1) if a_ else 1.0
            bb = synth.cell_coefficients(n_ ** 3, 2) if b_ else 1.0
            Aa = asm.with_dirichlet(la, asm.cartesian_operator(la, aa, bb))
            ma = la.dirichlet_mask()
            ba = np.where(ma, 0.0, synth.rhs_values(la.ndofs, 0))
            errs[name] = {"A_norm_rel_error": a_err(Aa, spla.spsolve(Aa.tocsc(), ba),
                                                    np.where(ma, 0.0, small[name]["x"])),
                          "gpu_iters": small[name]["iters"], "gpu_rel_res": small[name]["rel_res"]}
        res["errors_vs_oracle_direct_solve"] = errs
        # C5 input: the 27-sample triquadratic interpolant of alpha against alpha(x) at
        # the q = 14 Gauss-Lobatto points of every cell
        v = synth.perturbed_vertices(24, 3)
        smp = synth.c5_coefficient_samples(v, 24)
        xq, _ = oq.rule(14, "gll")
        interp = oq.sampled_values(smp, xq)                       # (ncells, q^3)
        mesh24 = Mesh(24, 24, 24, vertices=v)
        cv = mesh24.cell_vertices()
        worst = 0.0
        for c0 in range(0, cv.shape[0], 2048):
            X = []
            for k in range(c0, min(cv.shape[0], c0 + 2048)):
                Xk, _ = asm.trilinear_jacobian(cv[k], xq)
                X.append(Xk)
            X = np.stack(X)
            ex = synth.c5_alpha(X.reshape(-1, 3)).reshape(X.shape[0], -1)
            worst = max(worst, float(np.max(np.abs(interp[c0:c0 + X.shape[0]] - ex) / ex)))
        res["c5_alpha_interpolation_max_rel_error"] = worst
    out = {"value": pcg_value, "unit": "GDoF/s", "cores": cores, "kind": "oracle", "sample": res["pcg_sample"]}
    out.update({k: v for k, v in res.items() if k != "pcg_sample"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--only", choices=["c2", "c2-apply", "c2-relax", "c3", "c3-apply", "c5-apply", "table", "hmg", "hodge"],
                    default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-table", action="store_true", help="skip the Table hgrad-iter iteration study")
    ap.add_argument("--no-hmg", action="store_true", help="skip the h-multigrid coarse-solver study")
    ap.add_argument("--no-hodge", action="store_true", help="skip the Hodge-Laplacian MINRES study")
    ap.add_argument("--nrhs", type=int, default=4, help="right-hand sides of the C2 multi-vector solve (1: skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="copy 1 GiB once before the solves (outside the timed region), a plain copy "
                         "kernel of known size for scaling HBM byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path runs on a single MI355X "
              "(sharding across GPUs is designed, not built); rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2211_14284_amd import rz
    torch.cuda.init()
    ctx = rz.Context(0, torch.cuda.current_stream())
    if args.calib_copy:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        piece = args.only
        res = {}
        if piece == "c2":
            bench_c2(torch, rz, ctx, argparse.Namespace(**{**vars(args), "no_mixed": True}), res)
        elif piece == "c2-apply":
            alpha, beta, _ = workload(args.n, args.p)
            pb = rz.Problem(ctx, args.n, args.p, alpha, beta, omega=0.3)
            res["apply_ms_f64"] = time_apply(torch, pb, torch.float64, rz.F64, reps=args.steps)
            res["apply_ms_f32"] = time_apply(torch, pb, torch.float32, rz.F32, reps=args.steps)
            res["apply_ms_bf16"] = time_apply(torch, pb, torch.bfloat16, rz.BF16, reps=args.steps)
            pb.close()
        elif piece == "c2-relax":
            # the relaxation on 1 and on nrhs vectors (patch-solve launches over one and
            # over several vectors), for kernel traces and HBM counters
            alpha, beta, _ = workload(args.n, args.p)
            pb = rz.Problem(ctx, args.n, args.p, alpha, beta, omega=0.3)
            for k in (1, args.nrhs):
                r = torch.rand((pb.ndofs, k), dtype=torch.float64, device="cuda:0").squeeze(1)
                z = torch.empty_like(r)
                pb.relax(r, z)
                torch.cuda.synchronize()
                pb.timing(True)
                pb.timing_read()
                for _ in range(args.steps):
                    pb.relax(r, z)
                kt = pb.timing_read()
                pb.timing(False)
                res[f"nrhs{k}"] = {g: round(v[0] / max(v[1], 1), 4) for g, v in kt.items() if v[1]}
                del r, z
            pb.close()
        elif piece == "c3":
            res = bench_c3(torch, rz, ctx, args.steps, args.warmup)
        elif piece == "table":
            res = bench_table_hgrad_iter(torch, rz, ctx)
        elif piece == "hmg":
            res = bench_hmg(torch, rz, ctx, args.steps, args.warmup)
        elif piece == "hodge":
            res = bench_hodge(torch, rz, ctx, HODGE_CASES + HODGE_CASES_HMG)
        elif piece == "c3-apply":
            pb = rz.Problem(ctx, 16, 6, 1.0, 1.0, space="curl", omega=0.3)
            res["apply_ms_f64"] = time_apply(torch, pb, torch.float64, rz.F64, reps=args.steps)
            res["apply_ms_f32"] = time_apply(torch, pb, torch.float32, rz.F32, reps=args.steps)
            pb.close()
        elif piece == "c5-apply":
            import synth
            v = synth.perturbed_vertices(24, 3)
            pb = rz.Problem(ctx, 24, 8, synth.c5_coefficient_samples(v, 24), 1.0, vertices=v, omega=0.3)
            res["apply_ms_f64"] = time_apply(torch, pb, torch.float64, rz.F64, reps=args.steps)
            res["apply_ms_f32"] = time_apply(torch, pb, torch.float32, rz.F32, reps=args.steps)
            res["apply_ms_bf16"] = time_apply(torch, pb, torch.bfloat16, rz.BF16, reps=args.steps)
            pb.close()
        torch.cuda.synchronize()
        rz.close_all()
        print(json.dumps({"only": piece, **res}), flush=True)
        return
    out = {"metric": METRIC, "value": None, "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    bench_c2(torch, rz, ctx, args, out)
    gpu = {}
    log("C1")
    out["c1"], gpu["c1"] = bench_c1(torch, rz, ctx)
    if not args.no_c3:
        out["c3"] = bench_c3(torch, rz, ctx, max(1, args.steps // 2), 1)
    if not args.no_table:
        out["table_hgrad_iter"] = bench_table_hgrad_iter(torch, rz, ctx)
    if not args.no_hmg:
        out["hmg_coarse"] = bench_hmg(torch, rz, ctx, max(1, args.steps // 3), 1)
    if not args.no_hodge:
        out["table_hodge_iter"] = bench_hodge(torch, rz, ctx)
    if not args.no_c5:
        out["c5"] = bench_c5(torch, rz, ctx, max(1, args.steps // 2), 1)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, rz)
    if not args.no_cpu_baseline:
        gpu["small"] = gpu_small_solutions(torch, rz, ctx)
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(gpu)
    torch.cuda.synchronize()
    rz.close_all()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
