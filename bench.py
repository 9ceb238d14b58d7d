#!/usr/bin/env python
"""Benchmark of the H(grad) hot path on one MI355X.

Workload (default): Q_7 on a uniform 32^3 hexahedral mesh of the unit cube
(225^3 = 11,390,625 lattice DoFs), cellwise-constant alpha, beta log-uniform in
[1e-2, 1e2) (SplitMix64 seeds 1, 2), U[-1,1) right-hand side (seed 0), homogeneous
Dirichlet boundary.

One step = one PCG solve from x = 0 to a true relative residual of 1e-8 with the
p-multigrid V(1,1) preconditioner (statically condensed vertex-star relaxation
with IC patch factors, p=1 coarse solve), all vectors resident in HBM; setup is
done once before the timed region and reported separately.  Printed: one JSON
line with the FP64 solve throughput as `value`, plus the mixed-precision solve,
the operator-apply throughput, per-kernel times and the roofline of the dominant
kernel (HIP events on the library stream over the timed region), and the CPU
oracle timed on a bounded sample.
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
# HBM bytes per launch of a kernel group from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0, factors from a plain 1 GiB copy in the same run); the figure belongs
# to the kernel version it was taken on (profiles/pmc_patch_solve_hgrad_q7_n32.md)
MEASURED_TRAFFIC = {"patch": 2.281e9}
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


def kernel_bytes(pb, sz, n):
    """Algorithmic HBM bytes of one launch of each timed kernel group (element size sz)."""
    nd, ns, nnz, nrows, nc, p = pb.ndofs, pb.nslots, pb.nnz, pb.nrows, pb.ncells, pb.p
    niface = nd - nc * (p - 1) ** 3
    return {
        # x read once, y written once, 6 weights per cell
        "apply": 2 * nd * sz + 6 * nc * sz,
        # r read once, interface right-hand side written once
        "condense": (nd + niface) * sz,
        # every slot: its factor (off-diagonals and diagonal, stored once) read once,
        # its interface vector in and out; both sweeps stream the off-diagonals, the
        # second read served by the caches or counted by the HBM counters
        "patch": ns * (nnz + 2 * nrows) * sz,
        # patch solutions read once, r read once, z written once
        "expand": (ns * nrows + 2 * nd) * sz,
        # dense inverse blocks and coupling products of the coarse factorisation
        # (W, M, N per plane), each read once
        "coarse": 3 * (n - 1) * ((n - 1) ** 2) ** 2 * 8,
    }


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


def time_apply(torch, pb, dtype_t, code, reps=50, warm=10):
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


def c5_aux_variants(torch, rz, ctx, pb, b, x, n, p, train_seeds=(10, 11, 12, 13)):
    """FP64 PCG on the C5 problem with three separable auxiliaries: cell averages
    (default), the least-squares fit to the broken diagonals, and an MLP trained on
    meshes with other perturbation seeds (features -> log(fit / average))."""
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
        hp = rz.Problem(rz.Context(-1), n, p, synth.c5_coefficient_samples(v, n), 1.0, vertices=v)
        t, f, bs = hp.aux_data()
        hp.close()
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
    return res


def bench_c5(torch, rz, ctx, steps, warmup, n=24, p=8):
    """Q_8 on a 24^3 mesh with interior vertices perturbed by up to 0.15 h (seed 3),
    alpha = exp(0.5 sin 2pi x sin 2pi y sin 2pi z) sampled at 27 reference points per
    cell, beta = 1, U[-1,1) RHS (seed 0): PCG with the cell-averaged separable
    auxiliary in the relaxation, FP64 and mixed."""
    import synth
    v = synth.perturbed_vertices(n, 3)
    a = synth.c5_coefficient_samples(v, n)
    out = {"workload": f"H(grad) Q_{p} on a perturbed {n}^3 mesh (trilinear cells, interior vertices "
                       f"+-0.15h), alpha=exp(0.5 sin sin sin) sampled 27/cell, beta=1; "
                       f"cell-averaged separable auxiliary"}
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
            out["aux"] = c5_aux_variants(torch, rz, ctx, pb, b, x, n, p)
            out["gdofs_f64"] = round(pb.ndofs / (ms * 1e-3) / 1e9, 5)
            out["apply_ms_f64"] = round(time_apply(torch, pb, torch.float64, rz.F64), 4)
            out["apply_ms_f32"] = round(time_apply(torch, pb, torch.float32, rz.F32), 4)
            out["apply_gdofs_f64"] = round(pb.ndofs / (out["apply_ms_f64"] * 1e-3) / 1e9, 2)
            out["apply_gdofs_f32"] = round(pb.ndofs / (out["apply_ms_f32"] * 1e-3) / 1e9, 2)
        pb.close()
    return out


def bench_c3(torch, rz, ctx, n=16, p=6):
    """H(curl) NCE_6 on a uniform 16^3 mesh, alpha = beta = 1: operator apply throughput
    (the H(curl) relaxation is not built, so no solve)."""
    pb = rz.Problem(ctx, n, p, 1.0, 1.0, space="curl")
    out = {"workload": f"H(curl) NCE_{p} on {n}^3 uniform hex mesh, alpha=beta=1 (apply only)",
           "ndofs": pb.ndofs, "nfree": pb.nfree}
    for name, dt, code in (("f64", torch.float64, rz.F64), ("f32", torch.float32, rz.F32)):
        ms = time_apply(torch, pb, dt, code)
        out[f"apply_ms_{name}"] = round(ms, 4)
        out[f"apply_gdofs_{name}"] = round(pb.ndofs / (ms * 1e-3) / 1e9, 2)
    pb.close()
    return out


def bench_batched(torch, rz, nrhs=4, nctx=2, count=64):
    """The batched workload: 64 problems with (n, p) drawn per problem (n in 4..16,
    p in 3..9, streams 1000+i), 4 right-hand sides each (seeds 4i..4i+3), alpha =
    beta = 1.  Only H(grad) is built, so every member is solved as an H(grad) Riesz
    map of its drawn size and degree.  Sequential rz_solve calls vs rz_solve_batched
    over `nctx` contexts (streams); two streams measured fastest (1, 2, 4, 8 streams:
    0.94x, 1.42x, 1.09x, 0.94x of the sequential time)."""
    import synth
    streams = [torch.cuda.Stream() for _ in range(nctx)]
    ctxs = [rz.Context(0, s) for s in streams]
    log(f"batched: setting up {count} problems")
    t0 = time.perf_counter()
    probs, bs, xs, spec = [], [], [], []
    for i in range(count):
        space, n, p = synth.batch_spec(i)
        pb = rz.Problem(ctxs[i % nctx], n, p, 1.0, 1.0)
        probs.append(pb)
        spec.append((space, n, p))
        bs.append(torch.as_tensor(np.stack([synth.rhs_values(pb.ndofs, 4 * i + r) for r in range(nrhs)]),
                                  device="cuda:0"))
        xs.append(torch.zeros((nrhs, pb.ndofs), dtype=torch.float64, device="cuda:0"))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    dofs_rhs = sum(pb.ndofs for pb in probs) * nrhs
    log("batched: sequential solves")

    def sequential():
        for pb, b, x in zip(probs, bs, xs):
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
    out = {"workload": f"{count} H(grad) Riesz maps, n in 4..16, p in 3..9 (drawn per problem), "
                       f"{nrhs} RHS each, alpha=beta=1 (members drawn as curl/div solved as grad)",
           "problems": count, "rhs_per_problem": nrhs, "total_dofs_x_rhs": dofs_rhs,
           "spaces_drawn": {s: sum(1 for q in spec if q[0] == s) for s in ("grad", "curl", "div")},
           "setup_s": round(setup_s, 2), "sequential_s": round(t_seq, 4), "batched_s": round(t_con, 4),
           "contexts": nctx, "gdofs_rhs_per_s_sequential": round(dofs_rhs / t_seq / 1e9, 4),
           "gdofs_rhs_per_s_batched": round(dofs_rhs / t_con / 1e9, 4),
           "speedup": round(t_seq / t_con, 3), "iters_min_max": [min(iters), max(iters)],
           "max_rel_res": max(inf.rel_res for row in con for inf in row)}
    for pb in probs:
        pb.close()
    return out


def cpu_baseline(n=4, p=7, min_s=10.0):
    """The oracle's FP64 PCG (same method, same recipe) on a bounded sample."""
    from threadpoolctl import threadpool_limits
    import synth
    from oracle.lattice import Mesh, Lattice
    from oracle import assemble as asm, auxop, schwarz, pmg
    with threadpool_limits(limits=1):
        al = synth.cell_coefficients(n ** 3, 1)
        be = synth.cell_coefficients(n ** 3, 2)
        m = Mesh(n, n, n)
        lat, latc = Lattice(m, "grad", p), Lattice(m, "grad", 1)
        A = asm.with_dirichlet(lat, asm.cartesian_operator(lat, al, be))
        co = auxop.cartesian_coefficient_array(lat, al, be)
        R = schwarz.SCRelaxGrad(lat, auxop.separable_operator(lat, co))
        Pr = pmg.prolongation(lat, latc)
        cs = pmg.CoarseSolver(latc, asm.with_dirichlet(latc, asm.cartesian_operator(latc, al, be)))
        mask = lat.dirichlet_mask()
        v0 = np.where(mask, 0.0, synth.uniform_pm1(99, lat.ndofs))
        lam = pmg.lanczos_lambda_max(A, lambda r: np.where(mask, 0.0, R.apply(r)), v0)
        V = pmg.VCycle(lat, A, R, Pr, cs, pmg.omega_from_lambda(lam))
        b = np.where(mask, 0.0, synth.rhs_values(lat.ndofs, 0))
        # a bounded sample: repeat the solve until at least min_s seconds of CPU work
        reps, t = 0, 0.0
        while t < min_s:
            t0 = time.perf_counter()
            x, it, _ = pmg.pcg(A, b, V)
            t += time.perf_counter() - t0
            reps += 1
        t /= reps
    return {"value": lat.ndofs / t / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FP64 PCG to 1e-8 (same V(1,1)/IC/p-MG method and coefficient recipe), "
                      f"Q_{p} on {n}^3 cells = {lat.ndofs} DoFs, {it} iterations, setup excluded, "
                      f"{t:.3f} s per solve on 1 host thread, mean of {reps} repetitions"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-c5", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-c3", action="store_true")
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
    stream = torch.cuda.current_stream()
    ctx = rz.Context(0, stream)
    if args.calib_copy:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    alpha, beta, b = workload(args.n, args.p)
    log(f"setup FP64 problem n={args.n} p={args.p}")
    t0 = time.perf_counter()
    pb = rz.Problem(ctx, args.n, args.p, alpha, beta, precision=rz.PREC_F64)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup done in {setup_s:.2f} s; timing {args.steps} FP64 solves")
    bt = torch.as_tensor(b, device="cuda:0")
    x = torch.empty(pb.ndofs, dtype=torch.float64, device="cuda:0")
    ms, infos, kt = time_solves(torch, pb, bt, x, args.steps, args.warmup)
    iters = infos[-1].iters
    relres = max(i.rel_res for i in infos)
    # dominant kernel and its roofline (algorithmic bytes / average launch time)
    kb = kernel_bytes(pb, 8, args.n)
    dom = max(kt, key=lambda k: kt[k][0])
    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in kt.items()}
    roof = None
    if dom in kb and kt[dom][1]:
        ach = kb[dom] / (per_launch[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": MEASURED_TRAFFIC.get(dom) if args.p == 7 and args.n == 32 else None,
                "kernel": dom,
                "avg_launch_ms": round(per_launch[dom], 4), "algorithmic_bytes_per_launch": kb[dom]}
    log(f"FP64 solve {ms:.3f} ms, {iters} iterations; timing the apply")
    apply64 = time_apply(torch, pb, torch.float64, rz.F64)
    apply32 = time_apply(torch, pb, torch.float32, rz.F32)
    out = {
        "metric": METRIC, "value": round(pb.ndofs / (ms * 1e-3) / 1e9, 5), "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"H(grad) Q_{args.p} on {args.n}^3 uniform hex mesh, cellwise log-uniform "
                               f"alpha,beta in [1e-2,1e2), U[-1,1) RHS; PCG to rel. residual 1e-8",
                   "ndofs": pb.ndofs, "nfree": pb.nfree, "cells": pb.ncells, "p": args.p},
        "pcg_ms_f64": round(ms, 4), "iters_f64": iters, "rel_res_f64": relres,
        "setup_s_f64": round(setup_s, 3), "omega": pb.omega(),
        "apply_gdofs_f64": round(pb.ndofs / (apply64 * 1e-3) / 1e9, 2),
        "apply_gdofs_f32": round(pb.ndofs / (apply32 * 1e-3) / 1e9, 2),
        "apply_ms_f64": round(apply64, 4), "apply_ms_f32": round(apply32, 4),
        "kernel_ms_per_step_f64": {k: round(v[0] / args.steps, 4) for k, v in kt.items()},
        "kernel_launches_per_step_f64": {k: v[1] / args.steps for k, v in kt.items()},
        "roofline": roof,
    }
    pb.close()
    if not args.no_mixed:
        log("setup mixed-precision problem")
        t0 = time.perf_counter()
        pm = rz.Problem(ctx, args.n, args.p, alpha, beta, precision=rz.PREC_MIXED)
        torch.cuda.synchronize()
        out["setup_s_mixed"] = round(time.perf_counter() - t0, 3)
        msm, infm, ktm = time_solves(torch, pm, bt, x, args.steps, args.warmup)
        out["pcg_ms_mixed"] = round(msm, 4)
        out["iters_mixed"] = infm[-1].iters
        out["rel_res_mixed"] = max(i.rel_res for i in infm)
        out["kernel_ms_per_step_mixed"] = {k: round(v[0] / args.steps, 4) for k, v in ktm.items()}
        out["speedup_mixed_vs_f64"] = round(ms / msm, 3)
        pm.close()
        log("setup defect-correction problem (FP32 operator)")
        pd = rz.Problem(ctx, args.n, args.p, alpha, beta, precision=rz.PREC_DEFECT)
        msd, infd, ktd = time_solves(torch, pd, bt, x, args.steps, args.warmup)
        out["pcg_ms_defect"] = round(msd, 4)
        out["iters_defect_inner"] = infd[-1].iters
        out["rel_res_defect"] = max(i.rel_res for i in infd)
        out["kernel_ms_per_step_defect"] = {k: round(v[0] / args.steps, 4) for k, v in ktd.items()}
        out["speedup_defect_vs_f64"] = round(ms / msd, 3)
        pd.close()
    if not args.no_c5:
        out["c5"] = bench_c5(torch, rz, ctx, max(1, args.steps // 2), 1)
    if not args.no_c3:
        out["c3"] = bench_c3(torch, rz, ctx)
    if not args.no_batched:
        out["batched"] = bench_batched(torch, rz)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    torch.cuda.synchronize()
    rz.close_all()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
