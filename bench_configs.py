"""Measurement runs of the configurations other than the headline box beam (called by bench.py --workload).

sphere      4,096 points on the unit sphere, single layer, FP64, p = 6, leaf <= 64; full O(N^2) oracle.
cells       64 periodic-cell bodies (unit cube minus ellipsoids, 20k-200k points each) in ONE batched plan,
            single + double layer, FP32 (split FP16 with the compressed M2L with --precision split16); also 64
            separate plans; oracle on 1,000 targets per cell.  With --periodic the cells are the periodic
            metamaterial cells of Sec. 4.3 (the void/material faces only, every integral over the lattice
            images; fmm_plan_periodic), oracle: Ewald sums on 40 targets of 2 cells.
cantilever  8:1:1 cantilever with 64 spherical holes (~965k quadrature points): bem_solve (FP64, tol 1e-6)
            without and with the two-level preconditioner (--precond), then the stress at the 128^3 interior
            lattice; oracle rows of the matrix-vector product and stress on sampled points; with
            --full-residual every row of b - A x by direct sums.
metacell    the periodic metamaterial cell of Sec. 4.3: 100^3 voxels with a central spherical cavity (R_c 0.2,
            alpha_c 0.7, or --rc 0.3 --alpha-c 0.4), the single-iteration solution on the device (periodic surface,
            superposition solve, stress at every filled voxel centre, TD, volume-fraction rule) and the effective
            bulk modulus of the initial and of the new design against the Hashin-Shtrikman bound.
warmstart   Algorithm 1 on the 120 x 15 x 15 voxel beam for 20 iterations (C = 0.001: the load corner's stress
            concentration sets the TD range, and larger C removes a third of the beam at once); systems 11-20 solved
            from zero, from the previous solution mapped onto the new surface, and from the learned network.
Each prints one JSON line.
"""
import json
import os
import time

import numpy as np
import torch

from paper_1612_04082_amd import kfmm
from workloads import geometry as geo

G = 1.0
K = kfmm.moduli(G, 0.3)


def _t(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


def _time_evals(plan, kind, a, b, out, steps, warmup):
    for _ in range(warmup):
        plan.eval(kind, a, b, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.eval(kind, a, b, out)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _cores():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def sphere(args):
    from oracle import direct as od
    c = geo.sphere_cloud(4096, seed=1)
    plan = kfmm.FmmPlan(_t(c["src"]), _t(c["nrm"]), _t(c["w"]), K=K, G=G, p=6, leaf_max=64, precision=kfmm.FP64)
    a = _t(c["a"])
    out = torch.empty((4096, 3), dtype=torch.float64, device="cuda")
    ms = _time_evals(plan, kfmm.DISP, a, None, out, args.steps, args.warmup)
    tc = time.time()
    ref = od.direct(od.DISP, c["src"], c["src"], c["w"], a=c["a"], K=K, G=G, nthreads=_cores())
    tcpu = time.time() - tc
    got = out.cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return dict(metric="FMM target points/s", value=4096 / (ms * 1e-3), unit="target points/s", ms_per_step=ms,
                dtype="f64", config=dict(workload="unit-sphere cloud, 4096 points, single layer, p=6, leaf<=64"),
                rel_err=err, rel_err_inf=float(np.abs(got - ref).max() / np.abs(ref).max()),
                tree=plan.info(), cpu_baseline=dict(value=4096 / tcpu, unit="target points/s", cores=_cores(),
                                                    kind="oracle", sample="full 4096 x 4096"))


def cells(args):
    from oracle import direct as od
    prec = {"split16": kfmm.FP32_M2L_SPLIT16}.get(args.precision, kfmm.FP32)
    tol = args.m2l_tol if args.precision == "split16" else 0.0  # compressed M2L with the split-FP16 arithmetic
    cl = geo.periodic_cell_batch(64) if args.periodic else geo.cell_batch(64)
    cells_arg = [(0.0, 0.0, 0.0, 1.0)] * 64 if args.periodic else None
    src = np.concatenate([c["src"] for c in cl])
    nrm = np.concatenate([c["nrm"] for c in cl])
    w = np.concatenate([c["w"] for c in cl])
    a = np.concatenate([c["a"] for c in cl])
    b = np.concatenate([c["b"] for c in cl])
    off = np.concatenate([[0], np.cumsum([c["src"].shape[0] for c in cl])])
    n = src.shape[0]
    t0 = time.time()
    plan = kfmm.FmmPlan(_t(src), _t(nrm), _t(w), K=K, G=G, p=args.p, leaf_max=args.leaf, precision=prec,
                        batch_src=list(off), m2l_tol=tol, cells=cells_arg)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    da, db = _t(a), _t(b)
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    ms = _time_evals(plan, kfmm.DISP, da, db, out, args.steps, args.warmup)
    got = out.cpu().numpy()
    plan.close()
    # the same cells as 64 separate plans, evaluated back to back
    plans, bufs = [], []
    t0 = time.time()
    for c in cl:
        plans.append(kfmm.FmmPlan(_t(c["src"]), _t(c["nrm"]), _t(c["w"]), K=K, G=G, p=args.p, leaf_max=args.leaf,
                                  precision=prec, m2l_tol=tol, cells=cells_arg[:1] if cells_arg else None))
        bufs.append((_t(c["a"]), _t(c["b"]), torch.empty((c["src"].shape[0], 3), dtype=torch.float64, device="cuda")))
    torch.cuda.synchronize()
    plan_seq_s = time.time() - t0
    for p_, (x, y, o) in zip(plans, bufs):
        p_.eval(kfmm.DISP, x, y, o)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        for p_, (x, y, o) in zip(plans, bufs):
            p_.eval(kfmm.DISP, x, y, o)
    e1.record()
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / args.steps
    for p_ in plans:
        p_.close()
    # oracle on 1,000 targets per cell (free space), or Ewald sums on 100 targets of 4 cells (periodic)
    rng = np.random.default_rng(4)
    errs = []
    tc = time.time()
    n_ref = 0
    for g, c in enumerate(cl):
        if args.periodic and g % 32:
            continue
        idx = rng.choice(c["src"].shape[0], size=40 if args.periodic else 1000, replace=False)
        if args.periodic:
            from oracle import periodic as opd
            ref = opd.periodic(od.DISP, c["src"][idx], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G,
                               L=1.0, alpha_L=3.5, nthreads=_cores())
        else:
            ref = od.direct(od.DISP, c["src"][idx], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G,
                            nthreads=_cores())
        n_ref += len(idx)
        errs.append(float(np.linalg.norm(got[off[g]:off[g + 1]][idx] - ref) / np.linalg.norm(ref)))
    tcpu = time.time() - tc
    kind_cells = "periodic metamaterial cells" if args.periodic else "periodic-cell bodies"
    return dict(metric=f"FMM target points/s (64 {'periodic ' if args.periodic else ''}cells, one batched plan)",
                value=n / (ms * 1e-3),
                unit="target points/s", ms_per_step=ms,
                dtype={kfmm.FP32_M2L_SPLIT16: "f32+f16x2"}.get(prec, "f32"),
                config=dict(workload=f"64 {kind_cells}, {n} points, SL+DL, p={args.p}, leaf<={args.leaf}",
                            m2l_tol=tol),
                sequential=dict(ms_per_step=ms_seq, value=n / (ms_seq * 1e-3), plan_seconds=plan_seq_s),
                plan_seconds=plan_s, rel_err_max_cell=max(errs), rel_err_median_cell=float(np.median(errs)),
                cpu_baseline=dict(value=n_ref / tcpu, unit="target points/s", cores=_cores(), kind="oracle",
                                  sample=("40 targets of cells 0 and 32 x all sources of the cell, Ewald sums"
                                          if args.periodic else "1000 targets per cell x all sources of the cell")))


def cantilever(args):
    from oracle import bem as ob
    from oracle import direct as od
    M, holes = geo.cantilever_voxels(seed=3)
    h = 2.0 / 9.0
    prob = geo.cantilever_problem(M, h)
    T = prob["tri"].shape[0]
    dtri, dbc, dval = _t(prob["tri"]), _t(prob["bc_type"], torch.int8), _t(prob["bc_val"])
    # unpreconditioned and two-level preconditioned GMRES on the same system; the preconditioned solution
    # feeds the stress stage
    modes = {"none": [kfmm.PC_NONE], "two-level": [kfmm.PC_TWO_LEVEL],
             "both": [kfmm.PC_NONE, kfmm.PC_TWO_LEVEL]}[args.precond]
    solves = {}
    for pcm in modes:
        torch.cuda.synchronize()
        t0 = time.time()
        x, u, t, st = kfmm.bem_solve(dtri, dbc, dval, K=K, G=G, tol=1e-6, restart=200, max_iter=3000, p=8,
                                     leaf_max=128, precision=kfmm.FP64, svd_eps=args.svd_eps, allow_noconv=True,
                                     precond=pcm, m2l_tol=args.bem_m2l_tol)
        torch.cuda.synchronize()
        solve_s = time.time() - t0
        solves["two-level" if pcm == kfmm.PC_TWO_LEVEL else "none"] = dict(
            seconds=solve_s, iters=st["iters"], converged=st["converged"], rel_res=st["rel_res"],
            restarts=st["restarts"], t_setup_s=st["t_setup_s"], t_precond_s=st["t_precond_s"],
            pc_coarse_dim=st["pc_coarse_dim"], t_solve_s=st["t_solve_s"],
            ms_per_iteration=1e3 * st["t_solve_s"] / max(1, st["n_matvec"]))
        print(json.dumps({"solve": solves}), flush=True)
    # oracle rows of the product for a random unknown vector (direct FP64 sums + closed-form self blocks);
    # at the solution itself A x ~ b is a 1e4-fold cancellation and the relative row error is inflated
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(T, size=args.rows, replace=False))
    xs = rng.normal(size=(T, 3))
    tc = time.time()
    ref_rows = ob.matvec_rows(prob["tri"], prob["bc_type"], xs, rows, K, G, nthreads=_cores())
    t_rows = time.time() - tc
    gpu_full = kfmm.bem_matvec(dtri, dbc, dval, x=_t(xs), which=0, K=K, G=G, p=8, precision=kfmm.FP64,
                               svd_eps=args.svd_eps or 1e-7, m2l_tol=args.bem_m2l_tol).cpu().numpy()
    gpu_rows = gpu_full[rows]
    matvec_err = float(np.linalg.norm(gpu_rows - ref_rows) / np.linalg.norm(ref_rows))
    # residual floor of the solution measured with the exact operator: product error eps times
    # ||A|| ||x|| / ||b|| (||A|| estimated as ||A x_r|| / ||x_r|| on the random x_r above)
    scale_t = -G / ob.mean_edge(prob["tri"])
    xsol = x.cpu().numpy().copy()
    xsol[prob["bc_type"] == 0] /= scale_t  # solver units
    b_gpu = kfmm.bem_matvec(dtri, dbc, dval, which=1, K=K, G=G, p=8, precision=kfmm.FP64,
                            svd_eps=args.svd_eps or 1e-7, m2l_tol=args.bem_m2l_tol).cpu().numpy()
    kx = float(np.linalg.norm(gpu_full) / np.linalg.norm(xs) * np.linalg.norm(xsol) / np.linalg.norm(b_gpu))
    residual = dict(norm_A_x_over_b=kx, product_err_random=matvec_err, floor_estimate=matvec_err * kx)
    if args.full_residual:
        # every row of b - A x by direct FP64 sums over all quadrature points on the host cores
        tc = time.time()
        allrows = np.arange(T)
        ax_full = ob.matvec_rows(prob["tri"], prob["bc_type"], xsol, allrows, K, G, nthreads=_cores())
        print(json.dumps({"direct_product_rows_done_s": time.time() - tc}), flush=True)
        b_full = ob.rhs_rows(prob["tri"], prob["bc_type"], prob["bc_val"], allrows, K, G, nthreads=_cores())
        residual.update(direct_rel_res=float(np.linalg.norm(b_full - ax_full) / np.linalg.norm(b_full)),
                        direct_seconds=time.time() - tc,
                        rhs_fmm_vs_direct=float(np.linalg.norm(b_gpu.reshape(-1, 3) - b_full) / np.linalg.norm(b_full)))
        print(json.dumps({"residual": residual}), flush=True)
    # stress at the 128^3 lattice
    # stress at the 128^3 lattice: p = 9 (the derivative kernel needs one order more than displacement for
    # 1e-5 here: 9e-6 at p = 8, 3e-6 at p = 9 measured with random boundary data), FP32 M2L and near field
    # with FP64 pseudo-inverses and translations (with FP32 translations the error here is 1.4e-5); the first
    # call also builds the p = 9 operators, the second is the steady cost (tree, lists, evaluation)
    lat = geo.interior_lattice(M, h, n=128, holes=holes)
    dl = _t(lat)
    stress_times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.time()
        sig = kfmm.bem_stress(dtri, dbc, dval, u, t, dl, K=K, G=G, p=9, leaf_max=128,
                              precision=kfmm.FP32_TRANS64, m2l_tol=args.stress_m2l_tol)
        torch.cuda.synchronize()
        stress_times.append(time.time() - t0)
    stress_s = stress_times[1]
    sidx = np.sort(rng.choice(lat.shape[0], size=args.rows, replace=False))
    qp, qn, qw, qe = ob.quadrature(prob["tri"])
    un, tn = u.cpu().numpy(), t.cpu().numpy()
    tc = time.time()
    sref = od.direct(od.STRESS, lat[sidx], qp, qw, a=tn[qe], b=-un[qe], nrm=qn, K=K, G=G, nthreads=_cores())
    t_sig = time.time() - tc
    sg = sig.cpu().numpy()[sidx]
    stress_err = float(np.linalg.norm(sg - sref) / np.linalg.norm(sref))
    return dict(metric="BEM solve time (s), cantilever 8:1:1 with 64 holes", value=solve_s, unit="s",
                higher_is_better=False, dtype="f64",
                config=dict(workload=f"cantilever [0,32]x[0,4]^2, h=2/9, 64 holes: {T} elements, {16 * T} quadrature "
                                     f"points, {3 * T} unknowns; GMRES(200) tol 1e-6, FMM p=8 leaf<=128 FP64, "
                                     f"m2l_tol {args.bem_m2l_tol:g}",
                            precond=args.precond),
                svd_eps=args.svd_eps, gmres=solves,
                matvec_rows_rel_err=matvec_err, oracle_rows_seconds=t_rows, residual_vs_exact=residual,
                stress=dict(targets=int(lat.shape[0]), p=9, precision="fp32t64", m2l_tol=args.stress_m2l_tol,
                            seconds=stress_s,
                            seconds_first_call=stress_times[0], points_per_s=lat.shape[0] / stress_s,
                            rel_err=stress_err, oracle_seconds=t_sig),
                cpu_baseline=dict(value=args.rows / t_sig, unit="stress target points/s", cores=_cores(),
                                  kind="oracle", sample=f"{args.rows} lattice points x {16 * T} sources"))


def metacell(args):
    from paper_1612_04082_amd.alg1 import PeriodicCell
    n = args.cell_n
    M0 = geo.cavity_cell(n, args.rc)
    cell = PeriodicCell(n, p=args.p_bem, leaf_max=128, tol=1e-6, m2l_tol=args.bem_m2l_tol)
    cell.single_iteration(geo.cavity_cell(8, args.rc), args.alpha_c)  # operators of this p (first use)
    torch.cuda.synchronize()
    t0 = time.time()
    new, rec = cell.single_iteration(M0, args.alpha_c)
    torch.cuda.synchronize()
    it_s = time.time() - t0
    print(json.dumps({"single_iteration": rec, "seconds": it_s}), flush=True)
    out = cell.bulk_modulus(new)
    return dict(metric="periodic cell single-iteration time (s), 100^3 voxels", value=it_s, unit="s",
                higher_is_better=False, dtype="f64",
                config=dict(workload=f"periodic cell {n}^3 voxels, spherical cavity R_c={args.rc}, alpha_c={args.alpha_c}, "
                                     f"hydrostatic stress, FMM p={args.p_bem} leaf<=128 FP64, m2l_tol "
                                     f"{args.bem_m2l_tol:g}, GMRES tol 1e-6"),
                initial=rec, result=dict(void_fraction=out["void_fraction"], K_eff=out["K_eff"], K_hs=out["K_hs"],
                                         K_eff_over_hs=out["K_eff"] / out["K_hs"], T=out["T"], gmres=out["gmres"],
                                         t_solve_s=out["t_solve_s"]),
                initial_K_eff_over_hs=rec["K_eff"] / rec["K_hs"])


def warmstart(args):
    from paper_1612_04082_amd.alg1 import warm_start_study
    M0 = np.ones((120, 15, 15), bool)
    log = []
    pcm = kfmm.PC_NONE if args.precond == "none" else kfmm.PC_TWO_LEVEL
    rec = warm_start_study(M0, n_iter=args.iters, train_from=2, measure_from=args.measure_from, h=1.0, C=0.001,
                           tol_seq=1e-6, tol=1e-6, epochs=200, lr=1e-3, restart=200, p=args.p_bem, leaf_max=128,
                           precision=kfmm.FP64, precond=pcm, m2l_tol=args.bem_m2l_tol,
                           log=lambda r: (log.append(r), print(json.dumps(r), flush=True)))
    meas = [r for r in rec if "zero" in r]
    summ = {}
    for mode in ("zero", "prev", "net"):
        it = [r[mode]["iters"] for r in meas]
        sec = [r[mode]["seconds"] for r in meas]
        summ[mode] = dict(iters_mean=float(np.mean(it)), iters_std=float(np.std(it)), seconds_mean=float(np.mean(sec)),
                          seconds_std=float(np.std(sec)))
    return dict(metric="BEM solve time learned vs plain (s per solve, mean over measured iterations)",
                value=summ["net"]["seconds_mean"], unit="s", higher_is_better=False, dtype="f64",
                config=dict(workload=f"Algorithm 1 on 120x15x15 voxels, C=0.001, tol 1e-6, GMRES(200), "
                                     f"FMM p={args.p_bem} FP64, m2l_tol {args.bem_m2l_tol:g}",
                            precond="none" if pcm == kfmm.PC_NONE else "two-level"),
                summary=summ, speedup_vs_zero=summ["zero"]["seconds_mean"] / summ["net"]["seconds_mean"],
                speedup_vs_prev=summ["prev"]["seconds_mean"] / summ["net"]["seconds_mean"],
                iterations=[dict(iter=r["iter"], alpha=r.get("alpha"), T=r["T"]) for r in rec])


def run(args):
    fn = dict(sphere=sphere, cells=cells, cantilever=cantilever, warmstart=warmstart, metacell=metacell)[args.workload]
    line = fn(args)
    line.setdefault("higher_is_better", True)
    line.update(n_gpus=1, steps=args.steps, warmup=args.warmup, data="synthetic", vs_baseline=None)
    print(json.dumps(line), flush=True)
