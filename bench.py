"""Benchmark: KIFMM evaluation throughput (target points/s) on one MI355X.

Workload (the configuration the headline metric is quoted on): the 120 x 20 x 20 box-beam surface,
201,344 quadrature points with outward normals and area weights, targets = sources, random single-
and double-layer densities N(0,1); one step = one fmm_eval of the displacement of the combined
single + double layer (S2M, M2M, M2L, L2L, X, W, L2T, near field), p = 8 (the smallest order that reaches
1e-5 relative error on this surface; p = 6 and p = 7 stop near 1.5e-4 and 2.4e-5), leaf <= 256 (on this
surface leaf limits 96 and 128 give one tree, 160 to 256 another with 13% fewer boxes, depth 6 and 6%
fewer seconds per eval; 320 merges into 1,064 boxes and quadruples the near field).
Default arithmetic (--precision split16): point evaluations and translations in FP32 (M2M / L2L on
check potentials, factored pseudo-inverses), the M2L contraction on the FP16 matrix cores with operands
split into high and low FP16 parts; M2L compressed onto a shared basis with relative cutoff 3e-7 (463
directions, kept as 480 = the padded width of the contraction).  The plan (tree, lists, operators) is
built once outside the timed region, as the paper excludes tree construction from its per-pass rate.

Printed JSON line: metric/value/unit, timing, the relative L2 and max-norm errors of the timed loop's own
output on a 40,000-target sample against the FP64 oracle, the roofline of the dominant kernel (the M2L
contraction; bound = the larger of its algorithmic FLOP at the matrix peak and its algorithmic bytes at
the HBM peak, its launch time from HIP events recorded inside the library on the evaluation stream), the
whole evaluation's T_ideal / T_measured (every phase's algorithmic work at the peak of its unit, from
fmm_plan_work), and the oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks (TFLOP/s; HBM in TB/s).  Algorithmic FLOP are priced at the dense peak of the unit
# a phase runs on: the split-FP16 products at the FP16 dense matrix peak (the three FP16 products per
# algorithmic product are the implementation's cost, reported apart as the matrix-pipe utilisation).
HBM_TBS = 8.0
VALU_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split16": 157.3, "fp32t64": 157.3}
M2L_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split16": 2500.0, "fp32t64": 157.3}
TRANS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split16": 2500.0, "fp32t64": 78.6}
MFMA_PRODUCTS = {"split16": 3}  # matrix-core products per algorithmic product
KERNELS = {"fp64": "k_gemm_f<double>", "fp32": "k_gemm_f<float>", "fp32t64": "k_gemm_f<float>",
           "split16": "k_gemm_h3 (FP16 high/low split, 3 MFMA products)"}
PHASE_UNIT = {"permute": "hbm", "m2l_red": "hbm", "s2m": "valu", "s2l": "valu", "near": "valu", "leaf": "valu",
              "uc2ue": "trans", "m2m": "trans", "m2l_prep": "trans", "down": "trans", "m2l": "m2l"}


def phase_peak_tflops(phase, precision):
    u = PHASE_UNIT[phase]
    return {"hbm": None, "valu": VALU_TFLOPS[precision], "trans": TRANS_TFLOPS[precision],
            "m2l": M2L_TFLOPS[precision]}[u]


def ideal_ms(flops, nbytes, peak_tflops):
    """Roofline time of a phase: the larger of its FLOP at the unit's peak and its bytes at the HBM peak."""
    t_f = flops / (peak_tflops * 1e12) if peak_tflops else 0.0
    return max(t_f, nbytes / (HBM_TBS * 1e12)) * 1e3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# HBM bytes of one M2L launch of the default configuration, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch) scaled by the same counters on a 1024 MiB copy (factors 2.0 and 1.0); the summary is in
# profiles/m2l_split16_boxbeam_p8_leaf256.md.  Valid only for the kernel sources and the launch set-up (tile
# widths, in fmm.hip) it was measured on.
M2L_TRAFFIC = {"sources_sha256": "78cf899a0402fc685f47d45d84675d2037e3f7e00e630a5893eec5d68d18d4d9",
               "fetch_kib": 153057.6 * 2.0, "write_kib": 172768.0 * 1.0}
M2L_SOURCES = ("paper_1612_04082_amd/csrc/gemm_kernels.h", "paper_1612_04082_amd/csrc/gemm_h3.hip",
               "paper_1612_04082_amd/csrc/gemm.h", "paper_1612_04082_amd/csrc/fmm.hip")


def m2l_traffic_bytes(args):
    import hashlib
    if (args.precision, args.p, args.leaf, args.m2l_tol) != ("split16", 8, 256, 3e-7):
        return None
    h = hashlib.sha256()
    for f in M2L_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != M2L_TRAFFIC["sources_sha256"]:
        return None
    return (M2L_TRAFFIC["fetch_kib"] + M2L_TRAFFIC["write_kib"]) * 1024.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32", "split16", "fp32t64"], default="split16",
                    help="fp32t64: FP32 M2L with FP64 pseudo-inverses and translations")
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--leaf", type=int, default=256)
    ap.add_argument("--sample", type=int, default=40000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--m2l-tol", type=float, default=3e-7, help="shared-basis M2L compression cutoff (FP32); 0 = dense")
    ap.add_argument("--svd-eps", type=float, default=0.0, help="pseudo-inverse cutoff (0: library default)")
    ap.add_argument("--stress-m2l-tol", type=float, default=1e-7,
                    help="M2L compression cutoff of the cantilever's lattice stress (FP32 M2L; 0 = dense)")
    ap.add_argument("--bem-m2l-tol", type=float, default=1e-8,
                    help="M2L compression cutoff of the FP64 BEM products (cantilever, warmstart, metacell; 0 = dense)")
    ap.add_argument("--rows", type=int, default=2000, help="oracle sample for the cantilever workload")
    ap.add_argument("--precond", choices=["none", "two-level", "both"], default="both",
                    help="GMRES preconditioning of the cantilever workload")
    ap.add_argument("--full-residual", action="store_true",
                    help="cantilever: the solution's residual with every row of the product by direct FP64 sums")
    ap.add_argument("--iters", type=int, default=20, help="Algorithm 1 iterations for the warmstart workload")
    ap.add_argument("--measure-from", type=int, default=11)
    ap.add_argument("--p-bem", type=int, default=8, help="expansion order of the BEM solves in the warmstart workload")
    ap.add_argument("--periodic", action="store_true", help="cells workload: periodic metamaterial cells")
    ap.add_argument("--cell-n", type=int, default=100, help="voxels per axis of the metacell workload")
    ap.add_argument("--rc", type=float, default=0.2, help="initial cavity radius of the metacell workload")
    ap.add_argument("--alpha-c", type=float, default=0.7, help="volume fraction of the metacell workload")
    ap.add_argument("--workload", choices=["beam", "sphere", "cells", "cantilever", "warmstart", "metacell"],
                    default="beam",
                    help="beam: the headline line; the others measure the remaining configurations")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only copy one device buffer of this many MiB into another (a plain copy kernel of known "
                         "traffic, to scale the HBM byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU (there is no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy_mib > 0:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": n * 4, "calib_copy_bytes_written": n * 4}))
        return
    if args.workload != "beam":
        import bench_configs
        bench_configs.run(args)
        return

    import numpy as np
    import torch

    from paper_1612_04082_amd import kfmm
    from workloads import geometry as geo

    dev = torch.device("cuda:0")
    prec = {"fp64": kfmm.FP64, "fp32": kfmm.FP32, "split16": kfmm.FP32_M2L_SPLIT16,
            "fp32t64": kfmm.FP32_TRANS64}[args.precision]
    c = geo.box_beam_cloud(seed=2)
    n = c["src"].shape[0]
    t = lambda x: torch.tensor(x, dtype=torch.float64, device=dev)
    src, nrm, w, a, b = t(c["src"]), t(c["nrm"]), t(c["w"]), t(c["a"]), t(c["b"])
    G = 1.0
    K = kfmm.moduli(G, 0.3)
    t0 = time.time()
    plan = kfmm.FmmPlan(src, nrm, w, K=K, G=G, p=args.p, leaf_max=args.leaf, precision=prec, m2l_tol=args.m2l_tol)
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    info = plan.info()
    out = torch.empty((n, 3), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.eval(kfmm.DISP, a, b, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # inside the timed region the library records a pair of HIP events around each M2L launch on its
    # stream (nothing else changes)
    plan.profile("m2l")
    wall0 = time.time()
    e0.record(stream)
    for _ in range(args.steps):
        plan.eval(kfmm.DISP, a, b, out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ms = e0.elapsed_time(e1) / args.steps
    value = n / (ms * 1e-3)
    m2l_timed, m2l_calls = plan.phase_times()
    m2l_ms = m2l_timed["m2l"] / m2l_calls
    plan.profile(False)
    timed_out = out.cpu().numpy()  # the accuracy check below reads the timed loop's own result
    # phase timing: events recorded inside the library on the evaluation stream
    plan.profile(True)
    for _ in range(args.steps):
        plan.eval(kfmm.DISP, a, b, out)
    phases, calls = plan.phase_times()
    plan.profile(False)
    phases = {k: v / calls for k, v in phases.items()}
    work = plan.work(kfmm.DISP, True, True)
    # dominant kernel: the M2L contraction; its roofline is the larger of the algorithmic FLOP at the matrix
    # peak and the algorithmic bytes (operators, input and output vectors, each once) at the HBM peak
    m2l_flops, m2l_bytes = work["m2l"]
    peak_mfma = M2L_TFLOPS[args.precision]
    t_mfma = m2l_flops / (peak_mfma * 1e12)
    t_hbm = m2l_bytes / (HBM_TBS * 1e12)
    m2l_s = m2l_ms * 1e-3
    mfma_view = {"achieved": m2l_flops / m2l_s / 1e12, "peak": peak_mfma, "unit": "TFLOP/s",
                 "frac": t_mfma / m2l_s}
    hbm_view = {"achieved": m2l_bytes / m2l_s / 1e9, "peak": HBM_TBS * 1e3, "unit": "GB/s", "frac": t_hbm / m2l_s}
    main = hbm_view if t_hbm >= t_mfma else mfma_view
    roofline = {"bound": "hbm" if t_hbm >= t_mfma else "mfma",
                "kernel": f"M2L contraction ({KERNELS[args.precision]}, one launch per eval)",
                **main, "traffic": m2l_traffic_bytes(args),
                "flops_per_launch": m2l_flops, "bytes_per_launch": m2l_bytes, "avg_ms": m2l_ms,
                "avg_ms_alone": phases["m2l"], "mfma_view": mfma_view, "hbm_view": hbm_view}
    if args.precision in MFMA_PRODUCTS:
        roofline["mfma_pipe_util"] = MFMA_PRODUCTS[args.precision] * mfma_view["frac"]
    # whole evaluation: T_ideal = sum over phases of each phase's roofline time, against the timed step
    per_phase = {}
    t_ideal = 0.0
    for ph, (fl, by) in work.items():
        ti = ideal_ms(fl, by, phase_peak_tflops(ph, args.precision))
        t_ideal += ti
        if fl or by:
            per_phase[ph] = {"flops": fl, "bytes": by, "ideal_ms": ti, "measured_ms_alone": phases[ph],
                             "frac": ti / phases[ph] if phases[ph] > 0 else None}
    whole = {"t_ideal_ms": t_ideal, "t_measured_ms": ms, "frac": t_ideal / ms, "phases": per_phase,
             "peaks": {"hbm_TBs": HBM_TBS, "valu_TFLOPs": VALU_TFLOPS[args.precision],
                       "translations_TFLOPs": TRANS_TFLOPS[args.precision], "m2l_TFLOPs": peak_mfma}}
    # accuracy on a sample of targets vs the FP64 oracle (also the CPU baseline)
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(n, size=min(args.sample, n), replace=False))
    gpu_out = timed_out[idx]
    cpu_baseline = None
    rel_err = eps_inf = None
    if not args.no_cpu_baseline:
        from oracle import direct as od
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        tc = time.time()
        ref = od.direct(od.DISP, c["src"][idx], c["src"], c["w"], a=c["a"], b=c["b"], nrm=c["nrm"], K=K, G=G,
                        nthreads=cores)
        tcpu = time.time() - tc
        rel_err = float(np.linalg.norm(gpu_out - ref) / np.linalg.norm(ref))
        eps_inf = float(np.abs(gpu_out - ref).max() / np.abs(ref).max())
        pairs = float(len(idx)) * n
        cpu_baseline = {"value": len(idx) / tcpu, "unit": "target points/s", "cores": cores, "kind": "oracle",
                        "sample": f"{len(idx)} targets x {n} sources, FP64 direct sum (C, OpenMP), single + double "
                                  "layer", "seconds": tcpu, "pairs_per_s": pairs / tcpu, "cpu_model": cpu_model()}
    line = {
        "metric": "FMM target points/s at 1e-5 rel err",
        "value": value,
        "unit": "target points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "split16": "f32+f16x2",
                  "fp32t64": "f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "box-beam 120x20x20 surface, 201344 quadrature points, single+double layer "
                               f"displacement, targets=sources, p={args.p}, leaf<={args.leaf}",
                   "n_targets": n, "n_sources": n, "precision": args.precision, "p": args.p, "leaf_max": args.leaf,
                   "m2l_tol": args.m2l_tol, "m2l_rank": info.get("m2l_rank")},
        "rel_err": rel_err,
        "rel_err_source": "output of the timed (overlapped) evaluations",
        "eps_inf": eps_inf,
        "roofline": roofline,
        "roofline_whole_eval": whole,
        "cpu_baseline": cpu_baseline,
        "phases_ms": phases,
        "plan_seconds": plan_s,
        "tree": {k: info[k] for k in ("n_box", "n_leaf", "depth", "n_u_pairs", "n_v_pairs", "n_w_pairs",
                                      "n_x_pairs")},
        "wall_s": wall,
    }
    plan.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
