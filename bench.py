#!/usr/bin/env python3
"""Benchmark of the AMG-PCG solve phase on one MI355X.

Default workload (one step = one full solve to rtol 1e-6 from x0 = 0): the
7-point 3D Poisson problem on a 384^3 grid (56.6M unknowns, 395M nonzeros,
b = A x_true with x_true ~ U[0,1) seed 0), FP64 preconditioned CG with the
FP64 AMG V-cycle -- the largest single-GPU configuration, on which plain
FP64, the FP32 V-cycle inside FP64 flexible CG and the learned form are all
run. Each form is timed on the same problem and GPU and checked by its true
FP64 residual.

Printed: one JSON line with the time to solution (ms per step), the HBM
roofline of the dominant kernel, k_spmv_pfuse (the fused CG pass: direction
update, q = A p, deferred x update and p.q), from HIP events recorded on the
library's stream around each of its launches during timed solves (the rest
of the iteration runs back to back; launches issued past convergence, which
exit at entry, are not counted), and the CPU oracle's full solve of the same
problem on the host's cores.

Other workloads (not the headline line): --workload poisson256,
diffusion256 (lognormal coefficients, --az anisotropy), learned128 (collect
pairs, train the network, evaluate on held-out right-hand sides).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

METRIC = "time-to-rtol 1e-6 + SpMV/V-cycle HBM GB/s: FP64 vs mixed vs learned"
NET_FLOP_PER_CELL = 2 * 27 * (16 + 16 * 16 + 16)   # three 3x3x3 layers, 1 -> 16 -> 16 -> 1
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(ROOT, "paper_2406_19754_amd", "weights", "net_poisson128.ckpt")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_poisson384.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(info, form="fp64", fused=False, split=True, dia=True, split_update=True):
    """Algorithmic bytes per launch of the level-0 kernels (each array once, no padding).

    split: smoothing through A M^-1 (pre) and A P (post), the library default.
    dia: A and A M^-1 read from hacked DIA (8 bytes per FP64 entry, 4 per FP32
    entry) instead of hacked ELL (value + 4-byte index), when level 0 has it.
    """
    N = info["rows"][0]
    Z = info["nnz"][0]
    Zp = info["sp_nnz"][0] if info["levels"] > 1 else 0
    Nc = info["rows"][1] if info["levels"] > 1 else 0
    v = 8 if form == "fp64" else 4
    # pair restriction: the pre-smoothing pass also writes N/2 pair sums; the
    # restriction reads them with N/2 entries (value + index) instead of r with N
    pr = bool(info.get("pair_restrict", [0])[0]) and split
    hb = v * N // 2 if pr else 0
    rb = (N // 2) * (v + 4) + v * (N // 2) + v * Nc if pr else N * (v + 4) + v * N + v * Nc
    dia = dia and info["dia_slots"][0] > 0
    a64 = 8 if dia else 12          # the outer operator is always FP64
    av = v if dia else v + 4        # A M^-1 in the V-cycle's precision
    if split:
        # pre: A M^-1, r gathered (fused: r_old and q gathered, r_new written), r_0 written
        pre = (Z * av + 8 * N + v * N if not fused else Z * av + 2 * 8 * N + 8 * N + v * N) + hb
        # post: S P; b (FP64), minv, r_0 read; x_c gathered; z (FP64) written
        post = Zp * (v + 4) + 8 * N + 2 * v * N + v * Nc + 8 * N
    else:
        pre = Z * (v + 4) + 8 * N + v * N + v * N if not fused else Z * (v + 4) + 2 * 8 * N + v * N + 8 * N + v * N
        post = Z * (v + 4) + 8 * N + v * N + v * N + 4 * N + v * Nc + 8 * N
    if fused and split and split_update:
        # pass 2 as two kernels: r = r - alpha q (r_old, q read, r_new written),
        # then r_0 = r_new - (A M^-1) r_new (A M^-1, r_new gathered, r_0 written)
        pre2 = 3 * 8 * N + Z * av + 8 * N + v * N + hb
        return {
            "k_spmv_pfuse": Z * a64 + 2 * 8 * N + 2 * 8 * N + 2 * 8 * N,
            "k_rupdate + k_pre_s": pre2,
            "k_spmv_R": rb,
            "k_post_s": post,
        }
    if fused:
        return {
            # A; z and p_old gathered; p_new, q written; x read and written
            "k_spmv_pfuse": Z * a64 + 2 * 8 * N + 2 * 8 * N + 2 * 8 * N,
            "k_update_pre_s": pre,
            "k_spmv_R": rb,
            "k_post_s": post,
        }
    return {
        "spmv_dot": Z * a64 + 2 * 8 * N,                       # A, p gathered, q written
        "cg_update": 6 * 8 * N,                                # x, r, p, q read; x, r written
        "pre_smooth_l0": pre,
        "restrict_l0": rb,                                     # R (or R2), r_0 (or pair sums) gathered, b_1 written
        "post_smooth_l0": post,
        "dir_update": 3 * 8 * N,                               # z, p read; p written
    }


def mixed_kernel_bytes(info):
    """Algorithmic bytes per launch of the level-0 kernels of the mixed form:
    FP64 FCG(1) with the FP32 V-cycle, its output z kept in FP32, the update
    pass split in two, smoothing through A M^-1 (hacked DIA) and S P."""
    N, Z = info["rows"][0], info["nnz"][0]
    Zp = info["sp_nnz"][0] if info["levels"] > 1 else 0
    Nc = info["rows"][1] if info["levels"] > 1 else 0
    pr = bool(info.get("pair_restrict", [0])[0])
    return {
        # A (FP64); z (FP32), p_old, x, r_old read; p_new, q, x written
        "k_spmv_pfuse_fcg": Z * 8 + 4 * N + 3 * 8 * N + 3 * 8 * N,
        # r_old, q read; r_new (FP64) and its FP32 copy written
        "k_rupdate_r32": 3 * 8 * N + 4 * N,
        # A M^-1 (FP32), r gathered, r_0 written (+ N/2 pair sums)
        "k_pre_s_f32": Z * 4 + 4 * N + 4 * N + (2 * N if pr else 0),
        # R2 over pair sums (N/2 entries of value + index) or R over r_0; b_1 written
        "k_spmv_R_f32": ((N // 2) * 8 + 4 * (N // 2) if pr else N * 8 + 4 * N) + 4 * Nc,
        # S P; minv, b, r_0 (FP32) and q (FP64, for z.q) read; x_c gathered; z (FP32) written
        "k_post_s_f32": Zp * 8 + 3 * 4 * N + 8 * N + 4 * Nc + 4 * N,
    }


def source_hash():
    h = hashlib.sha256()
    for f in ["amg.hip", "kernels.h"]:
        h.update(open(os.path.join(ROOT, "paper_2406_19754_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel, n):
    """Per-launch HBM bytes of `kernel` from committed PMC counters, or None
    when the counters were taken on other kernel sources or another size."""
    try:
        t = json.load(open(TRAFFIC))
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash() or t.get("n") != n:
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def problem(workload, n, az, seed=0):
    from paper_2406_19754_amd import problems as P
    if workload.startswith("diffusion"):
        rp, col, val = P.diffusion7(n, seed=seed, sigma=1.5, az=az)
        desc = (f"3D lognormal diffusion -div(k grad u), FV 7-point, {n}^3, log k ~ N(0,1.5^2) seed {seed}, "
                f"a_z = {az}")
    else:
        rp, col, val = P.poisson7(n)
        desc = f"3D Poisson 7-point {n}^3"
    xt = P.x_true(n ** 3, 0)
    b = P.rhs_from_solution(rp, col, val, xt)
    return rp, col, val, xt, b, desc


def time_configs(args, psc, torch, rp, col, val, bd, x, ms64=None):
    """Time FP64 PCG and mixed FCG(1) with each --configs setting on the
    problem (b = bd); ms64: the headline FP64 time, for the speed-up."""
    forms = {}
    extra = {"smatch": dict(sweeps=3, smoothed_prol=True, smoother_sweeps=4),
             "vmatch": dict(sweeps=3, smoother_sweeps=2, vcycle_double=True),
             "vbm": dict(aggregation=psc.AGGR_VBM, vbm_theta=0.01, smoothed_prol=True, smoother_sweeps=4),
             "ainv": dict(smoother=psc.SMOOTH_AINV, ainv_tau=0.1),
             "invk": dict(smoother=psc.SMOOTH_INVK, invk_fill=0, invk_inv_fill=1),
             "invk00": dict(smoother=psc.SMOOTH_INVK, invk_fill=0, invk_inv_fill=0),
             "cheb1": dict(smoother=psc.SMOOTH_CHEB4, smoother_sweeps=1),
             "cheb2": dict(smoother=psc.SMOOTH_CHEB4, smoother_sweeps=2),
             "cheb3": dict(smoother=psc.SMOOTH_CHEB4, smoother_sweeps=3),
             # the paper's settings with its inexact coarsest solver (at most 40
             # l1-Jacobi PCG iterations), solved with FCG as in the paper
             "smatch_paper": dict(sweeps=3, smoothed_prol=True, smoother_sweeps=4, coarse_pcg_iters=40),
             "vmatch_paper": dict(sweeps=3, smoother_sweeps=2, vcycle_double=True, coarse_pcg_iters=40),
             "vbm_paper": dict(aggregation=psc.AGGR_VBM, vbm_theta=0.01, smoothed_prol=True, smoother_sweeps=4,
                               coarse_pcg_iters=40)}
    for cfg in [c for c in args.configs.split(",") if c]:
        t0 = time.time()
        # Host setup for every configuration hierarchy: one process that had
        # built a device-coarsened hierarchy ended with a host-side SIGSEGV
        # while building a second one with device coarsening (INVK(0,0),
        # 256^3); its cause is not found, so no run builds a second
        # device-coarsened hierarchy in one process.
        hs = psc.Hierarchy(rp, col, val, build_fp32=not args.no_mixed, use_graph=not args.no_graph,
                           setup_device=False,
                           setup_device_products=args.device_products, **extra[cfg])
        infs = hs.info()
        log(f"{cfg} hierarchy {infs['rows']} built in {time.time() - t0:.1f}s, "
            f"opcx {infs['operator_complexity']:.4f}")
        for form in ["fp64"] + ([] if args.no_mixed else ["mixed"]):
            inexact = extra[cfg].get("coarse_pcg_iters", 0) > 0

            def run_s():
                x.zero_()
                if form == "fp64" and not inexact:
                    return hs.pcg(bd, x, rtol=1e-6, maxit=500)
                return hs.fcg(bd, x, rtol=1e-6, maxit=500, prec=psc.FP64 if form == "fp64" else psc.FP32)
            for _ in range(args.warmup):
                run_s()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                rs = run_s()
            torch.cuda.synchronize()
            mss = (time.perf_counter() - t) * 1e3 / args.steps
            # one event-instrumented solve for the V-cycle's bandwidth
            hs.timing(True)
            run_s()
            torch.cuda.synchronize()
            vc_cnt, vc_ms = hs.timing_get()["vcycle"]
            hs.timing(False)
            vb = infs["vcycle_bytes_fp64" if form == "fp64" else "vcycle_bytes_fp32"]
            vgbs = vb / (vc_ms / vc_cnt * 1e-3) / 1e9 if vc_cnt else None
            log(f"{cfg} {form}: {mss:.2f} ms/solve, {rs['iters']} its, relres {rs['relres']:.2e}"
                + (f", V-cycle {vc_ms / vc_cnt:.3f} ms at {vgbs:.0f} GB/s" if vc_cnt else ""))
            forms[cfg + "_" + form] = {"ms": mss, "iters": rs["iters"], "relres": rs["relres"],
                                       "speedup_vs_fp64": ms64 / mss if ms64 else None,
                                       "operator_complexity": infs["operator_complexity"],
                                       "setup_s": infs["setup_seconds"],
                                       "vcycle_ms": vc_ms / vc_cnt if vc_cnt else None, "vcycle_gbs": vgbs}
            if infs["smoother"]:
                forms[cfg + "_" + form]["smoother_nnz_per_row"] = infs["smoother_nnz"][0] / infs["rows"][0]
        hs.close()
    return forms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson384",
                    choices=["poisson256", "poisson384", "diffusion256", "learned128"])
    ap.add_argument("--n", type=int, default=0, help="grid size per axis (default from the workload)")
    ap.add_argument("--az", type=float, default=1.0, help="z anisotropy of the diffusion workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (default: OMP_NUM_THREADS, else every core of the affinity mask)")
    ap.add_argument("--spmv-reps", type=int, default=100)
    ap.add_argument("--grid-max", type=int, default=0, help="workgroup cap of the streaming kernels")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-dia", action="store_true", help="read level operators from hacked ELL only")
    ap.add_argument("--no-dia-uniform", action="store_true",
                    help="hacked DIA with per-slice offset arrays instead of uniform offsets in the kernel argument")
    ap.add_argument("--mixed-fused", action="store_true",
                    help="FP32 V-cycle: fuse the residual update with the level-0 pre-smoothing")
    ap.add_argument("--fused-update", action="store_true",
                    help="FP64 forms: residual update and level-0 pre-smoothing in one pass (PSC_TUNE_FP64_SPLIT = 0)")
    ap.add_argument("--xcd-chunks", action="store_true",
                    help="give each accelerator die a contiguous chunk of the work (default: launch order)")
    ap.add_argument("--tail-rows", type=int, default=-1,
                    help="levels up to this many rows run in one workgroup (0: launch their kernels one by one)")
    ap.add_argument("--coarse-sweeps", type=int, default=30,
                    help="l1-Jacobi sweeps of a coarsest level left by a coarsening stall")
    ap.add_argument("--configs", default="",
                    help="comma-separated extra preconditioner settings to time with the same problem: "
                         "smatch (aggregates <= 8, smoothed prolongator, 4 sweeps), "
                         "vmatch (aggregates <= 8, tentative prolongator, 2 sweeps doubled per level), "
                         "vbm (strength-based aggregation, smoothed prolongator, 4 sweeps), "
                         "ainv (AINV smoother, drop tolerance 0.1), invk (INVK smoother, fill 0, inverse fill 1), "
                         "invk00 (INVK, no inverse fill), cheb1/cheb2/cheb3 (fourth-kind Chebyshev "
                         "polynomial smoother of degree 1/2/3), smatch_paper/vmatch_paper/vbm_paper (the paper's "
                         "settings with at most 40 l1-Jacobi PCG iterations on the coarsest level, FCG)")
    ap.add_argument("--only-configs", action="store_true",
                    help="time only the --configs settings (no headline solve; one JSON line of their results)")
    ap.add_argument("--rebuild-timing", action="store_true",
                    help="time a numeric-only rebuild (new coefficients on the same pattern) against the full "
                         "build, then solve with the rebuilt hierarchy (one JSON line)")
    ap.add_argument("--device-products", action="store_true",
                    help="smoothed-prolongator settings: form their sparse products on the GPU")
    ap.add_argument("--no-split", action="store_true",
                    help="smoothing sweeps gather through A, M^-1 and P instead of A M^-1 and A P")
    ap.add_argument("--unfused", action="store_true", help="one kernel per CG operation instead of the fused PCG iteration")
    ap.add_argument("--train-epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--crops", type=int, default=20000)
    ap.add_argument("--save-weights", default="")
    ap.add_argument("--eval-only", action="store_true",
                    help="learned128: evaluate the shipped weights without collecting pairs or training")
    ap.add_argument("--profile-mix", action="store_true",
                    help="run the kernel mix used for rocprofv3 counter passes: a plain 1 GiB device copy "
                         "(counter calibration), 10 SpMVs on A_0, one FP64 PCG and one mixed FCG solve")
    ap.add_argument("--oracle-child", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the solve path is not sharded across GPUs",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "learned128":
        return learned(args)
    if args.profile_mix:
        return profile_mix(args)
    if args.oracle_child:
        return oracle_child(args)

    import numpy as np
    import torch
    from paper_2406_19754_amd import psc

    n = args.n or {"poisson256": 256, "poisson384": 384, "diffusion256": 256}[args.workload]
    N = n ** 3
    t0 = time.time()
    rp, col, val, xt, b, desc = problem(args.workload, n, args.az)
    log(f"problem {desc} built in {time.time() - t0:.1f}s")
    if args.rebuild_timing:
        t0 = time.time()
        h = psc.Hierarchy(rp, col, val, build_fp32=not args.no_mixed)
        build_s = time.time() - t0
        log(f"hierarchy built in {build_s:.2f}s")
        # new coefficients on the same pattern: the operator scaled row and
        # column by a smooth positive field (s_i a_ij s_j stays SPD)
        sc = 1.0 + 0.5 * np.sin(np.arange(N) * (2 * np.pi / n))
        rows = np.repeat(np.arange(N), np.diff(rp))
        val2 = sc[rows] * val * sc[col]
        t0 = time.time()
        h.rebuild(val2)
        rebuild_s = time.time() - t0
        log(f"numeric rebuild in {rebuild_s:.2f}s ({build_s / rebuild_s:.1f}x faster than the build)")
        import scipy.sparse as sps
        A2 = sps.csr_matrix((val2, col, rp), shape=(N, N))
        bb = A2 @ xt
        bd = torch.from_numpy(bb).cuda()
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            x.zero_()
            h.pcg(bd, x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            x.zero_()
            r = h.pcg(bd, x)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / args.steps
        log(f"pcg on the rebuilt hierarchy: {ms:.2f} ms/solve, {r['iters']} its, relres {r['relres']:.2e}")
        print(json.dumps({"mode": "rebuild", "workload": desc, "build_s": build_s, "rebuild_s": rebuild_s,
                          "rebuild_seconds_lib": h.info()["rebuild_seconds"], "pcg_ms": ms, "iters": r["iters"],
                          "relres": r["relres"]}))
        return
    if args.only_configs:
        bd = torch.from_numpy(b).cuda()
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        forms = time_configs(args, psc, torch, rp, col, val, bd, x)
        print(json.dumps({"mode": "configs", "workload": desc, "steps": args.steps, "warmup": args.warmup,
                          "setup": "host", "forms": forms}))
        return
    t0 = time.time()
    h = psc.Hierarchy(rp, col, val, build_fp32=not args.no_mixed, use_graph=not args.no_graph,
                      coarse_sweeps=args.coarse_sweeps)
    if args.grid_max:
        h.tune(psc.TUNE_GRID_MAX, args.grid_max)
    if args.unfused:
        h.tune(psc.TUNE_FUSED_PCG, 0)
    if args.no_split:
        h.tune(psc.TUNE_SPLIT, 0)
    if args.no_dia:
        h.tune(psc.TUNE_DIA, 0)
    if args.no_dia_uniform:
        h.tune(psc.TUNE_DIA_UNIFORM, 0)
    if args.xcd_chunks:
        h.tune(psc.TUNE_XCD, 1)
    if args.mixed_fused:
        h.tune(psc.TUNE_MIXED_SPLIT, 0)
    if args.fused_update:
        h.tune(psc.TUNE_FP64_SPLIT, 0)
    if args.tail_rows >= 0:
        h.tune(psc.TUNE_TAIL, args.tail_rows)
    info = h.info()
    log(f"hierarchy {info['rows']} built in {time.time() - t0:.1f}s, opcx {info['operator_complexity']:.4f}")
    dev = torch.device("cuda:0")
    bd = torch.from_numpy(b).to(dev)
    x = torch.zeros(N, dtype=torch.float64, device=dev)
    net = None
    if not args.no_learned and os.path.exists(WEIGHTS) and not args.workload.startswith("diffusion"):
        net = psc.Net.load(WEIGHTS)
        net.set_grid((n, n, n))

    def run(form):
        x.zero_()
        if form == "fp64":
            return h.pcg(bd, x, rtol=1e-6, maxit=500)
        if form == "mixed":
            return h.fcg(bd, x, rtol=1e-6, maxit=500, prec=psc.FP32)
        if form == "fcg64":
            return h.fcg(bd, x, rtol=1e-6, maxit=500)
        if form == "learned_mixed":
            return h.fcg(bd, x, rtol=1e-6, maxit=500, net=net, prec=psc.FP32)
        return h.fcg(bd, x, rtol=1e-6, maxit=500, net=net)

    def timed(form, steps, warmup, events):
        """events: 0 graph replay (the headline), 1 HIP events around every
        level-0 kernel, 2 HIP events around the outer SpMV pass only."""
        for _ in range(warmup):
            run(form)
        h.timing(int(events))
        h.timing_get()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = None
        for _ in range(steps):
            res = run(form)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / steps
        kt = h.timing_get()
        h.timing(False)
        return ms, res, kt

    # Timed region: K solves replayed from the captured iteration graph (the
    # headline time to solution); then K solves launched kernel by kernel with
    # HIP events on the library's stream around every level-0 kernel (the
    # per-kernel table; the events add launch gaps, so these solves are not the
    # headline); then K solves with events around the outer SpMV pass only, the
    # rest of each iteration back to back as in a replay (the roofline).
    fused = not args.unfused and info["levels"] > 1
    ms64, r64, _ = timed("fp64", args.steps, args.warmup, False)
    log(f"fp64 pcg: {ms64:.2f} ms/solve, {r64['iters']} its, relres {r64['relres']:.2e}")
    xg = x.cpu().numpy()
    ms64e, r64e, kt64 = timed("fp64", args.steps, 0, 1)
    log(f"fp64 pcg, events around every level-0 kernel: {ms64e:.2f} ms/solve")
    assert r64e["iters"] == r64["iters"]
    ms64r, r64r, kt64r = timed("fp64", args.steps, 0, 2)
    log(f"fp64 pcg, events around the outer SpMV pass only: {ms64r:.2f} ms/solve")
    assert r64r["iters"] == r64["iters"]
    err_true = float(np.linalg.norm(xg - xt) / np.linalg.norm(xt))

    split_update = not args.fused_update and not args.no_split
    kb = kernel_bytes(info, "fp64", fused=fused, split=not args.no_split, dia=not args.no_dia,
                      split_update=split_update)
    tname = ({"spmv_dot": "k_spmv_pfuse", "pre_smooth_l0": "k_rupdate + k_pre_s" if split_update else "k_update_pre_s",
              "restrict_l0": "k_spmv_R", "post_smooth_l0": "k_post_s"} if fused else {})
    kernels = {}
    for name, (cnt, tot) in kt64.items():
        kname = tname.get(name, name)
        if cnt and kname in kb:
            avg = tot / cnt
            kernels[kname] = {"launches": cnt, "avg_ms": avg, "alg_bytes": kb[kname],
                              "gbs": kb[kname] / (avg * 1e-3) / 1e9}
    vc_cnt, vc_ms = kt64["vcycle"]
    vcycle_gbs = info["vcycle_bytes_fp64"] / (vc_ms / vc_cnt * 1e-3) / 1e9 if vc_cnt else None
    # the roofline kernel: the outer SpMV pass, timed alone
    dom = tname.get("spmv_dot", "spmv_dot")
    rc, rt = kt64r["spmv_dot"]
    d = {"launches": rc, "avg_ms": rt / rc, "alg_bytes": kb[dom], "gbs": kb[dom] / (rt / rc * 1e-3) / 1e9}
    log(f"{dom}: {rc} launches, {d['avg_ms'] * 1e3:.1f} us avg, {d['gbs']:.0f} GB/s "
        f"({d['gbs'] / HBM_PEAK_GBS:.3f} of peak)")

    # isolated SpMV loop on A_0 (the same kernel family)
    xs = torch.rand(N, dtype=torch.float64, device=dev)
    ys = torch.empty_like(xs)
    h.spmv(xs, ys)
    h.timing(True)
    h.timing_get()
    for _ in range(args.spmv_reps):
        h.spmv(xs, ys)
    ks = h.timing_get()["spmv_dot"]
    h.timing(0)
    spmv_ms = ks[1] / ks[0]
    spmv_gbs = info["spmv_bytes_fp64"] / (spmv_ms * 1e-3) / 1e9

    forms = {"fp64": {"ms": ms64, "iters": r64["iters"], "relres": r64["relres"],
                      "err_vs_x_true": err_true, "ms_event_instrumented": ms64e,
                      "vcycle_gbs": vcycle_gbs}}
    if not args.no_mixed:
        ms32, r32, _ = timed("mixed", args.steps, args.warmup, False)
        x32 = x.cpu().numpy()
        ms32e, _, kt32 = timed("mixed", args.steps, 0, True)
        log(f"mixed fcg: {ms32:.2f} ms/solve ({ms32e:.2f} instrumented), {r32['iters']} its, "
            f"relres {r32['relres']:.2e}")
        vc_cnt32, vc_ms32 = kt32["vcycle"]
        forms["mixed"] = {"ms": ms32, "ms_event_instrumented": ms32e, "iters": r32["iters"], "relres": r32["relres"],
                          "speedup_vs_fp64": ms64 / ms32,
                          "vcycle_gbs": info["vcycle_bytes_fp32"] / (vc_ms32 / vc_cnt32 * 1e-3) / 1e9
                          if vc_cnt32 else None,
                          "err_vs_fp64_x": float(np.linalg.norm(x32 - xg) / np.linalg.norm(xg))}
        if fused and split_update and not args.no_dia and info["dia_slots"][0] > 0:
            # per-kernel rates of the mixed form's level-0 kernels (its default path)
            kbm = mixed_kernel_bytes(info)
            tm = {"spmv_dot": ("k_spmv_pfuse_fcg",), "pre_smooth_l0": ("k_rupdate_r32", "k_pre_s_f32"),
                  "restrict_l0": ("k_spmv_R_f32",), "post_smooth_l0": ("k_post_s_f32",)}
            km = {}
            for name, parts in tm.items():
                cnt, tot = kt32.get(name, (0, 0.0))
                if cnt:
                    b = sum(kbm[p] for p in parts)
                    km[" + ".join(parts)] = {"launches": cnt, "avg_ms": tot / cnt, "alg_bytes": b,
                                             "gbs": b / (tot / cnt * 1e-3) / 1e9}
                    log(f"mixed {' + '.join(parts)}: {tot / cnt * 1e3:.1f} us avg, "
                        f"{km[' + '.join(parts)]['gbs'] / HBM_PEAK_GBS:.3f} of peak")
            forms["mixed"]["kernels"] = km
    forms.update(time_configs(args, psc, torch, rp, col, val, bd, x, ms64))
    if net is not None:
        # the learned forms run inside FCG(1): its plain FP64 time is their reference
        msf, rf, _ = timed("fcg64", args.steps, args.warmup, False)
        log(f"fp64 fcg (no network): {msf:.2f} ms/solve, {rf['iters']} its, relres {rf['relres']:.2e}")
        forms["fcg64"] = {"ms": msf, "iters": rf["iters"], "relres": rf["relres"], "speedup_vs_fp64": ms64 / msf}
        msl, rl, _ = timed("learned", args.steps, args.warmup, False)
        log(f"learned fcg: {msl:.2f} ms/solve, {rl['iters']} its, relres {rl['relres']:.2e}, "
            f"fallbacks {rl['fallbacks']}")
        forms["learned"] = {"ms": msl, "iters": rl["iters"], "relres": rl["relres"], "fallbacks": rl["fallbacks"],
                            "speedup_vs_fp64": ms64 / msl, "weights": os.path.relpath(WEIGHTS, ROOT)}
        if not args.no_mixed:
            msm, rm, _ = timed("learned_mixed", args.steps, args.warmup, False)
            log(f"learned fcg with FP32 V-cycle: {msm:.2f} ms/solve, {rm['iters']} its, fallbacks {rm['fallbacks']}")
            forms["learned_mixed"] = {"ms": msm, "iters": rm["iters"], "relres": rm["relres"],
                                      "fallbacks": rm["fallbacks"], "speedup_vs_fp64": ms64 / msm}
        forms["learned"]["net_apply"] = net_apply_timing(psc, torch, net, n, dev)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, n, r64, xg, ms64)

    out = {
        "metric": METRIC,
        "value": ms64,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{desc} ({N} unknowns, {info['nnz'][0]} nnz), FP64 PCG + matching-AMG "
                               "V(1,1) l1-Jacobi, aggregates <= 4, rtol 1e-6, b = A x_true, "
                               "x_true ~ U[0,1) seed 0, x0 = 0",
                   "levels": info["levels"], "rows": info["rows"],
                   "operator_complexity": info["operator_complexity"],
                   "setup_s": info["setup_seconds"]},
        "iters": r64["iters"],
        "relres": r64["relres"],
        "spmv_gbs": spmv_gbs,
        "spmv_frac": spmv_gbs / HBM_PEAK_GBS,
        "vcycle_gbs": vcycle_gbs,
        "forms": forms,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["gbs"] / HBM_PEAK_GBS, "traffic": traffic_for(dom, n),
                     "alg_bytes_per_launch": d["alg_bytes"], "avg_ms": d["avg_ms"], "launches": d["launches"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, n, r64, xg, ms64):
    """The CPU oracle (plain C, FP64 CSR) on the same problem: its own
    hierarchy build, then one full PCG solve to rtol 1e-6 from x0 = 0, timed
    with the host clock. Its row loops run on the host threads; dots,
    restrictions and the build are serial. It runs in a child process of its
    own (a fresh interpreter that never touches the GPU and regenerates the
    same seeded problem), so that the GPU process's runtime threads and heap
    play no part in it; a failure there leaves the GPU results standing.
    Also states how far the GPU's FP64 solution is from the oracle's."""
    import subprocess
    import tempfile
    import numpy as np
    threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) \
        or len(os.sched_getaffinity(0))
    base = {"value": None, "unit": "ms", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "gpu_iters": r64["iters"]}
    with tempfile.TemporaryDirectory() as td:
        np.save(os.path.join(td, "x_gpu.npy"), xg)
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", td, "--workload", args.workload,
               "--n", str(n), "--az", repr(args.az), "--cpu-threads", str(threads)]
        try:
            p = subprocess.run(cmd, stdout=subprocess.PIPE, timeout=1500)
        except subprocess.TimeoutExpired:
            log("cpu oracle: its process did not finish within 1500 s; no CPU baseline")
            return dict(base, error="oracle process timed out")
    if p.returncode != 0:
        log(f"cpu oracle: its process ended with status {p.returncode}; no CPU baseline")
        return dict(base, error=f"oracle process ended with status {p.returncode}")
    res = json.loads(p.stdout.decode().strip().splitlines()[-1])
    t_solve, t_setup = res["solve_s"], res["setup_s"]
    return dict(base, value=t_solve * 1e3, cores=res["threads"],
                sample=f"one full oracle PCG solve of the same {n}^3 problem to rtol 1e-6 from x0 = 0 "
                       f"({res['iters']} iterations; row loops on {res['threads']} threads, dots and restrictions "
                       f"serial), in a process of its own; its serial hierarchy build ({t_setup:.1f} s) is "
                       f"excluded like the GPU setup",
                oracle_iters=res["iters"], oracle_relres=res["relres"], oracle_setup_s=t_setup,
                x_gpu_vs_oracle=res["x_gpu_vs_oracle"], gpu_speedup=t_solve * 1e3 / ms64)


def oracle_child(args):
    """The oracle side of cpu_baseline, run as its own process: prints one
    JSON line with the oracle's times, iterations and the distance of the GPU
    solution (saved by the parent) from the oracle's."""
    import numpy as np
    import oracle
    n = args.n
    rp, col, val, xt, b, desc = problem(args.workload, n, args.az)
    oracle.set_threads(args.cpu_threads)
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    o = oracle.Hierarchy(rp, col, val)
    t_setup = time.perf_counter() - t0
    log(f"cpu oracle: hierarchy {o.sizes()} built in {t_setup:.1f}s (serial)")
    t0 = time.perf_counter()
    res = o.pcg(b, rtol=1e-6, maxit=500)
    t_solve = time.perf_counter() - t0
    xo = res["x"]
    xg = np.load(os.path.join(args.oracle_child, "x_gpu.npy"))
    diff = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    log(f"cpu oracle: PCG {res['iters']} its in {t_solve:.1f}s on {threads} threads, relres {res['relres']:.2e}; "
        f"|x_gpu - x_oracle|/|x_oracle| = {diff:.2e}")
    print(json.dumps({"solve_s": t_solve, "setup_s": t_setup, "iters": res["iters"], "relres": res["relres"],
                      "threads": threads, "x_gpu_vs_oracle": diff}), flush=True)


def profile_mix(args):
    import torch
    from paper_2406_19754_amd import psc
    n = args.n or {"poisson256": 256, "poisson384": 384, "diffusion256": 256}.get(args.workload, 384)
    N = n ** 3
    rp, col, val, xt, b, desc = problem(args.workload, n, args.az)
    h = psc.Hierarchy(rp, col, val, build_fp32=True)
    src = torch.rand(2 ** 27, dtype=torch.float64, device="cuda")   # 1 GiB read + 1 GiB written per copy
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    xs = torch.rand(N, dtype=torch.float64, device="cuda")
    ys = torch.empty_like(xs)
    for _ in range(10):
        h.spmv(xs, ys)
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    bd = torch.from_numpy(b).cuda()
    r1 = h.pcg(bd, x)
    x.zero_()
    r2 = h.fcg(bd, x, prec=psc.FP32)
    torch.cuda.synchronize()
    print(json.dumps({"profile_mix": desc, "copy_bytes_read": 2 ** 30, "copy_bytes_written": 2 ** 30,
                      "pcg": r1, "mixed": r2}), flush=True)


def net_apply_timing(psc, torch, net, n, dev, reps=10):
    """One network application z = s net(r/s) on the n^3 grid (psc_net_apply,
    host clock around `reps` calls, each ending in a stream synchronisation;
    the ||r|| reduction included), with the fused kernel and with one kernel
    per layer."""
    N = n ** 3
    r = torch.rand(N, dtype=torch.float64, device=dev) - 0.5
    z = torch.empty_like(r)
    out = {}
    for key, fused in (("per_layer_ms", 0), ("fused_ms", 1)):
        net.tune(psc.NET_TUNE_FUSED, fused)
        net.apply(r, z, (n, n, n))
        t = time.perf_counter()
        for _ in range(reps):
            net.apply(r, z, (n, n, n))
        out[key] = (time.perf_counter() - t) * 1e3 / reps
    out["fused_tflops"] = NET_FLOP_PER_CELL * N / (out["fused_ms"] * 1e-3) / 1e12
    log(f"network application at {n}^3: fused {out['fused_ms']:.2f} ms ({out['fused_tflops']:.0f} TFLOP/s), "
        f"one kernel per layer {out['per_layer_ms']:.2f} ms")
    return out


def learned(args):
    """Collect pairs on 128^3 Poisson, train the network, evaluate on held-out seeds."""
    import numpy as np
    import torch
    from paper_2406_19754_amd import learned as LR
    from paper_2406_19754_amd import problems as P
    from paper_2406_19754_amd import psc
    n = args.n or 128
    rp, col, val = P.poisson7(n)
    h = psc.Hierarchy(rp, col, val, build_fp32=True)
    if args.eval_only:
        # the shipped weights, no data collection or training
        net = psc.Net.load(WEIGHTS)
        losses, v0, v1, t_collect, t_train = np.zeros(0), None, None, 0.0, 0.0
    else:
        t0 = time.time()
        r, z = LR.collect_pairs(h, n, range(1, 65), range(101, 133), crops=args.crops, crop=40, seed=0)
        t_collect = time.time() - t0
        log(f"collected {r.shape[0]} crops in {t_collect:.1f}s")
        net = psc.Net(P.net_init(0))
        t0 = time.time()
        losses, v0, v1 = LR.train(net, r, z, epochs=args.train_epochs, batch=16, margin=3, lr=args.lr, seed=0,
                                  log=log, lr_min=args.lr * 0.02)
        t_train = time.time() - t0
        log(f"trained {len(losses)} steps in {t_train:.1f}s; validation MSE {v0:.4e} -> {v1:.4e}")
        if args.save_weights:
            os.makedirs(os.path.dirname(os.path.abspath(args.save_weights)), exist_ok=True)
            net.save(args.save_weights)
        del r, z
        torch.cuda.empty_cache()
    net.set_grid((n, n, n))
    ev = LR.evaluate(h, net, n, range(1001, 1009), kinds=("uniform",), reps=3)
    # cost of one network application vs one V-cycle on the same grid
    rr = torch.from_numpy(P.rhs_uniform(n ** 3, 5)).cuda()
    zz = torch.empty_like(rr)
    for fn in (lambda: net.apply(rr, zz, (n, n, n)), lambda: h.vcycle(rr, zz)):
        fn()
    t_net = t_vc = 0.0
    for name in ("net", "vc"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(20):
            net.apply(rr, zz, (n, n, n)) if name == "net" else h.vcycle(rr, zz)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) * 1e3 / 20
        t_net, t_vc = (dt, t_vc) if name == "net" else (t_net, dt)
    untrained = psc.Net(P.net_init(0))
    untrained.set_grid((n, n, n))
    ev_u = LR.evaluate(h, untrained, n, range(1001, 1003), kinds=("uniform",), reps=1)
    summary = {
        "workload": f"learned preconditioner, 3D Poisson 7-point {n}^3, held-out RHS U[-1,1] seeds 1001-1008",
        "crops": int(losses.size and args.crops), "collect_s": t_collect, "train_s": t_train,
        "train_steps": int(losses.size), "loss_first": float(losses[:20].mean()) if losses.size else None,
        "loss_last": float(losses[-20:].mean()) if losses.size else None, "val_mse_before": v0, "val_mse_after": v1,
        "pcg_iters": [e["pcg"]["iters"] for e in ev], "learned_iters": [e["learned"]["iters"] for e in ev],
        "pcg_ms": float(np.mean([e["pcg"]["ms"] for e in ev])),
        "learned_ms": float(np.mean([e["learned"]["ms"] for e in ev])),
        "learned_relres": max(e["learned"]["relres"] for e in ev),
        "learned_fallbacks": [e["learned"]["fallbacks"] for e in ev],
        "mixed_ms": float(np.mean([e["mixed"]["ms"] for e in ev])),
        "learned_mixed_ms": float(np.mean([e["learned_mixed"]["ms"] for e in ev])),
        "learned_mixed_iters": [e["learned_mixed"]["iters"] for e in ev],
        "untrained_iters": [e["learned"]["iters"] for e in ev_u],
        "net_apply_ms": t_net, "vcycle_ms": t_vc,
    }
    summary["speedup_learned_vs_pcg"] = summary["pcg_ms"] / summary["learned_ms"]
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
