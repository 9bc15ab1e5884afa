"""Benchmark of the WENO-TT hot path on one MI355X.

A step is one SSP-RK3 step of WENO-TT (per stage: the Lax-Friedrichs alpha estimated by a search
along grid lines, the role of tt_max_abs in eq. cfl-other; one rank-adaptive cross of the stage
value whose fiber kernel gathers the star stencil from the TT cores and applies Lax-Friedrichs
splitting and WENO5-JS; one TT-rounding; dynamic eps_TT). The default workload is
the 3D tilted Sod problem, 512^3 on [0,1]^3, transmissive, FP64, eps_TT(0) = 1e-6: Sod states
across a plane whose normal is e_x turned by a seeded angle (Sec. 5.5 shapes, eq. cfl-other
time step). dt = 0.5 h / alpha is taken from the state at the start of every step (inside the
timed region). The state evolves through warmup and timed steps from t = 0.

Printed: one JSON line with the dense-equivalent throughput (cells x steps / s), the
roofline of the dominant kernel class measured with HIP events on the library's stream
(with the other classes as a breakdown), the dense GPU WENO5 comparator run with the same
time steps, the L1 error of the density of both against the exact solution at the same time
(on the central box [0.25, 0.75]^3 for the tilted Sod problem) with the equal-L1 check, and the
oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dense-equiv cell-updates/s, WENO-TT vs dense WENO5 on GPU, at fixed L1 error"

PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="cells per dimension (0: the workload's own size)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--workload", default="sod3d_tilted",
                    choices=["sod3d_tilted", "quadrants2d", "wave3d", "sod3d", "blast_batch"],
                    help="sod3d_tilted (512^3) is the contract workload; the others are side measurements")
    ap.add_argument("--batch", type=int, default=32, help="states of the blast_batch workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy three times (the reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--precision", type=int, default=0, help="0 FP64 fiber path, 1 FP32 fiber path")
    ap.add_argument("--scheme", type=int, default=0,
                    help="0 stage cross (the contract line), 1 flux cross per direction, 2 LF-cross + WENO-crosses "
                         "as written in the paper (side measurements)")
    return ap.parse_args()


def cpu_baseline(flow, seconds, slab=64):
    """The oracle as it stands, on the host cores, over a bounded sample: whole steps of the full
    grid in 2D; in 3D whole steps of a slab of `slab` planes across the middle of the first axis
    (the same cells, states and per-cell work; its cut faces transmissive), so that the sample
    stays within the time budget (one oracle step of the full 512^3 grid takes about a minute on
    16 cores and ~30 GB of host memory)."""
    import numpy as np

    import oracle
    from oracle import tt_ref
    oracle.build(force=False)
    n, lo, hi = list(flow.n), list(flow.lo), list(flow.hi)
    cores = flow.cores
    note = ""
    if flow.ndim == 3 and n[0] > slab:
        a = (n[0] - slab) // 2
        h0 = flow.h[0]
        cores = [[comp[0][:, a:a + slab, :]] + list(comp[1:]) for comp in flow.cores]
        lo[0], hi[0], n[0] = flow.lo[0] + a * h0, flow.lo[0] + (a + slab) * h0, slab
        note = f" (planes {a}..{a + slab - 1} of the first axis, cut faces transmissive)"
    u = np.stack([tt_ref.tt_full(c) for c in cores])
    bcs = tuple(oracle.BC_PERIODIC if b == 0 else oracle.BC_TRANSMISSIVE for b in flow.bc)
    if note:
        bcs = (oracle.BC_TRANSMISSIVE,) + bcs[1:]
    P = oracle.Problem(tuple(n), tuple(lo), tuple(hi), bcs, gamma=flow.gamma)
    steps = 0
    t0 = time.perf_counter()
    while True:
        a = P.alpha(u)
        P.ssprk3(u, 0.5 * min(P.h) / a)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 1000:
            break
    cells = 1
    for m in n:
        cells *= m
    cores_used = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells * steps / el, "unit": "cell-updates/s", "cores": cores_used, "kind": "oracle",
            "sample": f"{steps} SSP-RK3 step(s) of the dense FP64 oracle from t=0 on "
                      f"{'x'.join(str(m) for m in n)} cells of the same initial state{note} ({el:.1f} s)"}


CLASS_NAMES = ["k_stage (fused star-stencil LF + WENO5-JS stage-value fiber kernel)",
               "k_prrlu (full-pivot rank-revealing LU of the cross blocks: k_prrlu_tile, k_prrlu_coop, "
               "k_prrlu_mw_step)",
               "k_hhqr (Householder TSQR of the rounding: k_qr_reg, k_hhqr)",
               "k_jacobi_lds (one-sided Jacobi SVD of the rounding)"]
CLASS_KEYS = ["k_stage", "k_prrlu", "k_hhqr", "k_jacobi_lds"]


def trace_mark(torch, dev):
    """A tiny torch kernel (an arange) outside the timed region, before its start and after its
    end, so that a kernel trace of this command can be cut to the timed steps."""
    torch.arange(3, device=dev, dtype=torch.int32)
    torch.cuda.synchronize()


def kernel_source_digest():
    """sha256 over the HIP sources: traffic taken from counters is valid only for these."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2405_12301_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, cls_key):
    """HBM bytes per class launch from the committed counter summary of this workload, or None
    when there is none or the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_digest():
        return None
    c = t.get("classes", {}).get(cls_key)
    return None if c is None else c.get("bytes_per_launch")


def roofline_of(cls_ms, cls_fl, cls_by, cls_n, steps, workload=None):
    ncls = len(cls_ms)
    breakdown = {}
    for i in range(ncls):
        entry = {"ms_per_step": cls_ms[i] / steps, "launches_per_step": cls_n[i] / steps,
                 "avg_launch_us": cls_ms[i] * 1e3 / max(cls_n[i], 1)}
        if cls_fl[i] > 0 and cls_ms[i] > 0:
            entry["tflops"] = cls_fl[i] / (cls_ms[i] * 1e-3) / 1e12
            entry["gbs_algorithmic"] = cls_by[i] / (cls_ms[i] * 1e-3) / 1e9
        breakdown[CLASS_KEYS[i]] = entry
    # dominant kernel: the class with the most device time among those with an algorithmic count
    dom = max((i for i in range(ncls) if cls_fl[i] > 0), key=lambda i: cls_ms[i])
    achieved = cls_fl[dom] / (cls_ms[dom] * 1e-3) / 1e12 if cls_ms[dom] > 0 else 0.0
    traffic = measured_traffic(workload, CLASS_KEYS[dom]) if workload else None
    return {"bound": "alu", "kernel": CLASS_NAMES[dom], "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
            "algorithmic_flops_per_launch": cls_fl[dom] / max(cls_n[dom], 1),
            "algorithmic_bytes_per_launch": cls_by[dom] / max(cls_n[dom], 1),
            "avg_launch_us": cls_ms[dom] * 1e3 / max(cls_n[dom], 1),
            "hbm_frac_algorithmic": cls_by[dom] / (cls_ms[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "breakdown": breakdown}


def blast_batch(args):
    """Side measurement: a batch of independent 3D spherical blasts with seeded grid sizes
    from {64,96,128,192,256}^3, stepped in lock-step by wenott_batch_rk3_step."""
    import torch

    import workloads
    from paper_2405_12301_amd import wenott as W

    W.load()
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    flows = [workloads.config4_blast_3d(seed=args.seed + i) for i in range(args.batch)]
    print(f"# generated {len(flows)} blast states in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    # their crosses stop at the cross-rank limit of 128 with sampled residuals above eps: an
    # explicit slack
    solvers = [W.Solver(f, W.default_opts(eps_mode=1, eps0=f.eps0, conv_slack=100.0)) for f in flows]
    for s in solvers:
        W.wenott_set_profiling(s.ctx, True)
    cells = sum(int(f.n[0]) * int(f.n[1]) * int(f.n[2]) for f in flows)
    hs = [min(f.h) for f in flows]

    def one_step():
        dts = [f.cfl * h / s.max_wavespeed() for f, h, s in zip(flows, hs, solvers)]
        W.wenott_batch_rk3_step([s.ctx for s in solvers], dts)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    ncls = 4
    cls_ms, cls_fl, cls_by, cls_n = [0.0] * ncls, [0.0] * ncls, [0.0] * ncls, [0] * ncls
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step()
        for s in solvers:
            inf = s.info()
            for i in range(ncls):
                cls_ms[i] += inf.class_ms[i]
                cls_fl[i] += inf.class_flops[i]
                cls_by[i] += inf.class_bytes[i]
                cls_n[i] += inf.class_launches[i]
        print(f"# step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ranks = [max(list(s.info().ranks)[:4]) for s in solvers]
    for s in solvers:
        s.close()
    out = {"metric": METRIC, "value": cells * args.steps / el, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"batch of {args.batch} 3D spherical blasts, grids from {{64..256}}^3 "
                                  f"(seeds {args.seed}..{args.seed + args.batch - 1}), transmissive, dynamic eps_TT "
                                  f"from 1e-6, CFL 0.5, lock-step batched stepping",
                      "cells_total": cells, "max_ranks": ranks},
           "roofline": roofline_of(cls_ms, cls_fl, cls_by, cls_n, args.steps)}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        n = 256 * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n * 8, "copies": 3}))
        return
    if args.workload == "blast_batch":
        blast_batch(args)
        return
    single_state(args)


def central_box_l1(rho_dev, flow, t, box):
    """mean |rho - rho_exact| over the cells whose centres lie in box (lo, hi) per dimension."""
    import numpy as np
    n = flow.n[0]
    xs = (np.arange(n) + 0.5) / n
    idx = np.nonzero((xs >= box[0]) & (xs <= box[1]))[0]
    a, b = int(idx[0]), int(idx[-1]) + 1
    got = rho_dev[a:b, a:b, a:b].cpu().numpy()
    return float(np.mean(np.abs(got - flow.exact_rho(t, box=box))))


def single_state(args):
    import numpy as np
    import torch

    import workloads
    from paper_2405_12301_amd import wenott as W

    W.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    box = None
    if args.workload == "sod3d_tilted":
        n = args.n or 512
        flow = workloads.config5_tilted_sod_3d(n, seed=args.seed)
        opts = W.default_opts(eps_mode=1, eps0=flow.eps0, precision=args.precision, scheme=args.scheme)
        box = (0.25, 0.75)
        wl = (f"3D tilted Sod {n}^3 on [0,1]^3 ({flow.note}), transmissive, dynamic eps_TT from 1e-6, CFL 0.5; "
              f"L1 of rho against the exact 1D Sod solution along the normal on [0.25,0.75]^3")
    elif args.workload == "quadrants2d":
        n = args.n or 512
        flow = workloads.config2_quadrants_2d(n, seed=args.seed)
        opts = W.default_opts(eps_mode=1, eps0=flow.eps0, precision=args.precision, scheme=args.scheme)
        wl = (f"four-quadrant Riemann problem 2D {n}x{n}, transmissive, seed {args.seed}, "
              f"dynamic eps_TT from 1e-8, CFL 0.5")
    elif args.workload == "wave3d":
        n = args.n or 256
        flow = workloads.config3_wave_3d(n, seed=args.seed)
        eps_w = 1e-10 if args.precision == 0 else 1e-6
        opts = W.default_opts(eps_mode=0, eps0=eps_w, precision=args.precision, scheme=args.scheme)
        wl = (f"3D smooth density wave {n}^3 with 8 Fourier modes, periodic, eps_TT {eps_w:g} fixed, CFL 0.5; "
              f"L1 error of rho against the exact (translated) solution reported for TT and dense")
    else:
        n = args.n or 256
        flow = workloads.sod_1d_like(3, n)
        opts = W.default_opts(eps_mode=0, eps0=1e-6, precision=args.precision, scheme=args.scheme)
        wl = f"3D Sod shock tube {n}^3 (axis-aligned, rank 1), transmissive, eps_TT 1e-6, CFL 0.5"
    print(f"# workload: {wl}", file=sys.stderr, flush=True)
    cells = 1
    for m in flow.n:
        cells *= m
    h = min(flow.h)
    solver = W.Solver(flow, opts)
    W.wenott_set_profiling(solver.ctx, True)

    dts = []
    for _ in range(args.warmup):
        a = solver.max_wavespeed()
        dts.append(flow.cfl * h / a)
        solver.step(dts[-1])
    torch.cuda.synchronize()
    print(f"# warmup done, ranks {list(solver.info().ranks)[:flow.ndim + 1]}", file=sys.stderr, flush=True)
    ncls = 4
    cls_ms = [0.0] * ncls
    cls_fl = [0.0] * ncls
    cls_by = [0.0] * ncls
    cls_n = [0] * ncls
    trace_mark(torch, dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = solver.max_wavespeed()
        dts.append(flow.cfl * h / a)
        solver.step(dts[-1])
        inf = solver.info()
        for i in range(ncls):
            cls_ms[i] += inf.class_ms[i]
            cls_fl[i] += inf.class_flops[i]
            cls_by[i] += inf.class_bytes[i]
            cls_n[i] += inf.class_launches[i]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    trace_mark(torch, dev)
    t_sim = float(sum(dts))
    info = solver.info()
    ranks = list(info.ranks)[:flow.ndim + 1]
    eps_now = info.eps
    print(f"# timed {args.steps} steps: {el * 1e3 / args.steps:.2f} ms/step, ranks {ranks}", file=sys.stderr,
          flush=True)
    l1 = None
    if flow.exact_rho is not None:
        rho_tt = solver.dense(device=True)[0]
        if box is not None:
            l1 = {"tt": central_box_l1(rho_tt, flow, t_sim, box), "t": t_sim, "box": list(box)}
        else:
            l1 = {"tt": float(np.mean(np.abs(rho_tt.cpu().numpy() - flow.exact_rho(t_sim)))), "t": t_sim}
        del rho_tt
    solver.close()

    roofline = roofline_of(cls_ms, cls_fl, cls_by, cls_n, args.steps,
                           f"{args.workload}_{n}" if args.precision == 0 else None)

    dense = None
    if not args.no_dense:
        # dense GPU WENO5 comparator on the same initial state with the same time steps
        s2 = W.Solver(flow, W.default_opts())
        u0 = s2.dense(device=True)
        s2.close()
        ctx = W.wenott_dense_init(flow.n, flow.lo, flow.hi, flow.gamma, flow.bc)
        for dt in dts[:args.warmup]:
            W.wenott_dense_rk3_step(ctx, u0, dt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for dt in dts[args.warmup:]:
            W.wenott_dense_max_wavespeed(ctx, u0)  # the TT step's dt rule reads alpha too
            W.wenott_dense_rk3_step(ctx, u0, dt)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        W.wenott_dense_destroy(ctx)
        if l1 is not None:
            if box is not None:
                l1["dense"] = central_box_l1(u0[0], flow, t_sim, box)
            else:
                l1["dense"] = float(np.mean(np.abs(u0[0].cpu().numpy() - flow.exact_rho(t_sim))))
            l1["equal_l1"] = bool(l1["tt"] <= 1.05 * l1["dense"])
        del u0
        dense = {"value": cells * args.steps / el2, "unit": "cell-updates/s", "ms_per_step": el2 * 1e3 / args.steps,
                 "note": "hand-written dense FP64 WENO5-JS + LF + SSP-RK3 on the same GPU, the same time steps"}
        print(f"# dense comparator {el2 * 1e3 / args.steps:.2f} ms/step", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": cells * args.steps / el,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32 fiber / f64 rounding",
        "data": "synthetic",
        "config": {"workload": wl,
                   "t_sim_end": t_sim, "ranks": ranks, "eps_tt": eps_now},
        "roofline": roofline,
        "dense_gpu_weno5": dense,
    }
    if dense is not None:
        out["tt_over_dense"] = out["value"] / dense["value"]
    if l1 is not None:
        out["l1_error_vs_exact"] = l1
    if not args.no_cpu_baseline and args.workload in ("sod3d_tilted", "quadrants2d"):
        out["cpu_baseline"] = cpu_baseline(flow, args.cpu_seconds)
    print(json.dumps(out))

if __name__ == "__main__":
    main()
