"""Benchmark: RBC cell-steps per second at residual <= 1e-6 on one MI355X.

Workload (default): the throughput configuration -- 100,000 red blood cells on the
642-vertex biconcave mesh, each randomly rotated with a Gaussian perturbation of its
initial positions (sigma = 2 % of the radius), driven by Stokes drag towards a per-cell
linear shear flow (rate U[100, 1000] 1/s) plus a Poiseuille profile across a cube sized
for 40 % volume fraction; dt = 1e-7 s, FP32 arithmetic with FP64 reductions.  The
inputs are synthetic and seeded (no dataset); the forces are recomputed every step
from the current state by a drag kernel, as a fluid solver would hand them over.

A step is one npFEM time step of every cell (Algorithm 1 of the paper: first guess,
L-BFGS iterations with the H~^-1 product on the matrix cores, line search, velocity
update, dissipation), with every cell converged to residual <= 1e-6.  Two forms are
timed on the same inputs and schedule: plain (start from the first guess y_n) and
learned (start from y_n + the correction predicted by the trained warm-start network,
inference included in the step); `value` is the faster one ("form" in the config).

    python bench.py [--steps K] [--warmup W] [--cells C] [--weights W.npy] [--no-cpu-baseline]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_FP32_PEAK_TFLOPS = 157.3  # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
N_CU = 256

# Algorithmic arithmetic of one objective + gradient evaluation, counted operation by
# operation from its formulas (add, mul, div, sqrt = 1 flop, fused multiply-add = 2):
# per directed edge 21 (curvature vectors) + 9 (bending gradient), per triangle corner
# 6 (gather), per triangle 237 single + 116 double (strain, SL(2) projection with three
# Newton steps, Skalak, corner gradients, energies, volume), per vertex 120 (of which 60
# in double: inertia, norms, residual sums).
EVAL_FP32_PER = {"dir_edge": 30, "corner": 6, "tri": 237, "vert": 60}
EVAL_FP64_PER = {"tri": 116, "vert": 60}


def eval_flops(n, nt, ne):
    f32 = EVAL_FP32_PER["dir_edge"] * 2 * ne + EVAL_FP32_PER["corner"] * 3 * nt + \
        EVAL_FP32_PER["tri"] * nt + EVAL_FP32_PER["vert"] * n
    f64 = EVAL_FP64_PER["tri"] * nt + EVAL_FP64_PER["vert"] * n
    return f32, f64


def measured_traffic():
    """HBM bytes per step launch from the committed counter summary, or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "step_kernel_throughput_100k_642.md")
    if not os.path.exists(prof):
        return None
    kv = {}
    for line in open(prof):
        if ":" in line and not line.startswith(" "):
            k, _, v = line.partition(":")
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ("npfem_kernels.hip", "npfem_internal.h"):
        with open(os.path.join(ROOT, "paper_1903_06479_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if kv.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def cell_step_flops(n, nt, ne, iters, evals, m):
    """(VALU FP32, VALU FP64, matrix-core) flops of one cell-step with the given mean
    iteration and evaluation counts: evaluations, the two-loop recursion and the
    iterate/history updates (8m + 10 flops per unknown per iteration), the dissipation
    (about 50 double flops per vertex), and (I + 1) products with the n x n inverses."""
    e32, e64 = eval_flops(n, nt, ne)
    f32 = evals * e32 + iters * (8 * m + 10) * 3 * n
    f64 = evals * e64 + 50 * n
    mfma = (iters + 1) * 2.0 * n * n * 3
    return f32, f64, mfma


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(n_cells: int):
    from rbc_inputs import workloads
    t0 = time.time()
    b = workloads.throughput(n_cells=n_cells) if n_cells == 100000 else \
        workloads.throughput(n_cells=100000, cells=np.arange(n_cells))
    log(f"[bench] generated {n_cells} cells in {time.time() - t0:.1f}s")
    return b


def cpu_baseline(b, n_sample: int, tol: float):
    """The FP64 oracle, as it stands, on the first n_sample cells for one step."""
    from threadpoolctl import threadpool_limits
    from rbc_inputs import workloads
    import oracle.model as om
    import oracle.step as ostep
    X, T = b.meshes[642]
    model = om.Model(X, T, om.Material(), workloads.DT_US)
    sl = slice(0, int(b.offsets[n_sample]))
    f = workloads.drag_forces(b, b.x, b.v)
    with threadpool_limits(limits=1):
        model.solve_Ht(np.zeros((642, 3)))
        model.solve_Mt(np.zeros((642, 3)))
        t0 = time.perf_counter()
        iters = []
        for c in range(n_sample):
            s = b.cell_slice(c)
            _, _, info = ostep.step(model, b.x[s], b.v[s], f[s], ostep.Params(tol=tol))
            iters.append(info.iterations)
        dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} cells of the 100,000-cell throughput workload, first step, "
                      f"FP64 NumPy/SciPy oracle, residual <= {tol:g}, one thread "
                      f"({dt:.1f}s, mean {np.mean(iters):.1f} iterations)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=100000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--cells-per-tile", type=int, default=0)
    ap.add_argument("--lbfgs-m", type=int, default=0, help="history length when not autotuned (0: plan default)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-check", type=int, default=0,
                    help="only copy a buffer of this many bytes 5 times (calibrates the HBM byte counters)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--fp32-products", action="store_true", help="FP32 instead of BF16 products with the inverses")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1903_06479_amd", "data", "warmstart_642.npy"),
                    help="trained warm-start network (FP32 parameters); empty string: plain form only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=320)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the cells are independent, "
              "so a multi-GPU run would shard them without any per-step exchange", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_check:
        a = torch.ones(args.copy_check // 4, dtype=torch.float32, device="cuda:0")
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": c.numel() * 4}), flush=True)
        return
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_params, CONVERGED

    b = make_inputs(args.cells)
    X, T = b.meshes[642]
    dev = torch.device("cuda:0")
    params = default_params(tol=args.tol, cells_per_tile=args.cells_per_tile,
                            inverse_bf16=0 if args.fp32_products else 1)
    t0 = time.time()
    mesh = Mesh(X, T)
    plan = Plan([mesh], workloads.DT_US, params=params)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    log(f"[bench] plan + batch in {time.time() - t0:.1f}s")
    x0 = torch.tensor(b.x, dtype=torch.float32, device=dev)
    v0 = torch.zeros_like(x0)
    zeta = torch.full((b.n_cells,), workloads.drag_coefficient(642), dtype=torch.float64, device=dev)
    rate = torch.tensor(b.shear_rate, dtype=torch.float64, device=dev)
    origin = torch.tensor(b.origin, dtype=torch.float64, device=dev)
    p = b.poiseuille
    x, v, f = x0.clone(), v0.clone(), torch.empty_like(x0)
    tuned = None
    if not args.no_autotune:
        batch.drag_forces(x, v, zeta, rate, origin, p["umax"], p["radius"], p["axis_y"], p["axis_z"], out=f)
        t0 = time.time()
        tuned = batch.autotune(x, v, f, max_lbfgs_m=5)
        log(f"[bench] autotune {time.time() - t0:.1f}s -> {tuned}")
    elif args.cells_per_tile or args.lbfgs_m:
        batch.schedule(cells_per_tile=args.cells_per_tile or None, lbfgs_m=args.lbfgs_m or None)
    if not args.no_graph:
        batch.set_graph(True)
    xo, vo = torch.empty_like(x0), torch.empty_like(x0)
    st = torch.empty(b.n_cells * 40, dtype=torch.uint8, device=dev)
    sched = batch.schedule()

    def run_form(form, net=None):
        """Warm-up, reset, then K timed steps of one form; HIP events around each step call
        (on the stream the kernels run on)."""
        nonlocal x, v, xo, vo

        def one_step(ev=None):
            nonlocal x, v, xo, vo
            batch.drag_forces(x, v, zeta, rate, origin, p["umax"], p["radius"], p["axis_y"], p["axis_z"], out=f)
            if ev is not None:
                ev[0].record()
            if net is None:
                batch.step(x, v, f, x_out=xo, v_out=vo, stats=st)
            else:
                batch.step_learned(net, x, v, f, x_out=xo, v_out=vo, stats=st)
            if ev is not None:
                ev[1].record()
            x, xo = xo, x
            v, vo = vo, v

        x.copy_(x0)
        v.copy_(v0)
        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        x.copy_(x0)
        v.copy_(v0)
        torch.cuda.synchronize()
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
        t_start = time.perf_counter()
        for k in range(args.steps):
            one_step(events[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kernel_ms = [a.elapsed_time(e) for a, e in events]
        s = Batch.stats_to_numpy(st)                    # last step (read after timing)
        res = {"value": b.n_cells * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
               "step_call_ms": float(np.mean(kernel_ms)),
               "iterations_mean": float(np.mean(s["iterations"])), "iterations_max": int(np.max(s["iterations"])),
               "evaluations_mean": float(np.mean(s["evaluations"])),
               "converged_fraction": float(np.mean((s["status"] & CONVERGED) != 0))}
        log(f"[bench] {form}: {res}")
        return res

    forms = {"plain": run_form("plain")}
    if args.weights:
        from paper_1903_06479_amd import Net
        net = Net(plan, np.load(args.weights))
        forms["learned"] = run_form("learned", net)
        # the network's own time (inference alone, same inputs)
        d = torch.empty_like(x0)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, e in ev:
            a.record()
            net.infer(batch, x0, v0, f, out=d)
            e.record()
        torch.cuda.synchronize()
        forms["learned"]["net_infer_ms"] = float(np.mean([a.elapsed_time(e) for a, e in ev[1:]]))
        forms["learned"]["weights"] = os.path.relpath(args.weights, ROOT)
    chosen = max(forms, key=lambda k: forms[k]["value"])
    pl = forms["plain"]
    n = 642
    mean_kernel_s = pl["step_call_ms"] / 1e3
    # roofline of the dominant kernel: the step kernel of the plain form
    I, E = pl["iterations_mean"], pl["evaluations_mean"]
    f32, f64, mfma = cell_step_flops(n, mesh.nt, mesh.ne, I, E, sched["lbfgs_m"])
    # vector arithmetic in FP32-equivalent flops: a double flop costs two single ones
    alu_flops = b.n_cells * (f32 + 2.0 * f64)
    io_bytes = b.n_cells * 60.0 * n                                  # x, v, f in; x, v out (FP32)
    roof = {"bound": "alu", "achieved": alu_flops / mean_kernel_s / 1e12, "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": None, "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"]
    if b.n_cells == 100000 and sched["cells_per_tile"] == 5 and sched["lbfgs_m"] == 2:
        roof["traffic"] = measured_traffic()
    ch = forms[chosen]
    out = {
        "metric": "RBC cell-steps/sec at residual <=1e-6, plain vs batched+learned warm start",
        "value": ch["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ch["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"throughput: {b.n_cells} RBCs x 642-vertex mesh, shear + Poiseuille drag, "
                               "dt=1e-7 s, FP32 bulk + FP64 reductions", "cells": b.n_cells, "mesh_vertices": n,
                   "form": chosen, "tol": args.tol, "schedule": sched,
                   "inverse_products": "fp32" if args.fp32_products else "bf16 off-diagonal + fp32 diagonal",
                   "hip_graph": not args.no_graph},
        "forms": forms,
        "roofline": roof,
        "roofline_kernel": "step kernel, plain form",
        "work_per_cell_step": {"valu_fp32_flops": f32, "valu_fp64_flops": f64, "mfma_flops": mfma,
                               "state_bytes": 60.0 * n},
        "mfma_TFLOPs": b.n_cells * mfma / mean_kernel_s / 1e12,
        "io_GBs": io_bytes / mean_kernel_s / 1e9,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(b, args.cpu_sample, args.tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
