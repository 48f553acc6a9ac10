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
# FP32 vector peak without packed instructions (the library is built with packed FP32
# disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz = 78.6 TFLOP/s; the
# published 157.3 TFLOP/s counts packed FP32.
VALU_FP32_PEAK_TFLOPS = 78.6
# products with the inverses (npfem_solver_params.inverse_bf16): FP32, dense BF16, banded BF16
PRODUCTS = {"fp32": 0, "bf16": 1, "band": 2}
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


def _cpu_worker(args):
    """One host process of the CPU baseline: oracle steps of its share of the sampled
    cells (first step of the throughput workload) until the deadline."""
    cells, tol, deadline_s = args
    from threadpoolctl import threadpool_limits
    from rbc_inputs import workloads
    import oracle.model as om
    import oracle.step as ostep
    with threadpool_limits(limits=1):
        sub = workloads.throughput(n_cells=100000, cells=cells)
        X, T = sub.meshes[642]
        model = om.Model(X, T, om.Material(), workloads.DT_US)
        model.solve_Ht(np.zeros((642, 3)))
        model.solve_Mt(np.zeros((642, 3)))
        f = workloads.drag_forces(sub, sub.x, sub.v)
        t0 = time.perf_counter()
        done, iters = 0, 0
        for c in range(sub.n_cells):
            s = sub.cell_slice(c)
            _, _, info = ostep.step(model, sub.x[s], sub.v[s], f[s], ostep.Params(tol=tol))
            done += 1
            iters += info.iterations
            if time.perf_counter() - t0 >= deadline_s:
                break
        return done, iters, time.perf_counter() - t0


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(tol: float, seconds: float, max_workers: int = 16):
    """The FP64 oracle as it stands, one process per usable host core (at most
    max_workers), each stepping its own cells of the throughput workload's first step
    for about `seconds`; cells are independent, so the rate is the sum over processes.
    Runs before the GPU is initialised (the worker processes never touch it)."""
    import multiprocessing as mp
    model, n_cpu, usable = host_cpu()
    workers = max(1, min(usable, max_workers))
    per = 4000                                    # more cells than any worker finishes
    jobs = [(np.arange(w, workers * per, workers), tol, seconds) for w in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    rate = sum(r[0] / r[2] for r in res)
    iters = sum(r[1] for r in res) / max(done, 1)
    return {"value": rate, "unit": "cell-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} cells of the 100,000-cell throughput workload's first step, FP64 NumPy/SciPy "
                      f"oracle (residual <= {tol:g}, mean {iters:.1f} iterations), one single-threaded process "
                      f"per core for about {seconds:.0f} s each ({wall:.1f} s wall); host: {model}, "
                      f"{n_cpu} logical CPUs, {usable} usable"}


# ---------------------------------------------------------------------------------
# The other configurations (one JSON line each): --config c1 | c2 | c3
# ---------------------------------------------------------------------------------

def _oracle_step(n_verts, x, v, f, tol=1e-12):
    from rbc_inputs import meshes, workloads
    import oracle.model as om
    import oracle.step as ostep
    X, T = meshes.rbc_mesh(n_verts)
    model = om.Model(X, T, om.Material(), workloads.DT_US)
    xr, vr, info = ostep.step(model, x, v, f, ostep.Params(tol=tol, polish=True))
    return xr, info


def config_c1(args):
    """One 258-vertex cell stretched by +-F (0..200 pN ramp over 200 steps), FP64,
    L-BFGS m = 5; positions against the oracle's trajectory at steps 50/100/150/200."""
    import torch
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_params, CONVERGED
    b = workloads.stretch(258)
    X, T = b.meshes[258]
    D = float(np.ptp(X[:, 0]))
    tol = min(args.tol, 1e-8)                       # the configuration's residual
    plan = Plan([Mesh(X, T)], workloads.DT_US,
                params=default_params(precision="fp64", tol=tol, lbfgs_m=5, noise_factor=64.0))
    batch = Batch(plan, np.zeros(1, np.int32))
    dev = torch.device("cuda:0")
    x = torch.tensor(b.x, dtype=torch.float64, device=dev)
    v = torch.zeros_like(x)
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "c1_stretch_oracle.json")
    if os.path.exists(gpath):
        golden = json.load(open(gpath))
    forces = [torch.tensor(workloads.stretch_forces(b, k, total_steps=200), dtype=torch.float64, device=dev)
              for k in range(1, 201)]
    iters, errs, conv = [], {}, True
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(200)]
    for k in range(1, 201):
        ev[k - 1][0].record()
        x, v, st = batch.step(x, v, forces[k - 1])
        ev[k - 1][1].record()
        s = Batch.stats_to_numpy(st)
        iters.append(int(s["iterations"][0]))
        conv = conv and bool(s["status"][0] == CONVERGED)
        if golden and str(k) in golden["x"]:
            errs[k] = float(np.abs(x.cpu().numpy() - np.array(golden["x"][str(k)])).max() / D)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(e) for a, e in ev]))
    return {"config": "c1", "workload": "stretch: 1 RBC x 258 vertices, +-F ramp 0-200 pN, 200 steps, FP64",
            "value": 1e3 / ms, "unit": "cell-steps/s", "step_ms": ms, "tol": tol,
            "iterations_mean": float(np.mean(iters)), "iterations_max": int(np.max(iters)),
            "all_converged": conv, "max_dx_over_D_vs_oracle": errs,
            "stretched_length_um": float(np.ptp(x.cpu().numpy()[:, 0])),
            "oracle_reference": "tests/golden/c1_stretch_oracle.json (residual 1e-12)" if golden else None}


def config_c2(args):
    """1,024 cells x 642 vertices in drag towards per-cell shear flows, FP32 (BF16
    products), 100 steps; sampled cells of the first step, and of the last step from the
    GPU's own state, against the oracle."""
    import torch
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_params, CONVERGED
    b = workloads.shear(n_cells=1024, seed=1002)
    X, T = b.meshes[642]
    D = float(np.ptp(X[:, 0]))
    plan = Plan([Mesh(X, T)], workloads.DT_US, params=default_params(tol=args.tol, inverse_bf16=PRODUCTS[args.products]))
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    dev = torch.device("cuda:0")
    t = lambda a, dt=torch.float64: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    zeta = torch.full((b.n_cells,), workloads.drag_coefficient(642), dtype=torch.float64, device=dev)
    rate, origin = t(b.shear_rate), t(b.origin)
    x0, v0 = t(b.x, torch.float32), t(b.v, torch.float32)
    # parity of the first step on sampled cells (inputs rounded to FP32 on both sides)
    f0 = batch.drag_forces(x0, v0, zeta, rate, origin)
    x1, _, st = batch.step(x0, v0, f0)
    xin, vin, fin, xo = (a.cpu().numpy().astype(np.float64) for a in (x0, v0, f0, x1))
    tuned = batch.autotune(x0, v0, f0, max_lbfgs_m=5)
    err = 0.0
    for c in (0, 511, 1023):
        sl = b.cell_slice(c)
        xr, _ = _oracle_step(642, xin[sl], vin[sl], fin[sl])
        err = max(err, float(np.abs(xo[sl] - xr).max() / D))
    x, v = x0.clone(), v0.clone()
    xo_, vo_ = torch.empty_like(x), torch.empty_like(v)
    f = torch.empty_like(x)
    from paper_1903_06479_amd import CELL_STATS_DTYPE
    stats = [torch.empty(b.n_cells * CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        batch.drag_forces(x, v, zeta, rate, origin, out=f)
        batch.step(x, v, f, x_out=xo_, v_out=vo_, stats=stats[k])
        x, xo_ = xo_, x
        v, vo_ = vo_, v
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S = [Batch.stats_to_numpy(s) for s in stats]
    it = np.concatenate([s["iterations"] for s in S])
    # the last step's inputs are the buffers swapped out after it
    xin, vin, fin, xo = (a.cpu().numpy().astype(np.float64) for a in (xo_, vo_, f, x))
    err_last = 0.0
    for c in (0, 511, 1023):
        sl = b.cell_slice(c)
        xr, _ = _oracle_step(642, xin[sl], vin[sl], fin[sl])
        err_last = max(err_last, float(np.abs(xo[sl] - xr).max() / D))
    return {"config": "c2", "workload": "shear: 1024 RBCs x 642 vertices, rates U[100,1000]/s, FP32 + BF16 products",
            "value": b.n_cells * args.steps / el, "unit": "cell-steps/s", "steps": args.steps,
            "ms_per_step": 1e3 * el / args.steps, "iterations_mean": float(it.mean()),
            "iterations_p99": float(np.percentile(it, 99)),
            "converged_fraction": float(np.mean(np.concatenate([(s["status"] & CONVERGED) != 0 for s in S]))),
            "first_step_max_dx_over_D_vs_oracle": err, "last_step_max_dx_over_D_vs_oracle": err_last,
            "oracle_cells": [0, 511, 1023],
            "schedule": batch.schedule(), "autotune_best_ms": tuned["best_ms"]}


def config_c3(args):
    """20,000 cells of 258/642/2562 vertices (30/50/20 %), random nodal forces plus
    Poiseuille drag, FP32 bulk (BF16 products) in one persistent launch; each step
    repeated in an all-FP64 plan (every mesh size) on the same inputs; one sampled cell
    of each mesh size against the oracle on the first step."""
    import torch
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_params, CONVERGED
    b = workloads.uneven(n_cells=20000)
    sizes = sorted(b.meshes)
    D = {n: float(np.ptp(b.meshes[n][0][:, 0])) for n in sizes}
    cm = np.array([sizes.index(int(n)) for n in b.cell_nverts], np.int32)
    meshes = [Mesh(*b.meshes[n]) for n in sizes]
    p32 = Plan(meshes, workloads.DT_US, params=default_params(tol=args.tol, inverse_bf16=PRODUCTS[args.products]))
    b32 = Batch(p32, cm)
    p64 = Plan(meshes, workloads.DT_US, params=default_params(precision="fp64", tol=args.tol))
    b64 = Batch(p64, cm)
    dev = torch.device("cuda:0")
    x, v = b.x.astype(np.float32).astype(np.float64), b.v.copy()
    err = {str(n): 0.0 for n in sizes}
    times, iters, conv, conv64 = [], [], [], []
    for k in range(args.c3_steps):
        f = workloads.drag_forces(b, x, v, step=k).astype(np.float32).astype(np.float64)
        xi, vi, fi = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (x, v, f))
        if k == 0:
            b32.autotune(xi, vi, fi, max_lbfgs_m=5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        xo, vo, st = b32.step(xi, vi, fi)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        s = Batch.stats_to_numpy(st)
        iters.append(s["iterations"])
        conv.append((s["status"] & CONVERGED) != 0)
        x32 = xo.cpu().numpy().astype(np.float64)
        # the same inputs (FP32 values) through the all-FP64 plan
        x64, _, s64 = b64.step(*(torch.tensor(a, dtype=torch.float64, device=dev) for a in (x, v, f)))
        conv64.append((Batch.stats_to_numpy(s64)["status"] & CONVERGED) != 0)
        x64 = x64.cpu().numpy()
        e_rows = np.abs(x32 - x64).max(axis=1)
        for i, n in enumerate(sizes):
            rows = np.repeat(cm == i, b.cell_nverts)
            err[str(n)] = max(err[str(n)], float(e_rows[rows].max() / D[n]))
        if k == 0:                      # one cell of each size: the oracle
            for n in sizes:
                c = int(np.nonzero(b.cell_nverts == n)[0][0])
                sl = b.cell_slice(c)
                xr, _ = _oracle_step(n, x[sl], v[sl], f[sl])
                err[f"{n}_vs_oracle_first_step"] = float(np.abs(x32[sl] - xr).max() / D[n])
        x, v = x32, vo.cpu().numpy().astype(np.float64)
        log(f"[c3] step {k + 1}: {times[-1]:.1f} ms")
    it = np.concatenate(iters)
    return {"config": "c3", "workload": "uneven: 20,000 RBCs of 258/642/2562 vertices (30/50/20 %), N(0,10 pN) "
                                        "nodal forces + Poiseuille drag, FP32 bulk + FP64 reductions",
            "value": b.n_cells / (float(np.mean(times)) / 1e3), "unit": "cell-steps/s", "steps": args.c3_steps,
            "step_ms": float(np.mean(times)), "iterations_mean": float(it.mean()),
            "converged_fraction": float(np.mean(np.concatenate(conv))),
            "converged_fraction_fp64": float(np.mean(np.concatenate(conv64))),
            "max_dx_over_D_fp32_vs_fp64_gpu": err, "schedule": b32.schedule()}


def config_solves(args):
    """The constant-matrix solves by four routes on the same right-hand sides: the products
    with the dense inverse in FP32, with its BF16 off-diagonal part (dense and banded in
    the reverse Cuthill-McKee order), and the paper's route, forward and back substitution
    with the banded Cholesky factor of H~ (FP32, on the matrix cores).  3 x 100,000 right-hand sides for the
    642-vertex mesh, 3 x 20,000 for the 2562-vertex one (one per coordinate and cell)."""
    import torch
    from rbc_inputs import meshes, workloads
    from paper_1903_06479_amd import Mesh, Plan, default_params
    dev = torch.device("cuda:0")
    out = {"config": "solves", "unit": "ns per right-hand side", "routes": {}}
    for n, rows in ((642, 300000), (2562, 60000)):
        X, T = meshes.rbc_mesh(n)
        g = torch.Generator(device=dev).manual_seed(n)
        res, ref = {}, None
        for name, mode in (("dense fp32 product", 0), ("dense bf16 product", 1), ("banded bf16 product", 2)):
            plan = Plan([Mesh(X, T)], workloads.DT_US, params=default_params(inverse_bf16=mode))
            npad = plan.n_pad(0)
            q = torch.zeros((rows, npad), dtype=torch.float32, device=dev)
            q[:, :n] = torch.randn((rows, n), generator=g, device=dev)
            g.manual_seed(n)
            o = torch.empty_like(q)
            us = _time_us(lambda: plan.apply_inverse(0, 0, q, o))
            res[name] = us * 1e3 / rows
            if mode == 0:
                ref = o[:4096].clone()
                work = torch.empty(plan.solve_factor_workspace(0, rows), dtype=torch.uint8, device=dev)
                us = _time_us(lambda: plan.solve_factor(0, 0, q, o, work=work))
                b = plan.factor_bandwidth(0)
                res["banded cholesky substitution"] = us * 1e3 / rows
                flops = 4.0 * n * b * rows
                res["substitution_half_bandwidth"] = b
                res["substitution_tflops_4nb"] = flops / us / 1e6
                # FP32 plans run the substitution on the matrix cores: dense FP32 MFMA peak
                res["substitution_frac_of_fp32_mfma_peak"] = flops / us / 1e6 / 157.3
                res["substitution_max_rel_diff_vs_fp32_product"] = float(
                    ((o[:4096] - ref).abs().max() / ref.abs().max()).item())
                del work
            del q, o
            torch.cuda.empty_cache()
        out["routes"][f"n={n}, {rows} right-hand sides"] = res
        log(f"[solves] n={n}: " + ", ".join(f"{k} {v:.3g}" for k, v in res.items()))
    return out


def _time_us(fn, reps=5):
    """Mean time of fn over reps calls after one untimed call, by events on the current
    stream (the stream the library launches on)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3


def elongation_index(lam, lam0, lam_inf):
    """Hochmuth's elongation index of the recovery experiment (eq. ElongationIndex):
    e = (lam - lam_inf)(lam0 + lam_inf) / ((lam + lam_inf)(lam0 - lam_inf))."""
    return (lam - lam_inf) * (lam0 + lam_inf) / ((lam + lam_inf) * (lam0 - lam_inf))


def config_recovery(args):
    """The fluid-free recovery experiment (section 4.2) on one 258-vertex cell, FP64,
    dt = 1 us: held at a stretching load of 50, 100 or 150 pN until steady, then released;
    lam = D_A / D_T (axial over transverse extent) is tracked and the elongation index
    e(t) fitted by exp(-t / t_c) (the printed exponent is garbled; it is read as 1).
    Run with the modified Skalak law (D = 35) and the original one (D = 0)."""
    import torch
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_material, default_params, CONVERGED
    b = workloads.stretch(258)
    X, T = b.meshes[258]
    lam_rest = float(np.ptp(X[:, 0]) / np.ptp(X[:, 1]))
    dt_us, hold, release = 1.0, args.rec_hold, args.rec_release
    dev = torch.device("cuda:0")
    out = {"config": "recovery", "workload": "recovery: 1 RBC x 258 vertices held at +-F on the 5 % end vertices, "
                                            f"then released; FP64, dt = {dt_us} us, {hold} + {release} steps",
           "lam_rest": lam_rest, "runs": []}
    for D in (35.0, 0.0):
        plan = Plan([Mesh(X, T)], dt_us, material=default_material(D=D),
                    params=default_params(precision="fp64", tol=1e-8, noise_factor=64.0))
        batch = Batch(plan, np.zeros(1, np.int32))
        for F in (50.0, 100.0, 150.0):
            x = torch.tensor(X, dtype=torch.float64, device=dev)
            v = torch.zeros_like(x)
            fs = [torch.tensor(workloads.recovery_forces(b, k, F, hold), dtype=torch.float64, device=dev)
                  for k in (1, hold + 1)]
            lam, iters, conv = [], [], True
            t0 = time.perf_counter()
            for k in range(1, hold + release + 1):
                x, v, st = batch.step(x, v, fs[0] if k <= hold else fs[1])
                s = Batch.stats_to_numpy(st)
                iters.append(int(s["iterations"][0]))
                conv = conv and bool(s["status"][0] & CONVERGED)
                xh = x.cpu().numpy()
                lam.append(float(np.ptp(xh[:, 0]) / np.ptp(xh[:, 1])))
            wall = time.perf_counter() - t0
            lam = np.array(lam)
            lam0 = lam[hold - 1]
            e = elongation_index(lam[hold:], lam0, lam_rest)
            t = dt_us * np.arange(1, release + 1)
            win = (e > 0.05) & (e < 0.8)
            tc = float(-1.0 / np.polyfit(t[win], np.log(e[win]), 1)[0]) if win.sum() >= 3 else None
            fit_dev = float(np.abs(e[win] - np.exp(-t[win] / tc)).max()) if tc else None
            out["runs"].append({"D": D, "F_pN": F, "lam_stretched": float(lam0), "hold_drift": float(lam[hold - 1] - lam[hold - 11]),
                                "t_c_us": tc, "max_dev_from_exp_fit": fit_dev,
                                "e_at_us": {str(int(tt)): float(ee) for tt, ee in zip(t, e) if int(tt) in (1, 2, 5, 10, 20, 50, 100, 200, 500)},
                                "iterations_mean": float(np.mean(iters)), "all_converged": conv,
                                "ms_per_step": 1e3 * wall / (hold + release)})
            log(f"[recovery] D={D} F={F}: lam {lam0:.3f}, t_c {tc} us, dev {fit_dev}")
    return out


def oracle_error(b, cells, xin, vin, fin, xout):
    """max |x - x_oracle| / D over the sampled cells: the oracle's stationary point (FP64,
    residual 1e-12) from the same (FP32) inputs the GPU step read."""
    from rbc_inputs import workloads
    import oracle.model as om
    import oracle.step as ostep
    X, T = b.meshes[642]
    model = om.Model(X, T, om.Material(), workloads.DT_US)
    D = float(np.ptp(X[:, 0]))
    err = 0.0
    for c in cells:
        sl = b.cell_slice(int(c))
        xr, _, _ = ostep.step(model, xin[sl], vin[sl], fin[sl], ostep.Params(tol=1e-12, polish=True))
        err = max(err, float(np.abs(xout[sl] - xr).max() / D))
    return err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", default="", choices=["", "c1", "c2", "c3", "recovery", "solves"],
                    help="run one of the other configurations instead of the throughput benchmark")
    ap.add_argument("--c3-steps", type=int, default=5)
    ap.add_argument("--rec-hold", type=int, default=400)
    ap.add_argument("--rec-release", type=int, default=600)
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
    ap.add_argument("--products", default="band", choices=["fp32", "bf16", "band"],
                    help="products with the inverses: FP32, BF16 off-diagonal (dense) or BF16 banded")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1903_06479_amd", "data", "warmstart_642.npy"),
                    help="trained warm-start network (FP32 parameters); empty string: plain form only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU-baseline time per host process")
    ap.add_argument("--oracle-cells", type=int, default=3, help="sampled cells checked against the oracle")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the cells are independent, "
              "so a multi-GPU run would shard them without any per-step exchange", file=sys.stderr)
        sys.exit(2)

    if args.copy_check:
        import torch
        a = torch.ones(args.copy_check // 4, dtype=torch.float32, device="cuda:0")
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": c.numel() * 4}), flush=True)
        return
    if args.config:
        cfg = {"c1": config_c1, "c2": config_c2, "c3": config_c3, "recovery": config_recovery,
               "solves": config_solves}[args.config]
        if args.config == "c2" and args.steps == 20:
            args.steps = 100
        print(json.dumps(cfg(args)), flush=True)
        return

    b = make_inputs(args.cells)
    cpu = None
    if not args.no_cpu_baseline:
        # the host processes are forked before anything initialises the GPU
        t0 = time.time()
        cpu = cpu_baseline(args.tol, args.cpu_seconds)
        log(f"[bench] cpu baseline {time.time() - t0:.1f}s -> {cpu['value']:.1f} cell-steps/s on {cpu['cores']} cores")

    import torch
    from rbc_inputs import workloads
    from paper_1903_06479_amd import Batch, Mesh, Plan, StatsTotal, default_params, CELL_STATS_DTYPE

    X, T = b.meshes[642]
    dev = torch.device("cuda:0")
    # a stream of the default priority: the step is captured into a HIP graph on it (the
    # NULL stream cannot be captured) and replayed on every later step
    stream = torch.cuda.Stream(device=dev)
    params = default_params(tol=args.tol, cells_per_tile=args.cells_per_tile,
                            inverse_bf16=PRODUCTS[args.products])
    t0 = time.time()
    mesh = Mesh(X, T)
    plan = Plan([mesh], workloads.DT_US, params=params)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    log(f"[bench] plan + batch in {time.time() - t0:.1f}s")
    with torch.cuda.stream(stream):
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
        st = torch.empty(b.n_cells * CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    sched = batch.schedule()

    def run_form(form, net=None):
        """Warm-up, reset, then K timed steps of one form; HIP events around each step call
        on the stream the kernels run on.  The per-cell statistics of every timed step are
        accumulated on the GPU (outside the events) and read after the timed region."""
        nonlocal x, v, xo, vo
        total = StatsTotal(dev, stream=stream)

        def one_step(ev=None):
            nonlocal x, v, xo, vo
            batch.drag_forces(x, v, zeta, rate, origin, p["umax"], p["radius"], p["axis_y"], p["axis_z"], out=f)
            if ev is not None:
                ev[0].record(stream)
            if net is None:
                batch.step(x, v, f, x_out=xo, v_out=vo, stats=st, stream=stream)
            else:
                batch.step_learned(net, x, v, f, x_out=xo, v_out=vo, stats=st, stream=stream)
            if ev is not None:
                ev[1].record(stream)
                total.add(st, b.n_cells, stream=stream)
            x, xo = xo, x
            v, vo = vo, v

        with torch.cuda.stream(stream):
            x.copy_(x0)
            v.copy_(v0)
            for _ in range(args.warmup):
                one_step()
            x.copy_(x0)
            v.copy_(v0)
        torch.cuda.synchronize()
        g0 = batch.graph_counts()
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
        t_start = time.perf_counter()
        with torch.cuda.stream(stream):
            for k in range(args.steps):
                one_step(events[k])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        g1 = batch.graph_counts()
        kernel_ms = [a.elapsed_time(e) for a, e in events]
        tot = total.read()
        cs = tot["cell_steps"]
        assert cs == b.n_cells * args.steps, tot
        res = {"value": cs / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
               "step_call_ms": float(np.mean(kernel_ms)),
               "iterations_mean": tot["iterations"] / cs, "iterations_max": tot["max_iterations"],
               "evaluations_mean": tot["evaluations"] / cs, "halvings_mean": tot["halvings"] / cs,
               "converged_fraction": 1.0 - tot["not_converged"] / cs,
               "not_converged_cell_steps": tot["not_converged"],
               "status_counts": dict(zip(("maxiter", "ls_fail", "nonfinite", "degenerate_tri"), tot["status_count"]),
                                     start_fallback=tot["start_fallback"]),
               "max_residual": tot["max_residual"],
               "stats_over": f"all {args.steps} timed steps ({cs} cell-steps)",
               "graph_captures_timed": g1["captures"] - g0["captures"],
               "graph_replays_timed": g1["replays"] - g0["replays"]}
        # the last timed step against the oracle on sampled cells: its inputs are (xo, vo, f)
        # after the final swap, its output x
        if args.oracle_cells > 0:
            ids = np.linspace(0, b.n_cells - 1, args.oracle_cells).round().astype(int)
            xin, vin, fin, xg = (a.cpu().numpy().astype(np.float64) for a in (xo, vo, f, x))
            res["max_dx_over_D_vs_oracle"] = oracle_error(b, ids, xin, vin, fin, xg)
            res["oracle_cells"] = ids.tolist()
        log(f"[bench] {form}: {res}")
        return res

    def eval_roofline():
        """The standalone objective-and-gradient kernel (one evaluation of every cell at
        x_n + u, u a small random displacement), timed alone: algorithmic bytes 48 n per
        cell (x_n, u and b in, the gradient out) plus 24 n for v and F_ext, from which b
        is formed."""
        with torch.cuda.stream(stream):
            u = 1e-3 * torch.randn_like(x0)
            batch.drag_forces(x0, v0, zeta, rate, origin, p["umax"], p["radius"], p["axis_y"], p["axis_z"], out=f)
            batch.eval(x0, v0, f, u, stream=stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
            for a, e in ev:
                a.record(stream)
                batch.eval(x0, v0, f, u, stream=stream)
                e.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(e) for a, e in ev]))
        n = 642
        by = b.n_cells * (48.0 + 24.0) * n
        e32, e64 = eval_flops(n, mesh.nt, mesh.ne)
        fl = b.n_cells * (e32 + 2.0 * e64)
        return {"kernel": "eval_kernel (one objective + gradient evaluation of every cell)", "ms": ms,
                "hbm": {"achieved": by / ms / 1e6, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": by / ms / 1e6 / HBM_PEAK_GBS, "bytes_per_cell": 72.0 * n},
                "alu": {"achieved": fl / ms / 1e9, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": fl / ms / 1e9 / VALU_FP32_PEAK_TFLOPS}}

    forms = {"plain": run_form("plain")}
    if args.weights:
        from paper_1903_06479_amd import Net
        net = Net(plan, np.load(args.weights))
        forms["learned"] = run_form("learned", net)
        # the network's own time (inference alone, same inputs)
        with torch.cuda.stream(stream):
            d = torch.empty_like(x0)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
            for a, e in ev:
                a.record(stream)
                net.infer(batch, x0, v0, f, out=d, stream=stream)
                e.record(stream)
        torch.cuda.synchronize()
        forms["learned"]["net_infer_ms"] = float(np.mean([a.elapsed_time(e) for a, e in ev[1:]]))
        forms["learned"]["weights"] = os.path.relpath(args.weights, ROOT)
    chosen = max(forms, key=lambda k: forms[k]["value"])
    pl = forms["plain"]
    n = 642
    mean_kernel_s = pl["step_call_ms"] / 1e3
    # roofline of the dominant kernel: the step kernel of the plain form.  Algorithmic
    # bytes per cell-step in the streaming form of the method: state in/out 60 n; per
    # iteration the two-loop recursion over the history (4 m 12 n + 36 n) and the
    # product's input and output (24 n); per evaluation x_n, u, b in and the gradient out
    # (48 n).
    I, E = pl["iterations_mean"], pl["evaluations_mean"]
    mh = sched["lbfgs_m"]
    cell_bytes = 60.0 * n + I * (4 * mh * 12 * n + 36 * n + 24 * n) + E * 48.0 * n
    roof = {"bound": "hbm", "achieved": b.n_cells * cell_bytes / mean_kernel_s / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": None, "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"]
    if b.n_cells == 100000 and sched["cells_per_tile"] == 5 and sched["lbfgs_m"] == 2:
        roof["traffic"] = measured_traffic()
    # the same kernel against the vector-arithmetic and matrix-core peaks
    f32, f64, mfma = cell_step_flops(n, mesh.nt, mesh.ne, I, E, mh)
    alu_flops = b.n_cells * (f32 + 2.0 * f64)         # a double flop costs two single ones
    roof_alu = {"achieved": alu_flops / mean_kernel_s / 1e12, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof_alu["frac"] = roof_alu["achieved"] / roof_alu["peak"]
    io_bytes = b.n_cells * 60.0 * n                                  # x, v, f in; x, v out (FP32)
    ch = forms[chosen]
    out = {
        "metric": "RBC cell-steps/sec at residual <=1e-6, plain vs batched+learned warm start",
        "value": ch["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ch["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"throughput: {b.n_cells} RBCs x 642-vertex mesh, shear + Poiseuille drag, "
                               "dt=1e-7 s, FP32 bulk + FP64 reductions", "cells": b.n_cells, "mesh_vertices": n,
                   "form": chosen, "tol": args.tol, "schedule": sched,
                   "inverse_products": {"fp32": "fp32", "bf16": "bf16 off-diagonal + fp32 diagonal",
                                        "band": "banded bf16 off-diagonal (RCM order) + fp32 diagonal"}[args.products],
                   "hip_graph": (not args.no_graph) and ch["graph_replays_timed"] == args.steps},
        "max_dx_over_D_vs_oracle": ch.get("max_dx_over_D_vs_oracle"),
        "forms": forms,
        "roofline": roof,
        "roofline_kernel": "step kernel, plain form",
        "roofline_alu": roof_alu,
        "roofline_eval": eval_roofline(),
        "algorithmic_bytes_per_cell_step": cell_bytes,
        "work_per_cell_step": {"valu_fp32_flops": f32, "valu_fp64_flops": f64, "mfma_flops": mfma,
                               "state_bytes": 60.0 * n},
        "mfma_TFLOPs": b.n_cells * mfma / mean_kernel_s / 1e12,
        "io_GBs": io_bytes / mean_kernel_s / 1e9,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
