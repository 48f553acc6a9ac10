"""Training and evaluation of the learned warm start on trajectories the solver itself
generates.  Every arithmetic step runs in the library (drag forces, first guess, the
step, the network's loss, gradient and Adam update); this module only orders the calls
and keeps the trajectories in device memory.

    python -m paper_1903_06479_amd.warmstart --out weights.npy [--epochs E] [--runs R]

trains the network on the shear-flow training workload (1,024 cells of the 642-vertex
mesh per run, shear rates U[50, 2000] 1/s, runs 0..R-1, 50 steps each), keeps the
parameters of the epoch with the lowest loss on the validation runs 150.., evaluates
them on the held-out runs 100..103 and writes the FP32 parameters.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import _native as N
from .solver import Batch, Mesh, Net, Plan, default_net_config, default_params


class Flow:
    """Per-cell drag towards shear + Poiseuille flow (the fluid's stand-in), on the GPU."""

    def __init__(self, batch: Batch, zeta, rate, origin, poiseuille=None):
        import torch
        dev = torch.device("cuda", batch.plan.device)
        t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float64), device=dev)
        self.batch = batch
        self.zeta, self.rate, self.origin = t(zeta), t(rate), t(origin)
        p = poiseuille or {"umax": 0.0, "radius": 1.0, "axis_y": 0.0, "axis_z": 0.0}
        self.p = (p["umax"], p["radius"], p["axis_y"], p["axis_z"])

    def forces(self, x, v, out=None):
        return self.batch.drag_forces(x, v, self.zeta, self.rate, self.origin, *self.p, out=out)


def collect(batch: Batch, flow: Flow, x0, v0, steps: int):
    """Run the plain solver for `steps` steps from (x0, v0); per step keep x_n, v_n, f,
    the converged x_{n+1} and the first guess u0 = y_n - x_n (device tensors)."""
    import torch
    traj = {k: [] for k in ("x", "v", "f", "x_next", "u0")}
    x, v = x0.clone(), v0.clone()
    iters = []
    for _ in range(steps):
        f = flow.forces(x, v)
        u0 = batch.first_guess(x, v, f)
        xn, vn, st = batch.step(x, v, f)
        iters.append(float(batch.stats_to_numpy(st)["iterations"].mean()))
        for k, t in (("x", x), ("v", v), ("f", f), ("x_next", xn), ("u0", u0)):
            traj[k].append(t)
        x, v = xn, vn
    torch.cuda.synchronize()
    traj["iterations"] = iters
    return traj


def dataset_loss(net: Net, batch: Batch, trajs: list, minibatch: int = 256) -> dict:
    """The loss over every (step, cell) sample of the trajectories, without an update: the
    mean over all samples, over the first steps (from the perturbed rest shapes) and over
    the later steps."""
    import torch
    dev = trajs[0]["x"][0].device
    n = batch.n_cells
    grad = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    sums = {"first": [0.0, 0], "later": [0.0, 0]}
    for tr in trajs:
        for s in range(len(tr["x"])):
            part = sums["first" if s == 0 else "later"]
            for c0 in range(0, n, minibatch):
                k = min(minibatch, n - c0)
                cells = torch.arange(c0, c0 + k, dtype=torch.int32, device=dev)
                loss, _ = net.loss_grad(batch, tr["x"][s], tr["v"][s], tr["f"][s], tr["x_next"][s], tr["u0"][s],
                                        cells=cells, grad=grad)
                part[0] += loss * k
                part[1] += k
    tot = sums["first"][0] + sums["later"][0]
    cnt = sums["first"][1] + sums["later"][1]
    return {"mean": tot / cnt, "first": sums["first"][0] / max(1, sums["first"][1]),
            "later": sums["later"][0] / max(1, sums["later"][1])}


def train(net: Net, batch: Batch, trajs: list, epochs: int, minibatch: int = 256, lr: float = 1e-3,
          lr_final: float = 1e-4, seed: int = 0, log=None, val: list | None = None):
    """Adam over (step, cell subset) minibatches of every trajectory, with the learning rate
    decaying geometrically from lr to lr_final.  With validation trajectories `val`, their
    whole loss is computed after every epoch and the network ends with the parameters of
    the best epoch.  Returns one record per epoch: the mean of the training losses sampled
    during the epoch and, with `val`, the validation losses."""
    import torch
    rng = np.random.default_rng(seed)
    dev = trajs[0]["x"][0].device
    n = batch.n_cells
    samples = [(r, s) for r in range(len(trajs)) for s in range(len(trajs[r]["x"]))]
    per_epoch = len(samples) * ((n + minibatch - 1) // minibatch)
    total = epochs * per_epoch
    history = []
    best = (np.inf, None, -1)
    it = 0
    for ep in range(epochs):
        t0 = time.time()
        losses = []
        for si in rng.permutation(len(samples)):
            r, s = samples[si]
            tr = trajs[r]
            perm = rng.permutation(n).astype(np.int32)
            for c0 in range(0, n, minibatch):
                cells = torch.tensor(perm[c0:c0 + minibatch], dtype=torch.int32, device=dev)
                want = (it % 50) == 0
                loss, g = net.loss_grad(batch, tr["x"][s], tr["v"][s], tr["f"][s], tr["x_next"][s], tr["u0"][s],
                                        cells=cells, want_loss=want)
                if want:
                    losses.append(loss)
                rate = lr * (lr_final / lr) ** (it / max(1, total - 1))
                net.adam_step(g, lr=rate)
                it += 1
        torch.cuda.synchronize()
        rec = {"epoch": ep + 1, "train_sampled": float(np.mean(losses))}
        if val:
            vl = dataset_loss(net, batch, val, minibatch)
            rec.update({"val": vl["mean"], "val_first": vl["first"], "val_later": vl["later"]})
            if vl["mean"] < best[0]:
                best = (vl["mean"], net.get_params(), ep + 1)
        history.append(rec)
        if log:
            log(f"[train] epoch {ep + 1}/{epochs}: {rec} ({time.time() - t0:.1f}s)")
    if best[1] is not None:
        net.set_params(best[1])
        if log:
            log(f"[train] kept the parameters of epoch {best[2]} (validation loss {best[0]:.4e})")
    return history


def compare(batch: Batch, net: Net, traj: dict, diameter: float, g_rel: float = 1e-6):
    """Plain and learned steps from the same states of a held-out trajectory: iterations,
    convergence, the position difference relative to the cell diameter and, where the two
    end more than 1e-5 D apart (different stationary points of a non-convex objective),
    whether the learned one has the higher objective g (beyond g_rel |g|)."""
    import torch
    it_p, it_l, dx, conv, fb = [], [], [], [], 0
    higher, lower = 0, 0
    off = batch.offsets
    for s in range(len(traj["x"])):
        x, v, f = traj["x"][s], traj["v"][s], traj["f"][s]
        xp, _, sp = batch.step(x, v, f)
        xl, _, sl = batch.step_learned(net, x, v, f)
        sp, sl = batch.stats_to_numpy(sp), batch.stats_to_numpy(sl)
        it_p.append(sp["iterations"].astype(np.float64))
        it_l.append(sl["iterations"].astype(np.float64))
        conv.append(bool(np.all(sp["status"] & N.CONVERGED) and np.all(sl["status"] & N.CONVERGED)))
        fb += int(np.sum((sl["status"] & N.START_FALLBACK) != 0))
        d = (xl - xp).abs().amax(dim=1).cpu().numpy()          # per vertex
        dcell = np.maximum.reduceat(d, off[:-1]) / diameter     # per cell
        dx.append(dcell)
        if np.any(dcell > 1e-5):
            _, tp = batch.eval(x, v, f, xp - x)
            _, tl = batch.eval(x, v, f, xl - x)
            gp, gl = tp[:, 0].cpu().numpy(), tl[:, 0].cpu().numpy()
            far = dcell > 1e-5
            higher += int(np.sum(far & (gl > gp + g_rel * np.abs(gp))))
            lower += int(np.sum(far & (gl <= gp + g_rel * np.abs(gp))))
    torch.cuda.synchronize()
    it_p, it_l, dx = np.concatenate(it_p), np.concatenate(it_l), np.concatenate(dx)
    return {"iterations_plain": float(it_p.mean()), "iterations_learned": float(it_l.mean()),
            "iterations_plain_p99": float(np.percentile(it_p, 99)),
            "iterations_learned_p99": float(np.percentile(it_l, 99)),
            "all_converged": all(conv), "max_dx_over_D": float(dx.max()),
            "median_dx_over_D": float(np.median(dx)),
            "cell_steps_dx_above_1e-5": int(np.sum(dx > 1e-5)),
            "dx_above_1e-5_learned_objective_higher": higher,
            "dx_above_1e-5_learned_objective_lower": lower,
            "start_fallback": fb,
            "first_step_max_dx_over_D": float(dx[:batch.n_cells].max()),
            "cell_steps": int(it_p.size)}


def init_params(config, seed: int = 0) -> np.ndarray:
    """He-style initial weights (zero biases, output layer scaled by 0.1), FP32, in the
    parameter order of the C ABI: W_e, b_e, per layer W_s, W_n, b, then W_d, b_d."""
    H, L = config.hidden, config.layers
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(H * 12) * np.sqrt(2.0 / 12), np.zeros(H)]
    for _ in range(L):
        parts += [rng.standard_normal(H * H) * np.sqrt(1.0 / H), rng.standard_normal(H * H) * np.sqrt(1.0 / H),
                  np.zeros(H)]
    parts += [rng.standard_normal(3 * H) * np.sqrt(1.0 / H) * 0.1, np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


def main(argv=None):
    import torch
    from rbc_inputs import workloads                # seeded synthetic workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--weights", default="", help="evaluate these FP32 parameters instead of training")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--runs", type=int, default=4)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--val-runs", type=int, default=1, help="validation runs 150.. (model selection)")
    ap.add_argument("--eval-runs", type=int, default=4)
    ap.add_argument("--eval-steps", type=int, default=10)
    ap.add_argument("--minibatch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--target-tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    b0 = workloads.training(0, n_cells=args.cells)
    X, T = b0.meshes[642]
    mesh = Mesh(X, T)
    cm = np.zeros(args.cells, np.int32)
    D = float(np.ptp(X[:, 0]))

    cfg = default_net_config()
    history, t_train = [], 0.0
    if args.weights:
        theta = np.load(args.weights)
    else:
        # training trajectories: FP64 solver, targets converged to target_tol
        plan64 = Plan([mesh], workloads.DT_US, params=default_params(precision="fp64", tol=args.target_tol))
        batch64 = Batch(plan64, cm)
        trajs = []
        t0 = time.time()
        for r in range(args.runs):
            b = workloads.training(r, n_cells=args.cells)
            flow = Flow(batch64, np.full(args.cells, workloads.drag_coefficient(642)), b.shear_rate, b.origin,
                        b.poiseuille)
            x, v = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (b.x, b.v))
            trajs.append(collect(batch64, flow, x, v, args.steps))
            log(f"[data] run {r}: {args.steps} steps, mean iterations {np.mean(trajs[-1]['iterations']):.2f} "
                f"({time.time() - t0:.1f}s)")
        val = []
        for r in range(args.val_runs):
            b = workloads.training(150 + r, n_cells=args.cells)
            flow = Flow(batch64, np.full(args.cells, workloads.drag_coefficient(642)), b.shear_rate, b.origin,
                        b.poiseuille)
            x, v = (torch.tensor(a, dtype=torch.float64, device=dev) for a in (b.x, b.v))
            val.append(collect(batch64, flow, x, v, args.steps))
            log(f"[data] validation run {150 + r}: {args.steps} steps ({time.time() - t0:.1f}s)")
        net64 = Net(plan64, init_params(cfg, args.seed), cfg)
        t0 = time.time()
        history = train(net64, batch64, trajs, args.epochs, args.minibatch, args.lr, args.lr_final, args.seed, log,
                        val=val)
        t_train = time.time() - t0
        theta = net64.get_params()
        if args.out:
            np.save(args.out, theta)
        del trajs, val
        torch.cuda.empty_cache()

    # held-out evaluation in the FP32 configuration of the throughput runs
    plan32 = Plan([mesh], workloads.DT_US, params=default_params(tol=1e-6, inverse_bf16=1))
    batch32 = Batch(plan32, cm)
    net32 = Net(plan32, theta, cfg)
    results = []
    for r in range(args.eval_runs):
        b = workloads.training(100 + r, n_cells=args.cells)
        flow = Flow(batch32, np.full(args.cells, workloads.drag_coefficient(642)), b.shear_rate, b.origin, b.poiseuille)
        x, v = (torch.tensor(a, dtype=torch.float32, device=dev) for a in (b.x, b.v))
        tr = collect(batch32, flow, x, v, args.eval_steps)
        results.append(compare(batch32, net32, tr, D))
        log(f"[eval] run {100 + r}: {results[-1]}")
    summary = {
        "train": {"runs": args.runs, "steps": args.steps, "cells": args.cells,
                  "samples": args.runs * args.steps * args.cells, "epochs": args.epochs,
                  "validation": {"runs": args.val_runs, "steps": args.steps},
                  "per_epoch": history, "seconds": t_train},
        "heldout": {
            "cells": args.eval_runs * args.cells, "steps": args.eval_steps,
            "iterations_plain": float(np.mean([r["iterations_plain"] for r in results])),
            "iterations_learned": float(np.mean([r["iterations_learned"] for r in results])),
            "max_dx_over_D": float(max(r["max_dx_over_D"] for r in results)),
            "cell_steps_dx_above_1e-5": int(sum(r["cell_steps_dx_above_1e-5"] for r in results)),
            "dx_above_1e-5_learned_objective_higher": int(sum(r["dx_above_1e-5_learned_objective_higher"]
                                                              for r in results)),
            "start_fallback": int(sum(r["start_fallback"] for r in results)),
            "first_step_max_dx_over_D": float(max(r["first_step_max_dx_over_D"] for r in results)),
            "all_converged": all(r["all_converged"] for r in results)},
    }
    print(json.dumps(summary), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
