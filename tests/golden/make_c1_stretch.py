"""Writes c1_stretch_oracle.json: the FP64 oracle's trajectory of the stretched cell
(one 258-vertex cell, +-F ramped 0..200 pN over 200 steps on the 5 % end vertices,
dt = 0.1 us), every step taken to its stationary point (residual <= 1e-12, with the
residual-decrease continuation once the Armijo test stops resolving g), with the
positions at steps 50, 100, 150 and 200 and the residual and status of every step.
Calls only the oracle and the seeded input generators.

    python tests/golden/make_c1_stretch.py      (about 15 minutes on one core)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from rbc_inputs import workloads          # noqa: E402
import oracle.model as om                 # noqa: E402
import oracle.step as ostep               # noqa: E402

STEPS = 200
CHECK = (50, 100, 150, 200)
TOL = 1e-12


def main():
    b = workloads.stretch(258)
    X, T = b.meshes[258]
    model = om.Model(X, T, om.Material(), workloads.DT_US)
    x, v = b.x.copy(), b.v.copy()
    out = {"description": __doc__.strip().splitlines()[0], "steps": STEPS, "tol": TOL,
           "iterations": [], "polish_iterations": [], "residual": [], "status": [], "x": {}}
    t0 = time.time()
    for k in range(1, STEPS + 1):
        f = workloads.stretch_forces(b, k, total_steps=STEPS)
        x, v, info = ostep.step(model, x, v, f, ostep.Params(tol=TOL, polish=True))
        if info.status != ostep.CONVERGED:
            raise RuntimeError(f"step {k} did not reach residual {TOL:g}: {info.residual:.3e}")
        out["iterations"].append(int(info.iterations))
        out["polish_iterations"].append(int(info.polish_iterations))
        out["residual"].append(float(info.residual))
        out["status"].append(int(info.status))
        if k in CHECK:
            out["x"][str(k)] = x.tolist()
        print(f"step {k}: {info.iterations} + {info.polish_iterations} iterations, residual "
              f"{info.residual:.2e} ({time.time() - t0:.0f}s)", flush=True)
    out["length_x_final"] = float(np.ptp(x[:, 0]))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_stretch_oracle.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
