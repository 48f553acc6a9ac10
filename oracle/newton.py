"""Brute-force Newton solve of grad g = 0 with a finite-difference Jacobian
(FP64 oracle, test only).

An independent route to the stationary point that Algorithm 1 converges to: no
L-BFGS, no H~, no line search.  The Jacobian of grad g is built column by column
from central differences of the gradient, so the cost is O(n) gradient evaluations
per Newton iteration and this is meant for the 12- and 42-vertex meshes only.
"""
from __future__ import annotations

import numpy as np

from .step import Objective


def newton_solve(obj: Objective, x0, tol: float = 1e-13, max_iter: int = 50, fd_step: float = 1e-6):
    x = np.array(x0, np.float64)
    n3 = x.size
    for _ in range(max_iter):
        _, grad, _ = obj(x)
        if obj.residual(x, grad) <= tol:
            return x, True
        J = np.zeros((n3, n3))
        for j in range(n3):
            e = np.zeros(n3)
            e[j] = fd_step
            gp = obj(x + e.reshape(x.shape))[1].ravel()
            gm = obj(x - e.reshape(x.shape))[1].ravel()
            J[:, j] = (gp - gm) / (2 * fd_step)
        J = 0.5 * (J + J.T)
        x = x - np.linalg.solve(J, grad.ravel()).reshape(x.shape)
    _, grad, _ = obj(x)
    return x, obj.residual(x, grad) <= tol
