"""The npFEM time step of one cell (FP64 oracle, test only): Algorithm 1.

  x^(1)  = x_n + h M~^-1 M v_n + h^2 M~^-1 F_ext          (first guess, eq. preOptimizationNewton)
  repeat: d = -H_k grad g(x^(k))                          (L-BFGS, Nocedal & Wright Alg. 7.4,
                                                           initial Hessian H~)
          alpha = 1, 1/2, 1/4 ... until sufficient decrease (line search)
  v_{n+1} = (x_{n+1} - x_n) / h, then the dissipation of section 2.1.4.

The objective is eq. GeneralizedObjectiveFunction,
  g(x) = 1/(2h^2) tr((x - y)^T M~ (x - y)) + sum E(x),
and its gradient eq. GeneralizedObjectiveFunctionDerivative,
  grad g(x) = M~ (x - y) / h^2 + grad E(x).

Readings where the paper is silent (see the design notes):
  * Convergence: r = |grad g| / (|M u / h^2| + |b| + |grad g - M u / h^2 + b| + B sqrt(A0))
    <= tol, with u = x - x_n, b = M v_n / h + F_ext (2-norms over all 3n entries) and
    the force floor B sqrt(A0) (Skalak modulus times the size of the rest membrane,
    which keeps r meaningful for a cell at rest).  The scale is the size of the terms
    that balance at the solution, so r does not depend on where the iteration started.
  * Line search: accept alpha when g decreases by at least c1 alpha grad g . d, up to
    the rounding noise of evaluating g (8 eps times the sum of the absolute values of
    its terms).  Halving alone cannot enforce the curvature condition, which only
    decides whether the (s, y) pair is stored (s . y > 1e-12 |s| |y|).
  * The L-BFGS history is cleared at every time step.  When 30 halvings fail, the
    history is cleared and the iteration retried with d = -H~^-1 grad g; if that also
    fails the step stops with status LS_FAIL.
  * The step's result is defined as the stationary point grad g = 0 (eq.
    GeneralizedObjectiveFunctionDerivative).  Near it, the decrease of g per iteration
    falls below the FP64 resolution of g itself long before grad g stops shrinking, so
    the Armijo test fails at residuals of 1e-9..1e-7 on a stretched cell.  With
    Params.polish the iteration then continues with the same L-BFGS directions but
    accepts a step when the residual (the scaled |grad g|) decreases; this reaches
    residual 1e-12 in a few iterations and is how the parity reference is computed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .model import Model
from .collision import collision_energy
from .energy import area_normaliser, collapsed_triangles, elastic_energy, volume_normaliser

CONVERGED, MAXITER, LS_FAIL, NONFINITE, DEGENERATE_TRI = 1, 2, 4, 8, 16


@dataclass
class Params:
    tol: float = 1e-6
    m: int = 5
    max_iter: int = 200
    max_halvings: int = 30
    c1: float = 1e-4
    noise_factor: float = 8.0
    polish: bool = False        # continue on residual decrease once Armijo stops (see above)
    max_polish: int = 100


@dataclass
class StepInfo:
    iterations: int = 0
    evaluations: int = 0
    residual: float = np.inf
    status: int = 0
    objective: float = 0.0
    history: list = field(default_factory=list)
    polish_iterations: int = 0


class Objective:
    """g, grad g and the residual of one step (fixed x_n, v_n, F_ext).  literal: the
    volume term with the paper's normaliser at the current x instead of at x_n."""

    def __init__(self, m: Model, x_n, v_n, f_ext, literal: bool = False, contacts=None):
        """contacts: None or (q, nrm, w_col), the collision term of collision.py with the
        partner positions q and normals nrm (cell-local) found at the start of the step."""
        self.m, self.x_n = m, np.asarray(x_n, np.float64)
        self.contacts = contacts
        h = m.h
        self.b = m.mass[:, None] * np.asarray(v_n, np.float64) / h + np.asarray(f_ext, np.float64)
        # y_n = x_n + h M~^-1 M v_n + h^2 M~^-1 F_ext = x_n + h^2 M~^-1 b
        self.y = self.x_n + h * h * m.solve_Mt(self.b)
        self.Gn = None if literal else volume_normaliser(self.x_n, m)
        self.GA = area_normaliser(self.x_n, m) if m.mat.k_area_global > 0 else None
        self.evaluations = 0

    def __call__(self, x):
        """Returns (g, grad g, rounding-noise scale of g)."""
        self.evaluations += 1
        m, h = self.m, self.m.h
        dx = x - self.y
        Mdx = m.Mt @ dx
        inertia = 0.5 * np.sum(dx * Mdx) / h ** 2
        E, gE, parts = elastic_energy(x, m, self.Gn, self.GA)
        if self.contacts is not None:
            Ec, gc = collision_energy(x, *self.contacts)
            E, gE, parts = E + Ec, gE + gc, parts + [Ec]
        grad = Mdx / h ** 2 + gE
        noise = abs(inertia) + sum(abs(p) for p in parts)
        return inertia + E, grad, noise

    def residual(self, x, grad) -> float:
        num = np.linalg.norm(grad)
        if num == 0.0:
            return 0.0
        Mu = self.m.mass[:, None] * (x - self.x_n) / self.m.h ** 2
        floor = self.m.mat.B * np.sqrt(self.m.tri_area.sum())
        den = np.linalg.norm(Mu) + np.linalg.norm(self.b) + np.linalg.norm(grad - Mu + self.b) + floor
        return num / den


def lbfgs_direction(grad, S, Y, rho, solve_H0):
    """Two-loop recursion (Nocedal & Wright Alg. 7.4) with H0^-1 = H~^-1."""
    q = grad.copy()
    alpha = []
    for s, y, r in zip(reversed(S), reversed(Y), reversed(rho)):
        a = r * np.sum(s * q)
        q -= a * y
        alpha.append(a)
    z = solve_H0(q)
    for s, y, r, a in zip(S, Y, rho, reversed(alpha)):
        bta = r * np.sum(y * z)
        z += s * (a - bta)
    return -z


def minimise(obj: Objective, x0, p: Params):
    """Quasi-Newton minimisation of g from x0 (Algorithm 1, the while loop)."""
    eps = np.finfo(np.float64).eps
    x = np.array(x0, np.float64)
    g, grad, noise = obj(x)
    info = StepInfo()
    info.residual = obj.residual(x, grad)
    if info.residual <= p.tol:
        info.status = CONVERGED
    S, Y, rho = [], [], []
    while not info.status and info.iterations < p.max_iter:
        d = lbfgs_direction(grad, S, Y, rho, obj.m.solve_Ht)
        gd = np.sum(grad * d)
        alpha, accepted = 1.0, False
        for _ in range(p.max_halvings + 1):
            xt = x + alpha * d
            gt, gradt, noiset = obj(xt)
            if gt <= g + p.c1 * alpha * gd + p.noise_factor * eps * max(noise, noiset):
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            if S:                      # retry with the plain preconditioned gradient
                S, Y, rho = [], [], []
                continue
            info.status = LS_FAIL
            break
        _store_pair(S, Y, rho, xt - x, gradt - grad, p.m)
        x, g, grad, noise = xt, gt, gradt, noiset
        info.iterations += 1
        info.residual = obj.residual(x, grad)
        info.history.append(info.residual)
        if info.residual <= p.tol:
            info.status = CONVERGED
    if p.polish and info.status != CONVERGED:
        x, g = _polish(obj, x, g, grad, p, info)
    if not info.status:
        info.status = MAXITER
    if np.any(collapsed_triangles(x, obj.m)):
        info.status |= DEGENERATE_TRI
    info.evaluations = obj.evaluations
    info.objective = g
    return x, info


def _store_pair(S, Y, rho, s, y, m):
    """Keep (s, y) when the curvature s . y is positive (relative to |s| |y|); at most
    the m newest pairs."""
    sy = np.sum(s * y)
    if sy > 1e-12 * np.linalg.norm(s) * np.linalg.norm(y):
        S.append(s), Y.append(y), rho.append(1.0 / sy)
        if len(S) > m:
            S.pop(0), Y.pop(0), rho.pop(0)


def _polish(obj: Objective, x, g, grad, p: Params, info: StepInfo):
    """Continue towards grad g = 0 once the Armijo test on g can no longer resolve
    progress: the same L-BFGS directions (initial Hessian H~, fresh history), the step
    halved until the residual decreases."""
    S, Y, rho = [], [], []
    r = info.residual
    for _ in range(p.max_polish):
        if r <= p.tol:
            break
        d = lbfgs_direction(grad, S, Y, rho, obj.m.solve_Ht)
        alpha, accepted = 1.0, False
        for _ in range(p.max_halvings + 1):
            xt = x + alpha * d
            gt, gradt, _ = obj(xt)
            rt = obj.residual(xt, gradt)
            if rt < r:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            if S:
                S, Y, rho = [], [], []
                continue
            break
        _store_pair(S, Y, rho, xt - x, gradt - grad, p.m)
        x, g, grad, r = xt, gt, gradt, rt
        info.polish_iterations += 1
        info.history.append(r)
    info.residual = r
    if r <= p.tol:
        info.status = CONVERGED
    return x, g


def dissipate(x, v, mass, kappa):
    """Post-convergence dissipation (section 2.1.4, after Mueller et al. 2007): damp
    the part of v that differs from the best-fit rigid motion by the factor kappa."""
    m = mass[:, None]
    M = mass.sum()
    x_cm = np.sum(m * x, axis=0) / M
    v_cm = np.sum(m * v, axis=0) / M
    r = x - x_cm
    Lang = np.sum(np.cross(r, m * v), axis=0)
    I = np.zeros((3, 3))
    for ri, mi in zip(r, mass):
        rt = np.array([[0, -ri[2], ri[1]], [ri[2], 0, -ri[0]], [-ri[1], ri[0], 0]])
        I += mi * rt @ rt.T
    omega = np.linalg.solve(I, Lang)
    dv = v_cm + np.cross(omega, r) - v
    return v + kappa * dv


def step(m: Model, x_n, v_n, f_ext, p: Params = Params(), x_start=None, literal: bool = False, contacts=None):
    """One npFEM step of one cell: returns (x_{n+1}, v_{n+1}, info)."""
    obj = Objective(m, x_n, v_n, f_ext, literal, contacts)
    x0 = obj.y if x_start is None else np.asarray(x_start, np.float64)
    x, info = minimise(obj, x0, p)
    v = (x - obj.x_n) / m.h
    v = dissipate(x, v, m.mass, m.mat.kappa)
    return x, v, info
