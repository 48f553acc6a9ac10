"""Membrane energies and their gradients (FP64 oracle, test only).

Each function returns (E, dE/dx) for positions x [n,3] of one cell.  The internal
force of section 2.1 is F_int = -dE/dx.

Readings (paper silent or ambiguous; see the design notes):
  * PD weights carry the factor 1/2, E = (w/2) ||G x - p||^2, which is what the
    expansion into L, J, S in eq. fullyDeveloped_g implies.
  * The SL(2) projection of the area energy is solved directly: with F = U S V^T
    (s1 >= s2 >= 0), the closest S* = diag(t, 1/t) minimises (s1-t)^2 + (s2-1/t)^2,
    whose stationarity condition is t^4 - s1 t^3 + s2 t - 1 = 0; the largest real
    root is the minimiser (tested by brute force).
  * The bending projection R X_g c with R in SO(3) closest to X_f c is the rotation of
    the rest Laplacian onto the current one, so p_i = |l0_i| l_i / |l_i| (the energy
    penalises the change of |l_i|, i.e. of the mean-curvature magnitude).
  * Volume: the projection p = x - C grad C / |grad C|^2 (section 2.1.2) is used with
    the normaliser |grad C|^2 frozen at x_n for the whole step, making the energy
    (k/2) C(x)^2 / G_n and its gradient k C(x) grad C(x) / G_n consistent.  At x = x_n
    this is exactly the paper's PD gradient k (x - p(x)).  The paper's own form, with
    the normaliser taken at the current x (energy (k/2) C^2 / |grad C(x)|^2 and force
    k (x - p(x))), is kept as the `literal` option; its force is not the derivative of
    its energy once C != 0.
  * Global area (optional, off by default): the same construction with the total area
    A(x) in place of the volume, E = (k_A/2) (A - A0)^2 / G_A, G_A = |grad A(x_n)|^2.
  * Collapsed triangles (deformed area below 1e-6 of the rest area) have no second
    in-plane direction (see model.py): the in-plane forces of such a triangle act only
    along its remaining edge direction, and it adds nothing to the area gradient (its
    normal, and the derivative of its area, are undefined).
"""
from __future__ import annotations

import numpy as np

from .model import Model, area_gradient, surface_area, triangle_frames, volume, volume_gradient


def sl2_projection(s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """Largest real root t of t^4 - s1 t^3 + s2 t - 1 (vectorised, s1 >= s2 >= 0)."""
    s1 = np.atleast_1d(np.asarray(s1, np.float64))
    s2 = np.atleast_1d(np.asarray(s2, np.float64))
    comp = np.zeros((len(s1), 4, 4))
    comp[:, 1, 0] = comp[:, 2, 1] = comp[:, 3, 2] = 1.0
    comp[:, 0, 0] = s1          # companion matrix of t^4 - s1 t^3 + 0 t^2 + s2 t - 1
    comp[:, 0, 1] = 0.0
    comp[:, 0, 2] = -s2
    comp[:, 0, 3] = 1.0
    roots = np.linalg.eigvals(comp)
    near_real = np.abs(roots.imag) <= 1e-6 * np.maximum(1.0, np.abs(roots))
    t = np.where(near_real, roots.real, -np.inf).max(axis=1)
    for _ in range(3):          # polish the root with Newton steps on the same polynomial
        f = t ** 4 - s1 * t ** 3 + s2 * t - 1.0
        df = 4 * t ** 3 - 3 * s1 * t ** 2 + s2
        ok = np.abs(df) > 1e-12
        t = np.where(ok, t - f / np.where(ok, df, 1.0), t)
    return t


COLLAPSE_RATIO = 1e-6


def collapsed_triangles(x: np.ndarray, m: Model) -> np.ndarray:
    """Triangles whose deformed area is below COLLAPSE_RATIO of their rest area."""
    a, b, c = x[m.tris[:, 0]], x[m.tris[:, 1]], x[m.tris[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(a - c, b - c), axis=1)
    return area < COLLAPSE_RATIO * m.tri_area


def _deformation(x: np.ndarray, m: Model):
    """F = D_s D_m^-1 in the deformed triangle's own 2D frame (Appendix B) and its SVD."""
    Ds, basis, _ = triangle_frames(x, m.tris, collapsed_triangles(x, m))
    F = Ds @ m.Dm_inv
    U, s, Vt = np.linalg.svd(F)
    return F, U, s, Vt, basis


def _scatter_triangle_grad(m: Model, basis: np.ndarray, dEdF: np.ndarray) -> np.ndarray:
    """Map dE/dF (2x2, deformed frame) to vertex gradients:
    [g_a g_b] = basis (dE/dF) D_m^-T, g_c = -g_a - g_b (section 2.1.3)."""
    H = basis @ dEdF @ np.transpose(m.Dm_inv, (0, 2, 1))     # [nt, 3, 2]
    g = np.zeros((m.n, 3))
    np.add.at(g, m.tris[:, 0], H[:, :, 0])
    np.add.at(g, m.tris[:, 1], H[:, :, 1])
    np.add.at(g, m.tris[:, 2], -H[:, :, 0] - H[:, :, 1])
    return g


def area_energy(x: np.ndarray, m: Model):
    """Local area preservation (section 2.1.2): E_t = (A_t C / 2) ||F - T||_F^2,
    T = U diag(t, 1/t) V^T the closest matrix of determinant one."""
    F, U, s, Vt, basis = _deformation(x, m)
    t = sl2_projection(s[:, 0], s[:, 1])
    Sstar = np.zeros_like(F)
    Sstar[:, 0, 0], Sstar[:, 1, 1] = t, 1.0 / t
    T = U @ Sstar @ Vt
    w = m.tri_area * m.mat.C
    E = 0.5 * np.sum(w * np.sum((F - T) ** 2, axis=(1, 2)))
    return E, _scatter_triangle_grad(m, basis, w[:, None, None] * (F - T))


def skalak_f(lam, B, D):
    return B / 8 * lam ** 4 - B / 4 * lam ** 2 + D / 4 * (lam - 1) ** 4


def skalak_df(lam, B, D):
    return B / 2 * (lam ** 3 - lam) + D * (lam - 1) ** 3


def skalak_energy(x: np.ndarray, m: Model):
    """Modified Skalak material (section 2.1.3): E_t = W_t (f(l1) + f(l2) + B/4),
    f = B/8 l^4 - B/4 l^2 + D/4 (l-1)^4; the constant B/4 makes E(rest) = 0 and
    does not change the force.  P = U diag(f'(l1), f'(l2)) V^T, forces -W_t P D_m^-T."""
    B, D = m.mat.B, m.mat.D
    F, U, s, Vt, basis = _deformation(x, m)
    E = np.sum(m.tri_area * (skalak_f(s[:, 0], B, D) + skalak_f(s[:, 1], B, D) + B / 4))
    Pd = np.zeros_like(F)
    Pd[:, 0, 0], Pd[:, 1, 1] = skalak_df(s[:, 0], B, D), skalak_df(s[:, 1], B, D)
    P = U @ Pd @ Vt
    return E, _scatter_triangle_grad(m, basis, m.tri_area[:, None, None] * P)


def bending_energy(x: np.ndarray, m: Model):
    """Bending (eq. BendingDiscretizedPotential): E_i = (k A_i / 2) |l_i - p_i|^2,
    l = G_bend x (cotangent Laplacian), p_i = |l0_i| l_i / |l_i|."""
    ell = m.G_bend @ x
    nrm = np.linalg.norm(ell, axis=1)
    # |l_i| = 0 leaves the rotation undetermined; p_i = 0 is taken there
    small = nrm <= 1e-30
    p = np.where(small[:, None], 0.0, m.ell0_norm[:, None] * ell / np.where(small, 1.0, nrm)[:, None])
    r = ell - p
    w = m.mat.k_bend * m.vor_area
    E = 0.5 * np.sum(w * np.sum(r * r, axis=1))
    return E, m.G_bend.T @ (w[:, None] * r)


def volume_energy(x: np.ndarray, m: Model, Gn: float | None):
    """Global volume (section 2.1.2): E = (k / 2) C(x)^2 / G_n, C = V - V0,
    gradient k C grad C / G_n with grad C = nbar / 3.  Gn = None: the paper's literal
    form, normaliser |grad C(x)|^2 at the current x and force k C grad C / |grad C(x)|^2
    (= k (x - p(x)), not the derivative of that energy once C != 0)."""
    C = volume(x, m.tris) - m.V0
    gC = volume_gradient(x, m.tris)
    G = float(np.sum(gC ** 2)) if Gn is None else Gn
    return 0.5 * m.mat.k_volume * C * C / G, m.mat.k_volume * C / G * gC


def volume_normaliser(x: np.ndarray, m: Model) -> float:
    return float(np.sum(volume_gradient(x, m.tris) ** 2))


def area_normaliser(x: np.ndarray, m: Model) -> float:
    return float(np.sum(area_gradient(x, m.tris, collapsed_triangles(x, m)) ** 2))


def global_area_energy(x: np.ndarray, m: Model, GA: float):
    """Global area (optional; section 2.1.2 notes it could be built like the volume
    term): E = (k_A / 2) (A - A0)^2 / G_A, gradient k_A (A - A0) grad A / G_A."""
    C = surface_area(x, m.tris) - m.A0
    gA = area_gradient(x, m.tris, collapsed_triangles(x, m))
    return 0.5 * m.mat.k_area_global * C * C / GA, m.mat.k_area_global * C / GA * gA


def elastic_energy(x: np.ndarray, m: Model, Gn: float | None, GA: float | None = None):
    """Sum of the membrane energies and of their gradients, plus the list of the
    individual energies (for the line search's rounding-noise estimate).  The global
    area term enters when k_area_global > 0 (GA its frozen normaliser)."""
    parts = [area_energy(x, m), skalak_energy(x, m), bending_energy(x, m), volume_energy(x, m, Gn)]
    if m.mat.k_area_global > 0:
        parts.append(global_area_energy(x, m, GA))
    return sum(p[0] for p in parts), sum(p[1] for p in parts), [p[0] for p in parts]
