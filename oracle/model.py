"""Rest data and constant matrices of one membrane mesh (FP64 oracle, test only).

Readings of the paper taken here (each is listed with its reason in the design notes):
  * Triangle reference frame: Appendix B builds D_m from the edges towards the third
    vertex, D_m = [X1 - X3, X2 - X3], in the triangle's own 2D frame.
  * Bending: the cotangent weights are (cot a + cot b) / 2 divided by the vertex area,
    the vertex area being the mixed Voronoi area of Meyer et al. (2003); the paper
    says "Voronoi area" without more detail (section 2.1.2, eq. BendingDiscretizedPotential).
  * Mass: the body's total mass rho * V0 is lumped on the vertices in proportion to
    their barycentric area (section 2.1, "weighting based on the area per vertex").
  * L = sum_i w_i G_i^T G_i (eq. fullyDeveloped_g) over the projective-dynamics
    elements: area triangles (w = A_t C), bending vertices (w = A_i k_b), the volume
    element (G = I, w = k_volume) and, when it is switched on, the global-area element
    (G = I, w = k_area_global), built like the volume one (section 2.1.2 says global
    area conservation could be imposed by the same approach; off by default).
  * A triangle whose deformed area is below 1e-6 of its rest area is taken as
    collapsed: its frame has no second in-plane direction (the direction normal to the
    collapse is undefined), so that direction carries no force.
  * Rayleigh damping C = beta_D L' with alpha_D = 0 (section 2.1.4), where L' is L
    without the volume identity so that rigid translations are not damped, and
    beta_D = beta * h (beta given in units of the time step).  Hence
    M~ = M + h C = M + beta h^2 L'.
  * H~ = M~ / h^2 + L + K_mat (section 2.1.1), n x n, shared by the three coordinates,
    where K_mat = sum_t A_t k_mat G_t^T G_t is the optional material contribution to
    the Hessian approximation (section 2.1.1, non-PD energies); it changes only the
    preconditioner, never the solution.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg


@dataclass
class Material:
    """Membrane material.  Defaults: the parameter reading used by the workloads
    (shear modulus 5.3 pN/um -> Skalak B = 2 mu_s; area stiffness 100 mu_s)."""
    B: float = 10.6          # Skalak B (pN/um)
    C: float = 530.0         # local area PD stiffness (pN/um)
    D: float = 35.0          # Skalak correction (pN/um)
    k_bend: float = 0.2      # bending (pN um)
    k_volume: float = 250.0  # global volume PD weight (pN/um)
    beta: float = 0.01       # Rayleigh beta_D in units of the time step
    kappa: float = 0.6       # post-convergence dissipation
    density: float = 1100.0  # fg / um^3
    k_mat: float | None = None  # material stiffness added to H~ (None -> B)
    k_area_global: float = 0.0  # global-area PD weight (pN/um); 0 = off, as in the paper

    @property
    def k_mat_value(self) -> float:
        return self.B if self.k_mat is None else self.k_mat


def triangle_frames(x: np.ndarray, tris: np.ndarray, collapsed=None):
    """Each triangle (a, b, c) isometrically embedded in its own 2D frame.

    Returns (D [nt,2,2], basis [nt,3,2], area [nt]) with D = [x_a - x_c, x_b - x_c]
    expressed in the orthonormal frame basis = [e1, e2], e1 along x_a - x_c and
    e2 = n x e1 in the triangle's plane (n the unit normal), so det D = 2 * area >= 0.
    Triangles flagged in `collapsed` get e2 = 0 (no second in-plane direction).
    """
    e1v = x[tris[:, 0]] - x[tris[:, 2]]
    e2v = x[tris[:, 1]] - x[tris[:, 2]]
    cr = np.cross(e1v, e2v)
    crn = np.linalg.norm(cr, axis=1, keepdims=True)
    area = 0.5 * crn[:, 0]
    l1 = np.linalg.norm(e1v, axis=1, keepdims=True)
    t1 = e1v / np.where(l1 > 0, l1, 1.0)
    nrm = cr / np.where(crn > 0, crn, 1.0)
    t2 = np.cross(nrm, t1)
    if collapsed is not None:
        t2[collapsed] = 0.0
    basis = np.stack([t1, t2], axis=2)                      # [nt, 3, 2]
    D = np.einsum("tik,tij->tkj", basis, np.stack([e1v, e2v], axis=2))
    return D, basis, area


def vertex_neighbours(n: int, tris: np.ndarray) -> list[list[int]]:
    nb = [set() for _ in range(n)]
    for a, b, c in tris:
        nb[a] |= {b, c}
        nb[b] |= {a, c}
        nb[c] |= {a, b}
    return [sorted(s) for s in nb]


def cotangent_weights(X: np.ndarray, tris: np.ndarray) -> dict:
    """omega_ij = (cot alpha_ij + cot beta_ij) / 2 for every undirected edge (i < j),
    alpha and beta being the angles opposite the edge in its two triangles."""
    w: dict[tuple[int, int], float] = {}
    for t in tris:
        for k in range(3):
            i, j, o = t[k], t[(k + 1) % 3], t[(k + 2) % 3]
            u, v = X[i] - X[o], X[j] - X[o]
            cot = np.dot(u, v) / np.linalg.norm(np.cross(u, v))
            key = (min(i, j), max(i, j))
            w[key] = w.get(key, 0.0) + 0.5 * cot
    return w


def mixed_voronoi_areas(X: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Meyer et al. (2003) mixed Voronoi area of every vertex."""
    A = np.zeros(len(X))
    for t in tris:
        P = X[t]
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        ang = []
        for k in range(3):
            u, v = P[(k + 1) % 3] - P[k], P[(k + 2) % 3] - P[k]
            ang.append(np.arccos(np.clip(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v), -1, 1)))
        obtuse = [a > np.pi / 2 for a in ang]
        for k in range(3):
            if not any(obtuse):
                j, l = (k + 1) % 3, (k + 2) % 3
                A[t[k]] += (np.sum((P[k] - P[j]) ** 2) / np.tan(ang[l])
                            + np.sum((P[k] - P[l]) ** 2) / np.tan(ang[j])) / 8.0
            elif obtuse[k]:
                A[t[k]] += area / 2.0
            else:
                A[t[k]] += area / 4.0
    return A


def volume(x: np.ndarray, tris: np.ndarray) -> float:
    """Divergence-theorem volume of a closed mesh, V = 1/9 sum_t A_t (x1+x2+x3).n_t
    (section 2.1.2), with A_t n_t = (x2 - x1) x (x3 - x1) / 2."""
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    an = 0.5 * np.cross(b - a, c - a)
    return float(np.sum(np.einsum("ij,ij->i", a + b + c, an)) / 9.0)


def surface_area(x: np.ndarray, tris: np.ndarray) -> float:
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    return float(0.5 * np.sum(np.linalg.norm(np.cross(b - a, c - a), axis=1)))


def area_gradient(x: np.ndarray, tris: np.ndarray, collapsed=None) -> np.ndarray:
    """grad of the total area: a triangle's area A_t = |(x_b - x_a) x (x_c - x_a)| / 2
    has dA_t/dx_a = n x (x_c - x_b) / 2 (n its unit normal), and cyclically for b, c.
    A collapsed triangle (flagged in `collapsed`) has no normal, and |n| no derivative:
    it contributes nothing."""
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    nn = np.linalg.norm(cr, axis=1, keepdims=True)
    n = cr / np.where(nn > 0, nn, 1.0)
    if collapsed is not None:
        n[collapsed] = 0.0
    g = np.zeros_like(x)
    np.add.at(g, tris[:, 0], 0.5 * np.cross(n, c - b))
    np.add.at(g, tris[:, 1], 0.5 * np.cross(n, a - c))
    np.add.at(g, tris[:, 2], 0.5 * np.cross(n, b - a))
    return g


def volume_gradient(x: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """grad V = nbar / 3, nbar_k = sum of A_t n_t over the triangles containing k
    (section 2.1.2; exact for a closed mesh)."""
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    an = 0.5 * np.cross(b - a, c - a)
    nbar = np.zeros_like(x)
    for k in range(3):
        np.add.at(nbar, tris[:, k], an)
    return nbar / 3.0


class Model:
    """Everything about one mesh + material + time step that is constant in time."""

    def __init__(self, X: np.ndarray, tris: np.ndarray, mat: Material, h: float):
        self.X = np.asarray(X, np.float64)
        self.tris = np.asarray(tris, np.int64)
        self.mat = mat
        self.h = float(h)
        n = self.n = len(self.X)

        # triangle rest data: D_m, D_m^-1, rest area (Appendix B)
        Dm, _, self.tri_area = triangle_frames(self.X, self.tris)
        self.Dm_inv = np.linalg.inv(Dm)

        # bending rest data (eq. BendingDiscretizedPotential)
        self.vor_area = mixed_voronoi_areas(self.X, self.tris)
        omega = cotangent_weights(self.X, self.tris)
        Gb = np.zeros((n, n))
        for (i, j), w in omega.items():
            Gb[i, j] += w / self.vor_area[i]
            Gb[j, i] += w / self.vor_area[j]
        Gb[np.arange(n), np.arange(n)] = -Gb.sum(axis=1)
        self.G_bend = Gb                                     # ell = G_bend @ x
        self.ell0_norm = np.linalg.norm(Gb @ self.X, axis=1)

        # lumped mass, area weighted (section 2.1)
        self.V0 = volume(self.X, self.tris)
        self.A0 = surface_area(self.X, self.tris)
        bary = np.zeros(n)
        for k in range(3):
            np.add.at(bary, self.tris[:, k], self.tri_area / 3.0)
        self.mass = mat.density * self.V0 * bary / bary.sum()

        # L = sum w G^T G (eq. fullyDeveloped_g), per coordinate, n x n.  A triangle's
        # G_t (2 x n) has, in row r, D_m^-1[0, r] at vertex a, D_m^-1[1, r] at b and
        # -(D_m^-1[0, r] + D_m^-1[1, r]) at c, so that G_t x = (D_s D_m^-1)^T.
        L = np.zeros((n, n))
        g = np.stack([self.Dm_inv[:, 0, :], self.Dm_inv[:, 1, :],
                      -self.Dm_inv[:, 0, :] - self.Dm_inv[:, 1, :]], axis=1)   # [nt, 3 corners, 2 rows]
        GtG = np.einsum("tir,tjr->tij", g, g)                 # G_t^T G_t, 3 x 3 per triangle
        rows = np.repeat(self.tris[:, :, None], 3, axis=2).ravel()
        cols = np.repeat(self.tris[:, None, :], 3, axis=1).ravel()
        np.add.at(L, (rows, cols), ((self.tri_area * mat.C)[:, None, None] * GtG).ravel())
        L += (Gb.T * (mat.k_bend * self.vor_area)) @ Gb
        self.L_damp = L.copy()                               # L' (no volume identity)
        L += (mat.k_volume + mat.k_area_global) * np.eye(n)
        self.L = L
        self.K_mat = np.zeros((n, n))
        np.add.at(self.K_mat, (rows, cols), ((self.tri_area * mat.k_mat_value)[:, None, None] * GtG).ravel())

        # M~ = M + h C, C = beta_D L', beta_D = beta h; H~ = M~ / h^2 + L
        self.Mt = np.diag(self.mass) + mat.beta * self.h ** 2 * self.L_damp
        self.Ht = self.Mt / self.h ** 2 + self.L + self.K_mat
        self._chol = {}

    def _factor(self, name: str):
        if name not in self._chol:          # prefactored once, on first use (section 2.1.1)
            self._chol[name] = scipy.linalg.cho_factor(getattr(self, name), lower=True)
        return self._chol[name]

    def solve_Ht(self, q: np.ndarray) -> np.ndarray:
        """H~^-1 q with the Cholesky factor computed once (section 2.1.1)."""
        return scipy.linalg.cho_solve(self._factor("Ht"), q)

    def solve_Mt(self, q: np.ndarray) -> np.ndarray:
        return scipy.linalg.cho_solve(self._factor("Mt"), q)
