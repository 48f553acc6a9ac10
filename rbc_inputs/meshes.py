"""Rest meshes for the red-blood-cell membrane: subdivided platonic spheres mapped
onto the Evans-Skalak biconcave profile.

This module only builds geometry (vertex coordinates and outward, counter-clockwise
triangles).  It contains none of the solver's arithmetic, and it is shared by the
CPU oracle, the tests and the benchmark as the one source of seeded inputs.

Sizes (closed triangulated spheres, V - E + F = 2):
  octahedron subdivided k times  : V = 4 * 4**k + 2   (k=2: 66, k=3: 258, k=4: 1026)
  icosahedron subdivided k times : V = 10 * 4**k + 2  (k=0: 12, k=1: 42, k=3: 642, k=4: 2562)

The membrane shape: the introduction of the paper quotes the healthy RBC geometry
(diameter 7.82 um, thickness 0.81 um at the dimple and 2.57 um at the rim, area
134 um^2, volume 94 um^3) and points to the Evans & Skalak (1980) analytic profile.
The profile used here is the commonly quoted parameterisation
    z(r) = +- D sqrt(1 - 4 r^2 / D^2) (a0 + a1 r^2 / D^2 + a2 r^4 / D^4)
with D = 7.82 um, a0 = 0.0518, a1 = 2.0026, a2 = -4.491 (these coefficients are not
printed in the paper; tests check that they reproduce the numbers it does print).
"""
from __future__ import annotations

import numpy as np

RBC_DIAMETER_UM = 7.82
ES_COEFFS = (0.0518, 2.0026, -4.491)


def _orient_outward(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip any triangle whose normal points towards the origin (convex input only)."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c) / 3.0) < 0
    out = tris.copy()
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def icosahedron() -> tuple[np.ndarray, np.ndarray]:
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
         [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
         [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array(
        [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, _orient_outward(v, f)


def octahedron() -> tuple[np.ndarray, np.ndarray]:
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int32)
    return v, _orient_outward(v, f)


def subdivide(verts: np.ndarray, tris: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """One 4-to-1 split; new vertices are edge midpoints pushed onto the unit sphere."""
    verts = [tuple(x) for x in verts]
    cache: dict[tuple[int, int], int] = {}

    def mid(i: int, j: int) -> int:
        key = (i, j) if i < j else (j, i)
        k = cache.get(key)
        if k is None:
            m = (np.asarray(verts[i]) + np.asarray(verts[j])) / 2.0
            m /= np.linalg.norm(m)
            verts.append(tuple(m))
            k = len(verts) - 1
            cache[key] = k
        return k

    out = []
    for a, b, c in tris:
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
    return np.asarray(verts, dtype=np.float64), np.asarray(out, dtype=np.int32)


def unit_sphere(n_verts: int) -> tuple[np.ndarray, np.ndarray]:
    """Closed unit-sphere triangulation with exactly n_verts vertices."""
    for base, mult in ((icosahedron, 10), (octahedron, 4)):
        k = 0
        while mult * 4 ** k + 2 < n_verts:
            k += 1
        if mult * 4 ** k + 2 == n_verts:
            v, f = base()
            for _ in range(k):
                v, f = subdivide(v, f)
            return v, f
    raise ValueError(f"no subdivided icosahedron/octahedron has {n_verts} vertices")


def evans_skalak(sphere_verts: np.ndarray, diameter: float = RBC_DIAMETER_UM,
                 coeffs: tuple[float, float, float] = ES_COEFFS) -> np.ndarray:
    """Map unit-sphere points onto the biconcave profile (symmetry axis z)."""
    x, y, z = sphere_verts.T
    s = np.clip(x * x + y * y, 0.0, 1.0)
    a0, a1, a2 = coeffs
    height = diameter * np.sqrt(1.0 - s) * (a0 + a1 * s / 4.0 + a2 * s * s / 16.0)
    return np.stack([0.5 * diameter * x, 0.5 * diameter * y, np.sign(z) * height], axis=1)


def rbc_mesh(n_verts: int) -> tuple[np.ndarray, np.ndarray]:
    """Rest RBC mesh (um) with n_verts vertices: (verts [n,3] float64, tris [nt,3] int32)."""
    v, f = unit_sphere(n_verts)
    return evans_skalak(v), f


def sphere_mesh(n_verts: int, radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    v, f = unit_sphere(n_verts)
    return radius * v, f


def edges_of(tris: np.ndarray) -> np.ndarray:
    """Unique undirected edges [ne, 2] (i < j)."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e.sort(axis=1)
    return np.unique(e, axis=0)
