"""Collision term between cells (FP64 oracle, test only): section 4.7, Proof of
Capability.

The paper adds, for every colliding vertex, a non-PD energy (w_col/2) |p_i - x_i|^2 with
force w_col (p_i - x_i), where the desired position p_i comes from the colliding
neighbours and their normals, re-checks at every iteration whether the vertex still
penetrates and drops the term when it does not, and gives the term no share of H~.

Readings (the paper does not define p_i or the neighbour search precisely):
  * Contacts are found once per step, from the positions at the start of the step (the
    other cells' positions are not updated within a step: cells are solved
    independently, as the explicit coupling of section 2.2 hands over x_n): vertex i of
    cell A is in contact with the nearest vertex j of any other cell within the cutoff
    distance, ties broken by the smaller global vertex index.
  * The neighbour's normal n_j is the unit area-weighted vertex normal of its cell at
    x_n (the sum of (x_b - x_a) x (x_c - x_a) over the triangles containing j).
  * p_i is x_i projected onto the tangent plane of the neighbour at y_j:
    p_i = x_i - d n_j with d = (x_i - y_j) . n_j; the vertex penetrates while d < 0.
    Dropping the term when d >= 0 makes the energy (w/2) min(d, 0)^2 and its gradient
    w min(d, 0) n_j, continuous, with no contribution to H~.
"""
from __future__ import annotations

import numpy as np


def vertex_normals(x: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Unit area-weighted vertex normals of one closed mesh."""
    a, b, c = x[tris[:, 0]], x[tris[:, 1]], x[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    nrm = np.zeros_like(x)
    for k in range(3):
        np.add.at(nrm, tris[:, k], cr)
    ln = np.linalg.norm(nrm, axis=1, keepdims=True)
    return nrm / np.where(ln > 0, ln, 1.0)


def detect(origins, xs, tris_list, cutoff: float):
    """Brute-force contact search over all pairs of vertices of different cells.

    origins [C,3] world origin of each cell, xs list of [n_c,3] cell-local positions,
    tris_list list of [nt_c,3] triangles.  Returns per cell (q [n_c,3], nrm [n_c,3],
    partner [n_c]) with q the partner vertex in the cell's local frame, nrm its normal
    (zero where there is no contact) and partner its global vertex index (-1: none).
    """
    world = [np.asarray(o, np.float64)[None, :] + np.asarray(x, np.float64) for o, x in zip(origins, xs)]
    normals = [vertex_normals(np.asarray(x, np.float64), np.asarray(t)) for x, t in zip(xs, tris_list)]
    offs = np.concatenate([[0], np.cumsum([len(x) for x in xs])])
    allw = np.concatenate(world)
    alln = np.concatenate(normals)
    cell_of = np.concatenate([np.full(len(x), c) for c, x in enumerate(xs)])
    out = []
    for c, w in enumerate(world):
        q = np.zeros_like(w)
        nr = np.zeros_like(w)
        partner = np.full(len(w), -1)
        other = cell_of != c
        idx = np.nonzero(other)[0]
        for i in range(len(w)):
            d = allw[idx] - w[i]
            d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
            inside = d2 < cutoff * cutoff
            if not np.any(inside):
                continue
            cand = idx[inside]
            dc = d2[inside]
            best = cand[np.lexsort((cand, dc))[0]]
            partner[i] = best
            q[i] = allw[best] - np.asarray(origins[c], np.float64)
            nr[i] = alln[best]
        out.append((q, nr, partner))
    return out


def collision_energy(x: np.ndarray, q: np.ndarray, nrm: np.ndarray, w: float):
    """E = (w/2) sum min(d_i, 0)^2, d_i = (x_i - q_i) . n_i, and its gradient
    w min(d_i, 0) n_i (vertices without a contact have n_i = 0)."""
    d = np.minimum(np.sum((x - q) * nrm, axis=1), 0.0)
    return 0.5 * w * float(np.sum(d * d)), w * d[:, None] * nrm
