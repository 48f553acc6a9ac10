"""Pins of the oracle's collision term (section 4.7): the brute-force contact search
against a k-d tree, the vertex normals on a sphere, the one-sided energy against finite
differences, and steps that push penetrating vertices out and agree with brute-force
Newton."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from rbc_inputs import meshes
from oracle import collision, newton, step
from oracle.model import Model, Material
from conftest import oracle_model


def overlapping_pair(n=258, gap=-0.6, seed=0):
    """Two rest cells side by side along z (the thin axis) with their faces `gap` apart
    (negative: overlapping)."""
    X, T = meshes.rbc_mesh(n)
    th = np.ptp(X[:, 2])
    rng = np.random.default_rng(seed)
    origins = np.array([[10.0, 20.0, 30.0], [10.0 + 0.3, 20.0 - 0.2, 30.0 + th + gap]])
    xs = [X + 0.01 * rng.standard_normal(X.shape), X + 0.01 * rng.standard_normal(X.shape)]
    return X, T, origins, xs


def test_contact_search_matches_kd_tree():
    X, T, origins, xs = overlapping_pair()
    cutoff = 0.45
    res = collision.detect(origins, xs, [T, T], cutoff)
    world = [o + x for o, x in zip(origins, xs)]
    for c in (0, 1):
        tree = cKDTree(world[1 - c])
        d, j = tree.query(world[c], distance_upper_bound=cutoff)
        q, nrm, partner = res[c]
        has = np.isfinite(d)
        assert np.array_equal(partner >= 0, has)
        assert has.sum() > 10
        off = 0 if c == 1 else len(X)                  # global index of the other cell's vertex
        np.testing.assert_array_equal(partner[has], j[has] + off)
        np.testing.assert_allclose(q[has], world[1 - c][j[has]] - origins[c], atol=1e-12)
        assert np.all(nrm[~has] == 0)


def test_vertex_normals_on_a_sphere():
    X, T = meshes.sphere_mesh(642, 2.0)
    nrm = collision.vertex_normals(X, T)
    radial = X / np.linalg.norm(X, axis=1, keepdims=True)
    assert np.min(np.sum(nrm * radial, axis=1)) > 0.999
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, rtol=1e-14)


def test_collision_energy_one_sided_and_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((50, 3))
    q = x + 0.1 * rng.standard_normal((50, 3))
    nrm = rng.standard_normal((50, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm[::7] = 0.0                                      # no contact there
    w = 300.0
    E, g = collision.collision_energy(x, q, nrm, w)
    d = np.sum((x - q) * nrm, axis=1)
    assert E == pytest.approx(0.5 * w * np.sum(np.minimum(d, 0) ** 2))
    assert np.all(g[d >= 0] == 0) and np.all(g[::7] == 0)
    h = 1e-7
    for i, k in [(1, 0), (2, 1), (10, 2), (33, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (collision.collision_energy(xp, q, nrm, w)[0] - collision.collision_energy(xm, q, nrm, w)[0]) / (2 * h)
        assert fd == pytest.approx(g[i, k], rel=1e-6, abs=1e-8)
    # moving every vertex out along its normal past the plane removes the term
    E2, g2 = collision.collision_energy(q + 0.01 * nrm, q, nrm, w)
    assert E2 == 0.0 and np.all(g2 == 0)


def test_step_with_contacts_pushes_out_and_matches_newton():
    """Two overlapping 42-vertex spheres, each stepped against the other's x_n: the
    collision term reduces the penetration relative to the step without it, and the
    result is the brute-force Newton stationary point of the same objective."""
    X, T = meshes.sphere_mesh(42, 1.5)
    mm = Model(X, T, Material(), 0.1)
    origins = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.6]])
    xs = [X.copy(), X.copy()]
    res = collision.detect(origins, xs, [T, T], 0.8)
    q, nrm, partner = res[0]
    assert np.sum(partner >= 0) >= 3
    pen0 = -np.minimum(np.sum((xs[0] - q) * nrm, axis=1), 0).min()
    assert pen0 > 0.1
    v0, f0 = np.zeros_like(X), np.zeros_like(X)
    contacts = (q, nrm, 2.0e5)                     # above m/h^2 (3.7e4 pN/um per vertex here)
    x1, _, info = step.step(mm, xs[0], v0, f0, step.Params(tol=1e-12, polish=True), contacts=contacts)
    assert info.status & step.CONVERGED
    pen1 = -np.minimum(np.sum((x1 - q) * nrm, axis=1), 0).min()
    assert pen1 < 0.8 * pen0
    xn, ok = newton.newton_solve(step.Objective(mm, xs[0], v0, f0, contacts=contacts), x1 + 1e-5)
    assert ok and np.abs(xn - x1).max() <= 1e-10 * np.ptp(X)
