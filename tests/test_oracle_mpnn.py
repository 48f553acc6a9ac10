"""Pins of the FP64 network oracle (oracle/mpnn.py) against facts that do not come
from its own formulas: a known rotation, rigid-motion invariance, the neighbour
structure of the octahedron, a weight setting that reduces the network to
(I + mean-adjacency) f checked by brute-force loops, finite differences of the loss,
the closed form of Adam's first step, and bfloat16 rounding ties."""
import numpy as np
import pytest

import oracle.mpnn as mp
from rbc_inputs import meshes

CFG = mp.NetConfig(hidden=16, layers=2)


def small_cell(seed=0, level=1):
    X, T = meshes.sphere_mesh(42 if level == 1 else 162)
    rng = np.random.default_rng(seed)
    n = len(X)
    m = rng.uniform(0.5, 1.5, n)
    x = X + 0.05 * rng.standard_normal((n, 3))
    v = rng.standard_normal((n, 3))
    F = rng.standard_normal((n, 3))
    return X, T, m, x, v, F


def random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c)],
                     [2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b)],
                     [2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d]])


def test_kabsch_recovers_a_known_rotation():
    X, T, m, _, _, _ = small_cell()
    rng = np.random.default_rng(1)
    Q = random_rotation(rng)
    x = X @ Q.T + np.array([3.0, -2.0, 0.5])
    R, xc, Xc = mp.kabsch(X, x, m)
    assert np.abs(R - Q).max() < 1e-12
    assert abs(np.linalg.det(R) - 1.0) < 1e-12
    np.testing.assert_allclose(xc, (m @ x) / m.sum(), atol=1e-14)


def test_features_invariant_under_rigid_motion_and_uniform_fields():
    """Rotating and translating the cell, adding a uniform velocity and a uniform
    acceleration (force m_i a) leaves every feature unchanged; the predicted
    correction rotates with the cell."""
    X, T, m, x, v, F = small_cell(2)
    h = 0.1
    rng = np.random.default_rng(3)
    Q = random_rotation(rng)
    f1, R1, s1 = mp.features(X, x, v, F, m, h, CFG)
    x2 = x @ Q.T + np.array([1.0, 2.0, 3.0])
    v2 = v @ Q.T + np.array([0.3, -0.1, 0.2])
    F2 = F @ Q.T + m[:, None] * np.array([0.5, 0.4, -0.7])
    f2, R2, s2 = mp.features(X, x2, v2, F2, m, h, CFG)
    np.testing.assert_allclose(f2, f1, atol=1e-10)
    assert abs(s2 - s1) <= 1e-12 * s1
    np.testing.assert_allclose(R2, Q @ R1, atol=1e-12)
    A = mp.neighbour_mean_matrix(len(X), T)
    theta = mp.init_params(CFG, 5)
    d1 = mp.predict_delta(theta, X, x, v, F, m, h, A, CFG)
    d2 = mp.predict_delta(theta, X, x2, v2, F2, m, h, A, CFG)
    np.testing.assert_allclose(d2, d1 @ Q.T, atol=1e-12 * np.abs(d1).max())


def test_neighbour_mean_on_the_octahedron():
    """Vertex +-e_k of the octahedron neighbours the four vertices off its axis."""
    X, T = meshes.octahedron()
    A = mp.neighbour_mean_matrix(6, T).toarray()
    for i in range(6):
        for j in range(6):
            same_axis = abs(abs(X[i] @ X[j]) - 1.0) < 1e-12
            assert A[i, j] == (0.0 if same_axis else 0.25)


def test_reduced_network_is_identity_plus_neighbour_mean():
    """With W_e = [I; 0], b_e = 10 (all pre-activations positive), W_s = 0, W_n = I in
    the first layer, zero later layers, W_d = [I_3 0] and b_d = -20, the output is
    o_i = f_i + mean_{j in N(i)} f_j on the first three features; the neighbour sets
    come from a loop over the triangle edges."""
    X, T, m, x, v, F = small_cell(4)
    n = len(X)
    H = CFG.hidden
    theta = np.zeros(mp.param_count(CFG))
    p = mp.unpack(theta, CFG)
    p["We"][:mp.N_FEAT, :] = np.eye(mp.N_FEAT)
    p["be"][:] = 10.0
    p["Wn0"][:] = np.eye(H)
    p["Wd"][:, :3] = np.eye(3)
    p["bd"][:] = -20.0
    f = np.random.default_rng(5).uniform(-1, 1, (n, mp.N_FEAT))
    o, _ = mp.forward(theta, f, mp.neighbour_mean_matrix(n, T), CFG)
    nbrs = [set() for _ in range(n)]
    for a, b, c in T:
        for i, j in ((a, b), (b, c), (c, a)):
            nbrs[i].add(j)
            nbrs[j].add(i)
    for i in range(n):
        ref = f[i, :3] + sum(f[j, :3] for j in nbrs[i]) / len(nbrs[i])
        np.testing.assert_allclose(o[i], ref, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    X, T, m, x, v, F = small_cell(seed + 10)
    n = len(X)
    A = mp.neighbour_mean_matrix(n, T)
    theta = mp.init_params(CFG, seed)
    theta += 0.05 * np.random.default_rng(seed).standard_normal(theta.size)   # biases non-zero too
    rng = np.random.default_rng(seed + 100)
    cells = []
    for c in range(2):
        f, R, s = mp.features(X, x + 0.01 * c, v, F, m, 0.1, CFG)
        cells.append((f, rng.standard_normal((n, 3))))
    L, g = mp.loss_and_grad(theta, cells, A, CFG)
    idx = rng.choice(theta.size, 60, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (mp.loss_and_grad(tp, cells, A, CFG)[0] - mp.loss_and_grad(tm, cells, A, CFG)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * (abs(fd) + 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-9, 0.0])
    th = np.array([1.0, 2.0, 3.0, 4.0])
    opt = mp.Adam(lr=0.01)
    t1, mo, ve = mp.adam_update(th, g, np.zeros(4), np.zeros(4), 1, opt)
    np.testing.assert_allclose(t1 - th, -opt.lr * g / (np.abs(g) + opt.eps), rtol=1e-12, atol=1e-18)
    # a second identical gradient keeps the step size (mhat = g, vhat = g^2 again)
    t2, _, _ = mp.adam_update(t1, g, mo, ve, 2, opt)
    np.testing.assert_allclose(t2 - t1, -opt.lr * g / (np.abs(g) + opt.eps), rtol=1e-9, atol=1e-18)


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38])
    out = mp.bf16_round(vals)
    np.testing.assert_array_equal(out[:5], [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5])
    assert np.isfinite(out[5])


def test_target_and_prediction_are_consistent():
    """If the network output equals the target, the predicted correction is delta."""
    X, T, m, x, v, F = small_cell(7)
    f, R, s = mp.features(X, x, v, F, m, 0.1, CFG)
    delta = np.random.default_rng(8).standard_normal((len(X), 3))
    t = mp.target(R, s, delta)
    np.testing.assert_allclose(s * (t @ R.T), delta, atol=1e-12)
