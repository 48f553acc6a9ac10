"""Pins of the oracle's time step: closed-form special cases, the local/global
identity of Appendix A, brute-force Newton, invariances, dissipation."""
import numpy as np
import pytest

from rbc_inputs import meshes
from oracle import energy, newton, step
from oracle.model import Model, Material, triangle_frames, volume, volume_gradient
from conftest import oracle_model
from test_oracle_energy import random_rotation


def random_inputs(m, seed, pert=0.1, vel=0.01, force=5.0):
    rng = np.random.default_rng(seed)
    return (m.X + pert * rng.standard_normal(m.X.shape), vel * rng.standard_normal(m.X.shape),
            force * rng.standard_normal(m.X.shape))


def test_rest_state_is_a_fixed_point():
    """Zero force at the rest shape: r = 0 at the first guess, so no iteration and
    x_{n+1} = x_n, v_{n+1} = 0 exactly."""
    m = oracle_model(642)
    x, v, info = step.step(m, m.X, np.zeros_like(m.X), np.zeros_like(m.X))
    assert info.iterations == 0 and info.status == step.CONVERGED
    np.testing.assert_array_equal(x, m.X)
    assert np.abs(v).max() == 0.0


def test_no_stiffness_gives_explicit_inertial_update():
    """With every stiffness zero the objective is the inertial term only and its
    minimiser is y_n (eq. preOptimizationNewton) = x_n + h v_n + h^2 F_ext / m."""
    X, T = meshes.sphere_mesh(42, 3.0)
    mat = Material(B=0.0, C=0.0, D=0.0, k_bend=0.0, k_volume=0.0, k_mat=0.0, kappa=0.0)
    m = Model(X, T, mat, 0.1)
    xn, vn, f = random_inputs(m, 1)
    x, v, info = step.step(m, xn, vn, f, step.Params(tol=1e-14))
    expect = xn + m.h * vn + m.h ** 2 * f / m.mass[:, None]
    np.testing.assert_allclose(x, expect, rtol=0, atol=1e-14)
    np.testing.assert_allclose(v, (expect - xn) / m.h, atol=1e-12)


def test_local_global_special_case():
    """Appendix A: with projective-dynamics energies only, the quasi-Newton step with
    alpha = 1 and no history is the local/global update
        x* = H~^-1 (J p + M~ y / h^2),
    where J p = sum_i w_i G_i^T p_i is assembled here from explicit element matrices
    and projections (area: T re-embedded in 3D; bending: |l0| l/|l|; volume:
    x - C grad C / |grad C|^2).  Evaluated at x = x_n."""
    X, T = meshes.rbc_mesh(66)
    m = Model(X, T, Material(B=0.0, D=0.0, k_mat=0.0), 0.1)
    xn, vn, f = random_inputs(m, 2, pert=0.08)
    obj = step.Objective(m, xn, vn, f)
    _, grad, _ = obj(xn)
    d = -m.solve_Ht(grad)

    n = m.n
    Jp = np.zeros((n, 3))
    Ds, basis, _ = triangle_frames(xn, m.tris)
    F = Ds @ m.Dm_inv
    U, s, Vt = np.linalg.svd(F)
    t = energy.sl2_projection(s[:, 0], s[:, 1])
    for k, (a, b, c) in enumerate(m.tris):
        G = np.zeros((2, n))
        for r in range(2):
            G[r, a] += m.Dm_inv[k, 0, r]
            G[r, b] += m.Dm_inv[k, 1, r]
            G[r, c] -= m.Dm_inv[k, 0, r] + m.Dm_inv[k, 1, r]
        Tk = U[k] @ np.diag([t[k], 1 / t[k]]) @ Vt[k]
        p = (basis[k] @ Tk).T                               # 2 x 3 projection in 3D
        Jp += m.tri_area[k] * m.mat.C * G.T @ p
    ell = m.G_bend @ xn
    p_b = m.ell0_norm[:, None] * ell / np.linalg.norm(ell, axis=1, keepdims=True)
    Jp += m.G_bend.T @ ((m.mat.k_bend * m.vor_area)[:, None] * p_b)
    gC = volume_gradient(xn, m.tris)
    C = volume(xn, m.tris) - m.V0
    Jp += m.mat.k_volume * (xn - C * gC / np.sum(gC * gC))
    x_star = m.solve_Ht(Jp + m.Mt @ obj.y / m.h ** 2)
    np.testing.assert_allclose(xn + d, x_star, rtol=0, atol=1e-11 * np.abs(x_star).max())


@pytest.mark.parametrize("n", [12, 42])
def test_brute_force_newton_agrees(n):
    X, T = meshes.sphere_mesh(n, 3.0)
    m = Model(X, T, Material(), 0.1)
    xn, vn, f = random_inputs(m, 3 + n, pert=0.2)
    xa, _, info = step.step(m, xn, vn, f, step.Params(tol=1e-13))
    assert info.status == step.CONVERGED
    xb, ok = newton.newton_solve(step.Objective(m, xn, vn, f), xn + 0.01)
    assert ok
    assert np.abs(xa - xb).max() <= 1e-10 * np.ptp(X)


def test_solution_independent_of_start_history_and_preconditioner():
    """The step's result is the stationary point of g: it does not depend on the
    starting point, on the history length m, or on the material term in H~."""
    m = oracle_model(258)
    xn, vn, f = random_inputs(m, 4, pert=0.04)
    ref, _, _ = step.step(m, xn, vn, f, step.Params(tol=1e-12))
    D = np.ptp(m.X)
    x1, _, _ = step.step(m, xn, vn, f, step.Params(tol=1e-12), x_start=xn + 0.002)
    x2, _, _ = step.step(m, xn, vn, f, step.Params(tol=1e-12, m=1))
    m0 = oracle_model(258, k_mat=0.0)
    x3, _, _ = step.step(m0, xn, vn, f, step.Params(tol=1e-12))
    for x in (x1, x2, x3):
        assert np.abs(x - ref).max() <= 1e-10 * D


def test_rigid_equivariance_of_the_step():
    m = oracle_model(258)
    xn, vn, f = random_inputs(m, 5, pert=0.04)
    R, t = random_rotation(7), np.array([2.0, -1.0, 0.5])
    x1, v1, _ = step.step(m, xn, vn, f, step.Params(tol=1e-12))
    x2, v2, _ = step.step(m, xn @ R.T + t, vn @ R.T, f @ R.T, step.Params(tol=1e-12))
    np.testing.assert_allclose(x2, x1 @ R.T + t, atol=1e-10 * np.ptp(m.X))
    np.testing.assert_allclose(v2, v1 @ R.T, atol=1e-9 * np.abs(v1).max())


def test_dissipation_properties():
    """Section 2.1.4: the post-convergence step conserves linear and angular
    momentum, leaves a rigid velocity field unchanged, kappa = 0 is a no-op and
    kappa = 1 is a projection (idempotent)."""
    rng = np.random.default_rng(6)
    m = oracle_model(258)
    x = m.X + 0.05 * rng.standard_normal(m.X.shape)
    v = rng.standard_normal(m.X.shape)
    w = step.dissipate(x, v, m.mass, 0.6)
    mm = m.mass[:, None]
    np.testing.assert_allclose((mm * w).sum(0), (mm * v).sum(0), atol=1e-9 * np.abs(mm * v).sum())
    xc = (mm * x).sum(0) / m.mass.sum()
    np.testing.assert_allclose(np.cross(x - xc, mm * w).sum(0), np.cross(x - xc, mm * v).sum(0),
                               atol=1e-9 * np.abs(mm * v).sum())
    rigid = np.array([0.3, -0.1, 0.2]) + np.cross(np.array([0.5, 1.0, -2.0]), x)
    np.testing.assert_allclose(step.dissipate(x, rigid, m.mass, 0.6), rigid, atol=1e-12)
    np.testing.assert_array_equal(step.dissipate(x, v, m.mass, 0.0), v)
    p = step.dissipate(x, v, m.mass, 1.0)
    np.testing.assert_allclose(step.dissipate(x, p, m.mass, 1.0), p, atol=1e-12)


def test_stretching_load_converges_and_elongates():
    """The optical-tweezers loading (section 4.1) pulls the cell along x: after one
    step with the full 200 pN load the axial extent grows and the transverse shrinks
    relative to rest, and every internal force stays balanced."""
    m = oracle_model(258)
    from rbc_inputs import workloads
    b = workloads.stretch()
    f = workloads.stretch_forces(b, 200)
    x, v, info = step.step(m, m.X, np.zeros_like(m.X), f, step.Params(tol=1e-8))
    assert info.status == step.CONVERGED
    assert np.ptp(x[:, 0]) > np.ptp(m.X[:, 0])


def test_step_momentum_balance():
    """Newton's law for the whole body: internal forces and the Rayleigh term cancel
    in the sum, so sum m v_{n+1} = sum m v_n + h sum F_ext, and the dissipation keeps it."""
    m = oracle_model(258)
    xn, vn, f = random_inputs(m, 9, pert=0.04, vel=0.02, force=3.0)
    x, v, info = step.step(m, xn, vn, f, step.Params(tol=1e-12))
    mm = m.mass[:, None]
    expect = (mm * vn).sum(0) + m.h * f.sum(0)
    np.testing.assert_allclose((mm * v).sum(0), expect, atol=1e-8 * np.abs(mm * vn).sum())


# ---- L-BFGS two-loop recursion -------------------------------------------------------

def test_lbfgs_direction_equals_dense_bfgs_inverse_update():
    """The two-loop recursion is a fast way to apply H_k, the inverse-Hessian
    approximation obtained by the BFGS inverse update (Nocedal & Wright eq. 6.17)
        H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T,  rho = 1 / (y . s),
    applied to H_0 once per stored pair, oldest first.  Here H_0 is an SPD matrix
    applied to each of the three coordinate columns (as H~^-1 is), built densely on the
    flattened 3n vector, and the direction must be -H_k g.  The secant condition
    H_k y_newest = s_newest holds as well.  A reversed loop, a wrong rho or a swapped
    s/y would break either check."""
    rng = np.random.default_rng(11)
    n, k = 7, 4
    A = rng.standard_normal((n, n))
    H0 = A @ A.T + n * np.eye(n)                      # SPD, applied per coordinate
    H0_inv = np.linalg.inv(H0)
    solve = lambda q: H0_inv @ q                      # q is [n, 3]
    Bq = rng.standard_normal((3 * n, 3 * n))
    Hess = Bq @ Bq.T + np.eye(3 * n)                  # a curvature model for the pairs
    S = [rng.standard_normal((n, 3)) for _ in range(k)]
    Y = [(Hess @ s.ravel()).reshape(n, 3) for s in S]
    rho = [1.0 / np.sum(s * y) for s, y in zip(S, Y)]
    g = rng.standard_normal((n, 3))
    # dense H_k on the row-major flattening (index 3 i + c): H_0 = H0_inv (x) I_3
    H = np.kron(H0_inv, np.eye(3))
    I = np.eye(3 * n)
    for s, y in zip(S, Y):
        s_, y_ = s.ravel(), y.ravel()
        r = 1.0 / (y_ @ s_)
        H = (I - r * np.outer(s_, y_)) @ H @ (I - r * np.outer(y_, s_)) + r * np.outer(s_, s_)
    d = step.lbfgs_direction(g, S, Y, rho, solve)
    np.testing.assert_allclose(d.ravel(), -H @ g.ravel(), rtol=1e-10, atol=1e-12 * np.abs(H @ g.ravel()).max())
    np.testing.assert_allclose(H @ Y[-1].ravel(), S[-1].ravel(), rtol=1e-10, atol=1e-12)
    # no pairs: the preconditioned gradient
    np.testing.assert_allclose(step.lbfgs_direction(g, [], [], [], solve), -H0_inv @ g, rtol=1e-14)


# ---- residual ---------------------------------------------------------------------------

def _tetrahedron():
    X = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])
    T = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    return X, T


def test_residual_hand_computed_tetrahedron():
    """Regular tetrahedron with edge 2 sqrt(2): faces of area 2 sqrt(3), total area
    8 sqrt(3), volume 8/3.  With density 3 the mass is 8, i.e. 2 per vertex; with
    h = 0.5, m/h^2 = 8.  Inputs: u = (1/8, 0, 0) on vertex 0 (so M u/h^2 = (1, 0, 0)),
    v = 0, F_ext = (0, 3, 4) on vertex 1 (|b| = 5), and a gradient (0, 9, 12) on
    vertex 3 (|grad| = 15).  Then grad - M u/h^2 + b has entries (-1, 0, 0), (0, 3, 4),
    (0, 9, 12): norm sqrt(251), and
        r = 15 / (1 + 5 + sqrt(251) + B sqrt(8 sqrt(3))).
    """
    X, T = _tetrahedron()
    m = Model(X, T, Material(density=3.0), 0.5)
    assert np.isclose(m.V0, 8.0 / 3.0) and np.allclose(m.mass, 2.0)
    u = np.zeros((4, 3))
    u[0, 0] = 1.0 / 8.0
    f = np.zeros((4, 3))
    f[1] = [0.0, 3.0, 4.0]
    grad = np.zeros((4, 3))
    grad[3] = [0.0, 9.0, 12.0]
    obj = step.Objective(m, X, np.zeros((4, 3)), f)
    expect = 15.0 / (1.0 + 5.0 + np.sqrt(251.0) + m.mat.B * np.sqrt(8.0 * np.sqrt(3.0)))
    assert obj.residual(X + u, grad) == pytest.approx(expect, rel=1e-14)
    assert obj.residual(X + u, np.zeros((4, 3))) == 0.0


def test_residual_and_step_invariant_under_change_of_units():
    """The residual is a ratio of forces, so it must not depend on the units.  Lengths
    scaled by L, masses by Mu and times by Tau: forces scale by Mu L / Tau^2, the
    moduli B, C, D, k_volume (force per length) by Mu / Tau^2, k_bend (energy) by
    Mu L^2 / Tau^2, the density by Mu / L^3; beta is in units of the time step.  The
    residual of the same physical state, and the converged step, must map onto each
    other."""
    m1 = oracle_model(258)
    xn, vn, f = random_inputs(m1, 21, pert=0.04, vel=0.02, force=3.0)
    Lf, Mu, Tau = 1e3, 1e-3, 1e3           # nm, ag (1e-21 kg), ns
    Ff = Mu * Lf / Tau ** 2
    mat = m1.mat
    mat2 = Material(B=mat.B * Mu / Tau ** 2, C=mat.C * Mu / Tau ** 2, D=mat.D * Mu / Tau ** 2,
                    k_bend=mat.k_bend * Mu * Lf ** 2 / Tau ** 2, k_volume=mat.k_volume * Mu / Tau ** 2,
                    beta=mat.beta, kappa=mat.kappa, density=mat.density * Mu / Lf ** 3)
    m2 = Model(m1.X * Lf, m1.tris, mat2, m1.h * Tau)
    np.testing.assert_allclose(m2.mass, m1.mass * Mu, rtol=1e-12)
    o1 = step.Objective(m1, xn, vn, f)
    o2 = step.Objective(m2, xn * Lf, vn * Lf / Tau, f * Ff)
    x = o1.y + 0.01 * np.random.default_rng(3).standard_normal(xn.shape)
    _, g1, _ = o1(x)
    _, g2, _ = o2(x * Lf)
    np.testing.assert_allclose(g2, g1 * Ff, rtol=1e-7, atol=1e-9 * np.abs(g1).max() * Ff)
    assert o2.residual(x * Lf, g2) == pytest.approx(o1.residual(x, g1), rel=1e-7)
    x1, _, _ = step.step(m1, xn, vn, f, step.Params(tol=1e-12, polish=True))
    x2, _, _ = step.step(m2, xn * Lf, vn * Lf / Tau, f * Ff, step.Params(tol=1e-12, polish=True))
    assert np.abs(x2 / Lf - x1).max() <= 1e-10 * np.ptp(m1.X)


# ---- the stationary point (parity reference) ------------------------------------------

def test_polish_reaches_the_stationary_point_of_a_stretched_cell():
    """Under a large stretching load the Armijo test on g stops resolving progress well
    above residual 1e-12 (g's FP64 rounding exceeds its decrease); the residual-decrease
    continuation then reaches 1e-12, and the point it reaches is the brute-force Newton
    solution of grad g = 0 (66-vertex mesh)."""
    X, T = meshes.rbc_mesh(66)
    m = Model(X, T, Material(), 0.1)
    from rbc_inputs import workloads
    n_end = int(np.ceil(0.05 * len(X)))
    f = np.zeros_like(X)
    order = np.argsort(X[:, 0])
    f[order[-n_end:], 0] = 400.0 / n_end
    f[order[:n_end], 0] = -400.0 / n_end
    xa, _, plain = step.step(m, X, np.zeros_like(X), f, step.Params(tol=1e-12))
    xb, _, info = step.step(m, X, np.zeros_like(X), f, step.Params(tol=1e-12, polish=True))
    assert info.status == step.CONVERGED and info.residual <= 1e-12
    xn, ok = newton.newton_solve(step.Objective(m, X, np.zeros_like(X), f), xb + 1e-4, tol=1e-12)
    assert ok
    assert np.abs(xb - xn).max() <= 1e-11 * np.ptp(X)
    if plain.status != step.CONVERGED:          # the plain run stopped early: polish moved it
        assert plain.residual > 1e-12


def test_mixed_voronoi_areas_partition_the_surface():
    """Meyer's mixed areas split every triangle among its corners, so they sum to the
    total area, on the RBC meshes, which have obtuse triangles (the branch that gives
    the obtuse corner half the area and the others a quarter).  Single triangles fix
    the values: equilateral 1/3 each; right isosceles 1/2 at the right angle and 1/4 at
    the others (the circumcentre lies on the hypotenuse, so both branches must agree
    there); an obtuse triangle 1/2, 1/4, 1/4."""
    from oracle.model import mixed_voronoi_areas
    for n in (258, 642):
        mm = oracle_model(n)
        P = mm.X[mm.tris]
        cosang = []
        for k in range(3):
            u, v = P[:, (k + 1) % 3] - P[:, k], P[:, (k + 2) % 3] - P[:, k]
            cosang.append(np.einsum("ij,ij->i", u, v))
        n_obtuse = int(np.sum(np.min(cosang, axis=0) < 0))
        assert n_obtuse > 0, n
        assert mm.vor_area.sum() == pytest.approx(mm.tri_area.sum(), rel=1e-12)
        assert np.all(mm.vor_area > 0)
    tri = np.array([[0, 1, 2]])
    eq = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [1.0, np.sqrt(3.0), 0.0]])
    np.testing.assert_allclose(mixed_voronoi_areas(eq, tri), np.full(3, np.sqrt(3.0) / 3), rtol=1e-13)
    right = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 2.0, 0.0]])      # area 2
    np.testing.assert_allclose(mixed_voronoi_areas(right, tri), [1.0, 0.5, 0.5], rtol=1e-12)
    obtuse = np.array([[0.0, 0.0, 0.0], [4.0, 0.0, 0.0], [-1.0, 1.0, 0.0]])     # area 2, obtuse at 0
    np.testing.assert_allclose(mixed_voronoi_areas(obtuse, tri), [1.0, 0.5, 0.5], rtol=1e-13)
