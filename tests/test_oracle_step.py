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
