"""Pins of the oracle's membrane energies against what the paper and the mathematics
fix: closed forms, invariants, finite differences, brute force."""
import numpy as np
import pytest

from rbc_inputs import meshes
from oracle import energy
from oracle.model import Model, Material, volume, volume_gradient
from conftest import oracle_model

TERMS = ["area", "skalak", "bending", "volume"]


def term(name, x, m, Gn):
    if name == "area":
        return energy.area_energy(x, m)
    if name == "skalak":
        return energy.skalak_energy(x, m)
    if name == "bending":
        return energy.bending_energy(x, m)
    return energy.volume_energy(x, m, Gn)


def deformed(m, scale=0.05, seed=0):
    rng = np.random.default_rng(seed)
    return m.X + scale * rng.standard_normal(m.X.shape)


def random_rotation(seed):
    q = np.random.default_rng(seed).standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


# ---- SL(2) projection --------------------------------------------------------------

def test_sl2_projection_is_global_minimiser_brute_force():
    """The largest root of t^4 - s1 t^3 + s2 t - 1 minimises (s1-t)^2 + (s2-1/t)^2
    over t > 0 (dense grid search + refinement, 4000 random singular-value pairs)."""
    rng = np.random.default_rng(3)
    s = np.sort(rng.uniform(0.0, 4.0, (4000, 2)), axis=1)[:, ::-1]
    s = np.concatenate([s, [[1, 1], [2, 2], [0.5, 0.5], [3, 0], [1.5, 1.5]]])
    t = energy.sl2_projection(s[:, 0], s[:, 1])
    grid = np.exp(np.linspace(np.log(1e-3), np.log(1e3), 20001))
    for (s1, s2), tt in zip(s, t):
        d = (s1 - grid) ** 2 + (s2 - 1 / grid) ** 2
        k = np.argmin(d)
        lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
        for _ in range(100):                                  # golden-section refinement
            a, b = lo + 0.382 * (hi - lo), lo + 0.618 * (hi - lo)
            if (s1 - a) ** 2 + (s2 - 1 / a) ** 2 < (s1 - b) ** 2 + (s2 - 1 / b) ** 2:
                hi = b
            else:
                lo = a
        best = 0.5 * (lo + hi)
        dbest = (s1 - best) ** 2 + (s2 - 1 / best) ** 2
        dt = (s1 - tt) ** 2 + (s2 - 1 / tt) ** 2
        assert dt <= dbest + 1e-12 * (1 + dbest)


def test_area_energy_uniform_scaling_closed_form():
    """F = s R with s <= 2 projects to R, so E = C A_total (s - 1)^2."""
    m = oracle_model(258)
    for s in (0.8, 1.0, 1.3, 1.9):
        E, _ = energy.area_energy(s * m.X, m)
        assert np.isclose(E, m.mat.C * m.tri_area.sum() * (s - 1) ** 2, rtol=1e-10, atol=1e-12)


def test_area_energy_zero_for_area_preserving_triangle_maps():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.]])
    T = np.array([[0, 1, 2], [1, 3, 2]])
    m = Model(X, T, Material(), 0.1)
    for a, sh in ((1.7, 0.0), (0.6, 0.4), (1.0, 2.0)):
        A = np.array([[a, sh, 0], [0, 1 / a, 0], [0, 0, 1.]])      # det 1 in the plane
        E, g = energy.area_energy(X @ A.T, m)
        assert abs(E) < 1e-20 and np.abs(g).max() < 1e-9


# ---- Skalak -----------------------------------------------------------------------

def test_skalak_valanis_landel_equals_invariant_form():
    """Section 2.1.3: with D = 0, f(l1) + f(l2) + B/4 equals B/4 (I1^2/2 + I1 - I2),
    I1 = l1^2 + l2^2 - 2, I2 = l1^2 l2^2 - 1, computed here from tr and det of
    F^T F (no SVD).  The D term is checked with eigenvalues of F^T F."""
    m = oracle_model(258)
    x = deformed(m, 0.08, 1)
    Ds, _, _ = __import__("oracle.model", fromlist=["x"]).triangle_frames(x, m.tris)
    F = Ds @ m.Dm_inv
    Cg = np.transpose(F, (0, 2, 1)) @ F
    I1 = np.trace(Cg, axis1=1, axis2=2) - 2
    I2 = np.linalg.det(Cg) - 1
    B, D = m.mat.B, m.mat.D
    lam = np.sqrt(np.linalg.eigvalsh(Cg))
    expect = np.sum(m.tri_area * (B / 4 * (0.5 * I1 ** 2 + I1 - I2) + D / 4 * np.sum((lam - 1) ** 4, axis=1)))
    E, _ = energy.skalak_energy(x, m)
    assert np.isclose(E, expect, rtol=1e-10)


def test_skalak_small_strain_shear_modulus():
    """Small principal strains e1, e2: E = A (B/2)(e1^2 + e2^2) + O(e^3), i.e. the
    in-plane shear modulus is B/2 (the reading behind B = 2 * 5.3 pN/um)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0.]])
    T = np.array([[0, 1, 2], [1, 3, 2]])
    m = Model(X, T, Material(), 0.1)
    e1, e2 = 1e-4, -3e-4
    E, _ = energy.skalak_energy(X @ np.diag([1 + e1, 1 + e2, 1]).T, m)
    assert np.isclose(E, 1.0 * m.mat.B / 2 * (e1 ** 2 + e2 ** 2), rtol=2e-3)


def test_skalak_drucker_stability():
    """Section 2.1.3: f'' > 0 for all stretches with the default B, D."""
    B, D = Material().B, Material().D
    lam = np.linspace(1e-3, 5, 100001)
    f2 = 1.5 * B * lam ** 2 - 0.5 * B + 3 * D * (lam - 1) ** 2
    assert f2.min() > 0
    num = (energy.skalak_df(lam + 1e-6, B, D) - energy.skalak_df(lam - 1e-6, B, D)) / 2e-6
    assert np.allclose(num, f2, rtol=1e-6, atol=1e-6)


# ---- bending ----------------------------------------------------------------------

def test_bending_uniform_scaling_closed_form():
    m = oracle_model(642)
    for s in (0.7, 1.0, 1.2):
        E, _ = energy.bending_energy(s * m.X, m)
        expect = 0.5 * m.mat.k_bend * np.sum(m.vor_area * m.ell0_norm ** 2) * (s - 1) ** 2
        assert np.isclose(E, expect, rtol=1e-10, atol=1e-14)


def test_sphere_laplacian_is_twice_mean_curvature():
    """Laplace-Beltrami of the coordinates is -2 H n, so |l0| -> 2 / R on a fine sphere."""
    m = oracle_model(2562, "sphere")
    R = 3.0
    assert abs(np.median(m.ell0_norm) - 2 / R) / (2 / R) < 0.01
    assert np.sum(m.vor_area) == pytest.approx(m.tri_area.sum(), rel=1e-12)


# ---- volume -----------------------------------------------------------------------

def test_volume_closed_forms():
    v, f = meshes.octahedron()
    assert np.isclose(volume(v, f), 4.0 / 3.0, rtol=1e-14)
    v, f = meshes.icosahedron()                       # circumradius 1
    a = np.linalg.norm(v[f[0, 0]] - v[f[0, 1]])
    assert np.isclose(volume(v, f), 5.0 / 12.0 * (3 + 5 ** 0.5) * a ** 3, rtol=1e-13)
    assert np.isclose(volume(v + [3.0, -2.0, 7.0], f), volume(v, f), rtol=1e-13)


def test_volume_gradient_exact_on_closed_mesh():
    m = oracle_model(258)
    x = deformed(m, 0.1, 4)
    g = volume_gradient(x, m.tris)
    h = 0.05   # V is affine in any single coordinate, so the central difference is exact
    for i, k in [(0, 0), (17, 1), (200, 2), (257, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        assert np.isclose((volume(xp, m.tris) - volume(xm, m.tris)) / (2 * h), g[i, k], rtol=1e-10, atol=1e-12)
    assert np.abs(g.sum(axis=0)).max() < 1e-12


# ---- common invariants of all four terms -------------------------------------------

@pytest.mark.parametrize("name", TERMS)
def test_zero_at_rest(name):
    m = oracle_model(642)
    Gn = energy.volume_normaliser(m.X, m)
    E, g = term(name, m.X, m, Gn)
    assert abs(E) < 1e-10 and np.abs(g).max() < 1e-10


@pytest.mark.parametrize("name", TERMS)
def test_finite_difference_gradient(name):
    m = oracle_model(258)
    x = deformed(m, 0.06, 2)
    Gn = energy.volume_normaliser(deformed(m, 0.03, 9), m)
    E, g = term(name, x, m, Gn)
    h = 1e-6
    rng = np.random.default_rng(5)
    for i, k in zip(rng.integers(0, m.n, 12), rng.integers(0, 3, 12)):
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (term(name, xp, m, Gn)[0] - term(name, xm, m, Gn)[0]) / (2 * h)
        assert np.isclose(fd, g[i, k], rtol=1e-5, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("name", TERMS)
def test_rigid_invariance_and_momentum(name):
    """Noether (section 2.1): rigid-motion invariant energies conserve linear and
    angular momentum, i.e. sum f = 0 and sum x x f = 0."""
    m = oracle_model(258)
    x = deformed(m, 0.06, 3)
    Gn = energy.volume_normaliser(m.X, m)
    E, g = term(name, x, m, Gn)
    R = random_rotation(11)
    E2, g2 = term(name, x @ R.T + [1.5, -4.0, 0.25], m, Gn)
    assert np.isclose(E, E2, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g2, g @ R.T, atol=1e-9 * max(1.0, np.abs(g).max()))
    scale = np.abs(g).max() * m.n
    assert np.abs(g.sum(axis=0)).max() < 1e-11 * scale
    assert np.abs(np.cross(x, g).sum(axis=0)).max() < 1e-10 * scale


# ---- matrices ---------------------------------------------------------------------

def test_mass_and_L_structure():
    m = oracle_model(642)
    assert np.isclose(m.mass.sum(), m.mat.density * m.V0, rtol=1e-13)
    assert np.allclose(m.L, m.L.T, atol=1e-9)
    assert np.allclose(m.L_damp @ np.ones(m.n), 0, atol=1e-8)
    assert np.allclose(m.L @ np.ones(m.n), m.mat.k_volume, atol=1e-8)
    w = np.linalg.eigvalsh(m.L_damp)
    assert w.min() > -1e-8 * w.max()
    np.linalg.cholesky(m.Ht)


def test_L_matches_quadratic_part_of_pd_energies():
    """u^T L' u equals twice the sum of the PD quadratic forms evaluated element by
    element: area triangles A_t C |E_u D_m^-1|^2 and bending vertices k A_i |G_i u|^2
    (eq. fullyDeveloped_g); K_mat likewise with A_t k_mat."""
    m = oracle_model(258)
    u = np.random.default_rng(8).standard_normal((m.n, 3))
    Eu = np.stack([u[m.tris[:, 0]] - u[m.tris[:, 2]], u[m.tris[:, 1]] - u[m.tris[:, 2]]], axis=2)
    Fu = Eu @ m.Dm_inv
    tri = np.sum(m.tri_area * m.mat.C * np.sum(Fu * Fu, axis=(1, 2)))
    mat = np.sum(m.tri_area * m.mat.k_mat_value * np.sum(Fu * Fu, axis=(1, 2)))
    assert np.isclose(np.sum(u * (m.K_mat @ u)), mat, rtol=1e-10)
    nb = meshes.edges_of(m.tris.astype(np.int32))
    ell = np.zeros_like(u)
    for i, j in nb:
        ell[i] += m.G_bend[i, j] * (u[j] - u[i])
        ell[j] += m.G_bend[j, i] * (u[i] - u[j])
    bend = np.sum(m.mat.k_bend * m.vor_area * np.sum(ell * ell, axis=1))
    assert np.isclose(np.sum(u * (m.L_damp @ u)), tri + bend, rtol=1e-10)


# ---- global area (optional term) -------------------------------------------------------

def test_area_gradient_euler_relation_and_invariances():
    """The total area is homogeneous of degree 2 in the positions (and the volume of
    degree 3), so Euler's relation fixes sum_k x_k . grad A_k = 2 A (and = 3 V for the
    volume), independently of how the gradients are formed; translation and rotation
    invariance give sum grad A = 0 and sum x x grad A = 0."""
    from oracle.model import area_gradient, surface_area
    m = oracle_model(642)
    x = deformed(m, 0.08, 12) + [2.0, -1.0, 0.5]
    gA, gV = area_gradient(x, m.tris), volume_gradient(x, m.tris)
    assert np.sum(x * gA) == pytest.approx(2.0 * surface_area(x, m.tris), rel=1e-12)
    assert np.sum(x * gV) == pytest.approx(3.0 * volume(x, m.tris), rel=1e-12)
    assert np.abs(gA.sum(axis=0)).max() < 1e-12 * np.abs(gA).sum()
    assert np.abs(np.cross(x, gA).sum(axis=0)).max() < 1e-12 * np.abs(x[:, None] * gA[:, :, None]).sum()
    h = 1e-6
    for i, k in [(0, 0), (100, 1), (641, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (surface_area(xp, m.tris) - surface_area(xm, m.tris)) / (2 * h)
        assert fd == pytest.approx(gA[i, k], rel=1e-6, abs=1e-9)


def test_global_area_energy_pins():
    """(k_A/2)(A - A0)^2 / G_A: zero with zero force at rest, its gradient against
    finite differences (G_A frozen), invariant under rigid motions, and a uniform
    scaling by s gives exactly (k_A/2)(s^2 - 1)^2 A0^2 / G_A."""
    m = oracle_model(258, k_area_global=40.0)
    GA = energy.area_normaliser(deformed(m, 0.03, 3), m)
    E0, g0 = energy.global_area_energy(m.X, m, GA)
    assert abs(E0) < 1e-12 * m.A0 ** 2 and np.abs(g0).max() < 1e-10
    s = 1.03
    Es, _ = energy.global_area_energy(s * m.X, m, GA)
    assert Es == pytest.approx(0.5 * 40.0 * (s * s - 1) ** 2 * m.A0 ** 2 / GA, rel=1e-10)
    x = deformed(m, 0.05, 4)
    E, g = energy.global_area_energy(x, m, GA)
    h = 1e-6
    for i, k in [(3, 0), (77, 1), (250, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (energy.global_area_energy(xp, m, GA)[0] - energy.global_area_energy(xm, m, GA)[0]) / (2 * h)
        assert fd == pytest.approx(g[i, k], rel=1e-5, abs=1e-7 * np.abs(g).max())
    R = random_rotation(5)
    E2, g2 = energy.global_area_energy(x @ R.T - 3.0, m, GA)
    assert E2 == pytest.approx(E, rel=1e-10)
    np.testing.assert_allclose(g2, g @ R.T, atol=1e-10 * np.abs(g).max())
    # the global-area element adds k_A I to L (G = I, like the volume element)
    assert np.allclose(m.L @ np.ones(m.n), m.mat.k_volume + 40.0, atol=1e-8)


def test_step_with_global_area_matches_brute_force_newton():
    from oracle import newton, step
    from oracle.model import Model, Material
    X, T = meshes.sphere_mesh(42, 3.0)
    mm = Model(X, T, Material(k_area_global=80.0), 0.1)
    rng = np.random.default_rng(13)
    xn = X + 0.1 * rng.standard_normal(X.shape)
    vn, f = 0.01 * rng.standard_normal(X.shape), 5.0 * rng.standard_normal(X.shape)
    xa, _, info = step.step(mm, xn, vn, f, step.Params(tol=1e-13, polish=True))
    assert info.status & step.CONVERGED
    xb, ok = newton.newton_solve(step.Objective(mm, xn, vn, f), xn + 0.01)
    assert ok and np.abs(xa - xb).max() <= 1e-10 * np.ptp(X)


# ---- the paper's literal volume normaliser ---------------------------------------------

def test_literal_volume_normaliser():
    """The literal form takes |grad C|^2 at the current x: at x = x_n it coincides with
    the frozen form; its force equals the paper's PD force k (x - p(x)) with the
    projection p(x) = x - C grad C / |grad C|^2 assembled explicitly; once C != 0 that
    force differs from the derivative of its own energy (which the frozen form avoids)."""
    m = oracle_model(258)
    xn = deformed(m, 0.04, 6)
    x = xn + 0.03 * np.random.default_rng(2).standard_normal(xn.shape)
    Gn = energy.volume_normaliser(xn, m)
    Ef, gf = energy.volume_energy(xn, m, Gn)
    El, gl = energy.volume_energy(xn, m, None)
    assert El == Ef and np.array_equal(gl, gf)
    C = volume(x, m.tris) - m.V0
    gC = volume_gradient(x, m.tris)
    p = x - C * gC / np.sum(gC * gC)
    _, gl = energy.volume_energy(x, m, None)
    np.testing.assert_allclose(gl, m.mat.k_volume * (x - p), rtol=0, atol=1e-9 * np.abs(gl).max())
    i, k, h = 10, 2, 1e-6
    xp, xm = x.copy(), x.copy()
    xp[i, k] += h
    xm[i, k] -= h
    fd = (energy.volume_energy(xp, m, None)[0] - energy.volume_energy(xm, m, None)[0]) / (2 * h)
    assert abs(C) > 1e-3 and abs(fd - gl[i, k]) > 1e-6 * abs(gl[i, k])


# ---- collapsed triangles --------------------------------------------------------------

def test_collapsed_triangle_reading():
    """A triangle squeezed to a segment (one vertex on the opposite edge) has no second
    in-plane direction: every term stays finite, its in-plane forces act along the
    segment only, and the step reports DEGENERATE_TRI when the final positions still
    hold a collapsed triangle."""
    from oracle import step
    m = oracle_model(66)
    x = m.X.copy()
    a, b, c = m.tris[5]
    x[c] = 0.5 * (x[a] + x[b])                       # triangle 5 collapses onto edge ab
    assert energy.collapsed_triangles(x, m)[5] and energy.collapsed_triangles(x, m).sum() >= 1
    for name in ("area", "skalak"):
        E, g = term(name, x, m, energy.volume_normaliser(x, m))
        assert np.isfinite(E) and np.all(np.isfinite(g))
    # the in-plane terms of triangle 5 alone: forces parallel to the segment a-b
    from oracle.model import Model
    single = Model.__new__(Model)
    single.__dict__.update(m.__dict__)
    single.tris = m.tris[5:6]
    single.Dm_inv, single.tri_area = m.Dm_inv[5:6], m.tri_area[5:6]
    for fn in (energy.area_energy, energy.skalak_energy):
        _, g = fn(x, single)
        d = (x[b] - x[a]) / np.linalg.norm(x[b] - x[a])
        for v in (a, b, c):
            assert np.linalg.norm(np.cross(g[v], d)) <= 1e-9 * max(1.0, np.linalg.norm(g[v]))
    # a step that cannot undo the collapse (vertices pinned by huge masses is not an
    # option here), so check the flag on the status of a minimisation that starts and
    # stops there: max_iter 0 iterations of work, the first guess kept
    obj = step.Objective(m, x, np.zeros_like(x), np.zeros_like(x))
    _, info = step.minimise(obj, x, step.Params(max_iter=0))
    assert info.status & step.DEGENERATE_TRI
