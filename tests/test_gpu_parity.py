"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by
element on the same seeded inputs.

Tolerances: positions within 1e-5 of the cell diameter in FP32 plans and 1e-10 in
FP64 plans; gradients and objectives within the FP32/FP64 rounding of their largest
terms (1e-5 / 1e-11 relative)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from rbc_inputs import workloads
from conftest import oracle_model

pytestmark = pytest.mark.gpu

DT = workloads.DT_US


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    yield


def dev():
    return torch.device("cuda:0")


def T(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def make(meshes, precision="fp32", **prm):
    from paper_1903_06479_amd import Mesh, Plan, default_params
    params = default_params(precision=precision, **prm)
    return Plan([Mesh(*m) for m in meshes], DT, params=params)


def oracle_step(model, xn, vn, f, tol=1e-12, x_start=None):
    """The oracle's stationary point of the step (residual <= tol, continuing on residual
    decrease where the Armijo test stops resolving g)."""
    import oracle.step as ostep
    return ostep.step(model, xn, vn, f, ostep.Params(tol=tol, polish=True), x_start=x_start)


# ---- the MFMA product with the dense inverses -------------------------------------

@pytest.mark.parametrize("precision,n,bf16", [("fp32", 642, 0), ("fp64", 258, 0), ("fp32", 258, 0), ("fp64", 642, 0),
                                              ("fp32", 642, 1), ("fp32", 2562, 1),
                                              ("fp32", 258, 2), ("fp32", 642, 2), ("fp32", 2562, 2)])
def test_apply_inverse_matches_oracle(precision, n, bf16):
    """The matrix-core product with the dense inverses.  BF16 products (exact FP32
    diagonal + BF16 off-diagonal part) are checked against the bound their rounding
    allows: 2^-7 of the off-diagonal contribution; the banded ones (bf16 = 2) may in
    addition drop entries below 1e-4 sqrt(A_ii A_jj), which bounds the dropped part of
    out[r][j] by 1e-4 sqrt(A_jj) sum_i |q[r][i]| sqrt(A_ii).  The 2562-vertex case runs
    the banded product in several k chunks."""
    m = oracle_model(n)
    plan = make([(m.X, m.tris)], precision, inverse_bf16=bf16)
    dt = torch.float64 if precision == "fp64" else torch.float32
    npad = plan.n_pad(0)
    rows = 53                                        # spans several 48-row launches + a ragged tail
    rng = np.random.default_rng(n)
    q = np.zeros((rows, npad))
    q[:, :n] = rng.standard_normal((rows, n))
    tol = 2e-6 if precision == "fp32" else 1e-13
    for which, Ainv in ((0, np.linalg.inv(m.Ht)), (1, DT * DT * np.linalg.inv(m.Mt))):
        ref = q[:, :n] @ Ainv
        out = plan.apply_inverse(0, which, T(q, dt)).cpu().numpy().astype(np.float64)
        if bf16:
            off = Ainv - np.diag(np.diag(Ainv))
            # both operands are rounded to BF16 (unit roundoff 2^-8 each)
            bound = 1.01 * 2.0 ** -7 * (np.abs(q[:, :n]) @ np.abs(off)) + 1e-6 * np.abs(ref)
            if bf16 == 2:
                sd = np.sqrt(np.abs(np.diag(Ainv)))
                bound += 1.0001e-4 * np.outer(np.abs(q[:, :n]) @ sd, sd)
            assert np.all(np.abs(out[:, :n] - ref) <= bound)
        else:
            scale = np.abs(ref).max()
            assert np.abs(out[:, :n] - ref).max() <= tol * scale * np.sqrt(n)
        assert np.abs(out[:, n:]).max() == 0.0


# ---- the paper's route: substitution with the banded Cholesky factor ---------------

@pytest.mark.parametrize("precision,n", [("fp32", 258), ("fp32", 642), ("fp32", 2562), ("fp64", 258),
                                         ("fp64", 642), ("fp64", 2562)])
def test_solve_factor_matches_oracle(precision, n):
    """out = A^-1 q by forward and back substitution with the banded Cholesky factor of
    A = H~ or M~/h^2 (reverse Cuthill-McKee order), against the oracle's solve.  Bound:
    a Cholesky solve returns x with (A + dA) x = q, |dA| <= gamma |L||L^T|
    (Higham, Accuracy and Stability of Numerical Algorithms, thm 10.4), gamma = (3b + 6) u
    for a factor of half bandwidth b rounded to unit roundoff u; by Cauchy-Schwarz
    (|L||L^T|)_ij <= sqrt(A_ii A_jj), and each row of |L||L^T| has at most 4b + 1
    non-zeros.  130 right-hand sides: three waves of 64, the last one ragged."""
    m = oracle_model(n)
    plan = make([(m.X, m.tris)], precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    npad = plan.n_pad(0)
    b = plan.factor_bandwidth(0)
    assert 0 < b < n // 2
    rows = 130
    rng = np.random.default_rng(n + 1)
    q = np.zeros((rows, npad))
    q[:, :n] = rng.standard_normal((rows, n))
    q = q.astype(np.float32).astype(np.float64) if precision == "fp32" else q
    gamma = 1.01 * (3 * b + 6) * u
    for which, A, solve in ((0, m.Ht, m.solve_Ht), (1, m.Mt / (DT * DT), lambda r: DT * DT * m.solve_Mt(r))):
        out = plan.solve_factor(0, which, T(q, dt)).cpu().numpy().astype(np.float64)
        assert np.abs(out[:, n:]).max() == 0.0
        x = out[:, :n]
        resid = np.abs(q[:, :n] - x @ A)                     # A symmetric
        sd = np.sqrt(np.diag(A))
        w = np.sort(np.abs(x) * sd, axis=1)[:, ::-1][:, :4 * b + 1].sum(axis=1)
        assert np.all(resid <= gamma * np.outer(w, sd))
        # against the oracle's solution: x - ref = A^-1 (A x - q)
        ref = solve(q[:, :n].T).T
        inv_norm = 1.0 / np.linalg.eigvalsh(A)[0]
        err = np.linalg.norm(x - ref, axis=1)
        assert np.all(err <= 1.01 * inv_norm * np.linalg.norm(resid, axis=1) + 1e-12 * np.linalg.norm(ref, axis=1))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_solve_factor_second_mesh_and_row_counts(precision):
    """A plan of two mesh types (258 and 642 vertices, different n_pad and bands): the
    solves of mesh index 1 with 1, 64 (one full wave) and 65 right-hand sides, each
    against the oracle's solve within the backward-error bound of
    test_solve_factor_matches_oracle; mesh index 0 is solved by its own factor."""
    from paper_1903_06479_amd import Mesh, Plan, default_params
    m0, m1 = oracle_model(258), oracle_model(642)
    plan = Plan([Mesh(m0.X, m0.tris), Mesh(m1.X, m1.tris)], DT, params=default_params(precision=precision))
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    rng = np.random.default_rng(11)
    for mi, m in ((1, m1), (0, m0)):
        n, npad, b = m.X.shape[0], plan.n_pad(mi), plan.factor_bandwidth(mi)
        gamma = 1.01 * (3 * b + 6) * u
        sd = np.sqrt(np.diag(m.Ht))
        for rows in (1, 64, 65):
            q = np.zeros((rows, npad))
            q[:, :n] = rng.standard_normal((rows, n))
            q = q.astype(np.float32).astype(np.float64) if precision == "fp32" else q
            out = plan.solve_factor(mi, 0, T(q, dt)).cpu().numpy().astype(np.float64)
            assert np.abs(out[:, n:]).max() == 0.0
            x = out[:, :n]
            resid = np.abs(q[:, :n] - x @ m.Ht)
            w = np.sort(np.abs(x) * sd, axis=1)[:, ::-1][:, :4 * b + 1].sum(axis=1)
            assert np.all(resid <= gamma * np.outer(w, sd)), (mi, rows)
            ref = m.solve_Ht(q[:, :n].T).T
            err = np.linalg.norm(x - ref, axis=1)
            inv_norm = 1.0 / np.linalg.eigvalsh(m.Ht)[0]
            assert np.all(err <= 1.01 * inv_norm * np.linalg.norm(resid, axis=1) + 1e-12 * np.linalg.norm(ref, axis=1))


@pytest.mark.parametrize("kind,n,k_mat", [("sphere", 642, None), ("rbc", 642, 0.0), ("rbc", 258, 0.0)])
def test_solve_factor_other_meshes_and_materials(kind, n, k_mat):
    """The factor route on a different H~: the sphere mesh (another vertex graph and
    band), and H~ without the material term (k_mat = 0, section 2.1.1), FP32, against the
    oracle's solve of its own H~ within the backward-error bound of
    test_solve_factor_matches_oracle."""
    from paper_1903_06479_amd import Mesh, Plan, default_material, default_params
    kw = {} if k_mat is None else {"k_mat": k_mat}
    m = oracle_model(n, kind=kind, **kw)
    mat = default_material(**({} if k_mat is None else {"k_mat": k_mat}))
    plan = Plan([Mesh(m.X, m.tris)], DT, material=mat, params=default_params())
    npad, b = plan.n_pad(0), plan.factor_bandwidth(0)
    gamma = 1.01 * (3 * b + 6) * 2.0 ** -24
    rng = np.random.default_rng(n + 7)
    rows = 70
    q = np.zeros((rows, npad))
    q[:, :n] = rng.standard_normal((rows, n))
    q = q.astype(np.float32).astype(np.float64)
    out = plan.solve_factor(0, 0, T(q, torch.float32)).cpu().numpy().astype(np.float64)
    assert np.abs(out[:, n:]).max() == 0.0
    x = out[:, :n]
    resid = np.abs(q[:, :n] - x @ m.Ht)
    sd = np.sqrt(np.diag(m.Ht))
    w = np.sort(np.abs(x) * sd, axis=1)[:, ::-1][:, :4 * b + 1].sum(axis=1)
    assert np.all(resid <= gamma * np.outer(w, sd))
    ref = m.solve_Ht(q[:, :n].T).T
    err = np.linalg.norm(x - ref, axis=1)
    inv_norm = 1.0 / np.linalg.eigvalsh(m.Ht)[0]
    assert np.all(err <= 1.01 * inv_norm * np.linalg.norm(resid, axis=1) + 1e-12 * np.linalg.norm(ref, axis=1))


def test_solve_factor_arguments_and_workspace_reuse():
    """Workspace size checks, rows = 0, a bad `which`, and one workspace reused by two
    calls of different sizes (the second smaller)."""
    from paper_1903_06479_amd._native import NpfemError
    m = oracle_model(642)
    plan = make([(m.X, m.tris)])
    npad = plan.n_pad(0)
    need = plan.solve_factor_workspace(0, 200)
    assert need == 256 * npad * 4
    work = torch.empty(need, dtype=torch.uint8, device=dev())
    rng = np.random.default_rng(5)
    q = np.zeros((200, npad), np.float32)
    q[:, :642] = rng.standard_normal((200, 642))
    big = plan.solve_factor(0, 0, T(q, torch.float32), work=work).cpu().numpy()
    small = plan.solve_factor(0, 0, T(q[:70], torch.float32), work=work).cpu().numpy()
    assert np.array_equal(small, big[:70])
    with pytest.raises(NpfemError):
        plan.solve_factor(0, 0, T(q, torch.float32), work=work[: need - 1])
    with pytest.raises(NpfemError):
        plan.solve_factor(0, 2, T(q, torch.float32), work=work)
    empty = torch.zeros((0, npad), dtype=torch.float32, device=dev())
    assert plan.solve_factor(0, 0, empty, work=work).shape == (0, npad)


# ---- objective and gradient -------------------------------------------------------

def eval_case(n, precision, n_cells=6, seed=3):
    import oracle.step as ostep
    from paper_1903_06479_amd import Batch
    m = oracle_model(n)
    rng = np.random.default_rng(seed)
    plan = make([(m.X, m.tris)], precision)
    batch = Batch(plan, np.zeros(n_cells, np.int32))
    dt = plan.torch_dtype
    xs, vs, fs, us = [], [], [], []
    for c in range(n_cells):
        xs.append(m.X @ workloads.random_rotation(rng).T + 0.05 * rng.standard_normal(m.X.shape))
        vs.append(0.01 * rng.standard_normal(m.X.shape))
        fs.append(2.0 * rng.standard_normal(m.X.shape))
        us.append(2e-3 * rng.standard_normal(m.X.shape))
    cat = lambda a: np.concatenate(a)
    # inputs rounded to the plan's precision first, so both sides see the same numbers
    rnd = (lambda a: a.astype(np.float32).astype(np.float64)) if precision == "fp32" else (lambda a: a)
    xs, vs, fs, us = ([rnd(a) for a in arr] for arr in (xs, vs, fs, us))
    grad, terms = batch.eval(T(cat(xs), dt), T(cat(vs), dt), T(cat(fs), dt), T(cat(us), dt))
    grad = grad.cpu().numpy().astype(np.float64)
    terms = terms.cpu().numpy()
    out = []
    for c in range(n_cells):
        obj = ostep.Objective(m, xs[c], vs[c], fs[c])
        x = xs[c] + us[c]
        g, gr, noise = obj(x)
        w = obj.y - obj.x_n
        g_u = g - 0.5 * np.sum(w * (m.Mt @ w)) / DT ** 2     # drop the constant of the inertial term
        Mu = m.mass[:, None] * us[c] / DT ** 2
        scale = max(np.abs(Mu).max(), np.abs(obj.b).max(), np.abs(gr - Mu + obj.b).max())
        out.append(dict(g=g_u, grad=gr, noise=noise, resid=obj.residual(x, gr), scale=scale,
                        gpu_grad=grad[c * n:(c + 1) * n], gpu_terms=terms[c]))
    return out


@pytest.mark.parametrize("precision,n,tol", [("fp32", 642, 2e-5), ("fp32", 258, 2e-5), ("fp64", 258, 1e-11),
                                             ("fp64", 642, 1e-11)])
def test_eval_matches_oracle(precision, n, tol):
    for c in eval_case(n, precision):
        assert np.abs(c["gpu_grad"] - c["grad"]).max() <= tol * c["scale"]
        assert abs(c["gpu_terms"][0] - c["g"]) <= tol * c["noise"]
        assert abs(c["gpu_terms"][7] - c["resid"]) <= max(tol * 10, 1e-3 * c["resid"])


# ---- the step -----------------------------------------------------------------------

def run_step(plan, cell_mesh, x, v, f, **kw):
    from paper_1903_06479_amd import Batch
    batch = Batch(plan, cell_mesh)
    dt = plan.torch_dtype
    xo, vo, st = batch.step(T(x, dt), T(v, dt), T(f, dt), **kw)
    torch.cuda.synchronize()
    return (xo.cpu().numpy().astype(np.float64), vo.cpu().numpy().astype(np.float64),
            batch.stats_to_numpy(st), batch)


def rounded(a, precision):
    return a.astype(np.float32).astype(np.float64) if precision == "fp32" else a


def test_step_fp32_shear_matches_oracle():
    """One FP32 step of 21 perturbed 642-vertex cells in drag towards shear flows
    (several tiles and a ragged tail) against the converged FP64 oracle."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=21, seed=1002)
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    plan = make([(X, Tr)], "fp32", cells_per_tile=5)
    xo, vo, st, _ = run_step(plan, np.zeros(21, np.int32), x, v, f)
    assert np.all(st["status"] == CONVERGED), st
    D = np.ptp(X[:, 0])
    for c in range(21):
        s = b.cell_slice(c)
        xr, vr, info = oracle_step(m, x[s], v[s], f[s])
        assert np.abs(xo[s] - xr).max() <= 1e-5 * D
        ur = xr - x[s]
        assert np.abs((xo[s] - x[s]) - ur).max() <= 1e-3 * np.abs(ur).max() + 1e-6
        assert np.abs(vo[s] - vr).max() <= 1e-3 * np.abs(vr).max() + 1e-5


def test_step_fp32_bf16_products_same_solution():
    """BF16 products with the inverses (dense or banded) only precondition the iteration:
    the converged positions agree with the FP32-product path and the oracle within
    tolerance."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=12, seed=77)
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    res = {}
    for bf in (0, 1, 2):
        xo, vo, st, _ = run_step(make([(X, Tr)], "fp32", inverse_bf16=bf), np.zeros(12, np.int32), x, v, f)
        assert np.all(st["status"] == CONVERGED), st
        res[bf] = (xo, st["iterations"])
    D = np.ptp(X[:, 0])
    for bf in (1, 2):
        assert np.abs(res[0][0] - res[bf][0]).max() <= 1e-5 * D
        assert res[bf][1].mean() <= res[0][1].mean() + 1.0
        for c in (0, 7):
            s = b.cell_slice(c)
            xr, _, _ = oracle_step(m, x[s], v[s], f[s])
            assert np.abs(res[bf][0][s] - xr).max() <= 1e-5 * D


def test_step_tile_size_and_repeat_bitwise():
    """Cells never interact, so the result of a cell must not depend on which tile it
    lands in, and two runs must agree bit for bit (no atomics in the arithmetic)."""
    b = workloads.shear(n_cells=23, seed=5)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    ref = None
    for tcells in (1, 5, 16, 21, 16):
        plan = make([(X, Tr)], "fp32", cells_per_tile=tcells)
        xo, vo, st, _ = run_step(plan, np.zeros(23, np.int32), x, v, f)
        if ref is None:
            ref = (xo, vo, st["iterations"])
        else:
            np.testing.assert_array_equal(xo, ref[0])
            np.testing.assert_array_equal(vo, ref[1])
            np.testing.assert_array_equal(st["iterations"], ref[2])


@pytest.mark.parametrize("lbfgs_m", [2, 8])
def test_cell_state_placement_is_bitwise_neutral(lbfgs_m):
    """A tile's per-cell L-BFGS state lives in LDS when that costs no workgroups per CU
    and in the workspace otherwise; at the 642-vertex mesh one tile (LDS) and 5 or 16
    cells per tile (the workspace, for history 8 or 2) must give identical bits."""
    b = workloads.shear(n_cells=23, seed=6)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    ref = None
    for tcells in (1, 5, 16):
        plan = make([(X, Tr)], "fp32", cells_per_tile=tcells, lbfgs_m=lbfgs_m)
        xo, vo, st, _ = run_step(plan, np.zeros(23, np.int32), x, v, f)
        if ref is None:
            ref = (xo, vo, st["iterations"])
        else:
            np.testing.assert_array_equal(xo, ref[0])
            np.testing.assert_array_equal(vo, ref[1])
            np.testing.assert_array_equal(st["iterations"], ref[2])


def test_large_mesh_tiles_build_and_agree():
    """2562-vertex cells use nearly all of a CU's LDS, so the cell states must fall back
    to the workspace where they do not fit (a batch of 16-cell tiles used to fail to
    build); 1- and 16-cell tiles converge and agree bit for bit."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=16, n_verts=2562, seed=7)
    X, Tr = b.meshes[2562]
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    ref = None
    for tcells in (16, 1):
        plan = make([(X, Tr)], "fp32", cells_per_tile=tcells, lbfgs_m=2)
        xo, vo, st, _ = run_step(plan, np.zeros(16, np.int32), x, v, f)
        assert np.all(st["status"] & CONVERGED), st["status"]
        if ref is None:
            ref = (xo, vo)
        else:
            np.testing.assert_array_equal(xo, ref[0])
            np.testing.assert_array_equal(vo, ref[1])


def test_step_fp64_stretch_trajectory():
    """The optical-tweezers load on one 258-vertex cell, FP64, ramped to 200 pN over
    20 steps; each side follows its own trajectory; positions within 1e-10 D."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.stretch()
    X, Tr = b.meshes[258]
    m = oracle_model(258)
    plan = make([(X, Tr)], "fp64", tol=1e-10)
    from paper_1903_06479_amd import Batch
    batch = Batch(plan, np.zeros(1, np.int32))
    xg, vg = T(X, torch.float64), T(np.zeros_like(X), torch.float64)
    xr, vr = X.copy(), np.zeros_like(X)
    D = np.ptp(X[:, 0])
    for k in range(1, 21):
        f = workloads.stretch_forces(b, k, total_steps=20)
        xg, vg, st = batch.step(xg, vg, T(f, torch.float64))
        xr, vr, _ = oracle_step(m, xr, vr, f)
        s = batch.stats_to_numpy(st)
        assert s["status"][0] == CONVERGED
        err = np.abs(xg.cpu().numpy() - xr).max() / D
        assert err <= 1e-10, (k, err)
    assert np.ptp(xr[:, 0]) > D                    # it did stretch


@pytest.mark.parametrize("bf16,tile", [(0, 0), (2, 0), (2, 7)])
def test_step_uneven_mesh_mix(bf16, tile):
    """258/642/2562-vertex cells in one launch (FP32) against the oracle: FP32 products,
    and banded BF16 products (the 2562-vertex products staged in several k chunks), also
    with 7-cell tiles (21 rows: two 16-row blocks per product)."""
    from paper_1903_06479_amd import Batch, CONVERGED
    b = workloads.uneven(n_cells=200, cells=np.arange(12))
    sizes = sorted(b.meshes)
    meshes = [b.meshes[k] for k in sizes]
    cm = np.array([sizes.index(int(k)) for k in b.cell_nverts], np.int32)
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v, step=0), "fp32")
    plan = make(meshes, "fp32", inverse_bf16=bf16)
    batch = Batch(plan, cm)
    if tile:
        batch.schedule(cells_per_tile=tile)
    xo, vo, st = batch.step(T(x, torch.float32), T(v, torch.float32), T(f, torch.float32))
    torch.cuda.synchronize()
    xo, st = xo.cpu().numpy().astype(np.float64), batch.stats_to_numpy(st)
    assert np.all(st["status"] == CONVERGED), st
    for c in range(b.n_cells):
        s = b.cell_slice(c)
        n = int(b.cell_nverts[c])
        m = oracle_model(n)
        xr, _, _ = oracle_step(m, x[s], v[s], f[s])
        assert np.abs(xo[s] - xr).max() <= 1e-5 * np.ptp(m.X[:, 0]), (c, n)


def test_empty_batch_and_bad_mesh_index_are_rejected():
    """A batch of no cells, or with a cell of an unknown mesh, is refused with an error at
    creation (NPFEM_E_INVALID), before anything is launched."""
    from paper_1903_06479_amd import Batch
    X, Tr = workloads.shear(n_cells=1).meshes[642]
    plan = make([(X, Tr)], "fp32")
    with pytest.raises(RuntimeError, match="n_cells"):
        Batch(plan, np.zeros(0, np.int32))
    with pytest.raises(RuntimeError, match="mesh index"):
        Batch(plan, np.array([0, 1], np.int32))


def test_rest_cells_stay_put_and_nonfinite_is_flagged():
    """Zero force at the rest shape: a cell at rest with v = 0, F = 0 converges at the
    first guess and does not move (the mesh is given in FP32-representable coordinates,
    so the FP32 inputs are exactly the rest shape).  A cell with a NaN coordinate is
    flagged and returned unchanged without disturbing its tile mates."""
    from paper_1903_06479_amd import CONVERGED, NONFINITE
    m = oracle_model(642)
    X32 = rounded(m.X, "fp32")
    # cells: exact rest, a translated copy (re-rounded in FP32, so strained at the 1e-7
    # level), exact rest, poisoned
    x = np.concatenate([X32, rounded(X32 + 1.0, "fp32"), X32, X32])
    x[3 * 642 + 7, 1] = np.nan
    v = np.zeros_like(x)
    f = np.zeros_like(x)
    plan = make([(X32, m.tris)], "fp32", cells_per_tile=5)
    xo, vo, st, _ = run_step(plan, np.zeros(4, np.int32), x, v, f)
    for c in (0, 2):
        s = slice(642 * c, 642 * (c + 1))
        assert st["status"][c] == CONVERGED and st["iterations"][c] == 0
        np.testing.assert_array_equal(xo[s], x[s])
        assert np.abs(vo[s]).max() == 0.0
    assert st["status"][1] == CONVERGED
    assert np.abs(xo[642:1284] - x[642:1284]).max() <= 1e-6 * np.ptp(X32[:, 0])
    assert st["status"][3] == NONFINITE
    np.testing.assert_array_equal(np.isnan(xo[1926:]), np.isnan(x[1926:]))
    np.testing.assert_array_equal(xo[1926:][~np.isnan(x[1926:])], x[1926:][~np.isnan(x[1926:])])


def test_user_guess_does_not_change_the_solution():
    b = workloads.shear(n_cells=5, seed=9)
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    plan = make([(X, Tr)], "fp32")
    dt = torch.float32
    ref = [oracle_step(m, x[b.cell_slice(c)], v[b.cell_slice(c)], f[b.cell_slice(c)])[0] for c in range(5)]
    u_exact = np.concatenate(ref) - x
    u_pert = u_exact + 1e-3 * np.random.default_rng(0).standard_normal(x.shape)
    D = np.ptp(X[:, 0])
    for guess in (u_exact, u_pert):
        xo, _, st, _ = run_step(plan, np.zeros(5, np.int32), x, v, f, u_guess=T(guess, dt))
        assert np.abs(xo - np.concatenate(ref)).max() <= 1e-5 * D
    assert st["iterations"].max() >= 1


def test_momentum_balance_on_gpu():
    """sum m v_{n+1} = sum m v_n + h sum F_ext for every cell (internal forces and the
    Rayleigh term cancel; the dissipation keeps momentum)."""
    b = workloads.shear(n_cells=8, seed=11)
    X, Tr = b.meshes[642]
    rng = np.random.default_rng(1)
    x, v = b.x, 0.01 * rng.standard_normal(b.x.shape)
    f = 3.0 * rng.standard_normal(b.x.shape)
    plan = make([(X, Tr)], "fp64", tol=1e-10)
    xo, vo, st, _ = run_step(plan, np.zeros(8, np.int32), x, v, f)
    mass = plan.masses(0)[:, None]
    for c in range(8):
        s = b.cell_slice(c)
        lhs = (mass * vo[s]).sum(0)
        rhs = (mass * v[s]).sum(0) + DT * f[s].sum(0)
        assert np.abs(lhs - rhs).max() <= 1e-8 * np.abs(mass * v[s]).sum()


def test_multistep_fp32_trajectory():
    """Ten coupled steps (forces recomputed from each side's own state) of four cells."""
    b = workloads.throughput(n_cells=100000, cells=[0, 1, 2, 3])
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    from paper_1903_06479_amd import Batch
    plan = make([(X, Tr)], "fp32")
    batch = Batch(plan, np.zeros(4, np.int32))
    x = rounded(b.x, "fp32")
    xg, vg = T(x, torch.float32), T(np.zeros_like(x), torch.float32)
    xr, vr = x.copy(), np.zeros_like(x)
    D = np.ptp(X[:, 0])
    for k in range(10):
        fg = workloads.drag_forces(b, xg.cpu().numpy().astype(np.float64), vg.cpu().numpy().astype(np.float64))
        fr = workloads.drag_forces(b, xr, vr)
        xg, vg, _ = batch.step(xg, vg, T(fg, torch.float32))
        for c in range(4):
            s = b.cell_slice(c)
            xr[s], vr[s], _ = oracle_step(m, xr[s], vr[s], fr[s])
    assert np.abs(xg.cpu().numpy() - xr).max() <= 1e-5 * D


def test_drag_forces_kernel_matches_inputs_module():
    b = workloads.throughput(n_cells=100000, cells=[5, 6, 7])
    X, Tr = b.meshes[642]
    from paper_1903_06479_amd import Batch
    plan = make([(X, Tr)], "fp64")
    batch = Batch(plan, np.zeros(3, np.int32))
    v = 0.01 * np.random.default_rng(2).standard_normal(b.x.shape)
    ref = workloads.drag_forces(b, b.x, v)
    p = b.poiseuille
    f = batch.drag_forces(T(b.x, torch.float64), T(v, torch.float64),
                          T(np.full(3, workloads.drag_coefficient(642)), torch.float64),
                          T(b.shear_rate, torch.float64), T(b.origin, torch.float64),
                          p["umax"], p["radius"], p["axis_y"], p["axis_z"])
    np.testing.assert_allclose(f.cpu().numpy(), ref, rtol=1e-12, atol=1e-12)


def test_graph_replay_matches_eager_launch():
    """The step captured in a HIP graph on a (non-NULL) stream and replayed gives the
    eager result bit for bit, on every replay, with unrelated eager work and
    synchronisations in between; a caller alternating between two buffer sets (x -> x',
    then x' -> x) captures each set once and replays it afterwards."""
    from paper_1903_06479_amd import Batch, CELL_STATS_DTYPE
    b = workloads.shear(n_cells=12, seed=21)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    ref = Batch(plan, np.zeros(12, np.int32))
    xi, vi, fi = T(x, torch.float32), T(v, torch.float32), T(f, torch.float32)
    xe, ve, _ = ref.step(xi, vi, fi)
    xe2, ve2, _ = ref.step(xe, ve, fi)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    g = Batch(plan, np.zeros(12, np.int32))
    g.set_graph(True)
    with torch.cuda.stream(side):
        xa, va = xi.clone(), vi.clone()
        xb, vb = torch.empty_like(xi), torch.empty_like(vi)
        st = torch.empty(12 * CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev())
        for rep in range(4):
            xa.copy_(xi)
            va.copy_(vi)
            xb.fill_(0.0)
            g.step(xa, va, fi, x_out=xb, v_out=vb, stats=st, stream=side)      # set 1
            junk = (xi * 2.0).sum()                                            # eager work in between
            side.synchronize()
            assert torch.equal(xb, xe) and torch.equal(vb, ve), rep
            g.step(xb, vb, fi, x_out=xa, v_out=va, stats=st, stream=side)      # set 2
            side.synchronize()
            assert torch.equal(xa, xe2) and torch.equal(va, ve2), rep
            assert float(junk) == float(junk)
    counts = g.graph_counts()
    assert counts == {"captures": 2, "replays": 6}, counts
    # the NULL stream cannot be captured: those calls launch directly
    g.step(xi, vi, fi)
    assert g.graph_counts() == counts


def test_autotuner_keeps_the_solution():
    from paper_1903_06479_amd import Batch, CONVERGED
    b = workloads.shear(n_cells=40, seed=23)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    f = rounded(workloads.drag_forces(b, x, v), "fp32")
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(40, np.int32))
    xi, vi, fi = T(x, torch.float32), T(v, torch.float32), T(f, torch.float32)
    x0, _, _ = batch.step(xi, vi, fi)
    best = batch.autotune(xi, vi, fi)
    assert best["cells_per_tile"] in (2, 3, 5, 10, 16, 21) and best["lbfgs_m"] in (2, 3, 5) and best["best_ms"] > 0
    x1, _, st = batch.step(xi, vi, fi)
    torch.cuda.synchronize()
    assert np.all(batch.stats_to_numpy(st)["status"] == CONVERGED)
    assert (x1 - x0).abs().max().item() <= 1e-5 * np.ptp(X[:, 0])
    batch.schedule(cells_per_tile=7, lbfgs_m=1)
    assert batch.schedule()["cells_per_tile"] == 7
    x2, _, st = batch.step(xi, vi, fi)
    torch.cuda.synchronize()
    assert (x2 - x0).abs().max().item() <= 1e-5 * np.ptp(X[:, 0])


def test_c1_stretch_200_steps_matches_oracle_trajectory():
    """The full stretch run (one 258-vertex cell, 200 steps, FP64, m = 5) against the
    oracle at the FP64 tolerance 1e-10 D:
      * as configured (residual 1e-8): every step converges, and each checkpoint step
        (50, 100, 150, 200) on its own -- the oracle stepped from the GPU's state before
        that step -- agrees with the GPU's result of that step, positions and velocities;
      * the trajectory: positions at the checkpoints against the oracle's own 200-step
        trajectory (tests/golden/c1_stretch_oracle.json, every oracle step at residual
        <= 1e-12).  Errors of successive steps compound along a trajectory: at residual
        1e-8 the GPU's trajectory drifts to about 1.5e-10 D by step 150 while each step
        is within 2e-12 D of the oracle's, so the trajectory is run at residual 1e-10,
        the residual that delivers 1e-10 D along all 200 steps."""
    import json, os
    import oracle.step as ostep
    from paper_1903_06479_amd import Batch, CONVERGED
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1_stretch_oracle.json")))
    assert max(golden["residual"]) <= 1e-12 and all(s == 1 for s in golden["status"])
    b = workloads.stretch()
    X, Tr = b.meshes[258]
    m = oracle_model(258)
    D = np.ptp(X[:, 0])
    forces = [workloads.stretch_forces(b, k, total_steps=200) for k in range(1, 201)]
    for tol in (1e-8, 1e-10):
        # the line-search slack covers the rounding of the GPU's FP64 sums of g
        # (per-thread partial sums, then a tree: up to ~13 ulps of sum|terms|)
        plan = make([(X, Tr)], "fp64", tol=tol, lbfgs_m=5, noise_factor=64.0)
        batch = Batch(plan, np.zeros(1, np.int32))
        xg, vg = T(X, torch.float64), T(np.zeros_like(X), torch.float64)
        for k in range(1, 201):
            x_prev, v_prev = xg.cpu().numpy(), vg.cpu().numpy()
            xg, vg, st = batch.step(xg, vg, T(forces[k - 1], torch.float64))
            s = batch.stats_to_numpy(st)
            assert s["status"][0] == CONVERGED, (tol, k, s)
            if str(k) not in golden["x"]:
                continue
            xk = xg.cpu().numpy()
            err_traj = np.abs(xk - np.array(golden["x"][str(k)])).max() / D
            if tol == 1e-8:
                xr, vr, info = ostep.step(m, x_prev, v_prev, forces[k - 1], ostep.Params(tol=1e-12, m=5, polish=True))
                assert info.status == ostep.CONVERGED
                err_step = np.abs(xk - xr).max() / D
                err_v = np.abs(vg.cpu().numpy() - vr).max() / (D / DT)
                print(f"residual 1e-8, step {k}: this step from the GPU's state {err_step:.2e} D, velocity "
                      f"{err_v:.2e} D/h; trajectory {err_traj:.2e} D")
                assert err_step <= 1e-10, (k, err_step)
                assert err_v <= 1e-10, (k, err_v)
            else:
                print(f"residual 1e-10, step {k}: trajectory {err_traj:.2e} D")
                assert err_traj <= 1e-10, (k, err_traj)


def test_throughput_full_size_sampled_cells():
    """The 100,000-cell throughput step in the benchmark's launch configuration (5 cells
    per tile, history 2, BF16 products, HIP graph): every cell converges, and sampled
    cells agree with the converged FP64 oracle on the same (FP32) inputs within 1e-5 D,
    for the first step from rest and for the second step from the GPU's own state (with
    velocities within the velocity that tolerance implies, 1e-5 D / h)."""
    from paper_1903_06479_amd import Batch, CONVERGED
    b = workloads.throughput(n_cells=100000)
    X, Tr = b.meshes[642]
    D = np.ptp(X[:, 0])
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    batch.schedule(cells_per_tile=5, lbfgs_m=2)
    batch.set_graph(True)
    x = T(b.x, torch.float32)
    v = torch.zeros_like(x)
    zeta = torch.full((b.n_cells,), workloads.drag_coefficient(642), dtype=torch.float64, device=dev())
    p = b.poiseuille
    f = batch.drag_forces(x, v, zeta, T(b.shear_rate, torch.float64), T(b.origin, torch.float64),
                          p["umax"], p["radius"], p["axis_y"], p["axis_z"])
    xo, vo, st = batch.step(x, v, f)
    xo, vo, st = batch.step(x, v, f, x_out=xo, v_out=vo, stats=st)       # graph replay
    torch.cuda.synchronize()
    s = batch.stats_to_numpy(st)
    assert np.all(s["status"] == CONVERGED)
    m = oracle_model(642)
    xi, vi, fi, xg = (a.cpu().numpy().astype(np.float64) for a in (x, v, f, xo))
    for c in (0, 49999, 99999):
        sl = b.cell_slice(c)
        xr, _, _ = oracle_step(m, xi[sl], vi[sl], fi[sl])
        assert np.abs(xg[sl] - xr).max() <= 1e-5 * D, c
    # second step, from the GPU's state after the first
    f2 = batch.drag_forces(xo, vo, zeta, T(b.shear_rate, torch.float64), T(b.origin, torch.float64),
                           p["umax"], p["radius"], p["axis_y"], p["axis_z"])
    x2, v2, st2 = batch.step(xo, vo, f2)
    torch.cuda.synchronize()
    assert np.all(batch.stats_to_numpy(st2)["status"] == CONVERGED)
    xi, vi, fi, xg, vg = (a.cpu().numpy().astype(np.float64) for a in (xo, vo, f2, x2, v2))
    for c in (1, 50000, 99998):
        sl = b.cell_slice(c)
        xr, vr, _ = oracle_step(m, xi[sl], vi[sl], fi[sl])
        assert np.abs(xg[sl] - xr).max() <= 1e-5 * D, c
        assert np.abs(vg[sl] - vr).max() <= 1e-5 * D / workloads.DT_US, c


def test_no_history_fp64_matches_oracle():
    """History length 0 (the preconditioned gradient H~^-1 grad g every iteration) on
    FP64 642-vertex plans, whose vector passes take the unfused path: no stored pair is
    ever read, and the step reaches the oracle's stationary point (computed with m = 0
    too) within 1e-10 D."""
    import oracle.step as ostep
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=3, seed=41)
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    f = workloads.drag_forces(b, b.x, b.v)
    plan = make([(X, Tr)], "fp64", tol=1e-10, lbfgs_m=0, noise_factor=64.0, cells_per_tile=2)
    xo, vo, st, _ = run_step(plan, np.zeros(3, np.int32), b.x, b.v, f)
    assert np.all(st["status"] == CONVERGED), st
    D = np.ptp(X[:, 0])
    for c in range(3):
        s = b.cell_slice(c)
        xr, vr, _ = ostep.step(m, b.x[s], b.v[s], f[s], ostep.Params(tol=1e-12, m=0, polish=True))
        assert np.abs(xo[s] - xr).max() <= 1e-10 * D, c


def test_stats_totals_match_per_cell_results():
    """The device totals of npfem_stats_accumulate over several steps equal the sums and
    maxima of the per-cell results read back after each step."""
    from paper_1903_06479_amd import Batch, StatsTotal, CONVERGED, MAXITER
    b = workloads.shear(n_cells=37, seed=61)
    X, Tr = b.meshes[642]
    plan = make([(X, Tr)], "fp32", max_iter=4)              # some cells stop at MAXITER
    batch = Batch(plan, np.zeros(37, np.int32))
    x, v = T(b.x, torch.float32), T(b.v, torch.float32)
    total = StatsTotal()
    per = []
    for k in range(3):
        f = T(workloads.drag_forces(b, x.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)),
              torch.float32)
        x, v, st = batch.step(x, v, f)
        total.add(st, 37)
        per.append(batch.stats_to_numpy(st))
    tot = total.read()
    s = np.concatenate(per)
    assert tot["cell_steps"] == 3 * 37
    assert tot["iterations"] == s["iterations"].sum() and tot["evaluations"] == s["evaluations"].sum()
    assert tot["halvings"] == s["halvings"].sum() and tot["max_iterations"] == s["iterations"].max()
    assert tot["not_converged"] == np.sum((s["status"] & CONVERGED) == 0)
    assert tot["status_count"][0] == np.sum((s["status"] & MAXITER) != 0) > 0
    assert tot["max_residual"] == s["residual"].max()


def test_fp64_plans_cover_the_2562_vertex_mesh():
    """FP64 plans of the 2562-vertex mesh keep the current cell's x_n and trial u in the
    workspace (they do not fit the LDS beside the triangle chunks): one FP64 step of an
    uneven batch of 258/642/2562-vertex cells against the oracle within 1e-10 D."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.uneven(n_cells=200, cells=np.arange(9))
    sizes = sorted(b.meshes)
    assert 2562 in sizes
    cm = np.array([sizes.index(int(k)) for k in b.cell_nverts], np.int32)
    f = workloads.drag_forces(b, b.x, b.v, step=0)
    plan = make([b.meshes[k] for k in sizes], "fp64", tol=1e-10, noise_factor=64.0, cells_per_tile=2)
    xo, vo, st, _ = run_step(plan, cm, b.x, b.v, f)
    assert np.all(st["status"] == CONVERGED), st
    for c in range(b.n_cells):
        s = b.cell_slice(c)
        n = int(b.cell_nverts[c])
        m = oracle_model(n)
        xr, vr, _ = oracle_step(m, b.x[s], b.v[s], f[s])
        D = np.ptp(m.X[:, 0])
        assert np.abs(xo[s] - xr).max() <= 1e-10 * D, (c, n)
        assert np.abs(vo[s] - vr).max() <= 1e-10 * D / DT, (c, n)


def test_c3_uneven_fp32_matches_all_fp64_gpu_run():
    """The uneven configuration at full size (20,000 cells: 6,000 x 258, 10,000 x 642,
    4,000 x 2562 vertices), FP32 bulk with BF16 products in one persistent launch,
    against an all-FP64 GPU run of the same steps on the same (FP32) inputs, every mesh
    size included: positions within 1e-5 D for two steps, every cell converged in both."""
    from paper_1903_06479_amd import Batch, CONVERGED
    b = workloads.uneven(n_cells=20000)
    sizes = sorted(b.meshes)
    cm = np.array([sizes.index(int(n)) for n in b.cell_nverts], np.int32)
    assert [int(np.sum(b.cell_nverts == n)) for n in sizes] == [6000, 10000, 4000]
    meshes = [b.meshes[n] for n in sizes]
    b32 = Batch(make(meshes, "fp32", inverse_bf16=1), cm)
    b64 = Batch(make(meshes, "fp64"), cm)
    Ds = np.array([np.ptp(b.meshes[n][0][:, 0]) for n in sizes])[cm]
    row_D = np.repeat(Ds, b.cell_nverts)
    x, v = rounded(b.x, "fp32"), rounded(b.v, "fp32")
    for k in range(2):
        f = rounded(workloads.drag_forces(b, x, v, step=k), "fp32")
        x32, v32, s32 = b32.step(T(x, torch.float32), T(v, torch.float32), T(f, torch.float32))
        x64, _, s64 = b64.step(T(x, torch.float64), T(v, torch.float64), T(f, torch.float64))
        torch.cuda.synchronize()
        for st in (s32, s64):
            assert np.all(Batch.stats_to_numpy(st)["status"] == CONVERGED)
        xa = x32.cpu().numpy().astype(np.float64)
        err = np.abs(xa - x64.cpu().numpy()).max(axis=1) / row_D
        for n_i, n in enumerate(sizes):
            rows = np.repeat(cm == n_i, b.cell_nverts)
            print(f"step {k + 1}, {n} vertices: max |x32 - x64| / D = {err[rows].max():.2e}")
        assert err.max() <= 1e-5
        x, v = xa, v32.cpu().numpy().astype(np.float64)


# ---- optional terms: global area, the paper's literal volume normaliser, collapses ------

def _plan_with(meshes, precision, k_area_global=0.0, literal=False, **prm):
    from paper_1903_06479_amd import Mesh, Plan, default_material, default_params, _native as N
    params = default_params(precision=precision, **prm)
    params.volume_normaliser = N.VOLUME_PAPER_LITERAL if literal else N.VOLUME_STEP_FROZEN
    return Plan([Mesh(*m) for m in meshes], DT, material=default_material(k_area_global=k_area_global),
                params=params)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
@pytest.mark.parametrize("literal", [False, True])
def test_eval_optional_terms_and_collapsed_triangle_match_oracle(precision, tol, literal):
    """Objective terms and gradient with the global-area term switched on (k_A = 60),
    with the frozen or the literal volume normaliser, on perturbed cells and on a cell
    whose x_n has a collapsed triangle (one vertex on the opposite edge): gradient,
    global-area energy, total area and the count of collapsed triangles against the
    oracle."""
    import oracle.step as ostep
    from oracle import energy
    from oracle.model import surface_area
    from paper_1903_06479_amd import Batch
    m = oracle_model(258, k_area_global=60.0)
    rng = np.random.default_rng(17)
    xs, vs, fs, us = [], [], [], []
    for c in range(4):
        x = m.X @ workloads.random_rotation(rng).T + 0.05 * rng.standard_normal(m.X.shape)
        if c == 3:
            a, b, k = m.tris[40]
            x[k] = 0.5 * (x[a] + x[b])
        xs.append(x)
        vs.append(0.01 * rng.standard_normal(m.X.shape))
        fs.append(2.0 * rng.standard_normal(m.X.shape))
        us.append(np.zeros(m.X.shape) if c == 3 else 2e-3 * rng.standard_normal(m.X.shape))
    rnd = (lambda a: a.astype(np.float32).astype(np.float64)) if precision == "fp32" else (lambda a: a)
    xs, vs, fs, us = ([rnd(a) for a in arr] for arr in (xs, vs, fs, us))
    plan = _plan_with([(m.X, m.tris)], precision, 60.0, literal)
    batch = Batch(plan, np.zeros(4, np.int32))
    dt = plan.torch_dtype
    cat = lambda a: T(np.concatenate(a), dt)
    grad, terms = batch.eval(cat(xs), cat(vs), cat(fs), cat(us))
    grad, terms = grad.cpu().numpy().astype(np.float64), terms.cpu().numpy()
    for c in range(4):
        obj = ostep.Objective(m, xs[c], vs[c], fs[c], literal=literal)
        x = xs[c] + us[c]
        _, gr, noise = obj(x)
        Mu = m.mass[:, None] * us[c] / DT ** 2
        scale = max(np.abs(Mu).max(), np.abs(obj.b).max(), np.abs(gr - Mu + obj.b).max())
        assert np.abs(grad[c * m.n:(c + 1) * m.n] - gr).max() <= tol * scale, c
        e_area, _ = energy.global_area_energy(x, m, obj.GA)
        assert abs(terms[c][8] - e_area) <= tol * noise, c
        assert terms[c][9] == pytest.approx(surface_area(x, m.tris), rel=10 * tol)
        assert terms[c][10] == energy.collapsed_triangles(x, m).sum(), c
    assert terms[3][10] >= 1


def test_step_with_global_area_fp64_matches_oracle():
    """FP64 steps with the global-area term (k_A = 60, k_A I in H~) reach the oracle's
    stationary point within 1e-10 D; the reported total area of x_{n+1} is its area."""
    from oracle.model import surface_area
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=3, n_verts=258, seed=81)
    X, Tr = b.meshes[258]
    m = oracle_model(258, k_area_global=60.0)
    f = workloads.drag_forces(b, b.x, b.v)
    plan = _plan_with([(X, Tr)], "fp64", 60.0, tol=1e-10, noise_factor=64.0)
    xo, vo, st, _ = run_step(plan, np.zeros(3, np.int32), b.x, b.v, f)
    assert np.all(st["status"] == CONVERGED), st
    D = np.ptp(X[:, 0])
    for c in range(3):
        s = b.cell_slice(c)
        xr, vr, _ = oracle_step(m, b.x[s], b.v[s], f[s])
        assert np.abs(xo[s] - xr).max() <= 1e-10 * D, c
        assert st["area"][c] == pytest.approx(surface_area(xo[s], m.tris), rel=1e-12)


def test_literal_volume_normaliser_step():
    """The paper's literal normaliser (|grad V(x)|^2 at the current x) on FP64 steps of
    drag-driven cells: compared with the oracle's literal step, and the distance to the
    frozen-normaliser result reported.  Its force is not the derivative of its energy,
    so the line search may stop short (LS_FAIL); cells that converge must agree with the
    oracle within 1e-10 D."""
    from paper_1903_06479_amd import CONVERGED
    b = workloads.shear(n_cells=4, n_verts=258, seed=83)
    X, Tr = b.meshes[258]
    m = oracle_model(258)
    f = workloads.drag_forces(b, b.x, b.v)
    xl, _, sl, _ = run_step(_plan_with([(X, Tr)], "fp64", literal=True, tol=1e-10, noise_factor=64.0),
                            np.zeros(4, np.int32), b.x, b.v, f)
    xf, _, sf, _ = run_step(_plan_with([(X, Tr)], "fp64", tol=1e-10, noise_factor=64.0),
                            np.zeros(4, np.int32), b.x, b.v, f)
    D = np.ptp(X[:, 0])
    import oracle.step as ostep
    for c in range(4):
        s = b.cell_slice(c)
        xr, _, info = ostep.step(m, b.x[s], b.v[s], f[s], ostep.Params(tol=1e-12, polish=True), literal=True)
        print(f"cell {c}: GPU status {sl['status'][c]}, residual {sl['residual'][c]:.1e}; "
              f"literal vs frozen {np.abs(xl[s] - xf[s]).max() / D:.2e} D; "
              f"GPU vs oracle (literal) {np.abs(xl[s] - xr).max() / D:.2e} D")
        if sl["status"][c] & CONVERGED:
            assert np.abs(xl[s] - xr).max() <= 1e-10 * D, c
        assert sf["status"][c] == CONVERGED


# ---- line-search and iteration-control paths ---------------------------------------------

@pytest.mark.parametrize("case", ["halving", "retry", "ls_fail", "maxiter"])
def test_line_search_and_iteration_control_paths(case):
    """Each branch of the iteration control, reached through ordinary inputs on FP64
    plans and checked against the oracle taking the same branch:
      halving: c1 = 0.6 rejects alpha = 1 (a quadratic model needs alpha <= 2 (1 - c1)
               times the model's curvature ratio), so steps are halved, yet the step
               reaches the stationary point;
      retry:   c1 = 0.52 without halvings: plain H~ directions pass, some L-BFGS
               directions fail, the history is cleared and the step retried, and it
               still converges (with max_halvings = 0 every failed line search costs
               one evaluation, so the failures are evaluations - 1 - iterations);
      ls_fail: c1 = 0.6 without halvings: the first (plain) direction fails with no
               history to clear: LS_FAIL, x_{n+1} = y_n;
      maxiter: max_iter = 1: MAXITER after one iteration, the oracle's first iterate."""
    import oracle.step as ostep
    from paper_1903_06479_amd import CONVERGED, LS_FAIL, MAXITER
    cfg = {"halving": dict(c1=0.6, max_halvings=30), "retry": dict(c1=0.52, max_halvings=0),
           "ls_fail": dict(c1=0.6, max_halvings=0), "maxiter": dict(max_iter=1)}[case]
    b = workloads.shear(n_cells=3, n_verts=258, seed=91)
    X, Tr = b.meshes[258]
    m = oracle_model(258)
    f = workloads.drag_forces(b, b.x, b.v)
    plan = make([(X, Tr)], "fp64", tol=1e-10, lbfgs_m=5, noise_factor=64.0, **cfg)
    xo, vo, st, _ = run_step(plan, np.zeros(3, np.int32), b.x, b.v, f)
    D = np.ptp(X[:, 0])
    for c in range(3):
        s = b.cell_slice(c)
        p = ostep.Params(tol=1e-10, m=5, noise_factor=64.0, **cfg)
        xr, vr, info = ostep.step(m, b.x[s], b.v[s], f[s], p)
        it, ev, status = int(st["iterations"][c]), int(st["evaluations"][c]), int(st["status"][c])
        failed = ev - 1 - it
        print(f"{case} cell {c}: GPU status {status} it {it} ev {ev} halvings {st['halvings'][c]}; "
              f"oracle status {info.status} it {info.iterations} ev {info.evaluations}")
        if case in ("halving", "retry"):
            assert status == CONVERGED and info.status == ostep.CONVERGED
            xr, _, _ = oracle_step(m, b.x[s], b.v[s], f[s])          # the stationary point
            assert np.abs(xo[s] - xr).max() <= 1e-10 * D, c
            if case == "halving":
                # every halving costs one evaluation; most iterations needed one
                assert st["halvings"][c] == ev - 1 - it and 2 * st["halvings"][c] >= it > 0
            else:
                assert failed >= 1
        elif case == "ls_fail":
            assert status == LS_FAIL and info.status == ostep.LS_FAIL
            assert it == 0 and ev == 2 and info.evaluations == 2
            assert np.abs(xo[s] - xr).max() <= 1e-12 * D and np.abs(vo[s] - vr).max() <= 1e-10 * D / DT
        else:
            assert status == MAXITER and info.status == ostep.MAXITER and it == 1 == info.iterations
            assert np.abs(xo[s] - xr).max() <= 1e-10 * D and np.abs(vo[s] - vr).max() <= 1e-10 * D / DT


# ---- H~ variants (the preconditioner only) -------------------------------------------------

def test_hessian_approximation_variants_reach_the_same_point():
    """H~ with and without the material term k_mat (section 2.1.1), applied in FP64 or
    as FP32 / BF16-off-diagonal products: the preconditioner changes the iteration
    counts, never the stationary point (FP64 within 1e-10 D of the oracle, FP32 within
    1e-5 D)."""
    from paper_1903_06479_amd import Mesh, Plan, default_material, default_params, CONVERGED
    b = workloads.shear(n_cells=4, seed=97)
    X, Tr = b.meshes[642]
    f = workloads.drag_forces(b, b.x, b.v)
    D = np.ptp(X[:, 0])
    m = oracle_model(642)
    ref = [oracle_step(m, b.x[b.cell_slice(c)], b.v[b.cell_slice(c)], f[b.cell_slice(c)])[0] for c in range(4)]
    for k_mat in (0.0, -1.0):
        for precision, bf16, tol in (("fp64", 0, 1e-10), ("fp32", 0, 1e-5), ("fp32", 1, 1e-5)):
            plan = Plan([Mesh(X, Tr)], DT, material=default_material(k_mat=k_mat),
                        params=default_params(precision=precision, inverse_bf16=bf16,
                                              tol=1e-10 if precision == "fp64" else 1e-6,
                                              noise_factor=64.0 if precision == "fp64" else 8.0))
            x, v, ff = (rounded(a, precision) for a in (b.x, b.v, f))
            xo, _, st, _ = run_step(plan, np.zeros(4, np.int32), x, v, ff)
            assert np.all(st["status"] == CONVERGED), (k_mat, precision, bf16)
            err = max(np.abs(xo[b.cell_slice(c)] - ref[c]).max() for c in range(4)) / D
            print(f"k_mat {'B' if k_mat < 0 else 0}, {precision}{' bf16' if bf16 else ''}: "
                  f"iterations {st['iterations'].tolist()}, max |x - x_oracle| / D = {err:.2e}")
            assert err <= tol


# ---- collisions (section 4.7) ---------------------------------------------------------------

def _overlapping_cluster(k=6):
    """Cells of the uneven (20,000-cell, 40 % volume fraction) workload that overlap:
    a seed cell and its nearest neighbours by origin, all within reach of each other."""
    b_all = workloads.uneven(n_cells=20000)
    o = b_all.origin
    from scipy.spatial import cKDTree
    tree = cKDTree(o)
    dist, idx = tree.query(o, k=2)
    seed = int(np.argmin(dist[:, 1]))
    _, near = tree.query(o[seed], k=k)
    cells = np.sort(near)
    return workloads.uneven(n_cells=20000, cells=cells)


def _oracle_contacts(b, x, cutoff):
    from oracle import collision
    xs = [x[b.cell_slice(c)] for c in range(b.n_cells)]
    tris = [b.meshes[int(n)][1] for n in b.cell_nverts]
    return collision.detect(b.origin, xs, tris, cutoff)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_contact_search_matches_oracle(precision):
    """The hashed-grid contact search against the oracle's brute force on overlapping
    cells of the uneven workload: the same vertices have contacts, with the same
    partner (its position in the cell frame) and normal; where two candidates are at
    the same distance to rounding, either is accepted."""
    b = _overlapping_cluster()
    sizes = sorted(b.meshes)
    cm = np.array([sizes.index(int(n)) for n in b.cell_nverts], np.int32)
    from paper_1903_06479_amd import Batch
    plan = make([b.meshes[n] for n in sizes], precision)
    batch = Batch(plan, cm)
    x = rounded(b.x, precision)
    cutoff = 0.6
    q, n, count = batch.detect_contacts(T(b.origin, torch.float64), T(x, plan.torch_dtype), cutoff, count=True)
    q, n = q.cpu().numpy().astype(np.float64), n.cpu().numpy().astype(np.float64)
    ref = _oracle_contacts(b, x, cutoff)
    total = 0
    for c in range(b.n_cells):
        s = b.cell_slice(c)
        rq, rn, partner = ref[c]
        has = partner >= 0
        total += int(has.sum())
        world = b.origin[c] + x[s]
        dref = np.linalg.norm(rq - x[s], axis=1)
        near_cut = np.abs(dref - cutoff) < 1e-9 * cutoff
        gpu_has = np.any(n[s] != 0, axis=1)
        assert np.array_equal(gpu_has[~near_cut], has[~near_cut]), c
        both = has & gpu_has
        same = np.all(np.abs(q[s][both] - rq[both]) <= 1e-6 * (1 if precision == "fp32" else 1e-6), axis=1)
        dg = np.linalg.norm(q[s][both] - x[s][both], axis=1)
        assert np.all(same | (np.abs(dg - dref[both]) <= 1e-12 * cutoff)), c
        tol_n = 1e-6 if precision == "fp32" else 1e-12
        assert np.all(np.abs(n[s][both][same] - rn[both][same]).max(initial=0.0) <= tol_n), c
    assert total > 50 and abs(count - total) <= 2


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_with_contacts_matches_oracle(precision):
    """One step of the overlapping cluster with the collision term (w = 2e4 pN/um)
    against the oracle's step with the oracle's contacts: positions within 1e-10 D
    (FP64) or 1e-5 D (FP32); and the collision term reduces the deepest penetration
    relative to the step without it."""
    from paper_1903_06479_amd import Batch, CONVERGED
    b = _overlapping_cluster()
    sizes = sorted(b.meshes)
    cm = np.array([sizes.index(int(n)) for n in b.cell_nverts], np.int32)
    fp64 = precision == "fp64"
    plan = make([b.meshes[n] for n in sizes], precision, tol=1e-10 if fp64 else 1e-6,
                noise_factor=64.0 if fp64 else 8.0)
    batch = Batch(plan, cm)
    dt = plan.torch_dtype
    x, v = rounded(b.x, precision), rounded(b.v, precision)
    f = rounded(workloads.drag_forces(b, x, v, step=0), precision)
    w = 2.0e4
    q, n = batch.detect_contacts(T(b.origin, torch.float64), T(x, dt), 0.6)
    xo, vo, st = batch.step_contacts(T(x, dt), T(v, dt), T(f, dt), q, n, w)
    x0, _, _ = batch.step(T(x, dt), T(v, dt), T(f, dt))
    torch.cuda.synchronize()
    s = Batch.stats_to_numpy(st)
    assert np.all(s["status"] == CONVERGED), s
    xo, x0 = xo.cpu().numpy().astype(np.float64), x0.cpu().numpy().astype(np.float64)
    qn, nn = q.cpu().numpy().astype(np.float64), n.cpu().numpy().astype(np.float64)
    import oracle.step as ostep
    worst_with, worst_without = 0.0, 0.0
    for c in range(b.n_cells):
        sl = b.cell_slice(c)
        m = oracle_model(int(b.cell_nverts[c]))
        contacts = (qn[sl], nn[sl], w)
        xr, _, info = ostep.step(m, x[sl], v[sl], f[sl], ostep.Params(tol=1e-12, polish=True), contacts=contacts)
        D = np.ptp(m.X[:, 0])
        err = np.abs(xo[sl] - xr).max() / D
        print(f"cell {c} ({b.cell_nverts[c]} vertices): {int(np.sum(np.any(nn[sl] != 0, axis=1)))} contacts, "
              f"|x - x_oracle| / D = {err:.2e}")
        assert err <= (1e-10 if fp64 else 1e-5), c
        pen = lambda y: -np.minimum(np.sum((y - qn[sl]) * nn[sl], axis=1), 0).min(initial=0.0)
        worst_with = max(worst_with, pen(xo[sl]))
        worst_without = max(worst_without, pen(x0[sl]))
    print(f"deepest penetration: {worst_without:.3e} um without the term, {worst_with:.3e} um with it")
    assert worst_with < worst_without


# ---- the recovery workload (original and modified Skalak) -------------------------------------

@pytest.mark.parametrize("D", [35.0, 0.0])
def test_recovery_hold_and_release_match_oracle(D):
    """The fluid-free recovery experiment (one 258-vertex cell, dt = 1 us, FP64) with the
    modified (D = 35) and the original (D = 0) Skalak law: four steps held at 100 pN,
    then four released; every step against the oracle stepped from the GPU's state, and
    the eight-step trajectory against the oracle's own, within 1e-10 D."""
    import oracle.step as ostep
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_material, default_params, CONVERGED
    b = workloads.stretch(258)
    X, Tr = b.meshes[258]
    m = oracle_model(258, h=1.0, D=D)
    plan = Plan([Mesh(X, Tr)], 1.0, material=default_material(D=D),
                params=default_params(precision="fp64", tol=1e-10, noise_factor=64.0))
    batch = Batch(plan, np.zeros(1, np.int32))
    D_len = np.ptp(X[:, 0])
    xg, vg = T(X, torch.float64), T(np.zeros_like(X), torch.float64)
    xr, vr = X.copy(), np.zeros_like(X)
    p = ostep.Params(tol=1e-12, polish=True)
    for k in range(1, 9):
        f = workloads.recovery_forces(b, k, 100.0, hold_steps=4)
        xp, vp = xg.cpu().numpy(), vg.cpu().numpy()
        xg, vg, st = batch.step(xg, vg, T(f, torch.float64))
        assert batch.stats_to_numpy(st)["status"][0] == CONVERGED, k
        xs, _, _ = ostep.step(m, xp, vp, f, p)
        xr, vr, _ = ostep.step(m, xr, vr, f, p)
        e_step = np.abs(xg.cpu().numpy() - xs).max() / D_len
        e_traj = np.abs(xg.cpu().numpy() - xr).max() / D_len
        lam = np.ptp(xg.cpu().numpy()[:, 0]) / np.ptp(xg.cpu().numpy()[:, 1])
        print(f"D={D} step {k}: lambda {lam:.4f}, this step {e_step:.2e} D, trajectory {e_traj:.2e} D")
        assert e_step <= 1e-10 and e_traj <= 1e-10, k
