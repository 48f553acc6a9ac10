"""GPU parity of the learned warm start (first guess, network inference, loss and
gradient, Adam, the learned step) against the FP64 oracle, through the C ABI.

The GPU applies the weight matrices in BF16 and stores activations in BF16 (FP32
accumulation); the oracle runs in FP64 with the same BF16-rounded weight matrices and
FP32 biases.  Each BF16 rounding of an activation has relative error <= 2^-9, and the
network rounds features, the neighbour means and every layer's output (about 10
roundings along any path); rounding errors of independent sign add in quadrature
(sqrt(10) 2^-9 = 6.2e-3), so outputs and gradients are compared in the relative L2
norm with a bound of 1e-2 (single parameter blocks, which sum fewer terms: 3e-2)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle.mpnn as mp
from rbc_inputs import workloads
from conftest import oracle_model

pytestmark = pytest.mark.gpu

DT = workloads.DT_US
REL = 1e-2


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-test] {request.node.nodeid}", flush=True)
    yield


def dev():
    return torch.device("cuda:0")


def T(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def rounded(a, precision="fp32"):
    return a.astype(np.float32).astype(np.float64) if precision == "fp32" else a


def gpu_params(cfg, seed, scale=1.0):
    """Random parameters with BF16-exact weight matrices and FP32 biases."""
    theta = mp.init_params(cfg, seed)
    rng = np.random.default_rng(seed + 1)
    theta += 0.05 * rng.standard_normal(theta.size)
    p = mp.unpack(theta, cfg)
    for k in p:
        if k.startswith("W"):
            p[k][:] = mp.bf16_round(p[k]) * 1.0
        else:
            p[k][:] = p[k].astype(np.float32)
    p["Wd"][:] = mp.bf16_round(p["Wd"] * scale)
    return theta


def make(meshes, precision="fp32", **prm):
    from paper_1903_06479_amd import Mesh, Plan, default_params
    return Plan([Mesh(*m) for m in meshes], DT, params=default_params(precision=precision, **prm))


def relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_first_guess_matches_oracle():
    from paper_1903_06479_amd import Batch
    b = workloads.shear(n_cells=5, seed=31)
    X, Tr = b.meshes[642]
    m = oracle_model(642)
    f = workloads.drag_forces(b, b.x, b.v)
    plan = make([(X, Tr)], "fp64")
    batch = Batch(plan, np.zeros(5, np.int32))
    u0 = batch.first_guess(T(b.x, torch.float64), T(b.v, torch.float64), T(f, torch.float64)).cpu().numpy()
    import oracle.step as ostep
    for c in range(5):
        s = b.cell_slice(c)
        y = ostep.Objective(m, b.x[s], b.v[s], f[s]).y
        ref = y - b.x[s]            # carries the rounding of x_n + u and its subtraction
        assert np.abs(u0[s] - ref).max() <= 1e-10 * np.abs(ref).max() + 4e-16 * np.abs(b.x[s]).max()


@pytest.mark.parametrize("precision,n_verts,variant", [("fp32", 642, "lds"), ("fp64", 642, "lds"),
                                                      ("fp32", 642, "memory"), ("fp32", 2562, "auto")])
def test_inference_matches_oracle(precision, n_verts, variant, monkeypatch):
    """delta of every cell (world frame) against the oracle network on the same inputs,
    for the LDS-resident forward variant and the one that gathers from memory (forced by
    NPFEM_NET_NO_LDS, and taken by itself for the 2562-vertex mesh)."""
    from paper_1903_06479_amd import Batch, Net
    if variant == "memory":
        monkeypatch.setenv("NPFEM_NET_NO_LDS", "1")
    cfg = mp.NetConfig()
    b = workloads.shear(n_cells=7 if n_verts == 642 else 3, n_verts=n_verts, seed=41)
    X, Tr = b.meshes[n_verts]
    m = oracle_model(n_verts)
    dt = torch.float64 if precision == "fp64" else torch.float32
    x, v = rounded(b.x, precision), rounded(b.v, precision)
    f = rounded(workloads.drag_forces(b, x, v), precision)
    plan = make([(X, Tr)], precision)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    theta = gpu_params(cfg, 3)
    net = Net(plan, theta.astype(np.float32))
    assert np.array_equal(net.get_params(), theta.astype(np.float32))
    delta = net.infer(batch, T(x, dt), T(v, dt), T(f, dt)).cpu().numpy().astype(np.float64)
    A = mp.neighbour_mean_matrix(len(X), Tr)
    for c in range(b.n_cells):
        s = b.cell_slice(c)
        ref = mp.predict_delta(theta, X, x[s], v[s], f[s], m.mass, DT, A, cfg)
        assert relerr(delta[s], ref) <= REL, (c, relerr(delta[s], ref))


def test_inference_on_a_mixed_batch_matches_oracle():
    """Resident inference over more cells than workgroups, with the 258- and 642-vertex
    meshes interleaved: each workgroup carries several cells in turn and restages the
    neighbour lists when the mesh type changes.  Sampled cells (every 7th and the last
    40, which are each workgroup's second or third cell) against the oracle network."""
    from paper_1903_06479_amd import Batch, Net
    cfg = mp.NetConfig()
    b = workloads.uneven(n_cells=700, seed=43, sizes=(258, 642), counts=(0.5, 0.5))
    sizes = sorted(b.meshes)
    rng = np.random.default_rng(43)
    x = rounded(b.x)
    v = rounded(0.05 * rng.standard_normal(b.x.shape))
    f = rounded(workloads.drag_forces(b, x, v) + 5.0 * rng.standard_normal(b.x.shape))
    plan = make([b.meshes[n] for n in sizes], "fp32")
    cm = np.array([sizes.index(int(n)) for n in b.cell_nverts], np.int32)
    assert 0 < cm.sum() < len(cm)
    batch = Batch(plan, cm)
    theta = gpu_params(cfg, 5)
    net = Net(plan, theta.astype(np.float32))
    delta = net.infer(batch, T(x), T(v), T(f)).cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(delta))
    models = {n: oracle_model(n) for n in sizes}
    mats = {n: mp.neighbour_mean_matrix(len(b.meshes[n][0]), b.meshes[n][1]) for n in sizes}
    for c in sorted(set(range(0, b.n_cells, 7)) | set(range(b.n_cells - 40, b.n_cells))):
        n = int(b.cell_nverts[c])
        s = b.cell_slice(c)
        ref = mp.predict_delta(theta, b.meshes[n][0], x[s], v[s], f[s], models[n].mass, DT, mats[n], cfg)
        assert relerr(delta[s], ref) <= REL, (c, n, relerr(delta[s], ref))


def test_loss_and_gradient_match_oracle():
    """Loss and gradient of a minibatch (a list of batch cells) against the oracle."""
    from paper_1903_06479_amd import Batch, Net
    import oracle.step as ostep
    cfg = mp.NetConfig()
    n_cells = 6
    b = workloads.shear(n_cells=n_cells, seed=43)
    X, Tr = b.meshes[642]
    m = oracle_model(len(X))
    x, v = b.x, b.v
    f = workloads.drag_forces(b, x, v)
    plan = make([(X, Tr)], "fp64")
    batch = Batch(plan, np.zeros(n_cells, np.int32))
    theta = gpu_params(cfg, 5)
    net = Net(plan, theta.astype(np.float32))
    rng = np.random.default_rng(7)
    x_next = x + 1e-4 * rng.standard_normal(x.shape)      # any converged-looking target
    u0 = batch.first_guess(T(x, torch.float64), T(v, torch.float64), T(f, torch.float64))
    cells = np.array([4, 1, 2], np.int32)
    loss, grad = net.loss_grad(batch, T(x, torch.float64), T(v, torch.float64), T(f, torch.float64),
                               T(x_next, torch.float64), u0, cells=T(cells, torch.int32))
    u0 = u0.cpu().numpy()
    A = mp.neighbour_mean_matrix(len(X), Tr)
    data = []
    for c in cells:
        s = b.cell_slice(int(c))
        feats, R, sc = mp.features(X, x[s], v[s], f[s], m.mass, DT, cfg)
        delta = x_next[s] - x[s] - u0[s]
        y = ostep.Objective(m, x[s], v[s], f[s]).y
        assert np.abs((x[s] + u0[s]) - y).max() <= 1e-10 * np.abs(y - x[s]).max() + 4e-16 * np.abs(x[s]).max()
        data.append((feats, mp.target(R, sc, delta)))
    Lr, gr = mp.loss_and_grad(theta, data, A, cfg)
    g = grad.cpu().numpy().astype(np.float64)
    print(f"loss rel. error {abs(loss - Lr) / Lr:.2e}, gradient rel. L2 error {relerr(g, gr):.2e}")
    assert abs(loss - Lr) <= REL * Lr
    assert relerr(g, gr) <= REL
    # block by block (each weight matrix and bias vector)
    pg, pr = mp.unpack(g, cfg), mp.unpack(gr, cfg)
    for k in pr:
        assert relerr(pg[k], pr[k]) <= 3 * REL, (k, relerr(pg[k], pr[k]))


def test_gradient_is_deterministic_and_adam_matches_oracle():
    from paper_1903_06479_amd import Batch, Net
    cfg = mp.NetConfig()
    b = workloads.shear(n_cells=4, seed=47)
    X, Tr = b.meshes[642]
    f = workloads.drag_forces(b, b.x, b.v)
    plan = make([(X, Tr)], "fp32")
    batch = Batch(plan, np.zeros(4, np.int32))
    theta = gpu_params(cfg, 9).astype(np.float32)
    net = Net(plan, theta)
    xs = [T(a) for a in (b.x, b.v, f)]
    x_next = T(b.x + 1e-4)
    u0 = batch.first_guess(*xs)
    l1, g1 = net.loss_grad(batch, *xs, x_next, u0)
    l2, g2 = net.loss_grad(batch, *xs, x_next, u0)
    assert l1 == l2 and torch.equal(g1, g2)
    net.adam_step(g1, lr=1e-3)
    net.adam_step(g1, lr=1e-3)
    th2 = net.get_params().astype(np.float64)
    g = g1.cpu().numpy().astype(np.float64)
    t_ref, mo, ve = mp.adam_update(theta.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, mp.Adam(lr=1e-3))
    t_ref, _, _ = mp.adam_update(t_ref, g, mo, ve, 2, mp.Adam(lr=1e-3))
    assert np.abs(th2 - t_ref).max() <= 1e-6 * (1 + np.abs(t_ref).max())
    net.set_params(theta)                      # resets the optimiser
    net.adam_step(g1, lr=1e-3)
    t1, _, _ = mp.adam_update(theta.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, mp.Adam(lr=1e-3))
    assert np.abs(net.get_params() - t1).max() <= 1e-6 * (1 + np.abs(t1).max())


def test_learned_step_reaches_the_plain_solution():
    """Starting from y_n + delta changes only the path: the converged positions agree
    with the plain step within the FP32 tolerance, for any network output."""
    from paper_1903_06479_amd import Batch, Net, CONVERGED, START_FALLBACK
    cfg = mp.NetConfig()
    b = workloads.shear(n_cells=9, seed=53)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x), rounded(b.v)
    f = rounded(workloads.drag_forces(b, x, v))
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(9, np.int32))
    net = Net(plan, gpu_params(cfg, 11).astype(np.float32))
    xi, vi, fi = T(x), T(v), T(f)
    xp, vp, sp = batch.step(xi, vi, fi)
    xl, vl, sl = batch.step_learned(net, xi, vi, fi)
    torch.cuda.synchronize()
    sp, sl = batch.stats_to_numpy(sp), batch.stats_to_numpy(sl)
    assert np.all(sp["status"] == CONVERGED) and np.all((sl["status"] & ~np.uint32(START_FALLBACK)) == CONVERGED)
    D = np.ptp(X[:, 0])
    assert (xl - xp).abs().max().item() <= 1e-5 * D
    # the learned start is y_n + delta: with delta = 0 (zero output layer) the step is the plain one
    th = gpu_params(cfg, 11).astype(np.float32)
    p = mp.unpack(th, cfg)
    p["Wd"][:] = 0.0
    p["bd"][:] = 0.0
    net.set_params(th)
    x0, v0, s0 = batch.step_learned(net, xi, vi, fi)
    torch.cuda.synchronize()
    assert torch.equal(x0, xp) and torch.equal(v0, vp)
    s0 = batch.stats_to_numpy(s0)
    np.testing.assert_array_equal(s0["iterations"], sp["iterations"])
    # g(y_n + 0) = g(y_n): the learned start is kept, at the cost of one more evaluation
    assert np.all(s0["status"] == CONVERGED)
    np.testing.assert_array_equal(s0["evaluations"], sp["evaluations"] + 1)


def test_learned_start_that_raises_the_objective_falls_back_to_y_n():
    """A network whose corrections are far too large (output layer scaled by 1000) raises
    g at y_n + delta in every cell: every cell starts from y_n instead, reports
    NPFEM_START_FALLBACK, and ends bit for bit where the plain step ends."""
    from paper_1903_06479_amd import Batch, Net, CONVERGED, START_FALLBACK
    cfg = mp.NetConfig()
    b = workloads.shear(n_cells=9, seed=53)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x), rounded(b.v)
    f = rounded(workloads.drag_forces(b, x, v))
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(9, np.int32))
    theta = gpu_params(cfg, 11, scale=1000.0).astype(np.float32)
    net = Net(plan, theta)
    xi, vi, fi = T(x), T(v), T(f)
    xp, vp, sp = batch.step(xi, vi, fi)
    xl, vl, sl = batch.step_learned(net, xi, vi, fi)
    delta = net.infer(batch, xi, vi, fi)
    torch.cuda.synchronize()
    sp, sl = batch.stats_to_numpy(sp), batch.stats_to_numpy(sl)
    assert delta.abs().max().item() > 1e-3 * np.ptp(X[:, 0])
    assert np.all(sl["status"] == CONVERGED | START_FALLBACK), sl["status"]
    assert torch.equal(xl, xp) and torch.equal(vl, vp)
    np.testing.assert_array_equal(sl["iterations"], sp["iterations"])
    np.testing.assert_array_equal(sl["evaluations"], sp["evaluations"] + 1)


def test_learned_form_on_a_rough_first_step():
    """The first step of a held-out run of the training workload (cells placed with a
    perturbed rest shape, where the bending projection makes g non-convex), with the
    committed weights: every cell converges; where the learned and plain steps end at
    different stationary points (more than 1e-5 D apart; one cell of 1,024 here), the
    learned one has the lower objective g."""
    import os
    from paper_1903_06479_amd import Batch, Net, CONVERGED
    from paper_1903_06479_amd import warmstart as ws
    b = workloads.training(101, n_cells=1024)
    X, Tr = b.meshes[642]
    D = float(np.ptp(X[:, 0]))
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = Net(plan, np.load(os.path.join(root, "paper_1903_06479_amd", "data", "warmstart_642.npy")))
    flow = ws.Flow(batch, np.full(b.n_cells, workloads.drag_coefficient(642)), b.shear_rate, b.origin, b.poiseuille)
    tr = ws.collect(batch, flow, T(b.x), T(b.v), 1)
    r = ws.compare(batch, net, tr, D)
    print(r)
    assert r["all_converged"]
    assert r["cell_steps_dx_above_1e-5"] <= 2, r
    assert r["dx_above_1e-5_learned_objective_higher"] == 0, r


def test_training_reduces_the_loss():
    """A few Adam steps on one minibatch of solver targets lower its loss."""
    from paper_1903_06479_amd import Batch, Net
    cfg = mp.NetConfig()
    b = workloads.shear(n_cells=8, seed=59)
    X, Tr = b.meshes[642]
    x, v = rounded(b.x), rounded(b.v)
    f = rounded(workloads.drag_forces(b, x, v))
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(8, np.int32))
    xi, vi, fi = T(x), T(v), T(f)
    xn, _, _ = batch.step(xi, vi, fi)
    u0 = batch.first_guess(xi, vi, fi)
    net = Net(plan, mp.init_params(cfg, 1).astype(np.float32))
    losses = []
    for it in range(30):
        loss, g = net.loss_grad(batch, xi, vi, fi, xn, u0)
        losses.append(loss)
        net.adam_step(g, lr=3e-3)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0], losses


def test_trained_network_cuts_iterations_on_held_out_cells():
    """The committed weights (trained on runs 0-3 of the training workload) on cells of a
    held-out run (100), over its first 4 steps: fewer quasi-Newton iterations than the
    plain start, every cell converged, the same positions (median within 1e-6 of the cell
    diameter), and no cell-step where the learned start ends at a different stationary
    point with a higher objective than the plain one."""
    import os
    from paper_1903_06479_amd import Batch, Net
    from paper_1903_06479_amd import warmstart as ws
    b = workloads.training(100, n_cells=256)
    X, Tr = b.meshes[642]
    plan = make([(X, Tr)], "fp32", inverse_bf16=1)
    batch = Batch(plan, np.zeros(b.n_cells, np.int32))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = Net(plan, np.load(os.path.join(root, "paper_1903_06479_amd", "data", "warmstart_642.npy")))
    flow = ws.Flow(batch, np.full(b.n_cells, workloads.drag_coefficient(642)), b.shear_rate, b.origin, b.poiseuille)
    tr = ws.collect(batch, flow, T(b.x), T(b.v), 4)
    r = ws.compare(batch, net, tr, float(np.ptp(X[:, 0])))
    print(r)
    assert r["all_converged"]
    assert r["iterations_learned"] <= r["iterations_plain"] - 0.3, r
    assert r["dx_above_1e-5_learned_objective_higher"] == 0, r
    assert r["median_dx_over_D"] <= 1e-6, r


def test_loss_grad_rejects_a_bad_cell_index_before_any_launch():
    """An out-of-range index in the training cell list is refused with
    NPFEM_E_INVALID, and no kernel has run: the gradient buffer is untouched."""
    from paper_1903_06479_amd import Batch, Net
    from paper_1903_06479_amd import _native as N
    b = workloads.shear(n_cells=4, seed=51)
    X, Tr = b.meshes[642]
    plan = make([(X, Tr)])
    batch = Batch(plan, np.zeros(4, np.int32))
    net = Net(plan, mp.init_params(mp.NetConfig(), 3).astype(np.float32))
    x, v = T(b.x), T(b.v)
    grad = torch.full((net.n_params,), 7.0, dtype=torch.float32, device=dev())
    for bad in ([0, 4], [-1], [1, 2, 100000]):
        cells = torch.tensor(bad, dtype=torch.int32, device=dev())
        with pytest.raises(N.NpfemError, match="invalid argument"):
            net.loss_grad(batch, x, v, v, x, v, cells=cells, grad=grad)
    torch.cuda.synchronize()
    assert torch.all(grad == 7.0)
    cells = torch.tensor([3, 0], dtype=torch.int32, device=dev())
    loss, g = net.loss_grad(batch, x, v, v, x, v, cells=cells, grad=grad)
    assert np.isfinite(loss) and torch.isfinite(g).all()
