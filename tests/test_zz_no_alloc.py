"""The allocation-free step (npfem_step_noalloc, through the C ABI) against npfem_step:
the same inputs give the same bits, on two calls in a row with the second on a smaller
batch, after an FP64 call has left other contents in the shared scratch array."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from rbc_inputs import workloads

pytestmark = pytest.mark.gpu


def _case(n_cells, seed, precision="fp32", **prm):
    from paper_1903_06479_amd import Batch, Mesh, Plan, default_params, CELL_STATS_DTYPE
    b = workloads.shear(n_cells=n_cells, seed=seed)
    X, Tr = b.meshes[642]
    plan = Plan([Mesh(X, Tr)], workloads.DT_US, params=default_params(precision=precision, **prm))
    batch = Batch(plan, np.zeros(n_cells, np.int32))
    dt = plan.torch_dtype
    dev = torch.device("cuda:0")
    x = torch.tensor(b.x, dtype=dt, device=dev)
    v = torch.tensor(0.01 * np.random.default_rng(seed).standard_normal(b.x.shape), dtype=dt, device=dev)
    f = torch.tensor(workloads.drag_forces(b, b.x, b.v), dtype=dt, device=dev)
    st_ref = torch.empty(n_cells * CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    st_na = torch.empty_like(st_ref)
    return plan, batch, x, v, f, st_ref, st_na


def _check(batch, x, v, f, st_ref, st_na):
    xr, vr, _ = batch.step(x, v, f, stats=st_ref)
    xo, vo = torch.full_like(x, float("nan")), torch.full_like(v, float("nan"))
    st_na.fill_(0xFF)
    batch.step_noalloc(x, v, f, xo, vo, stats=st_na)
    torch.cuda.synchronize()
    assert torch.equal(xo, xr) and torch.equal(vo, vr)
    assert torch.equal(st_na, st_ref)
    from paper_1903_06479_amd import Batch, CONVERGED
    assert np.all(Batch.stats_to_numpy(st_na)["status"] & CONVERGED)


def test_noalloc_step_matches_step_twice_then_smaller():
    # an FP64 call first, so the scratch holds other data when the FP32 calls start
    _, b64, *bufs64 = _case(7, 70, "fp64", tol=1e-9, cells_per_tile=3)
    _check(b64, *bufs64)
    # two calls in a row: 45 cells, then 11 (the second reuses what the first left)
    _, big, *bufs = _case(45, 71, "fp32", inverse_bf16=1, cells_per_tile=5, lbfgs_m=2)
    _check(big, *bufs)
    _, small, *bufs = _case(11, 72, "fp32", inverse_bf16=1, cells_per_tile=5, lbfgs_m=2)
    _check(small, *bufs)


def test_noalloc_step_reduces_the_grid_for_a_large_batch():
    """A batch whose persistent grid needs more workspace than the scratch array holds
    runs on fewer workgroups and still gives the same bits as npfem_step."""
    _, batch, *bufs = _case(2100, 73, "fp32", inverse_bf16=1, cells_per_tile=5, lbfgs_m=2)
    assert batch.schedule()["grid_blocks"] * 5 * 9 * 3 * 672 * 4 > 64 << 20
    _check(batch, *bufs)
