"""Seeded inputs: mesh topology, the biconcave shape against the paper's printed
geometry, workload reproducibility."""
import json
import os

import numpy as np
import pytest

from rbc_inputs import meshes, workloads

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rbc_geometry.json")))


@pytest.mark.parametrize("n", [12, 42, 66, 258, 642, 1026, 2562])
def test_mesh_counts_closed_oriented(n):
    v, f = meshes.rbc_mesh(n)
    assert len(v) == n and len(f) == 2 * n - 4
    # every directed edge appears once and its reverse once: closed, consistently oriented
    d = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    s = {tuple(e) for e in d}
    assert len(s) == len(d)
    assert all((b, a) in s for a, b in s)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    assert np.einsum("ij,ij->i", a, np.cross(b, c)).sum() > 0      # outward


def test_evans_skalak_matches_printed_geometry():
    """Introduction: area 134 um^2, volume 94 um^3, diameter 7.82 um, thickness
    0.81 um at the dimple and 2.57 um at the rim."""
    v, f = meshes.rbc_mesh(2562)
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6
    assert abs(area - GOLDEN["surface_area_um2"]) / GOLDEN["surface_area_um2"] < 0.01
    assert abs(vol - GOLDEN["volume_um3"]) / GOLDEN["volume_um3"] < 0.01
    assert abs(np.ptp(v[:, 0]) - GOLDEN["diameter_um"]) < 1e-9
    # analytic profile thickness (the mesh samples it)
    s = np.linspace(0, 1, 200001)
    a0, a1, a2 = meshes.ES_COEFFS
    thick = 2 * GOLDEN["diameter_um"] * np.sqrt(1 - s) * (a0 + a1 * s / 4 + a2 * s * s / 16)
    assert abs(thick[0] - GOLDEN["thickness_dimple_um"]) < 0.005
    assert abs(thick.max() - GOLDEN["thickness_rim_um"]) < 0.01


def test_shear_subset_reproducible():
    full = workloads.shear(n_cells=12, seed=7)
    sub = workloads.shear(n_cells=12, seed=7, cells=[3, 10])
    for k, c in enumerate([3, 10]):
        np.testing.assert_array_equal(sub.x[sub.cell_slice(k)], full.x[full.cell_slice(c)])
        assert sub.shear_rate[k] == full.shear_rate[c]
    again = workloads.shear(n_cells=12, seed=7)
    np.testing.assert_array_equal(again.x, full.x)


def test_perturbation_size():
    b = workloads.shear(n_cells=4, seed=1)
    rest = b.meshes[642][0]
    for c in range(4):
        x = b.x[b.cell_slice(c)]
        # remove the rotation (Kabsch) and measure the residual spread
        H = rest.T @ x
        U, _, Vt = np.linalg.svd(H)
        R = (U @ Vt).T
        if np.linalg.det(R) < 0:
            U[:, -1] *= -1
            R = (U @ Vt).T
        resid = x - rest @ R.T
        assert abs(resid.std() - 0.02 * workloads.RBC_RADIUS_UM) < 0.01


def test_stretch_forces_balanced_and_ramped():
    b = workloads.stretch()
    f = workloads.stretch_forces(b, 200)
    assert np.allclose(f.sum(axis=0), 0)
    assert np.isclose(f[f[:, 0] > 0, 0].sum(), 200.0)
    assert (f[:, 0] > 0).sum() == 13
    assert np.isclose(workloads.stretch_forces(b, 100)[f[:, 0] > 0, 0].sum(), 100.0)


def test_uneven_mix_and_forces():
    b = workloads.uneven(n_cells=200, cells=np.arange(40))
    assert set(b.cell_nverts) <= {258, 642, 2562}
    f1 = workloads.drag_forces(b, b.x, b.v, step=3)
    f2 = workloads.drag_forces(b, b.x, b.v, step=3)
    f3 = workloads.drag_forces(b, b.x, b.v, step=4)
    np.testing.assert_array_equal(f1, f2)
    assert not np.allclose(f1, f3)
    assert abs(f1[:, 1].std() - 10.0) < 0.5
