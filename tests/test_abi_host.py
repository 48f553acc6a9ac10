"""The C-ABI library on the host (no GPU): every declared symbol is exported, mesh
validation and the host's FP64 rest data (an implementation independent of the
oracle's) agree with the oracle."""
import os
import re

import numpy as np
import pytest

from rbc_inputs import meshes
from conftest import ROOT, oracle_model

from paper_1903_06479_amd import _native as N
from paper_1903_06479_amd.solver import Mesh


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "npfem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(npfem_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = N.lib()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(N._SIGNATURES)


def test_status_strings_and_defaults():
    L = N.lib()
    assert L.npfem_status_string(0) == b"ok"
    assert L.npfem_status_string(-2) == b"invalid mesh"
    from paper_1903_06479_amd import default_material, default_params
    m, p = default_material(), default_params()
    assert (m.B, m.C, m.D, m.k_bend, m.k_volume, m.kappa) == (10.6, 530.0, 35.0, 0.2, 250.0, 0.6)
    assert p.lbfgs_m == 5 and p.tol == 1e-6 and p.precision == N.FP32


def test_mesh_validation_errors():
    v, f = meshes.rbc_mesh(66)
    with pytest.raises(N.NpfemError, match="invalid mesh"):
        Mesh(v, f[:-1])                                   # open surface
    g = f.copy()
    g[0] = g[0, ::-1]
    with pytest.raises(N.NpfemError, match="invalid mesh"):
        Mesh(v, g)                                        # one triangle flipped
    with pytest.raises(N.NpfemError, match="invalid mesh"):
        Mesh(v, f[:, ::-1].copy())                        # all flipped: negative volume
    g = f.copy()
    g[3, 1] = len(v) + 5
    with pytest.raises(N.NpfemError, match="invalid mesh"):
        Mesh(v, g)
    w = v.copy()
    w[5] = np.nan
    with pytest.raises(N.NpfemError, match="invalid mesh"):
        Mesh(w, f)


def test_solve_entry_points_reject_a_null_plan():
    """The product and factor-solve entry points check their plan before any device
    call (no GPU is touched): a NULL plan is NPFEM_E_INVALID, and the workspace query
    returns -1."""
    from ctypes import c_void_p
    L = N.lib()
    nul = c_void_p(0)
    assert L.npfem_solve_factor_workspace(nul, 0, 10) == -1
    assert L.npfem_solve_factor(nul, 0, 0, nul, nul, 10, nul, 0, nul, nul) == -1
    assert L.npfem_last_error() == b"solve_factor: NULL plan"
    assert L.npfem_apply_inverse(nul, 0, 0, nul, nul, 10, nul, nul) == -1
    assert L.npfem_last_error() == b"apply_inverse: NULL plan"


@pytest.mark.parametrize("n", [258, 642])
def test_host_rest_data_matches_oracle(n):
    m = oracle_model(n)
    mesh = Mesh(m.X, m.tris)
    assert (mesh.n, mesh.nt, mesh.ne) == (n, 2 * n - 4, 3 * n - 6)
    assert np.isclose(mesh.rest_volume, m.V0, rtol=1e-13)
    assert np.isclose(mesh.rest_area, m.tri_area.sum(), rtol=1e-13)
    rd = mesh.rest_data()
    np.testing.assert_allclose(rd["vor_area"], m.vor_area, rtol=1e-11)
    np.testing.assert_allclose(rd["ell0"], m.ell0_norm, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(rd["tri_area"], m.tri_area, rtol=1e-12)
    np.testing.assert_allclose(rd["dminv"], m.Dm_inv, rtol=1e-11, atol=1e-12)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets the C
    compiler gives the header's structs."""
    import ctypes
    import subprocess
    structs = {"npfem_material": N.Material, "npfem_solver_params": N.SolverParams,
               "npfem_net_config": N.NetConfig}
    np_structs = {"npfem_cell_stats": N.CELL_STATS_DTYPE, "npfem_stats_total": N.STATS_TOTAL_DTYPE}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "npfem.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    for name, dt in np_structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in dt.names:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
    for name, dt in np_structs.items():
        assert int(got[name]) == dt.itemsize, name
        for f in dt.names:
            assert int(got[f"{name}.{f}"]) == dt.fields[f][1], (name, f)
