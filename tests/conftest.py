import os
import sys
from functools import lru_cache

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


@lru_cache(maxsize=None)
def oracle_model(n_verts: int, kind: str = "rbc", h: float = 0.1, **mat_kw):
    """Cached oracle Model for a mesh (kind 'rbc' or 'sphere')."""
    from rbc_inputs import meshes
    from oracle.model import Model, Material
    X, T = meshes.rbc_mesh(n_verts) if kind == "rbc" else meshes.sphere_mesh(n_verts, 3.0)
    return Model(X, T, Material(**dict(mat_kw)), h)
