"""Seeded synthetic workloads for the batched RBC step (units: um, us, pN, fg).

Every array here is an *input* to the step: rest meshes, initial positions and
velocities, and the external nodal forces that a fluid solver would hand over
(explicit coupling: forces are computed from the state at time t).  The fluid is not
simulated; it is replaced by analytic flow fields and Stokes drag, so the shapes,
magnitudes and spatial structure of the forcing resemble the paper's shear and
Poiseuille experiments without needing the lattice-Boltzmann solver.

Workloads
  stretch  : one 258-vertex cell at rest, equal and opposite forces ramped 0-200 pN
             on the 5 % of vertices at each end of the x axis (optical-tweezers load).
  recovery : the same cell held at a constant stretching load, then released (the
             fluid-free recovery experiment; the forces are recovery_forces).
  shear    : N cells of one mesh, random rotation, Gaussian perturbation of the
             initial positions (sigma = 2 % of the radius), centres on a lattice,
             drag towards a per-cell linear shear flow, rate U[100, 1000] 1/s.
  uneven   : 20,000 cells drawn 30/50/20 % from 258/642/2562-vertex meshes, random
             rotations, uniform centres in a cube sized for 40 % volume fraction,
             N(0, 10 pN) random nodal forces redrawn every step plus Poiseuille drag.
  training : shear workload with rates U[50, 2000] 1/s (learned warm start data).
  throughput: 100,000 cells of the 642 mesh, as ``shear`` plus Poiseuille drag,
             centres uniform in a cube sized for 40 % volume fraction.

Each cell draws from its own counter-addressed stream
``SeedSequence(seed, spawn_key=(cell,))`` so any subset of a large batch can be
regenerated exactly without generating the rest.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import rbc_mesh, RBC_DIAMETER_UM

DT_US = 0.1                      # 1e-7 s
RBC_RADIUS_UM = RBC_DIAMETER_UM / 2.0
RBC_VOLUME_UM3 = 94.1
PLASMA_VISCOSITY = 1.2e3         # 1.2 mPa s in pN us / um^2
POISEUILLE_UMAX = 5.0e-3         # 5 mm/s in um/us


def drag_coefficient(n_verts: int) -> float:
    """Stokes drag of a sphere of the cell radius, shared equally by the vertices."""
    return 6.0 * np.pi * PLASMA_VISCOSITY * RBC_RADIUS_UM / n_verts


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def cell_rng(seed: int, cell: int, step: int | None = None) -> np.random.Generator:
    key = (cell,) if step is None else (cell, step + 1)
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=key)))


@dataclass
class Batch:
    """A batch of cells.  Positions are cell-local (origin near the cell centre);
    ``origin`` holds the float64 world position of each local frame."""
    name: str
    meshes: dict                      # n_verts -> (rest_verts [n,3], tris [nt,3])
    cell_nverts: np.ndarray           # [C] mesh size per cell
    offsets: np.ndarray               # [C+1] vertex offsets into the concatenated arrays
    x: np.ndarray                     # [V,3] float64 local positions
    v: np.ndarray                     # [V,3] float64 velocities
    origin: np.ndarray                # [C,3] float64
    shear_rate: np.ndarray            # [C] 1/us (0 = none)
    poiseuille: dict | None = None    # {"umax", "radius", "axis_y", "axis_z"}
    random_force_sigma: float = 0.0   # pN, per node per component, redrawn per step
    seed: int = 0
    cells: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))  # global ids

    @property
    def n_cells(self) -> int:
        return len(self.cell_nverts)

    def cell_slice(self, c: int) -> slice:
        return slice(int(self.offsets[c]), int(self.offsets[c + 1]))


def _assemble(name, meshes, nverts, xs, origins, rates, cells, seed, **kw) -> Batch:
    offsets = np.zeros(len(nverts) + 1, np.int64)
    offsets[1:] = np.cumsum(nverts)
    x = np.concatenate(xs) if xs else np.zeros((0, 3))
    return Batch(name=name, meshes=meshes, cell_nverts=np.asarray(nverts, np.int64),
                 offsets=offsets, x=x, v=np.zeros_like(x), origin=np.asarray(origins, float).reshape(-1, 3),
                 shear_rate=np.asarray(rates, float), cells=np.asarray(cells, np.int64), seed=seed, **kw)


def _placed_cell(rest: np.ndarray, rng: np.random.Generator, perturb: float) -> np.ndarray:
    rot = random_rotation(rng)
    x = rest @ rot.T
    if perturb > 0:
        x = x + perturb * rng.standard_normal(x.shape)
    return x


# ---------------------------------------------------------------------------------
# Workload builders
# ---------------------------------------------------------------------------------

def stretch(n_verts: int = 258) -> Batch:
    meshes = {n_verts: rbc_mesh(n_verts)}
    rest = meshes[n_verts][0]
    return _assemble("stretch", meshes, [n_verts], [rest.copy()], [np.zeros(3)], [0.0], [0], 0)


def stretch_forces(batch: Batch, step: int, total_steps: int = 200, f_max: float = 200.0) -> np.ndarray:
    """Nodal forces at step k = 1..total_steps: +-F_k/n_end along x on the
    ceil(5 %) of rest vertices with the largest / smallest x, F_k = f_max k / total."""
    n = int(batch.cell_nverts[0])
    rest = batch.meshes[n][0]
    n_end = int(np.ceil(0.05 * n))
    order = np.argsort(rest[:, 0], kind="stable")
    f = np.zeros((n, 3))
    fk = f_max * step / total_steps
    f[order[-n_end:], 0] = fk / n_end
    f[order[:n_end], 0] = -fk / n_end
    return f


def recovery_forces(batch: Batch, step: int, f_stretch: float = 100.0, hold_steps: int = 300) -> np.ndarray:
    """The recovery experiment's load (section 4.2): the stretching forces +-f_stretch on
    the end vertices held for steps 1..hold_steps, then released (zero afterwards)."""
    if step <= hold_steps:
        return stretch_forces(batch, 1, total_steps=1, f_max=f_stretch)
    n = int(batch.cell_nverts[0])
    return np.zeros((n, 3))


def shear(n_cells: int = 1024, n_verts: int = 642, seed: int = 1002, cells=None,
          rate_range=(100.0, 1000.0), perturb_frac: float = 0.02, lattice=(16, 8, 8),
          spacing: float = 10.0) -> Batch:
    meshes = {n_verts: rbc_mesh(n_verts)}
    rest = meshes[n_verts][0]
    cells = np.arange(n_cells) if cells is None else np.asarray(cells)
    xs, origins, rates = [], [], []
    nx, ny, nz = lattice
    for c in cells:
        rng = cell_rng(seed, int(c))
        xs.append(_placed_cell(rest, rng, perturb_frac * RBC_RADIUS_UM))
        rates.append(rng.uniform(*rate_range) * 1e-6)        # 1/s -> 1/us
        i, j, k = int(c) % nx, (int(c) // nx) % ny, (int(c) // (nx * ny)) % nz
        origins.append(spacing * np.array([i, j, k], float))
    return _assemble("shear", meshes, [n_verts] * len(cells), xs, origins, rates, cells, seed)


def _cube_side(n_cells: int, fraction: float = 0.40) -> float:
    return (n_cells * RBC_VOLUME_UM3 / fraction) ** (1.0 / 3.0)


def uneven(n_cells: int = 20000, seed: int = 1003, cells=None,
           sizes=(258, 642, 2562), counts=(0.3, 0.5, 0.2)) -> Batch:
    meshes = {n: rbc_mesh(n) for n in sizes}
    per = [int(round(c * n_cells)) for c in counts]
    per[-1] = n_cells - sum(per[:-1])
    types = np.concatenate([np.full(k, n) for k, n in zip(per, sizes)])
    np.random.Generator(np.random.PCG64(seed)).shuffle(types)
    side = _cube_side(n_cells)
    cells = np.arange(n_cells) if cells is None else np.asarray(cells)
    xs, origins = [], []
    for c in cells:
        rng = cell_rng(seed, int(c))
        n = int(types[c])
        xs.append(_placed_cell(meshes[n][0], rng, 0.0))
        origins.append(rng.uniform(0.0, side, 3))
    used = sorted({int(types[c]) for c in cells})
    return _assemble("uneven", {n: meshes[n] for n in used}, [int(types[c]) for c in cells], xs,
                     origins, np.zeros(len(cells)), cells, seed,
                     poiseuille={"umax": POISEUILLE_UMAX, "radius": side / 2, "axis_y": side / 2,
                                 "axis_z": side / 2},
                     random_force_sigma=10.0)


def throughput(n_cells: int = 100000, n_verts: int = 642, seed: int = 1005, cells=None) -> Batch:
    meshes = {n_verts: rbc_mesh(n_verts)}
    rest = meshes[n_verts][0]
    side = _cube_side(n_cells)
    cells = np.arange(n_cells) if cells is None else np.asarray(cells)
    xs, origins, rates = [], [], []
    for c in cells:
        rng = cell_rng(seed, int(c))
        xs.append(_placed_cell(rest, rng, 0.02 * RBC_RADIUS_UM))
        rates.append(rng.uniform(100.0, 1000.0) * 1e-6)
        origins.append(rng.uniform(0.0, side, 3))
    return _assemble("throughput", meshes, [n_verts] * len(cells), xs, origins, rates, cells, seed,
                     poiseuille={"umax": POISEUILLE_UMAX, "radius": side / 2, "axis_y": side / 2,
                                 "axis_z": side / 2})


def training(run: int, n_cells: int = 1024, cells=None) -> Batch:
    """Learned-warm-start data: shear workload, rates U[50, 2000] 1/s.
    Runs 0-3 are training (seeds 4000-4003), runs 100-103 held out (4100-4103)."""
    seed = 4000 + run
    b = shear(n_cells=n_cells, seed=seed, cells=cells, rate_range=(50.0, 2000.0))
    b.name = "training"
    return b


# ---------------------------------------------------------------------------------
# External forces (the fluid's stand-in), computed from the state at time t
# ---------------------------------------------------------------------------------

def drag_forces(batch: Batch, x: np.ndarray, v: np.ndarray, step: int = 0) -> np.ndarray:
    """zeta (u_flow(x) - v) per vertex, plus the workload's random nodal forces.

    u_flow = [shear_rate_c * z_local + u_P(rho)] e_x, with the Poiseuille profile
    u_P = umax (1 - rho^2 / R^2) for rho < R (rho = distance from the tube axis,
    which runs along x), else 0.
    """
    f = np.zeros_like(x)
    for c in range(batch.n_cells):
        s = batch.cell_slice(c)
        n = int(batch.cell_nverts[c])
        zeta = drag_coefficient(n)
        ux = batch.shear_rate[c] * x[s, 2]
        if batch.poiseuille is not None:
            p = batch.poiseuille
            wy = batch.origin[c, 1] + x[s, 1] - p["axis_y"]
            wz = batch.origin[c, 2] + x[s, 2] - p["axis_z"]
            rho2 = wy * wy + wz * wz
            ux = ux + np.where(rho2 < p["radius"] ** 2, p["umax"] * (1.0 - rho2 / p["radius"] ** 2), 0.0)
        f[s, 0] = zeta * (ux - v[s, 0])
        f[s, 1] = -zeta * v[s, 1]
        f[s, 2] = -zeta * v[s, 2]
        if batch.random_force_sigma > 0:
            rng = cell_rng(batch.seed, int(batch.cells[c]), step)
            f[s] += batch.random_force_sigma * rng.standard_normal((n, 3))
    return f
