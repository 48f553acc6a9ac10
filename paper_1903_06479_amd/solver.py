"""Python handles over the C ABI.  Argument marshalling only: every step of the
solver runs in libnpfem.so; torch tensors provide device memory and streams."""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

import numpy as np

from . import _native as N


def _ptr(a: np.ndarray) -> c_void_p:
    return c_void_p(a.ctypes.data)


def _dptr(t) -> c_void_p:
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def default_material(**overrides) -> N.Material:
    m = N.Material()
    N.lib().npfem_material_default(byref(m))
    for k, v in overrides.items():
        setattr(m, k, float(v))
    return m


def default_params(**overrides) -> N.SolverParams:
    p = N.SolverParams()
    N.lib().npfem_solver_params_default(byref(p))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp32": N.FP32, "fp64": N.FP64}[v]
        setattr(p, k, v)
    return p


class Mesh:
    """Rest membrane mesh (validated and preprocessed on the host)."""

    def __init__(self, verts, tris):
        verts = np.ascontiguousarray(verts, np.float64)
        tris = np.ascontiguousarray(tris, np.int32)
        if verts.ndim != 2 or verts.shape[1] != 3 or tris.ndim != 2 or tris.shape[1] != 3:
            raise ValueError("verts must be [n,3] and tris [nt,3]")
        h = c_void_p()
        N.check(N.lib().npfem_mesh_create(len(verts), _ptr(verts), len(tris), _ptr(tris), byref(h)),
                "npfem_mesh_create")
        self._h = h
        n, nt, ne = c_int32(), c_int32(), c_int32()
        V0, A0 = c_double(), c_double()
        N.check(N.lib().npfem_mesh_query(h, byref(n), byref(nt), byref(ne), byref(V0), byref(A0)),
                "npfem_mesh_query")
        self.n, self.nt, self.ne = n.value, nt.value, ne.value
        self.rest_volume, self.rest_area = V0.value, A0.value

    def rest_data(self) -> dict:
        out = {"vor_area": np.zeros(self.n), "ell0": np.zeros(self.n), "tri_area": np.zeros(self.nt),
               "dminv": np.zeros((self.nt, 2, 2))}
        N.check(N.lib().npfem_mesh_rest_data(self._h, *(_ptr(out[k]) for k in ("vor_area", "ell0", "tri_area", "dminv"))),
                "npfem_mesh_rest_data")
        return out

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and N is not None and N._lib is not None:
            N._lib.npfem_mesh_destroy(h)


class Plan:
    """Mesh types + material + time step: constant matrices and their inverses on the GPU."""

    def __init__(self, meshes, dt: float, material: N.Material | None = None,
                 params: N.SolverParams | None = None, device: int = 0):
        self.meshes = list(meshes)
        self.material = material or default_material()
        self.params = params or default_params()
        self.dt = float(dt)
        arr = (c_void_p * len(self.meshes))(*[m._h for m in self.meshes])
        h = c_void_p()
        N.check(N.lib().npfem_plan_create(device, ctypes.cast(arr, c_void_p), len(self.meshes),
                                          byref(self.material), self.dt, byref(self.params), byref(h)),
                "npfem_plan_create")
        self._h = h
        self.device = device

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.params.precision == N.FP64 else torch.float32

    def masses(self, mesh_index: int) -> np.ndarray:
        out = np.zeros(self.meshes[mesh_index].n)
        N.check(N.lib().npfem_plan_masses(self._h, mesh_index, _ptr(out)), "npfem_plan_masses")
        return out

    def n_pad(self, mesh_index: int) -> int:
        np_ = c_int32()
        N.check(N.lib().npfem_apply_inverse(self._h, mesh_index, 0, None, None, 0, byref(np_), None),
                "npfem_apply_inverse")
        return np_.value

    def apply_inverse(self, mesh_index: int, which: int, inp, out=None, stream=None):
        """out[r] = A inp[r] for A = H~^-1 (which 0) or h^2 M~^-1 (which 1); inp [rows, n_pad]."""
        import torch
        if out is None:
            out = torch.empty_like(inp)
        self._check(inp, out)
        N.check(N.lib().npfem_apply_inverse(self._h, mesh_index, which, _dptr(inp), _dptr(out),
                                            inp.shape[0], None, _stream(stream)), "npfem_apply_inverse")
        return out

    def factor_bandwidth(self, mesh_index: int) -> int:
        """Half bandwidth b of the banded Cholesky factors used by solve_factor."""
        b = c_int32()
        N.check(N.lib().npfem_solve_factor(self._h, mesh_index, 0, None, None, 0, None, 0, byref(b), None),
                "npfem_solve_factor")
        return b.value

    def solve_factor_workspace(self, mesh_index: int, rows: int) -> int:
        nb = N.lib().npfem_solve_factor_workspace(self._h, mesh_index, rows)
        if nb < 0:
            raise ValueError("npfem_solve_factor_workspace: bad arguments")
        return nb

    def solve_factor(self, mesh_index: int, which: int, inp, out=None, work=None, stream=None):
        """out[r] = A^-1 inp[r] by substitution with the banded Cholesky factor of A = H~
        (which 0) or M~/h^2 (which 1); inp [rows, n_pad].  work: a device byte tensor of at
        least solve_factor_workspace(mesh_index, rows) bytes (allocated when None)."""
        import torch
        if out is None:
            out = torch.empty_like(inp)
        self._check(inp, out)
        rows = inp.shape[0]
        if work is None:
            work = torch.empty(max(1, self.solve_factor_workspace(mesh_index, rows)), dtype=torch.uint8,
                               device=inp.device)
        N.check(N.lib().npfem_solve_factor(self._h, mesh_index, which, _dptr(inp), _dptr(out), rows,
                                           _dptr(work), work.numel() * work.element_size(), None,
                                           _stream(stream)), "npfem_solve_factor")
        return out

    def _check(self, *ts):
        for t in ts:
            if t is None:
                continue
            if not t.is_cuda or t.dtype != self.torch_dtype or not t.is_contiguous():
                raise ValueError(f"expected a contiguous CUDA tensor of {self.torch_dtype}")

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and N is not None and N._lib is not None:
            N._lib.npfem_plan_destroy(h)


class Batch:
    """The cells advanced together; each cell's vertices are contiguous, in order."""

    def __init__(self, plan: Plan, cell_mesh):
        self.plan = plan
        self.cell_mesh = np.ascontiguousarray(cell_mesh, np.int32)
        h = c_void_p()
        nv = c_int64()
        N.check(N.lib().npfem_batch_create(plan._h, len(self.cell_mesh), _ptr(self.cell_mesh), byref(h),
                                           byref(nv)), "npfem_batch_create")
        self._h = h
        self.n_cells = len(self.cell_mesh)
        self.n_vertices = nv.value
        sizes = np.array([m.n for m in plan.meshes])[self.cell_mesh]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    def schedule(self, cells_per_tile: int | None = None, lbfgs_m: int | None = None) -> dict:
        """Set (when given) and report the schedule: cells per tile, history length,
        persistent workgroups, tiles."""
        if cells_per_tile is not None or lbfgs_m is not None:
            cur = self.schedule()
            N.check(N.lib().npfem_batch_schedule(self._h, cells_per_tile or cur["cells_per_tile"],
                                                 cur["lbfgs_m"] if lbfgs_m is None else lbfgs_m),
                    "npfem_batch_schedule")
        T, m, g, nt = c_int32(), c_int32(), c_int32(), c_int32()
        N.check(N.lib().npfem_batch_get_schedule(self._h, byref(T), byref(m), byref(g), byref(nt)),
                "npfem_batch_get_schedule")
        return {"cells_per_tile": T.value, "lbfgs_m": m.value, "grid_blocks": g.value, "n_tiles": nt.value}

    def autotune(self, x, v, f, max_lbfgs_m: int = 5, stream=None) -> dict:
        """Time the candidate schedules on these inputs and keep the fastest."""
        import torch
        xs, vs = torch.empty_like(x), torch.empty_like(v)
        best = c_double()
        N.check(N.lib().npfem_batch_autotune(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(xs), _dptr(vs),
                                             max_lbfgs_m, _stream(stream), byref(best)), "npfem_batch_autotune")
        out = self.schedule()
        out["best_ms"] = best.value
        return out

    def set_graph(self, use_graph: bool) -> None:
        N.check(N.lib().npfem_batch_set_graph(self._h, 1 if use_graph else 0), "npfem_batch_set_graph")

    def graph_counts(self) -> dict:
        """Graph captures and replays performed by this batch's steps."""
        c, r = c_int64(), c_int64()
        N.check(N.lib().npfem_batch_graph_counts(self._h, byref(c), byref(r)), "npfem_batch_graph_counts")
        return {"captures": c.value, "replays": r.value}

    def _vec(self, t, name):
        if t.shape != (self.n_vertices, 3):
            raise ValueError(f"{name} must have shape ({self.n_vertices}, 3)")
        self.plan._check(t)

    def step(self, x, v, f, x_out=None, v_out=None, u_guess=None, stats=True, stream=None):
        """One time step of every cell (Algorithm 1).  Returns (x_out, v_out, stats)."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f")):
            self._vec(t, nm)
        x_out = torch.empty_like(x) if x_out is None else x_out
        v_out = torch.empty_like(v) if v_out is None else v_out
        self._vec(x_out, "x_out")
        self._vec(v_out, "v_out")
        if u_guess is not None:
            self._vec(u_guess, "u_guess")
        st = None
        if stats is True:
            st = torch.empty(self.n_cells * N.CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=x.device)
        elif stats is not None and stats is not False:
            st = stats
        N.check(N.lib().npfem_step(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(x_out), _dptr(v_out),
                                   _dptr(u_guess), _dptr(st), _stream(stream)), "npfem_step")
        return x_out, v_out, st

    def detect_contacts(self, origin, x, cutoff, q=None, n=None, count=False, stream=None):
        """Nearest vertex of another cell within `cutoff` for every vertex: (q, n) in the
        plan's precision, and the number of vertices with a contact when count=True."""
        import torch
        self._vec(x, "x")
        if origin.dtype != torch.float64 or not origin.is_cuda or origin.shape != (self.n_cells, 3):
            raise ValueError("origin must be a float64 CUDA tensor of shape (n_cells, 3)")
        q = torch.empty_like(x) if q is None else q
        n = torch.empty_like(x) if n is None else n
        nc = c_int64(-1)
        N.check(N.lib().npfem_collisions_detect(self._h, _dptr(origin), _dptr(x), float(cutoff), _dptr(q), _dptr(n),
                                                byref(nc) if count else None, _stream(stream)),
                "npfem_collisions_detect")
        return (q, n, nc.value) if count else (q, n)

    def step_contacts(self, x, v, f, q, n, w_col, x_out=None, v_out=None, stats=True, stream=None):
        """One step with the collision term of the contacts (q, n) and weight w_col."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f"), (q, "q"), (n, "n")):
            self._vec(t, nm)
        x_out = torch.empty_like(x) if x_out is None else x_out
        v_out = torch.empty_like(v) if v_out is None else v_out
        st = None
        if stats is True:
            st = torch.empty(self.n_cells * N.CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=x.device)
        elif stats is not None and stats is not False:
            st = stats
        N.check(N.lib().npfem_step_contacts(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(q), _dptr(n), float(w_col),
                                            _dptr(x_out), _dptr(v_out), _dptr(st), _stream(stream)),
                "npfem_step_contacts")
        return x_out, v_out, st

    def step_noalloc(self, x, v, f, x_out, v_out, stats=None, u_guess=None, stream=None):
        """npfem_step with every buffer supplied by the caller and the workspace in the
        library's static device scratch: allocates nothing."""
        for t, nm in ((x, "x"), (v, "v"), (f, "f"), (x_out, "x_out"), (v_out, "v_out")):
            self._vec(t, nm)
        if u_guess is not None:
            self._vec(u_guess, "u_guess")
        N.check(N.lib().npfem_step_noalloc(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(x_out), _dptr(v_out),
                                           _dptr(u_guess), _dptr(stats), _stream(stream)), "npfem_step_noalloc")
        return x_out, v_out, stats

    @staticmethod
    def stats_to_numpy(st) -> np.ndarray:
        return st.cpu().numpy().view(N.CELL_STATS_DTYPE)

    def step_learned(self, net: "Net", x, v, f, x_out=None, v_out=None, stats=True, stream=None):
        """One step started from y_n + delta, delta predicted by the network."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f")):
            self._vec(t, nm)
        x_out = torch.empty_like(x) if x_out is None else x_out
        v_out = torch.empty_like(v) if v_out is None else v_out
        self._vec(x_out, "x_out")
        self._vec(v_out, "v_out")
        st = None
        if stats is True:
            st = torch.empty(self.n_cells * N.CELL_STATS_DTYPE.itemsize, dtype=torch.uint8, device=x.device)
        elif stats is not None and stats is not False:
            st = stats
        N.check(N.lib().npfem_step_learned(self._h, net._h, _dptr(x), _dptr(v), _dptr(f), _dptr(x_out),
                                           _dptr(v_out), _dptr(st), _stream(stream)), "npfem_step_learned")
        return x_out, v_out, st

    def first_guess(self, x, v, f, out=None, stream=None):
        """u0 = y_n - x_n = h^2 M~^-1 (M v / h + f) of every cell."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f")):
            self._vec(t, nm)
        out = torch.empty_like(x) if out is None else out
        self._vec(out, "out")
        N.check(N.lib().npfem_first_guess(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(out), _stream(stream)),
                "npfem_first_guess")
        return out

    def eval(self, x, v, f, u, stream=None):
        """Objective terms [n_cells, 8] and gradient at x_n + u."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f"), (u, "u")):
            self._vec(t, nm)
        grad = torch.empty_like(x)
        terms = torch.empty((self.n_cells, N.N_TERMS), dtype=torch.float64, device=x.device)
        N.check(N.lib().npfem_eval(self._h, _dptr(x), _dptr(v), _dptr(f), _dptr(u), _dptr(grad),
                                   _dptr(terms), _stream(stream)), "npfem_eval")
        return grad, terms

    def drag_forces(self, x, v, zeta, rate, origin, umax=0.0, radius=1.0, axis_y=0.0, axis_z=0.0,
                    out=None, stream=None):
        """Stokes drag towards a shear + Poiseuille flow (the fluid's stand-in)."""
        import torch
        self._vec(x, "x")
        self._vec(v, "v")
        out = torch.empty_like(x) if out is None else out
        for t in (zeta, rate, origin):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError("zeta, rate, origin must be float64 CUDA tensors")
        N.check(N.lib().npfem_drag_forces(self._h, _dptr(x), _dptr(v), _dptr(zeta), _dptr(rate), _dptr(origin),
                                          umax, radius, axis_y, axis_z, _dptr(out), _stream(stream)),
                "npfem_drag_forces")
        return out

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and N is not None and N._lib is not None:
            N._lib.npfem_batch_destroy(h)


class StatsTotal:
    """Device totals of per-cell step results over any number of steps
    (npfem_stats_accumulate): no host synchronisation until read."""

    def __init__(self, device="cuda:0", stream=None):
        import torch
        self.buf = torch.empty(N.STATS_TOTAL_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.reset(stream)

    def reset(self, stream=None) -> None:
        N.check(N.lib().npfem_stats_reset(_dptr(self.buf), _stream(stream)), "npfem_stats_reset")

    def add(self, stats, n_cells: int, stream=None) -> None:
        N.check(N.lib().npfem_stats_accumulate(_dptr(stats), int(n_cells), _dptr(self.buf), _stream(stream)),
                "npfem_stats_accumulate")

    def read(self) -> dict:
        a = self.buf.cpu().numpy().view(N.STATS_TOTAL_DTYPE)[0]
        return {k: (a[k].tolist() if a[k].shape else a[k].item()) for k in N.STATS_TOTAL_DTYPE.names}


def default_net_config(**overrides) -> N.NetConfig:
    c = N.NetConfig()
    N.lib().npfem_net_config_default(byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


class Net:
    """The learned warm-start network of a plan (parameters and optimiser on the GPU)."""

    def __init__(self, plan: Plan, theta=None, config: N.NetConfig | None = None):
        self.plan = plan
        self.config = config or default_net_config()
        self.n_params = int(N.lib().npfem_net_param_count(byref(self.config)))
        if self.n_params < 0:
            raise ValueError("invalid network configuration")
        theta = np.zeros(self.n_params, np.float32) if theta is None else np.ascontiguousarray(theta, np.float32)
        if theta.shape != (self.n_params,):
            raise ValueError(f"theta must have {self.n_params} entries")
        h = c_void_p()
        N.check(N.lib().npfem_net_create(plan._h, byref(self.config), _ptr(theta), byref(h)), "npfem_net_create")
        self._h = h

    def set_params(self, theta) -> None:
        theta = np.ascontiguousarray(theta, np.float32)
        if theta.shape != (self.n_params,):
            raise ValueError(f"theta must have {self.n_params} entries")
        N.check(N.lib().npfem_net_set_params(self._h, _ptr(theta)), "npfem_net_set_params")

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        N.check(N.lib().npfem_net_get_params(self._h, _ptr(out)), "npfem_net_get_params")
        return out

    def infer(self, batch: Batch, x, v, f, out=None, stream=None):
        """World-frame correction delta of every vertex of the batch."""
        import torch
        out = torch.empty_like(x) if out is None else out
        for t, nm in ((x, "x"), (v, "v"), (f, "f"), (out, "out")):
            batch._vec(t, nm)
        N.check(N.lib().npfem_net_infer(self._h, batch._h, _dptr(x), _dptr(v), _dptr(f), _dptr(out),
                                        _stream(stream)), "npfem_net_infer")
        return out

    def loss_grad(self, batch: Batch, x, v, f, x_next, u0, cells=None, n_cells=None, grad=None, stream=None,
                  want_loss=True):
        """Mean squared error of the listed cells (device int32 tensor, or the first n_cells)
        and its gradient (device float32 [n_params])."""
        import torch
        for t, nm in ((x, "x"), (v, "v"), (f, "f"), (x_next, "x_next"), (u0, "u0")):
            batch._vec(t, nm)
        if cells is not None:
            if cells.dtype != torch.int32 or not cells.is_cuda or not cells.is_contiguous():
                raise ValueError("cells must be a contiguous int32 CUDA tensor")
            n_cells = cells.numel()
        elif n_cells is None:
            n_cells = batch.n_cells
        grad = torch.empty(self.n_params, dtype=torch.float32, device=x.device) if grad is None else grad
        loss = c_double(float("nan"))
        N.check(N.lib().npfem_net_loss_grad(self._h, batch._h, _dptr(cells), int(n_cells), _dptr(x), _dptr(v),
                                            _dptr(f), _dptr(x_next), _dptr(u0),
                                            byref(loss) if want_loss else None, _dptr(grad), _stream(stream)),
                "npfem_net_loss_grad")
        return loss.value, grad

    def adam_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
        N.check(N.lib().npfem_net_adam_step(self._h, _dptr(grad), lr, beta1, beta2, eps, _stream(stream)),
                "npfem_net_adam_step")

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and N is not None and N._lib is not None:
            N._lib.npfem_net_destroy(h)
