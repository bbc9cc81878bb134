"""ctypes binding of libfmbem.so (the C ABI declared in include/fmbem.h).

Argument marshalling only: every step of the operator and the solve runs in
the HIP library.  PyTorch tensors provide device memory and streams.  There is
no fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as ct
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmbem.so")

FP64, FP32 = 0, 1
BURTON_MILLER, CBIE = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of device memory", 4: "device error",
          5: "not converged", 6: "workspace too small"}


class FmbemError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class CellMesh(ct.Structure):
    _fields_ = [("n_vertices", ct.c_int32), ("vertices", ct.POINTER(ct.c_double)),
                ("n_triangles", ct.c_int32), ("triangles", ct.POINTER(ct.c_int32))]


class PlanDesc(ct.Structure):
    _fields_ = [("grid", ct.c_int32 * 3), ("pitch", ct.c_double * 3), ("k", ct.c_double),
                ("order", ct.c_int32), ("formulation", ct.c_int32), ("alpha_re", ct.c_double),
                ("alpha_im", ct.c_double), ("near_radius", ct.c_int32 * 3), ("fft_shape", ct.c_int32 * 3),
                ("precisions", ct.c_uint32), ("dft_schedule", ct.c_int32), ("halfspace", ct.c_int32),
                ("plane_z", ct.c_double), ("reflection_re", ct.c_double), ("reflection_im", ct.c_double),
                ("tile_shape", ct.c_int32 * 3), ("exact", ct.c_int32),
                ("near_levels", ct.c_int32), ("near_order", ct.c_int32)]


DFT_SCHEDULE = {"auto": 0, "axes": 1, "fused": 2, "gemm": 3, "mfma": 4, "fft": 5}


class PlanInfo(ct.Structure):
    _fields_ = [("n_dof_cell", ct.c_int32), ("n_cells", ct.c_int32), ("n_dof", ct.c_int64), ("p", ct.c_int32),
                ("fft_shape", ct.c_int32 * 3), ("n_near", ct.c_int32), ("n_far", ct.c_int32),
                ("precisions", ct.c_uint32), ("resident_bytes", ct.c_size_t),
                ("workspace_bytes_per_rhs", ct.c_size_t * 2), ("scale", ct.c_double),
                ("near_levels", ct.c_int32), ("near_order", ct.c_int32), ("near_boxes", ct.c_int64),
                ("near_m2l_pairs", ct.c_int64), ("near_p2p_entries", ct.c_int64), ("near_macs_per_rhs", ct.c_double),
                ("near_max_tasks", ct.c_int32)]


class SolveOpts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("restart", ct.c_int32), ("max_iters", ct.c_int32),
                ("max_refinements", ct.c_int32), ("inner_precision", ct.c_int32), ("inner_tol", ct.c_double),
                ("orthogonalization", ct.c_int32)]


ORTHO = {"dgks": 0, "twice": 1, "once": 2}


class SolveInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("refinements", ct.c_int32), ("rel_residual", ct.c_double)]


class EngineTiming(ct.Structure):
    _fields_ = [("rounds", ct.c_int64), ("member_rounds", ct.c_int64), ("admitted", ct.c_int64),
                ("retired", ct.c_int64), ("enqueue_s", ct.c_double), ("admit_s", ct.c_double),
                ("wait_s", ct.c_double), ("retire_s", ct.c_double)]


EXPORTS = ["fmbem_plan_create", "fmbem_plan_query", "fmbem_plan_destroy", "fmbem_plan_export", "fmbem_matvec",
           "fmbem_solve", "fmbem_incident_plane_wave", "fmbem_incident_point_source", "fmbem_plan_profile",
           "fmbem_plan_profile_read", "fmbem_status_string", "fmbem_solve_batch", "fmbem_engine_create",
           "fmbem_engine_submit", "fmbem_engine_step", "fmbem_engine_poll", "fmbem_engine_stats",
           "fmbem_engine_destroy", "fmbem_solver_create", "fmbem_solver_run", "fmbem_solver_graph_stats",
           "fmbem_solver_destroy", "fmbem_incident_at_points", "fmbem_field", "fmbem_insertion_loss",
           "fmbem_matvec_noalloc", "fmbem_engine_timing_read"]
NOALLOC_WORKSPACE_BYTES = 64 << 20   # FMBEM_NOALLOC_WORKSPACE_BYTES
STAGES = tuple(f"{s}_{p}" for p in ("fp64", "fp32") for s in ("near", "reduce", "fft", "m2l", "ifft", "l2t"))

_lib = None


def load():
    """Load libfmbem.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_12050_amd.build`")
    lib = ct.CDLL(LIB_PATH)
    vp = ct.c_void_p
    lib.fmbem_plan_create.argtypes = [ct.POINTER(CellMesh), ct.POINTER(PlanDesc), vp, ct.POINTER(vp)]
    lib.fmbem_plan_query.argtypes = [vp, ct.POINTER(PlanInfo)]
    lib.fmbem_plan_destroy.argtypes = [vp]
    lib.fmbem_plan_export.argtypes = [vp, ct.c_int32, vp, ct.c_size_t]
    lib.fmbem_matvec.argtypes = [vp, ct.c_int32, ct.c_int32, vp, vp, vp, ct.c_size_t, vp]
    lib.fmbem_matvec_noalloc.argtypes = [vp, ct.c_int32, ct.c_int32, vp, vp, vp]
    lib.fmbem_solve.argtypes = [vp, ct.POINTER(SolveOpts), ct.c_int32, vp, vp, ct.POINTER(SolveInfo), vp]
    lib.fmbem_solver_create.argtypes = [vp, ct.POINTER(SolveOpts), ct.c_int32, ct.c_int32, ct.POINTER(vp)]
    lib.fmbem_solver_run.argtypes = [vp, vp, vp, ct.POINTER(SolveInfo), vp]
    lib.fmbem_solver_graph_stats.argtypes = [vp, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64)]
    lib.fmbem_solver_destroy.argtypes = [vp]
    lib.fmbem_engine_create.argtypes = [ct.c_size_t, ct.c_int32, vp, ct.POINTER(vp)]
    lib.fmbem_engine_submit.argtypes = [vp, vp, ct.POINTER(SolveOpts), ct.c_int32, vp, vp, ct.POINTER(ct.c_int64)]
    lib.fmbem_engine_step.argtypes = [vp]
    lib.fmbem_engine_poll.argtypes = [vp, ct.c_int64, ct.POINTER(ct.c_int32), ct.POINTER(SolveInfo)]
    lib.fmbem_engine_stats.argtypes = [vp, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_size_t)]
    lib.fmbem_engine_timing_read.argtypes = [vp, ct.POINTER(EngineTiming)]
    lib.fmbem_engine_destroy.argtypes = [vp]
    lib.fmbem_solve_batch.argtypes = [ct.c_int32, ct.POINTER(vp), ct.POINTER(SolveOpts), ct.POINTER(ct.c_int32),
                                      ct.POINTER(vp), ct.POINTER(vp), ct.POINTER(SolveInfo), vp]
    lib.fmbem_incident_plane_wave.argtypes = [vp, ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, vp, vp]
    lib.fmbem_incident_point_source.argtypes = [vp, ct.c_int32, ct.POINTER(ct.c_double), ct.c_double, vp, vp]
    dp = ct.POINTER(ct.c_double)
    lib.fmbem_incident_at_points.argtypes = [vp, ct.c_int32, ct.c_int32, dp, ct.c_double, ct.c_int32, dp, vp, vp]
    lib.fmbem_field.argtypes = [vp, ct.c_int32, vp, ct.c_int32, dp, vp, vp, vp]
    lib.fmbem_insertion_loss.argtypes = [ct.c_int32, ct.c_int32, vp, vp, vp, vp]
    lib.fmbem_plan_profile.argtypes = [vp, ct.c_uint32, ct.c_int32]
    lib.fmbem_plan_profile_read.argtypes = [vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)]
    lib.fmbem_status_string.argtypes = [ct.c_int32]
    lib.fmbem_status_string.restype = ct.c_char_p
    for f in EXPORTS:
        if f != "fmbem_status_string":
            getattr(lib, f).restype = ct.c_int32
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != 0:
        raise FmbemError(status, where)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def solve_opts(tol=1e-8, restart=30, max_iters=1000, max_refinements=20, inner="fp64", inner_tol=1e-5,
               ortho="dgks") -> SolveOpts:
    return SolveOpts(tol, restart, max_iters, max_refinements, _precision(inner), inner_tol, ORTHO[ortho])


def check_vectors(n_dof: int, dtype, x, y=None, what=("x", "y")) -> int:
    """Validate caller tensors before any launch (the C ABI takes raw pointers, so this is the
    only guard against writes past an allocation): x, and y when given, must be contiguous
    device tensors of ``dtype`` holding the same whole number R >= 1 of [n_dof] vectors.
    Returns R; raises ValueError otherwise."""
    for name, t in zip(what, (x, y)):
        if t is None:
            continue
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    R = x.numel() // n_dof
    if R < 1 or R * n_dof != x.numel():
        raise ValueError(f"{what[0]} size {x.numel()} is not a positive multiple of the DOF count {n_dof}")
    if y is not None and y.numel() != x.numel():
        raise ValueError(f"{what[1]} must hold as many elements as {what[0]} ({y.numel()} != {x.numel()})")
    return R


def _info_dicts(info):
    return [dict(iterations=i.iterations, refinements=i.refinements, rel_residual=i.rel_residual) for i in info]


def solve_batch(problems, stream=None, raise_on_not_converged=True):
    """Solve several independent problems in lockstep with grouped launches.

    problems: list of (plan, b, x or None, options dict for solve_opts).  Returns the
    list of (x, infos) in the same order."""
    import torch
    n = len(problems)
    if n == 0:
        return []
    plans = (ct.c_void_p * n)()
    opts = (SolveOpts * n)()
    nr = (ct.c_int32 * n)()
    bp = (ct.c_void_p * n)()
    xp = (ct.c_void_p * n)()
    xs = []
    for i, (plan, b, x, kw) in enumerate(problems):
        R = check_vectors(plan.n_dof, torch.complex128, b, x, ("b", "x"))
        if x is None:
            x = torch.zeros_like(b)
        plans[i] = plan._h
        opts[i] = solve_opts(**(kw or {}))
        nr[i] = R
        bp[i] = b.data_ptr()
        xp[i] = x.data_ptr()
        xs.append(x)
    info = (SolveInfo * sum(nr))()
    lib = load()
    st = lib.fmbem_solve_batch(n, plans, opts, nr, bp, xp, info, _stream_ptr(stream))
    if st != 0 and (st != 5 or raise_on_not_converged):
        check(st, "fmbem_solve_batch")
    out, off = [], 0
    for i in range(n):
        out.append((xs[i], _info_dicts(info[off:off + nr[i]])))
        off += nr[i]
    return out


class Solver:
    """Persistent solver for repeated solves with one plan and RHS count (buffers allocated
    once; optional HIP-graph replay of the Arnoldi steps)."""

    def __init__(self, plan, n_rhs: int = 1, graphs: bool = False, **opts):
        self._lib = load()
        self.plan = plan
        self.n_rhs = int(n_rhs)
        o = solve_opts(**opts)
        h = ct.c_void_p()
        check(self._lib.fmbem_solver_create(plan._h, ct.byref(o), self.n_rhs, 1 if graphs else 0, ct.byref(h)),
              "fmbem_solver_create")
        self._h = h

    def close(self):
        if self._h:
            self._lib.fmbem_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, b, x=None, stream=None, raise_on_not_converged=True):
        import torch
        if check_vectors(self.plan.n_dof, torch.complex128, b, x, ("b", "x")) != self.n_rhs:
            raise ValueError("b does not match the solver's right-hand-side count")
        if x is None:
            x = torch.zeros_like(b)
        info = (SolveInfo * self.n_rhs)()
        st = self._lib.fmbem_solver_run(self._h, ct.c_void_p(b.data_ptr()), ct.c_void_p(x.data_ptr()), info,
                                        _stream_ptr(stream))
        if st != 0 and (st != 5 or raise_on_not_converged):
            check(st, "fmbem_solver_run")
        return x, _info_dicts(info)

    def graph_stats(self):
        g, r = ct.c_int32(), ct.c_int64()
        check(self._lib.fmbem_solver_graph_stats(self._h, ct.byref(g), ct.byref(r)), "fmbem_solver_graph_stats")
        return dict(graphs=g.value, replays=r.value)


class Engine:
    """Serving engine (continuous batching of solve requests, admission by device bytes).

    submit() queues a request and returns a ticket; step() advances every admitted
    problem by one operator application; poll() returns None while pending, else
    (x, infos, status).  The engine keeps b and x alive until the ticket is polled."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 16, stream=None):
        self._lib = load()
        self._stream = stream
        h = ct.c_void_p()
        check(self._lib.fmbem_engine_create(int(hbm_budget_bytes), int(max_slots), _stream_ptr(stream),
                                            ct.byref(h)), "fmbem_engine_create")
        self._h = h
        self._held = {}

    def close(self):
        if self._h:
            self._lib.fmbem_engine_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, plan, b, x=None, **opts) -> int:
        import torch
        R = check_vectors(plan.n_dof, torch.complex128, b, x, ("b", "x"))
        if x is None:
            x = torch.zeros_like(b)
        o = solve_opts(**opts)
        t = ct.c_int64()
        check(self._lib.fmbem_engine_submit(self._h, plan._h, ct.byref(o), R, ct.c_void_p(b.data_ptr()),
                                            ct.c_void_p(x.data_ptr()), ct.byref(t)), "fmbem_engine_submit")
        self._held[t.value] = (plan, b, x, R)
        return t.value

    def step(self):
        check(self._lib.fmbem_engine_step(self._h), "fmbem_engine_step")

    def poll(self, ticket: int):
        plan, b, x, R = self._held[ticket]
        done = ct.c_int32()
        info = (SolveInfo * R)()
        st = self._lib.fmbem_engine_poll(self._h, ticket, ct.byref(done), info)
        if not done.value:
            check(st, "fmbem_engine_poll")
            return None
        del self._held[ticket]
        return x, _info_dicts(info), st

    def stats(self):
        a, q, u = ct.c_int32(), ct.c_int32(), ct.c_size_t()
        check(self._lib.fmbem_engine_stats(self._h, ct.byref(a), ct.byref(q), ct.byref(u)), "fmbem_engine_stats")
        return dict(active=a.value, queued=q.value, bytes_in_use=u.value)

    def timing(self):
        t = EngineTiming()
        check(self._lib.fmbem_engine_timing_read(self._h, ct.byref(t)), "fmbem_engine_timing_read")
        return {name: getattr(t, name) for name, _ in EngineTiming._fields_}


def _precision(p) -> int:
    if p in (FP64, "fp64", "f64", "complex128"):
        return FP64
    if p in (FP32, "fp32", "f32", "complex64"):
        return FP32
    raise ValueError(p)


class Plan:
    """A device-resident FMPBEM operator (fmbem_plan_create)."""

    def __init__(self, vertices, triangles, grid, pitch, k, order, formulation="bm", alpha=None,
                 near_radius=(1, 1, 1), fft_shape=(0, 0, 0), precisions=("fp64", "fp32"), stream=None,
                 dft_schedule="auto", halfspace=None, tile_shape=(0, 0, 0), exact=False, near_levels=0,
                 near_order=0):
        """halfspace: None (full space) or (plane_z, R_p): the half-space Green's function with the
        plane z = plane_z and reflection coefficient R_p.  tile_shape: forced tile shapes of the
        near-field, L2T and M2L GEMM launches (0 = autotuned, v = shape v - 1).  exact: the exact
        periodic BEM operator (every block integrated, n x n blocks per bin) instead of the fast
        multipole one; order is then ignored.  near_levels >= 1: the multilevel near field of
        FMPBEM2 with that many subdivisions of the cell box and truncation near_order (0:
        min(order, 7))."""
        lib = load()
        self._lib = lib
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        t = np.ascontiguousarray(triangles, dtype=np.int32)
        mesh = CellMesh(v.shape[0], v.ctypes.data_as(ct.POINTER(ct.c_double)), t.shape[0],
                        t.ctypes.data_as(ct.POINTER(ct.c_int32)))
        d = PlanDesc()
        for a in range(3):
            d.grid[a] = int(grid[a])
            d.pitch[a] = float(pitch[a])
            d.near_radius[a] = int(near_radius[a])
            d.fft_shape[a] = int(fft_shape[a])
        d.k = float(k)
        d.order = int(order)
        d.formulation = {"bm": BURTON_MILLER, "cbie": CBIE}[formulation]
        if alpha is None:
            d.alpha_re = d.alpha_im = math.nan
        else:
            d.alpha_re, d.alpha_im = float(np.real(alpha)), float(np.imag(alpha))
        d.precisions = sum(1 << _precision(p) for p in precisions)
        d.dft_schedule = DFT_SCHEDULE[dft_schedule]
        for a in range(3):
            d.tile_shape[a] = int(tile_shape[a])
        d.exact = 1 if exact else 0
        d.near_levels = int(near_levels)
        d.near_order = int(near_order)
        if halfspace is not None:
            zg, rp = halfspace
            d.halfspace = 1
            d.plane_z = float(zg)
            d.reflection_re, d.reflection_im = float(np.real(rp)), float(np.imag(rp))
        h = ct.c_void_p()
        check(lib.fmbem_plan_create(ct.byref(mesh), ct.byref(d), _stream_ptr(stream), ct.byref(h)),
              "fmbem_plan_create")
        self._h = h
        info = PlanInfo()
        check(lib.fmbem_plan_query(h, ct.byref(info)), "fmbem_plan_query")
        self.info = {f: getattr(info, f) for f, _ in PlanInfo._fields_}
        self.info["fft_shape"] = tuple(info.fft_shape)
        self.info["workspace_bytes_per_rhs"] = tuple(info.workspace_bytes_per_rhs)
        self.n = info.n_dof_cell
        self.n_cells = info.n_cells
        self.n_dof = info.n_dof
        self.p = info.p

    @classmethod
    def from_workload(cls, w, precisions=("fp64", "fp32"), stream=None, **kw):
        return cls(w.vertices, w.triangles, w.lattice.grid, w.lattice.pitch, w.k, w.order, w.formulation,
                   near_radius=w.near_radius, precisions=precisions, stream=stream, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fmbem_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- inspection
    def export(self, what: str) -> np.ndarray:
        n, p = self.n, self.p
        B = int(np.prod(self.info["fft_shape"]))
        shapes = {"S": (0, (self.info["n_near"], n, n), np.complex128), "V0": (1, (p, n), np.complex128),
                  "U0": (2, (n, p), np.complex128), "Lambda": (3, (B, p, p), np.complex128),
                  "near_offsets": (4, (self.info["n_near"], 3), np.int32)}
        code, shape, dt = shapes[what]
        out = np.zeros(shape, dtype=dt)
        check(self._lib.fmbem_plan_export(self._h, code, out.ctypes.data_as(ct.c_void_p), out.nbytes),
              "fmbem_plan_export")
        return out

    # ---------------------------------------------------------------- profiling
    def profile(self, stages=None, period: int = 1):
        """Start recording the named stages (None: all; [] stops), e.g. ["near_fp32"], on every
        period-th operator application."""
        if stages is None:
            mask = (1 << len(STAGES)) - 1
        else:
            mask = 0
            for s in stages:
                mask |= 1 << STAGES.index(s)
        check(self._lib.fmbem_plan_profile(self._h, mask, int(period)), "fmbem_plan_profile")

    def profile_read(self):
        """{stage: (total ms, launches)} of the operator applications since profile()."""
        ms = (ct.c_double * len(STAGES))()
        cnt = (ct.c_int64 * len(STAGES))()
        check(self._lib.fmbem_plan_profile_read(self._h, ms, cnt), "fmbem_plan_profile_read")
        return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}

    # ---------------------------------------------------------------- operator
    def workspace(self, n_rhs: int, precision="fp64"):
        import torch
        nb = n_rhs * self.info["workspace_bytes_per_rhs"][_precision(precision)]
        return torch.empty(max(nb, 256), dtype=torch.uint8, device="cuda")

    def matvec(self, x, y=None, precision="fp64", workspace=None, stream=None):
        """y = A x for x of shape [R, n_cells, n_dof_cell] (or [R, N]) on the device."""
        import torch
        pr = _precision(precision)
        dt = torch.complex128 if pr == FP64 else torch.complex64
        R = check_vectors(self.n_dof, dt, x, y)
        if y is None:
            y = torch.empty_like(x)
        if workspace is None:
            workspace = self.workspace(R, pr)
        elif not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous CUDA tensor")
        check(self._lib.fmbem_matvec(self._h, pr, R, ct.c_void_p(x.data_ptr()), ct.c_void_p(y.data_ptr()),
                                     ct.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                     _stream_ptr(stream)),
              "fmbem_matvec")
        return y

    def matvec_noalloc(self, x, y, precision="fp64", stream=None):
        """y = A x through fmbem_matvec_noalloc (workspace in the library's static device array,
        nothing allocated); x and y are caller-owned contiguous device tensors of equal size."""
        import torch
        pr = _precision(precision)
        dt = torch.complex128 if pr == FP64 else torch.complex64
        if y is None:
            raise ValueError("y must be given (the call allocates nothing)")
        R = check_vectors(self.n_dof, dt, x, y)
        check(self._lib.fmbem_matvec_noalloc(self._h, pr, R, ct.c_void_p(x.data_ptr()), ct.c_void_p(y.data_ptr()),
                                             _stream_ptr(stream)), "fmbem_matvec_noalloc")
        return y

    def solve(self, b, x=None, tol=1e-8, restart=30, max_iters=1000, max_refinements=20, inner="fp64",
              inner_tol=1e-5, ortho="dgks", stream=None, raise_on_not_converged=True):
        import torch
        R = check_vectors(self.n_dof, torch.complex128, b, x, ("b", "x"))
        if x is None:
            x = torch.zeros_like(b)
        o = solve_opts(tol, restart, max_iters, max_refinements, inner, inner_tol, ortho)
        info = (SolveInfo * R)()
        st = self._lib.fmbem_solve(self._h, ct.byref(o), R, ct.c_void_p(b.data_ptr()), ct.c_void_p(x.data_ptr()),
                                   info, _stream_ptr(stream))
        if st != 0 and (st != 5 or raise_on_not_converged):
            check(st, "fmbem_solve")
        return x, [dict(iterations=i.iterations, refinements=i.refinements, rel_residual=i.rel_residual)
                   for i in info]

    def incident_plane_wave(self, directions, amplitude=1.0, stream=None):
        import torch
        d = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
        out = torch.empty((d.shape[0], self.n_cells, self.n), dtype=torch.complex128, device="cuda")
        check(self._lib.fmbem_incident_plane_wave(self._h, d.shape[0], d.ctypes.data_as(ct.POINTER(ct.c_double)),
                                                  float(amplitude), ct.c_void_p(out.data_ptr()),
                                                  _stream_ptr(stream)), "fmbem_incident_plane_wave")
        return out

    def incident_point_source(self, sources, amplitude=1.0, stream=None):
        import torch
        s = np.ascontiguousarray(np.atleast_2d(sources), dtype=np.float64)
        out = torch.empty((s.shape[0], self.n_cells, self.n), dtype=torch.complex128, device="cuda")
        check(self._lib.fmbem_incident_point_source(self._h, s.shape[0], s.ctypes.data_as(ct.POINTER(ct.c_double)),
                                                    float(amplitude), ct.c_void_p(out.data_ptr()),
                                                    _stream_ptr(stream)), "fmbem_incident_point_source")
        return out

    def incident_at_points(self, kind, sources, points, amplitude=1.0, stream=None):
        """Incident pressure at points (fmbem_incident_at_points); kind "plane_wave" (sources =
        unit directions) or "point_source" (sources = positions).  Returns complex128 [R, M]."""
        import torch
        kinds = {"plane_wave": 0, "point_source": 1}
        if kind not in kinds:
            raise ValueError(f"kind must be one of {sorted(kinds)}")
        src = np.ascontiguousarray(np.atleast_2d(sources), dtype=np.float64)
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        if src.shape[1] != 3 or pts.shape[1] != 3:
            raise ValueError("sources and points must be [.., 3]")
        out = torch.empty((src.shape[0], pts.shape[0]), dtype=torch.complex128, device="cuda")
        dp = ct.POINTER(ct.c_double)
        check(self._lib.fmbem_incident_at_points(self._h, kinds[kind], src.shape[0], src.ctypes.data_as(dp),
                                                 float(amplitude), pts.shape[0], pts.ctypes.data_as(dp),
                                                 ct.c_void_p(out.data_ptr()), _stream_ptr(stream)),
              "fmbem_incident_at_points")
        return out

    def field(self, x, points, p_inc=None, stream=None):
        """Pressure at points of the fluid from the surface pressure x ([R, C, n] or [R, N],
        complex128 on the device): fmbem_field.  p_inc ([R, M] complex128 on the device) is
        added when given.  Returns complex128 [R, M]."""
        import torch
        if x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous complex128 device tensor")
        R = x.shape[0] if x.dim() > 1 else 1
        if x.numel() != R * self.n_cells * self.n:
            raise ValueError("x must hold [R][n_cells][n] values")
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        if pts.shape[1] != 3:
            raise ValueError("points must be [M, 3]")
        M = pts.shape[0]
        if p_inc is not None:
            if p_inc.dtype != torch.complex128 or not p_inc.is_cuda or not p_inc.is_contiguous() \
                    or p_inc.numel() != R * M:
                raise ValueError("p_inc must be a contiguous complex128 device tensor of R x M values")
        out = torch.empty((R, M), dtype=torch.complex128, device="cuda")
        check(self._lib.fmbem_field(self._h, R, ct.c_void_p(x.data_ptr()), M,
                                    pts.ctypes.data_as(ct.POINTER(ct.c_double)),
                                    ct.c_void_p(p_inc.data_ptr() if p_inc is not None else 0),
                                    ct.c_void_p(out.data_ptr()), _stream_ptr(stream)), "fmbem_field")
        return out


def insertion_loss(p_inc, p, stream=None):
    """IL in dB per right-hand side over the observation points (fmbem_insertion_loss);
    p_inc, p: complex128 device tensors [R, M].  Returns float64 [R] on the device."""
    import torch
    for t in (p_inc, p):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("p_inc and p must be contiguous complex128 device tensors")
    if p_inc.shape != p.shape or p.dim() not in (1, 2):
        raise ValueError("p_inc and p must have the same shape [R, M]")
    R, M = (1, p.shape[0]) if p.dim() == 1 else p.shape
    il = torch.empty(R, dtype=torch.float64, device="cuda")
    lib = load()
    check(lib.fmbem_insertion_loss(R, M, ct.c_void_p(p_inc.data_ptr()), ct.c_void_p(p.data_ptr()),
                                   ct.c_void_p(il.data_ptr()), _stream_ptr(stream)), "fmbem_insertion_loss")
    return il
