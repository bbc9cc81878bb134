"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol that include/fmbem.h declares, rejects invalid arguments before any
device work, and the Python layer fails loudly when the library is missing."""
import ctypes as ct
import math
import os
import re

import numpy as np
import pytest

import paper_2201_12050_amd as fm
from paper_2201_12050_amd import _lib
from workloads import icosphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "fmbem.h")).read()
    return set(re.findall(r"\b(fmbem_[a-z_0-9]+)\s*\(", text))


def test_exports_every_declared_symbol():
    declared = _declared()
    assert declared == set(_lib.EXPORTS)
    lib = ct.CDLL(_lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name


def _desc(**kw):
    d = _lib.PlanDesc()
    for a in range(3):
        d.grid[a] = (3, 3, 1)[a]
        d.pitch[a] = 0.3
        d.near_radius[a] = 1
        d.fft_shape[a] = 0
    d.k = 10.0
    d.order = 4
    d.formulation = 0
    d.alpha_re = d.alpha_im = math.nan
    d.precisions = 3
    for key, v in kw.items():
        if key in ("grid", "pitch", "fft_shape", "near_radius", "tile_shape"):
            for a in range(3):
                getattr(d, key)[a] = v[a]
        else:
            setattr(d, key, v)
    return d


def _mesh(v, t):
    v = np.ascontiguousarray(v, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.int32)
    return _lib.CellMesh(v.shape[0], v.ctypes.data_as(ct.POINTER(ct.c_double)), t.shape[0],
                         t.ctypes.data_as(ct.POINTER(ct.c_int32))), (v, t)


@pytest.mark.parametrize("case", ["null", "bad_index", "degenerate", "order", "fft", "k", "grid", "formulation",
                                  "nan_vertex", "radius", "dft_schedule", "halfspace_flag", "halfspace_grid",
                                  "halfspace_crossing", "halfspace_nan", "tile_shape_high", "tile_shape_negative"])
def test_plan_create_rejects_invalid_arguments(case):
    lib = fm.load()
    v, t = icosphere(1, 0.1)
    out = ct.c_void_p()
    if case == "null":
        assert lib.fmbem_plan_create(None, None, None, ct.byref(out)) == 1
        return
    desc = _desc()
    if case == "bad_index":
        t = t.copy(); t[3, 1] = v.shape[0]
    elif case == "degenerate":
        t = t.copy(); t[5, 2] = t[5, 1]
    elif case == "nan_vertex":
        v = v.copy(); v[0, 0] = np.nan
    elif case == "order":
        desc = _desc(order=21)
    elif case == "fft":
        desc = _desc(fft_shape=(4, 0, 0))   # needs >= 2*3-1 = 5
    elif case == "k":
        desc = _desc(k=0.0)
    elif case == "grid":
        desc = _desc(grid=(0, 3, 1))
    elif case == "formulation":
        desc = _desc(formulation=7)
    elif case == "radius":
        desc = _desc(near_radius=(4, 1, 1))
    elif case == "dft_schedule":
        desc = _desc(dft_schedule=6)
    elif case == "halfspace_flag":
        desc = _desc(halfspace=2, plane_z=0.2)
    elif case == "halfspace_grid":        # the second layer (z up to 0.4) crosses z = 0.2
        desc = _desc(halfspace=1, plane_z=0.2, grid=(3, 3, 2))
    elif case == "halfspace_crossing":    # the sphere of radius 0.1 crosses z = 0.05
        desc = _desc(halfspace=1, plane_z=0.05, reflection_re=1.0)
    elif case == "halfspace_nan":
        desc = _desc(halfspace=1, plane_z=math.nan)
    elif case == "tile_shape_high":
        desc = _desc(tile_shape=(0, 0, 11))
    elif case == "tile_shape_negative":
        desc = _desc(tile_shape=(-1, 0, 0))
    mesh, keep = _mesh(v, t)
    assert lib.fmbem_plan_create(ct.byref(mesh), ct.byref(desc), None, ct.byref(out)) == 1
    assert out.value is None


@pytest.mark.parametrize("case", ["levels_negative", "levels_high", "order_high", "order_negative"])
def test_multilevel_descriptor_rejects_invalid_values(case):
    lib = fm.load()
    v, t = icosphere(1, 0.1)
    kw = {"levels_negative": dict(near_levels=-1), "levels_high": dict(near_levels=9),
          "order_high": dict(near_levels=2, near_order=8), "order_negative": dict(near_levels=2, near_order=-1)}[case]
    mesh, keep = _mesh(v, t)
    out = ct.c_void_p()
    assert lib.fmbem_plan_create(ct.byref(mesh), ct.byref(_desc(**kw)), None, ct.byref(out)) == 1
    assert out.value is None


@pytest.mark.parametrize("case", ["exact", "halfspace", "radius", "outside_box", "at_leaf_centre"])
def test_multilevel_descriptor_rejects_unsupported_combinations(case):
    # FMPBEM2 needs near radius 1, the full space, the multipole far field and every collocation
    # point inside the cell's lattice box, off its leaf centre (checked before any device work)
    lib = fm.load()
    v, t = icosphere(1, 0.1)
    kw = dict(near_levels=2)
    if case == "exact":
        kw["exact"] = 1
    elif case == "halfspace":
        kw.update(halfspace=1, plane_z=-0.2)
    elif case == "radius":
        kw["near_radius"] = (2, 1, 1)
    elif case == "outside_box":
        kw["pitch"] = (0.15, 0.15, 0.15)   # the sphere of radius 0.1 leaves the box
    elif case == "at_leaf_centre":
        # one triangle whose centroid is the centre of its level-2 leaf
        c = np.array([0.0375, 0.0375, 0.0375])
        v = np.array([c + [0.01, 0, 0], c + [-0.005, 0.008, 0], c + [-0.005, -0.008, 0]])
        t = np.array([[0, 1, 2]])
    mesh, keep = _mesh(v, t)
    out = ct.c_void_p()
    assert lib.fmbem_plan_create(ct.byref(mesh), ct.byref(_desc(**kw)), None, ct.byref(out)) == 2
    assert out.value is None


def test_other_entry_points_reject_null_plan():
    lib = fm.load()
    assert lib.fmbem_matvec(None, 0, 1, None, None, None, 0, None) == 1
    assert lib.fmbem_matvec_noalloc(None, 0, 1, None, None, None) == 1
    assert lib.fmbem_plan_query(None, None) == 1
    assert lib.fmbem_plan_destroy(None) == 1
    assert lib.fmbem_plan_export(None, 0, None, 0) == 1
    assert lib.fmbem_solve(None, None, 1, None, None, None, None) == 1
    assert lib.fmbem_solve_batch(0, None, None, None, None, None, None, None) == 1
    assert lib.fmbem_engine_create(0, 1, None, None) == 1
    assert lib.fmbem_engine_submit(None, None, None, 1, None, None, None) == 1
    assert lib.fmbem_engine_step(None) == 1
    assert lib.fmbem_engine_poll(None, 1, None, None) == 1
    assert lib.fmbem_engine_stats(None, None, None, None) == 1
    assert lib.fmbem_engine_timing_read(None, None) == 1
    assert lib.fmbem_engine_destroy(None) == 1
    assert lib.fmbem_solver_create(None, None, 1, 0, None) == 1
    assert lib.fmbem_solver_run(None, None, None, None, None) == 1
    assert lib.fmbem_solver_graph_stats(None, None, None) == 1
    assert lib.fmbem_solver_destroy(None) == 1
    assert lib.fmbem_status_string(7) == b"request exceeds the engine's memory budget"
    assert lib.fmbem_incident_plane_wave(None, 1, None, 1.0, None, None) == 1
    assert lib.fmbem_incident_at_points(None, 0, 1, None, 1.0, 1, None, None, None) == 1
    assert lib.fmbem_field(None, 1, None, 1, None, None, None, None) == 1
    assert lib.fmbem_insertion_loss(1, 1, None, None, None, None) == 1
    assert lib.fmbem_insertion_loss(0, 1, 8, 8, 8, None) == 1
    assert lib.fmbem_status_string(5) == b"not converged"
    assert lib.fmbem_status_string(99) == b"unknown status"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2201_12050_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f


def test_struct_layouts_match_header(tmp_path):
    # every ctypes mirror of a header struct has the C compiler's size and field offsets
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"fmbem_cell_mesh": _lib.CellMesh, "fmbem_plan_desc": _lib.PlanDesc, "fmbem_plan_info": _lib.PlanInfo,
               "fmbem_solve_opts": _lib.SolveOpts, "fmbem_solve_info": _lib.SolveInfo,
               "fmbem_engine_timing": _lib.EngineTiming}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmbem.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ct.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


class _FakeDeviceTensor:
    """Stand-in for a device tensor (dtype, is_cuda, contiguity, element count) so that the
    binding's argument checks run without a GPU."""

    def __init__(self, numel, dtype, cuda=True, contiguous=True):
        self._n, self.dtype, self.is_cuda, self._c = numel, dtype, cuda, contiguous

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c


@pytest.mark.parametrize("case", ["ok", "ok_no_y", "x_dtype", "y_dtype", "x_host", "y_host", "y_strided",
                                  "x_ragged", "x_empty", "y_short", "y_long"])
def test_binding_checks_vectors_before_launch(case):
    import torch
    c128, c64 = torch.complex128, torch.complex64
    n_dof = 40
    x = _FakeDeviceTensor(3 * n_dof, c128)
    y = _FakeDeviceTensor(3 * n_dof, c128)
    if case == "ok_no_y":
        y = None
    elif case == "x_dtype":
        x = _FakeDeviceTensor(3 * n_dof, c64)
    elif case == "y_dtype":          # a complex64 output for an FP64 apply would be written past its end
        y = _FakeDeviceTensor(3 * n_dof, c64)
    elif case == "x_host":
        x = _FakeDeviceTensor(3 * n_dof, c128, cuda=False)
    elif case == "y_host":
        y = _FakeDeviceTensor(3 * n_dof, c128, cuda=False)
    elif case == "y_strided":
        y = _FakeDeviceTensor(3 * n_dof, c128, contiguous=False)
    elif case == "x_ragged":         # R would be floored silently
        x = _FakeDeviceTensor(3 * n_dof + 7, c128)
    elif case == "x_empty":
        x = _FakeDeviceTensor(0, c128)
    elif case == "y_short":
        y = _FakeDeviceTensor(2 * n_dof, c128)
    elif case == "y_long":
        y = _FakeDeviceTensor(4 * n_dof, c128)
    if case.startswith("ok"):
        assert _lib.check_vectors(n_dof, c128, x, y) == 3
    else:
        with pytest.raises(ValueError):
            _lib.check_vectors(n_dof, c128, x, y)


def test_binding_entry_points_use_the_vector_check():
    # every method that hands caller tensors to the library validates them first
    import inspect
    for fn in (_lib.Plan.matvec, _lib.Plan.matvec_noalloc, _lib.Plan.solve, _lib.Solver.run, _lib.Engine.submit,
               _lib.solve_batch):
        assert "check_vectors(" in inspect.getsource(fn), fn.__qualname__
