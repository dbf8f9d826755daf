"""CPU-side checks of the C ABI: the library loads, exports every function
include/subdiv.h declares, and its host-only entry points behave. No call
here touches a GPU."""
import ctypes
import os
import re

import pytest

from paper_1809_06047_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "subdiv.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(subdiv_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1809_06047_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "subdiv_refine" in names and "subdiv_plan" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding misses {n}"


def test_struct_layouts_match_header():
    # sizes the header implies on x86-64 (natural alignment)
    assert ctypes.sizeof(_lib.subdiv_mesh) == 4 * 4 + 3 * 8 + 8 + 2 * 8
    assert ctypes.sizeof(_lib.subdiv_level_info) == 5 * 8 + 2 * 4
    assert ctypes.sizeof(_lib.subdiv_level_out) == 4 * 8
    assert _lib.subdiv_plan_info.workspace_bytes.offset == 24 + 11 * 48


def test_host_entry_points(lib):
    assert lib.subdiv_version() == 1000
    assert lib.subdiv_strerror(-3) == b"non-manifold or inconsistently oriented mesh"
    assert lib.subdiv_last_error() == b""
    # workspace bound: grows with levels, zero on invalid input or int32 overflow
    b1 = lib.subdiv_workspace_bound(10242, 17408, 55296, 829, 0, 1, 0)
    b6 = lib.subdiv_workspace_bound(10242, 17408, 55296, 829, 0, 6, 0)
    assert 0 < b1 < b6
    assert lib.subdiv_workspace_bound(10242, 17408, 55296, 0, 0, 0, 0) == 0
    assert lib.subdiv_workspace_bound(10242, 17408, 55296, 0, 7, 2, 0) == 0
    assert lib.subdiv_workspace_bound(10242, 17408, 55296, 0, 0, 12, 0) == 0   # 4^11 H > int32
    assert lib.subdiv_workspace_bound(10242, 17408, 55296, 0, 0, 9, 0) == 0    # H_9 = 4^8 H_0 > int32


def test_plan_rejects_bad_arguments_without_device(lib):
    """Argument checks happen on the host before any device work."""
    info = _lib.subdiv_plan_info()
    m = _lib.subdiv_mesh()
    assert lib.subdiv_plan(None, 0, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    assert lib.subdiv_plan(ctypes.byref(m), 0, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    m.num_vertices, m.num_faces, m.face_order = 4, 1, 5
    m.face_verts = m.positions = 16  # never dereferenced: the order check fails first
    assert lib.subdiv_plan(ctypes.byref(m), 0, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    m.face_order = 4
    assert lib.subdiv_plan(ctypes.byref(m), 5, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    assert lib.subdiv_plan(ctypes.byref(m), 0, 0, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    assert lib.subdiv_refine(ctypes.byref(m), ctypes.byref(info), None, None, 0, None) == _lib.INVALID_ARG
    m.face_verts = 16 + 4  # face tables are read as int4 rows: 16-byte alignment is required
    assert lib.subdiv_plan(ctypes.byref(m), 0, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    assert lib.subdiv_workspace_bound(4, 1, 4, 0, 0, 1, 0) > 0  # sizes alone carry no pointers


def test_later_entry_points_reject_bad_arguments_without_device(lib):
    """Vertex data, selection, extraction and the backward check their
    arguments and the plan's state on the host before any device work."""
    info = _lib.subdiv_plan_info()   # never planned: stamp 0
    info.levels = 1                  # so that the mesh arguments pass and the state is what fails
    m = _lib.subdiv_mesh()
    m.num_vertices, m.num_faces, m.face_order = 4, 1, 4
    m.face_verts = m.positions = 16  # never dereferenced
    ws = ctypes.c_void_p(256)
    assert lib.subdiv_refine_vertex_data(ctypes.byref(m), ctypes.byref(info), ws, 0, ws, ws, 1, None) == \
        _lib.INVALID_ARG                                          # dim < 1
    assert lib.subdiv_refine_vertex_data(ctypes.byref(m), ctypes.byref(info), ws, 2, ws, ws, 1, None) == \
        _lib.STATE                                                # no kept state
    sel = _lib.subdiv_selection()
    assert lib.subdiv_select(ctypes.byref(m), ctypes.byref(info), None, 1, ws, 1, None, None) == _lib.INVALID_ARG
    assert lib.subdiv_select(ctypes.byref(m), ctypes.byref(info), None, 0, ws, 1, ctypes.byref(sel), None) == \
        _lib.INVALID_ARG                                          # rings < 1
    assert lib.subdiv_select(ctypes.byref(m), ctypes.byref(info), None, 1, ws, 1, ctypes.byref(sel), None) == \
        _lib.STATE                                                # not planned
    assert sel.num_vertices == 0
    ext = _lib.subdiv_extraction()
    assert lib.subdiv_extract(ctypes.byref(m), ctypes.byref(info), ctypes.byref(sel), None, ws, 1, None) == \
        _lib.INVALID_ARG
    assert lib.subdiv_extract(ctypes.byref(m), ctypes.byref(info), ctypes.byref(sel), ctypes.byref(ext), ws, 1,
                              None) == _lib.STATE
    assert lib.subdiv_backward(ctypes.byref(m), ctypes.byref(info), ws, ws, ws, 1, None) == _lib.STATE
    assert lib.subdiv_refine_positions(ctypes.byref(m), ctypes.byref(info), None, ws, 1, None) == _lib.INVALID_ARG


def test_creases_by_scheme_without_device(lib):
    """Creases: Catmull-Clark and Loop take them, sqrt(3) rejects them on the
    host, and batches take them for Catmull-Clark only (their workspace bound
    is 0 otherwise)."""
    info = _lib.subdiv_plan_info()
    m = _lib.subdiv_mesh()
    m.num_vertices, m.num_faces, m.face_order = 3, 1, 3
    m.face_verts = m.positions = 16  # never dereferenced: the crease check fails first
    m.num_creases = 1
    m.crease_verts = m.crease_sharpness = 16
    assert lib.subdiv_plan(ctypes.byref(m), 2, 1, 0, None, 0, ctypes.byref(info), None) == _lib.INVALID_ARG
    arr = (_lib.subdiv_mesh * 1)(m)
    assert lib.subdiv_batch_workspace_bound(arr, 1, 1, 1, 0) == 0      # Loop batch with creases
    assert lib.subdiv_batch_workspace_bound(arr, 1, 2, 1, 0) == 0      # sqrt(3) batch with creases
    m.num_creases = 0
    m.crease_verts = m.crease_sharpness = None
    arr = (_lib.subdiv_mesh * 1)(m)
    assert lib.subdiv_batch_workspace_bound(arr, 1, 1, 1, 0) > 0
    # the bound of a creased Loop cage covers the crease tables of every level
    assert lib.subdiv_workspace_bound(3, 1, 3, 1, 1, 3, 0) > lib.subdiv_workspace_bound(3, 1, 3, 0, 1, 3, 0)
