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
    assert lib.subdiv_version() == 1001
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
    one = (ctypes.c_int * 1)(1)
    loop, sqrt3 = (ctypes.c_int * 1)(1), (ctypes.c_int * 1)(2)
    assert lib.subdiv_batch_workspace_bound(arr, loop, one, 1, None, 0) == 0     # Loop batch with creases
    assert lib.subdiv_batch_workspace_bound(arr, sqrt3, one, 1, None, 0) == 0    # sqrt(3) batch with creases
    m.num_creases = 0
    m.crease_verts = m.crease_sharpness = None
    arr = (_lib.subdiv_mesh * 1)(m)
    assert lib.subdiv_batch_workspace_bound(arr, loop, one, 1, None, 0) > 0
    # the bound of a creased Loop cage covers the crease tables of every level
    assert lib.subdiv_workspace_bound(3, 1, 3, 1, 1, 3, 0) > lib.subdiv_workspace_bound(3, 1, 3, 0, 1, 3, 0)


def test_state_calls_need_a_refinement_in_that_workspace(lib):
    """A plan that keeps its state, but with no subdiv_refine enqueued into
    the workspace (the order plan, then backward / positions / vertex data):
    the library's host-side record of the workspace has no kept state, so
    every call that reads it returns SUBDIV_STATE before any device work
    (the never-written level tables would otherwise be read as indices).
    subdiv_state_destroy knows no state there either."""
    info = _lib.subdiv_plan_info()
    info.levels, info.scheme, info.flags = 2, 0, 2   # Catmull-Clark, SUBDIV_FLAG_KEEP_STATE
    info.priv_stamp = 1 << 60                        # looks planned; no such plan ever ran
    m = _lib.subdiv_mesh()
    m.num_vertices, m.num_faces, m.face_order = 4, 1, 4
    m.face_verts = m.positions = 16                  # never dereferenced
    info.priv_mesh_verts = 16
    ws = ctypes.c_void_p(1 << 20)
    info.priv_ws = ws.value
    outs = (_lib.subdiv_level_out * 3)()
    outs[2].positions = 16
    assert lib.subdiv_backward(ctypes.byref(m), ctypes.byref(info), ws, ws, ws, 1 << 30, None) == _lib.STATE
    assert lib.subdiv_refine_positions(ctypes.byref(m), ctypes.byref(info), outs, ws, 1 << 30, None) == _lib.STATE
    assert lib.subdiv_refine_vertex_data(ctypes.byref(m), ctypes.byref(info), ws, 3, ws, ws, 1 << 30, None) == \
        _lib.STATE
    sel = _lib.subdiv_selection()
    assert lib.subdiv_select(ctypes.byref(m), ctypes.byref(info), None, 1, ws, 1 << 30, ctypes.byref(sel),
                             None) == _lib.STATE
    assert lib.subdiv_state_destroy(ctypes.byref(info), ws) == _lib.STATE
    assert lib.subdiv_state_destroy(None, ws) == _lib.INVALID_ARG
    assert lib.subdiv_state_destroy(ctypes.byref(info), None) == _lib.INVALID_ARG


def test_batch_arguments_without_device(lib):
    """Per-mesh schemes and level counts: the host-only bound grows with
    either, rejects bad entries, and a mismatched member plan (never made,
    another cage) is refused before any device work."""
    tri = _lib.subdiv_mesh()
    tri.num_vertices, tri.num_faces, tri.face_order = 4, 4, 3
    tri.face_verts = tri.positions = 16
    quad = _lib.subdiv_mesh()
    quad.num_vertices, quad.num_faces, quad.face_order = 8, 6, 4
    quad.face_verts = quad.positions = 32
    arr = (_lib.subdiv_mesh * 3)(tri, quad, tri)
    sc = (ctypes.c_int * 3)(1, 0, 2)
    lv = (ctypes.c_int * 3)(2, 3, 1)
    b = lib.subdiv_batch_workspace_bound(arr, sc, lv, 3, None, 0)
    assert b > 0
    lv2 = (ctypes.c_int * 3)(2, 4, 1)
    assert lib.subdiv_batch_workspace_bound(arr, sc, lv2, 3, None, 0) > b
    bad = (ctypes.c_int * 3)(1, 0, 3)
    assert lib.subdiv_batch_workspace_bound(arr, bad, lv, 3, None, 0) == 0      # scheme out of range
    assert lib.subdiv_batch_workspace_bound(arr, sc, (ctypes.c_int * 3)(2, 0, 1), 3, None, 0) == 0   # 0 levels
    assert lib.subdiv_batch_workspace_bound(arr, sc, lv, 3, None, 4) == 0       # KEEP_STATE is not for batches
    plans = (_lib.subdiv_plan_info * 3)()
    assert lib.subdiv_batch_workspace_bound(arr, sc, lv, 3, plans, 0) == 0      # never planned
    outs = (_lib.subdiv_level_out * 3)()
    for o in outs:
        o.face_verts = o.positions = 64
    assert lib.subdiv_refine_batch(arr, sc, lv, 3, plans, outs, ctypes.c_void_p(1 << 20), 1 << 30, None) == \
        _lib.STATE
    for i, (m, s, l) in enumerate([(tri, 1, 2), (quad, 0, 3), (tri, 2, 1)]):
        p = plans[i]
        p.priv_stamp, p.priv_mesh_verts, p.scheme, p.levels = 1 << 61, m.face_verts, s, l
        p.level[0].num_vertices, p.level[0].num_faces = m.num_vertices, m.num_faces
        p.level[0].num_halfedges = m.num_faces * m.face_order
    plans[1].levels = 2                                                          # fewer levels than asked for
    assert lib.subdiv_refine_batch(arr, sc, lv, 3, plans, outs, ctypes.c_void_p(1 << 20), 1 << 30, None) == \
        _lib.STATE
    plans[1].levels = 3
    plans[2].priv_mesh_verts = 48                                                # another cage
    assert lib.subdiv_refine_batch(arr, sc, lv, 3, plans, outs, ctypes.c_void_p(1 << 20), 1 << 30, None) == \
        _lib.STATE
    plans[2].priv_mesh_verts = 16
    assert lib.subdiv_refine_batch(arr, sc, lv, 3, plans, outs, ctypes.c_void_p(1 << 20), 16, None) == \
        _lib.WORKSPACE


def test_tuning_table_host_calls(lib, tmp_path):
    """The launch-shape table: load, lookup by size bucket, single entries,
    malformed files rejected with the table unchanged (host-only calls)."""
    names = _lib.tuning_kernels()
    assert "lag2_group" in names and "loopl_face" in names and "bw_vertex" in names
    t = tmp_path / "t.json"
    t.write_text('{"device": "gfx950", "note": {"x": [1, 2.5, "y"]}, '
                 '"kernels": {"lag2_group": [[1000, 64], [100000, 128], [-1, 512]], "lag_edge": [[-1, 128]]}}')
    _lib.tuning_load(str(t))
    assert _lib.tuning_source() == str(t)
    assert _lib.tuning_block("lag2_group", 10) == 64
    assert _lib.tuning_block("lag2_group", 1000) == 64
    assert _lib.tuning_block("lag2_group", 1001) == 128
    assert _lib.tuning_block("lag2_group", 10 ** 9) == 512
    assert _lib.tuning_block("lag_edge", 5) == 128
    assert _lib.tuning_block("loop_face", 5) == 256  # no entry: the default
    bad = tmp_path / "bad.json"
    for text in ('{"kernels": {"lag2_group": [[10, 96]]}}',          # not a supported block
                 '{"kernels": {"nope": [[10, 64]]}}',                 # unknown kernel
                 '{"kernels": {"lag_edge": [[100, 64], [10, 128]]}}',  # unordered buckets
                 '{"kernels": {"lag_edge": [[100, 64]]'):             # truncated
        bad.write_text(text)
        with pytest.raises(_lib.SubdivError) as e:
            _lib.tuning_load(str(bad))
        assert e.value.status == _lib.INVALID_ARG
        assert _lib.tuning_block("lag2_group", 10) == 64  # unchanged
    _lib.tuning_set("loop_face", 128)
    _lib.tuning_set("loop_face", 512, max_items=100)
    assert _lib.tuning_block("loop_face", 50) == 512 and _lib.tuning_block("loop_face", 5000) == 128
    with pytest.raises(_lib.SubdivError):
        _lib.tuning_set("loop_face", 100)
    _lib.tuning_set("*", 64)
    assert all(_lib.tuning_block(n, 12345) == 64 for n in names)
    _lib.tuning_load(None)
    assert _lib.tuning_source() == "built-in"
    assert all(_lib.tuning_block(n, 12345) == 256 for n in names)
    default = os.path.join(ROOT, "paper_1809_06047_amd", "tuning_gfx950.json")
    _lib.tuning_load(default if os.path.exists(default) else None)


def test_kobbelt_scheme_host_checks(lib):
    """sqrt(3) with the boundary cycle (scheme 3): sizes bounded like the other
    schemes; batches and kept state refused without touching the device."""
    assert lib.subdiv_workspace_bound(162, 304, 912, 0, 3, 4, 0) > 0
    assert lib.subdiv_workspace_bound(162, 304, 912, 0, 4, 4, 0) == 0
    assert lib.subdiv_workspace_bound(162, 304, 912, 0, 3, 4, 0) >= lib.subdiv_workspace_bound(162, 304, 912, 0, 2, 4, 0)
