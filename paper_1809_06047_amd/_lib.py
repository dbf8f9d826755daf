"""ctypes view of the C ABI in include/subdiv.h (argument marshalling only).

Loading fails loudly when libsubdiv.so has not been built: there is no CPU
fallback anywhere in the product path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsubdiv.so")

CATMULL_CLARK, LOOP, SQRT3, SQRT3_KOBBELT = 0, 1, 2, 3
SCHEMES = {"cc": CATMULL_CLARK, "catmull-clark": CATMULL_CLARK, "loop": LOOP, "sqrt3": SQRT3,
           "sqrt3k": SQRT3_KOBBELT}

STATIC_WORKSPACE_BYTES = 64 << 20  # SUBDIV_STATIC_WORKSPACE_BYTES
OK, INVALID_ARG, SCHEME_MESH, NONMANIFOLD, DEGENERATE, BAD_CREASE, WORKSPACE, HIP, STATE = 0, -1, -2, -3, -4, -5, \
    -6, -7, -8
MAX_LEVELS = 10
MAX_VALENCE = 1024
FLAG_REBUILD_EACH_LEVEL = 1
SELECT_CLOSE_PINCHES = 1
FLAG_KEEP_STATE = 2

c_i32, c_i64, c_u32, c_u64, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, \
    ctypes.c_void_p, ctypes.c_size_t


class subdiv_mesh(ctypes.Structure):
    _fields_ = [("num_vertices", c_i32), ("num_faces", c_i32), ("face_order", c_i32), ("num_halfedges", c_i32),
                ("face_offsets", c_vp), ("face_verts", c_vp), ("positions", c_vp), ("num_creases", c_i32),
                ("crease_verts", c_vp), ("crease_sharpness", c_vp)]


class subdiv_level_info(ctypes.Structure):
    _fields_ = [("num_vertices", c_i64), ("num_edges", c_i64), ("num_faces", c_i64), ("num_halfedges", c_i64),
                ("num_boundary_edges", c_i64), ("face_order", c_i32), ("max_creases", c_i32)]


class subdiv_plan_info(ctypes.Structure):
    _fields_ = [("scheme", c_i32), ("levels", c_i32), ("flags", c_u32), ("max_valence", c_i32),
                ("max_sharpness", ctypes.c_float), ("reserved0", c_i32),
                ("level", subdiv_level_info * (MAX_LEVELS + 1)), ("workspace_bytes", c_sz),
                ("priv_mesh_verts", c_vp), ("priv_ws", c_vp), ("priv_stamp", c_u64)]


class subdiv_level_out(ctypes.Structure):
    _fields_ = [("face_verts", c_vp), ("positions", c_vp), ("edge_verts", c_vp), ("crease_sharpness", c_vp)]


class subdiv_stage_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("level", c_i32), ("launches", c_i32), ("total_ms", ctypes.c_double)]


class subdiv_selection(ctypes.Structure):
    _fields_ = [("num_vertices", c_i32), ("num_faces", c_i32), ("num_halfedges", c_i32), ("num_creases", c_i32),
                ("face_order", c_i32), ("rings", c_i32), ("flags", c_u32), ("priv_stamp", c_u64), ("priv_ws", c_vp)]


class subdiv_extraction(ctypes.Structure):
    _fields_ = [("face_offsets", c_vp), ("face_verts", c_vp), ("positions", c_vp), ("crease_verts", c_vp),
                ("crease_sharpness", c_vp), ("vertex_map", c_vp), ("face_map", c_vp), ("seed_flags", c_vp)]


class subdiv_kernel_time(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_char * 24), ("kernel", ctypes.c_char * 24), ("level", c_i32), ("block", c_i32),
                ("items", c_i64), ("launches", c_i32), ("reserved0", c_i32), ("total_ms", ctypes.c_double)]


# every function the header declares, with its signature
SIGNATURES = {
    "subdiv_workspace_bound": (c_sz, [c_i32, c_i32, c_i64, c_i32, ctypes.c_int, ctypes.c_int, c_u32]),
    "subdiv_plan": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.c_int, ctypes.c_int, c_u32, c_vp, c_sz,
                                   ctypes.POINTER(subdiv_plan_info), c_vp]),
    "subdiv_refine": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info),
                                     ctypes.POINTER(subdiv_level_out), c_vp, c_sz, c_vp]),
    "subdiv_refine_static": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info),
                                            ctypes.POINTER(subdiv_level_out), c_vp]),
    "subdiv_refine_positions": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info),
                                               ctypes.POINTER(subdiv_level_out), c_vp, c_sz, c_vp]),
    "subdiv_refine_vertex_data": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info),
                                                 c_vp, ctypes.c_int, c_vp, c_vp, c_sz, c_vp]),
    "subdiv_backward": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info), c_vp, c_vp,
                                       c_vp, c_sz, c_vp]),
    "subdiv_rcm_order": (ctypes.c_int, [c_i32, c_i32, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "subdiv_select": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info), c_vp, ctypes.c_int,
                                     c_vp, c_sz, ctypes.POINTER(subdiv_selection), c_vp]),
    "subdiv_select_ex": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info), c_vp,
                                        ctypes.c_int, c_u32, c_vp, c_sz, ctypes.POINTER(subdiv_selection), c_vp]),
    "subdiv_extract": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(subdiv_plan_info),
                                      ctypes.POINTER(subdiv_selection), ctypes.POINTER(subdiv_extraction), c_vp, c_sz,
                                      c_vp]),
    "subdiv_batch_workspace_bound": (c_sz, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                             ctypes.POINTER(subdiv_plan_info), c_u32]),
    "subdiv_plan_batch": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), ctypes.c_int, c_u32, c_vp, c_sz,
                                         ctypes.POINTER(subdiv_plan_info), c_vp]),
    "subdiv_refine_batch": (ctypes.c_int, [ctypes.POINTER(subdiv_mesh), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                           ctypes.POINTER(subdiv_plan_info), ctypes.POINTER(subdiv_level_out), c_vp,
                                           c_sz, c_vp]),
    "subdiv_state_destroy": (ctypes.c_int, [ctypes.POINTER(subdiv_plan_info), c_vp]),
    "subdiv_timing_enable": (None, [ctypes.c_int]),
    "subdiv_timing_select": (None, [ctypes.c_char_p, ctypes.c_int]),
    "subdiv_timing_read": (ctypes.c_int, [ctypes.POINTER(subdiv_stage_time), ctypes.c_int]),
    "subdiv_timing_read_kernels": (ctypes.c_int, [ctypes.POINTER(subdiv_kernel_time), ctypes.c_int]),
    "subdiv_tuning_load": (ctypes.c_int, [ctypes.c_char_p]),
    "subdiv_tuning_set": (ctypes.c_int, [ctypes.c_char_p, c_i64, ctypes.c_int]),
    "subdiv_tuning_block": (ctypes.c_int, [ctypes.c_char_p, c_i64]),
    "subdiv_tuning_source": (ctypes.c_char_p, []),
    "subdiv_tuning_kernel_name": (ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, ctypes.c_int]),
    "subdiv_last_error": (ctypes.c_char_p, []),
    "subdiv_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "subdiv_version": (ctypes.c_int, []),
}

_lib = None


def load():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_06047_amd.build` "
                              "(there is no fallback path)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SubdivError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        lib = load()
        msg = lib.subdiv_strerror(status).decode()
        if status in (HIP, WORKSPACE, INVALID_ARG) and lib.subdiv_last_error():
            msg += ": " + lib.subdiv_last_error().decode()
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


def timing_enable(on: bool = True):
    load().subdiv_timing_enable(1 if on else 0)


def timing_select(stage=None, level: int = -1):
    """Time only `stage` at `level` (-1: every level); None times every stage."""
    load().subdiv_timing_select(stage.encode() if stage else None, int(level))


def timing_read(max_out: int = 512):
    """{(stage, level): (launches, total_ms)} recorded since the last read."""
    buf = (subdiv_stage_time * max_out)()
    n = load().subdiv_timing_read(buf, max_out)
    if n < 0:
        raise SubdivError(n, "subdiv_timing_read")
    return {(buf[i].name.decode(), buf[i].level): (buf[i].launches, buf[i].total_ms) for i in range(n)}


def timing_read_kernels(max_out: int = 1024):
    """[(stage, level, kernel, items, block, launches, total_ms)] recorded since the last read."""
    buf = (subdiv_kernel_time * max_out)()
    n = load().subdiv_timing_read_kernels(buf, max_out)
    if n < 0:
        raise SubdivError(n, "subdiv_timing_read_kernels")
    return [(buf[i].stage.decode(), buf[i].level, buf[i].kernel.decode(), buf[i].items, buf[i].block,
             buf[i].launches, buf[i].total_ms) for i in range(n)]


def tuning_kernels():
    """Names of the tunable kernels."""
    out, i = [], 0
    buf = ctypes.create_string_buffer(32)
    while load().subdiv_tuning_kernel_name(i, buf, 32) == OK:
        out.append(buf.value.decode())
        i += 1
    return out


def tuning_load(path=None):
    check(load().subdiv_tuning_load(path.encode() if path else None), "subdiv_tuning_load")


def tuning_set(kernel: str, block: int, max_items: int = -1):
    check(load().subdiv_tuning_set(kernel.encode(), int(max_items), int(block)), "subdiv_tuning_set")


def tuning_block(kernel: str, items: int) -> int:
    b = load().subdiv_tuning_block(kernel.encode(), int(items))
    if b < 0:
        raise SubdivError(b, "subdiv_tuning_block")
    return b


def tuning_source() -> str:
    return load().subdiv_tuning_source().decode()


def check(status: int, where: str):
    if status != OK:
        raise SubdivError(status, where)
