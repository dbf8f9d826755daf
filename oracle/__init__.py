"""FP64 serial CPU oracle for AlSub refinement (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package. The product library never does: it shares no
code with the oracle and fails loudly when its own HIP build is missing.

The arithmetic lives in ``oracle.cpp`` (C++17, compiled with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes
and loops over levels. See the header of ``oracle.cpp`` for the paper
sections each rule follows and for the readings taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

CATMULL_CLARK, LOOP, SQRT3 = 0, 1, 2
# sqrt(3) with Kobbelt's two-step boundary cycle: the sqrt(3) step (fixed
# boundary) from even levels, the trisection step (code 3) from odd ones
SQRT3_KOBBELT = 3
TRISECT_STEP = 3
SCHEMES = {"cc": CATMULL_CLARK, "loop": LOOP, "sqrt3": SQRT3, "sqrt3k": SQRT3_KOBBELT}


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (serial, FP64, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp, ip, dp, lp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), \
            ctypes.POINTER(ctypes.c_int64)
        lib.oracle_step.restype = vp
        lib.oracle_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, dp, ctypes.c_int, ip, dp,
                                    ctypes.c_int, ip]
        lib.oracle_counts.argtypes = [vp, lp]
        lib.oracle_mesh.argtypes = [vp, ip, ip, dp]
        lib.oracle_edges.argtypes = [vp, ip]
        lib.oracle_creases.argtypes = [vp, ip, dp]
        lib.oracle_R.argtypes = [vp, lp, ip, dp]
        lib.oracle_free.argtypes = [vp]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None and a.size else None


@dataclasses.dataclass
class Level:
    """One level of a refinement: a polygon mesh with FP64 positions."""
    offsets: np.ndarray          # (F+1,) int32
    verts: np.ndarray            # (H,) int32
    positions: np.ndarray        # (V, 3) float64
    crease_verts: np.ndarray     # (C, 2) int32, rows (lo, hi) sorted by (hi, lo)
    crease_sharp: np.ndarray     # (C,) float64
    edges: Optional[np.ndarray] = None   # (E, 2) (lo, hi) of THIS level in edge-id order
    n_boundary: int = 0                  # boundary edges of THIS level
    R: object = None                     # scipy CSR R_k mapping this level's parent to it

    @property
    def num_vertices(self):
        return int(self.positions.shape[0])

    @property
    def num_faces(self):
        return int(self.offsets.shape[0] - 1)

    def face_table(self, order: int) -> np.ndarray:
        return self.verts.reshape(-1, order)


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle rejected the mesh, status {status}")
        self.status = status


def level_from_mesh(mesh) -> Level:
    """FP64 copy of a float32 cage (the same rounded inputs the GPU sees)."""
    m = mesh.general()
    cv = np.zeros((0, 2), np.int32) if m.crease_verts is None else np.asarray(m.crease_verts, np.int32)
    cs = np.zeros((0,), np.float64) if m.crease_sharp is None else np.asarray(m.crease_sharp, np.float32).astype(
        np.float64)
    return Level(offsets=np.asarray(m.offsets, np.int32), verts=np.asarray(m.verts, np.int32),
                 positions=np.asarray(m.positions, np.float32).astype(np.float64), crease_verts=cv,
                 crease_sharp=cs)


def step(lvl: Level, scheme: int, want_R: bool = False) -> Level:
    """One refinement step; also fills lvl.edges / lvl.n_boundary (the input
    level's edge enumeration) as a side result."""
    lib = _load()
    off = np.ascontiguousarray(lvl.offsets, np.int32)
    fv = np.ascontiguousarray(lvl.verts, np.int32)
    P = np.ascontiguousarray(lvl.positions, np.float64)
    cv = np.ascontiguousarray(lvl.crease_verts, np.int32).reshape(-1)
    cs = np.ascontiguousarray(lvl.crease_sharp, np.float64)
    status = ctypes.c_int(0)
    h = lib.oracle_step(int(scheme), int(P.shape[0]), int(off.shape[0] - 1), _ptr(off, ctypes.c_int),
                        _ptr(fv, ctypes.c_int), _ptr(P, ctypes.c_double), int(cs.shape[0]), _ptr(cv, ctypes.c_int),
                        _ptr(cs, ctypes.c_double), int(bool(want_R)), ctypes.byref(status))
    try:
        if status.value != 0:
            raise OracleError(status.value)
        c = np.zeros(7, np.int64)
        lib.oracle_counts(h, _ptr(c, ctypes.c_int64))
        V, F, H, C, E, NB, NNZ = (int(x) for x in c)
        o_off = np.empty(F + 1, np.int32)
        o_fv = np.empty(H, np.int32)
        o_P = np.empty((V, 3), np.float64)
        lib.oracle_mesh(h, _ptr(o_off, ctypes.c_int), _ptr(o_fv, ctypes.c_int), _ptr(o_P, ctypes.c_double))
        edges = np.empty((E, 2), np.int32)
        lib.oracle_edges(h, _ptr(edges, ctypes.c_int))
        o_cv = np.empty((C, 2), np.int32)
        o_cs = np.empty(C, np.float64)
        if C:
            lib.oracle_creases(h, _ptr(o_cv, ctypes.c_int), _ptr(o_cs, ctypes.c_double))
        R = None
        if want_R:
            import scipy.sparse as sp
            ptr = np.empty(V + 1, np.int64)
            col = np.empty(NNZ, np.int32)
            val = np.empty(NNZ, np.float64)
            lib.oracle_R(h, _ptr(ptr, ctypes.c_int64), _ptr(col, ctypes.c_int), _ptr(val, ctypes.c_double))
            R = sp.csr_matrix((val, col, ptr), shape=(V, lvl.num_vertices))
    finally:
        lib.oracle_free(h)
    lvl.edges = edges
    lvl.n_boundary = NB
    return Level(offsets=o_off, verts=o_fv, positions=o_P, crease_verts=o_cv, crease_sharp=o_cs, R=R)


def refine(mesh, scheme, levels: int, want_R: bool = False) -> List[Level]:
    """Levels 0..levels of the refinement of a float32 cage (level 0 = the
    cage in FP64). scheme: 0/1/2/3 or 'cc'/'loop'/'sqrt3'/'sqrt3k' (sqrt(3)
    with Kobbelt's boundary cycle: levels 1, 3, ... by the sqrt(3) step,
    levels 2, 4, ... by the trisection step)."""
    s = SCHEMES.get(scheme, scheme)
    out = [level_from_mesh(mesh) if not isinstance(mesh, Level) else mesh]
    for k in range(levels):
        sk = s if s != SQRT3_KOBBELT else (SQRT3 if k % 2 == 0 else TRISECT_STEP)
        out.append(step(out[-1], sk, want_R))
    return out


def status_of(mesh, scheme) -> int:
    """Status the oracle reports for one step of `mesh` (0 = accepted)."""
    try:
        step(level_from_mesh(mesh), SCHEMES.get(scheme, scheme))
        return 0
    except OracleError as e:
        return e.status
