"""Oracle of selective subdivision's extraction step (test infrastructure
only, like the rest of this package).

Sec. 3.4 ("Selective and Feature Adaptive Subdivision") of the paper, written
with the mesh matrix M (rows = vertices, columns = faces, one non-zero per
face corner):
  * x_0 marks the selected vertices: by default the extraordinary ones, whose
    valence n = M 1 (eq:vo, the number of incident faces) is not four;
  * q_i = M^T x_i marks the faces with a selected corner, and
    x_{i+1} = M q_i the corners of those faces; after `rings` rounds
  * X keeps the rows of the identity at the vertices of x_rings and X-ring
    the columns at the faces of q_{rings-1}; the extracted cage is
    M' = X M X-ring with vertex data P' = X P.
Deleting rows and columns of the identity keeps the surviving vertices and
faces in their original order, so the extracted vertex of rank r is the r-th
selected vertex, and a face keeps its corners in their cyclic order. The
paper leaves the creases of the extracted cage implicit; the reading taken
here keeps every crease whose edge is an edge of an extracted face, with its
endpoints renumbered (the edge survives exactly when such a face does).

The products are scipy sparse products of the literal matrices, in FP64 over
0/1 entries (exact).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Extracted:
    offsets: np.ndarray        # (F'+1,) int32
    verts: np.ndarray          # (H',) int32, extracted vertex ids
    positions: np.ndarray      # (V', 3) float32, copied
    crease_verts: np.ndarray   # (C', 2) int32, extracted ids, sorted by (min, max)
    crease_sharp: np.ndarray   # (C',) float32
    vertex_map: np.ndarray     # (V',) cage vertex of each extracted vertex
    face_map: np.ndarray       # (F',) cage face of each extracted face


def mesh_matrix(mesh) -> sp.csc_matrix:
    """M: V x F, M[v, f] = 1 for every corner v of face f (Sec. 3.1)."""
    faces = mesh.face_list()
    rows = np.concatenate([np.asarray(f, np.int64) for f in faces]) if faces else np.zeros(0, np.int64)
    cols = np.repeat(np.arange(len(faces)), [len(f) for f in faces])
    return sp.csc_matrix((np.ones(rows.size), (rows, cols)), shape=(mesh.num_vertices, len(faces)))


def _pinched(faces, star, q, v) -> bool:
    """The selected faces around v form more than one fan: taking two selected
    faces of v as joined when they share an edge at v, they fall into more
    than one component."""
    sel = [f for f in star[v] if q[f]]
    if len(sel) < 2:
        return False
    edges_at_v = {}
    for f in sel:
        c = faces[f]
        i = c.index(v)
        for w in (c[(i + 1) % len(c)], c[i - 1]):
            edges_at_v.setdefault(w, []).append(f)
    parent = {f: f for f in sel}

    def root(f):
        while parent[f] != f:
            f = parent[f]
        return f
    for fs in edges_at_v.values():
        for g in fs[1:]:
            parent[root(g)] = root(fs[0])
    return len({root(f) for f in sel}) > 1


def close_pinches(mesh, x, q, max_passes: int = 16):
    """Pinch closing (a reading: the paper's extraction does not meet the case
    of two selected regions touching at one vertex, whose extraction would not
    be manifold there): every selected vertex whose selected faces form more
    than one fan gets its whole star selected, q <- q + faces of those stars
    and x <- M q, pass after pass, each pass reading the previous one's
    selection, until no such vertex is left."""
    faces = mesh.face_list()
    star = [[] for _ in range(mesh.num_vertices)]
    for f, c in enumerate(faces):
        for v in c:
            star[v].append(f)
    M = mesh_matrix(mesh)
    for _ in range(max_passes):
        pinch = [v for v in np.flatnonzero(x) if _pinched(faces, star, q, int(v))]
        if not pinch:
            return x, q
        q = q.copy()
        for v in pinch:
            q[star[v]] = True
        x = (M @ q.astype(np.float64)) > 0
    raise ValueError("selection still pinched after every pass")


def select(mesh, rings: int = 1, seed: Optional[np.ndarray] = None, close: bool = False):
    """(x_rings, q_rings-1) as boolean vectors over the cage's vertices and
    faces (with `close`, pinches closed afterwards)."""
    if rings < 1:
        raise ValueError("rings >= 1")
    M = mesh_matrix(mesh)
    if seed is None:
        valence = np.asarray(M @ np.ones(M.shape[1])).ravel()   # n = M 1
        x = (valence != 4).astype(np.float64)
    else:
        x = (np.asarray(seed) != 0).astype(np.float64)
    q = None
    for _ in range(rings):
        q = (M.T @ x) > 0                      # q_i = M^T x_i
        x = (M @ q.astype(np.float64)) > 0     # x_{i+1} = M q_i
        x = x.astype(np.float64)
    if close:
        return close_pinches(mesh, x > 0, q)
    return x > 0, q


def extract(mesh, rings: int = 1, seed: Optional[np.ndarray] = None, dtype=np.float32,
            close: bool = False) -> Extracted:
    """M' = X M X-ring and P' = X P for the selection of `select` (positions
    copied in `dtype`; with `close`, pinches closed)."""
    xs, qs = select(mesh, rings, seed, close)
    vsel = np.flatnonzero(xs).astype(np.int32)
    fsel = np.flatnonzero(qs).astype(np.int32)
    newid = np.full(mesh.num_vertices, -1, np.int64)
    newid[vsel] = np.arange(vsel.size)
    faces = mesh.face_list()
    kept = [[int(newid[v]) for v in faces[f]] for f in fsel]
    assert all(v >= 0 for f in kept for v in f), "every corner of a selected face is selected"
    sizes = np.array([len(f) for f in kept], np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    verts = np.array([v for f in kept for v in f], np.int32)
    P = np.asarray(mesh.positions, dtype)[vsel]
    # creases on edges of the extracted faces
    edges = set()
    for f in kept:
        for j in range(len(f)):
            a, b = f[j], f[(j + 1) % len(f)]
            edges.add((min(a, b), max(a, b)))
    cv, cs = [], []
    if mesh.crease_verts is not None:
        for (a, b), s in zip(np.asarray(mesh.crease_verts), np.asarray(mesh.crease_sharp, np.float32)):
            na, nb = int(newid[a]), int(newid[b])
            if na >= 0 and nb >= 0 and (min(na, nb), max(na, nb)) in edges and s > 0:
                cv.append((min(na, nb), max(na, nb)))
                cs.append(s)
    order = sorted(range(len(cv)), key=lambda i: cv[i])
    crease_verts = np.array([cv[i] for i in order], np.int32).reshape(-1, 2)
    crease_sharp = np.array([cs[i] for i in order], np.float32)
    return Extracted(offsets=offsets, verts=verts, positions=P, crease_verts=crease_verts,
                     crease_sharp=crease_sharp, vertex_map=vsel, face_map=fsel)


class _Region:
    """A level's mesh for the selection: faces, FP64 positions, no creases."""

    def __init__(self, offsets, verts, positions):
        self.offsets = np.asarray(offsets, np.int64)
        self.verts = np.asarray(verts, np.int64)
        self.positions = np.asarray(positions, np.float64)
        self.num_vertices = self.positions.shape[0]
        self.crease_verts = None
        self.crease_sharp = None

    def face_list(self):
        o = self.offsets
        return [self.verts[o[i]:o[i + 1]].tolist() for i in range(len(o) - 1)]


@dataclasses.dataclass
class AdaptiveLevel:
    region: Extracted          # the extraction of level k (maps into level k's mesh), FP64 positions
    refined: object            # the region refined one Catmull-Clark level (an oracle Level)
    seed: np.ndarray           # (V_{k+1},) seed flags of the refined region's vertices


def adaptive(mesh, levels: int, rings: int = 1, seed: Optional[np.ndarray] = None):
    """Feature-adaptive refinement, Sec. 3.4 applied level after level: select
    and extract the region `rings` rings around the seeds, refine only the
    region one Catmull-Clark level (the oracle's step, FP64 throughout), and
    carry the seeds - the cage's extraordinary vertices unless given - to the
    refined region, where the extracted vertices keep their ids and the new
    points are not seeds. Every selection closes its pinches (see
    close_pinches). Stops early when a selection is empty."""
    from . import CATMULL_CLARK, Level, level_from_mesh, step
    lv0 = level_from_mesh(mesh)
    cur = _Region(lv0.offsets, lv0.verts, lv0.positions)
    if seed is None:
        M = mesh_matrix(cur)
        seed = (np.asarray(M @ np.ones(M.shape[1])).ravel() != 4).astype(np.uint8)
    out = []
    for _ in range(int(levels)):
        e = extract(cur, rings, seed, dtype=np.float64, close=True)
        if e.vertex_map.size == 0:
            break
        lv = step(Level(offsets=e.offsets, verts=e.verts, positions=e.positions,
                        crease_verts=np.zeros((0, 2), np.int32), crease_sharp=np.zeros(0)), CATMULL_CLARK)
        nseed = np.zeros(lv.num_vertices, np.uint8)
        nseed[:e.vertex_map.size] = np.asarray(seed)[e.vertex_map]
        out.append(AdaptiveLevel(region=e, refined=lv, seed=nseed))
        cur = _Region(lv.offsets, lv.verts, lv.positions)
        seed = nseed
    return out
