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


def select(mesh, rings: int = 1, seed: Optional[np.ndarray] = None):
    """(x_rings, q_rings-1) as boolean vectors over the cage's vertices and faces."""
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
    return x > 0, q


def extract(mesh, rings: int = 1, seed: Optional[np.ndarray] = None) -> Extracted:
    """M' = X M X-ring and P' = X P for the selection of `select`."""
    xs, qs = select(mesh, rings, seed)
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
    P = np.asarray(mesh.positions, np.float32)[vsel]
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
