"""Oracle of the mesh reordering of Sec. 4.5 (test infrastructure only).

The paper applies reverse Cuthill-McKee (Cuthill and McKee 1969, reversed
as George 1971) to the graph Laplacian of the mesh, i.e. to its vertex
graph, permutes the rows (vertices) of M with it, and sorts the columns
(faces) by their first non-zero entry. The paper does not fix the start
vertex or the order among equals; the reading taken here:
  * the start of every connected component is its unvisited vertex of
    smallest degree, the smaller id first;
  * a dequeued vertex appends its unvisited neighbours by increasing
    (degree, id);
  * the whole Cuthill-McKee sequence is reversed: new id of the vertex at
    position i is V - 1 - i;
  * a face's key is the smallest new id among its corners ("first non-zero"
    of its permuted column); faces are ordered by (key, old id);
  * a face keeps its corners in their cyclic order, starting at the same
    corner.
Degree = number of distinct neighbours over the faces' edges.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def neighbours(mesh):
    nb = [set() for _ in range(mesh.num_vertices)]
    for f in mesh.face_list():
        for j in range(len(f)):
            a, b = f[j], f[(j + 1) % len(f)]
            nb[a].add(b)
            nb[b].add(a)
    return nb


def rcm_order(mesh):
    """(vertex_perm, face_perm): new id -> old id, for vertices and faces."""
    nb = neighbours(mesh)
    V = mesh.num_vertices
    deg = np.array([len(s) for s in nb])
    seen = np.zeros(V, bool)
    seq = []
    by_degree = sorted(range(V), key=lambda v: (deg[v], v))
    for s in by_degree:
        if seen[s]:
            continue
        seen[s] = True
        q = deque([s])
        while q:
            v = q.popleft()
            seq.append(v)
            for w in sorted((w for w in nb[v] if not seen[w]), key=lambda w: (deg[w], w)):
                seen[w] = True
                q.append(w)
    vperm = np.array(seq[::-1], np.int32)
    newid = np.empty(V, np.int64)
    newid[vperm] = np.arange(V)
    faces = mesh.face_list()
    key = [min(newid[v] for v in f) for f in faces]
    fperm = np.array(sorted(range(len(faces)), key=lambda f: (key[f], f)), np.int32)
    return vperm, fperm


def bandwidth(mesh, vperm=None):
    """max |new(a) - new(b)| over the edges (the bandwidth of the Laplacian)."""
    V = mesh.num_vertices
    newid = np.arange(V) if vperm is None else np.empty(V, np.int64)
    if vperm is not None:
        newid[vperm] = np.arange(V)
    bw = 0
    for f in mesh.face_list():
        for j in range(len(f)):
            bw = max(bw, abs(int(newid[f[j]]) - int(newid[f[(j + 1) % len(f)]])))
    return bw
