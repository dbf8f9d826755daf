"""Seeded synthetic input meshes.

This module only builds inputs: control cages (face tables, positions, crease
tags) and request traces. It holds none of the refinement arithmetic and is
shared, read-only, by the FP64 oracle tests, the GPU tests and the benchmark.

Every generator is deterministic given ``seed`` (``numpy.random.default_rng``).
Jitter is i.i.d. Gaussian per coordinate with the given *standard deviation*.
Positions are rounded to float32 once, here, so that both the GPU path and the
oracle see bit-identical inputs.

Meshes use the layout of the paper's mesh matrix M (Sec. 3.2): one column per
face, row indices = the face's vertices in counter-clockwise cyclic order.
``offsets`` is the CSC column pointer (``None`` when every face has the same
order, the reduced form of Sec. 4.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Mesh:
    """A polygon cage in mesh-matrix (CSC) form."""
    positions: np.ndarray                 # (V, 3) float32
    verts: np.ndarray                     # (H,) int32, row indices of M
    offsets: Optional[np.ndarray] = None  # (F+1,) int32 column pointer, or None
    face_order: int = 0                   # uniform order when offsets is None
    crease_verts: Optional[np.ndarray] = None   # (C, 2) int32
    crease_sharp: Optional[np.ndarray] = None   # (C,) float32
    name: str = ""

    @property
    def num_vertices(self) -> int:
        return int(self.positions.shape[0])

    @property
    def num_faces(self) -> int:
        if self.offsets is not None:
            return int(self.offsets.shape[0] - 1)
        return int(self.verts.shape[0] // self.face_order)

    @property
    def num_halfedges(self) -> int:
        return int(self.verts.shape[0])

    @property
    def num_creases(self) -> int:
        return 0 if self.crease_verts is None else int(self.crease_verts.shape[0])

    def face_list(self):
        """Faces as a list of int lists (small meshes / tests only)."""
        if self.offsets is None:
            return self.verts.reshape(-1, self.face_order).tolist()
        o = self.offsets
        return [self.verts[o[i]:o[i + 1]].tolist() for i in range(len(o) - 1)]

    def general(self) -> "Mesh":
        """Same mesh with an explicit column pointer."""
        if self.offsets is not None:
            return self
        F = self.num_faces
        off = (np.arange(F + 1, dtype=np.int64) * self.face_order).astype(np.int32)
        return dataclasses.replace(self, offsets=off, face_order=0)


# --------------------------------------------------------------------------
# small helpers
# --------------------------------------------------------------------------

def _undirected_edges(faces: np.ndarray) -> np.ndarray:
    """Unique undirected edges (lo, hi) of a uniform face table, sorted."""
    c = faces.shape[1]
    a = faces.reshape(-1)
    b = np.roll(faces, -1, axis=1).reshape(-1)
    pairs = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)
    return np.unique(pairs, axis=0)


def _jitter(P: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    return (P + rng.normal(0.0, sigma, size=P.shape)).astype(np.float32)


def _orient_outward(P: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """Flip faces of a star-shaped closed surface so normals point away from 0."""
    a, b, c = (P[faces[:, i]] for i in range(3))
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a + b + c) < 0
    out = faces.copy()
    out[flip] = out[flip][:, ::-1]
    return out


# --------------------------------------------------------------------------
# base shapes
# --------------------------------------------------------------------------

def torus(n_major: int = 16, n_minor: int = 16, R: float = 1.0, r: float = 0.3):
    """Regular quad torus. Vertex (i, j) has index n_minor*i + j, at
    ((R + r cos phi_j) cos th_i, (R + r cos phi_j) sin th_i, r sin phi_j).
    Quad (i,j),(i+1,j),(i+1,j+1),(i,j+1) (indices mod n) has an outward normal.
    Returns (P float64 (V,3), faces int32 (F,4))."""
    i = np.arange(n_major)[:, None]
    j = np.arange(n_minor)[None, :]
    th = 2.0 * np.pi * i / n_major
    ph = 2.0 * np.pi * j / n_minor
    x = (R + r * np.cos(ph)) * np.cos(th)
    y = (R + r * np.cos(ph)) * np.sin(th)
    z = np.broadcast_to(r * np.sin(ph), x.shape)
    P = np.stack([x, y, z], axis=-1).reshape(-1, 3)

    def vid(a, b):
        return (a % n_major) * n_minor + (b % n_minor)

    ii, jj = np.meshgrid(np.arange(n_major), np.arange(n_minor), indexing="ij")
    ii, jj = ii.reshape(-1), jj.reshape(-1)
    faces = np.stack([vid(ii, jj), vid(ii + 1, jj), vid(ii + 1, jj + 1), vid(ii, jj + 1)], axis=1)
    return P, faces.astype(np.int32)


def icosahedron():
    """Unit icosahedron, 12 vertices / 20 outward-oriented triangles."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    P = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    return P, _orient_outward(P, F)


def icosphere(level: int):
    """Icosahedron followed by `level` 4-way midpoint splits, every new vertex
    projected to the unit sphere. level 5: V=10,242 F=20,480; level 6:
    V=40,962 F=81,920."""
    P, F = icosahedron()
    for _ in range(level):
        V = P.shape[0]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        he = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 1)  # (F,3,2)
        key = np.sort(he, axis=2).reshape(-1, 2)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        inv = inv.reshape(-1, 3)
        mid = P[uniq[:, 0]] + P[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        mab, mbc, mca = V + inv[:, 0], V + inv[:, 1], V + inv[:, 2]
        F = np.concatenate([np.stack([a, mab, mca], 1), np.stack([b, mbc, mab], 1),
                            np.stack([c, mca, mbc], 1), np.stack([mab, mbc, mca], 1)], 0).astype(np.int32)
        P = np.concatenate([P, mid], 0)
    return P, F


def geodesic_sphere(freq: int):
    """Class-I geodesic sphere: each icosahedron face split into freq^2
    triangles on a barycentric grid, vertices projected to the unit sphere.
    F = 20 freq^2, V = 10 freq^2 + 2. freq = 2^L reproduces icosphere(L)'s counts.

    A grid point of face (A, B, C) at (i, j) has integer weights (n-i-j, i, j)
    on those corners; points with equal weights on the 12 corners are one
    vertex, numbered in order of first appearance (faces in order, i outer,
    j inner). Its position is the weighted sum of its corners in ascending
    corner order, normalised."""
    P0, F0 = icosahedron()
    n = int(freq)
    if n < 1:
        raise ValueError("freq must be >= 1")
    I, J = np.array([(i, j) for i in range(n + 1) for j in range(n + 1 - i)], dtype=np.int64).T
    lp = np.full((n + 2, n + 2), -1, np.int64)
    lp[I, J] = np.arange(I.size)
    nf, npt = F0.shape[0], I.size
    W = np.zeros((nf, npt, 12), np.int64)
    for f in range(nf):
        A, B, C = (int(x) for x in F0[f])
        W[f, :, A] += n - I - J
        W[f, :, B] += I
        W[f, :, C] += J
    uniq, first, inv = np.unique(W.reshape(-1, 12), axis=0, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    ids = rank[inv.reshape(-1)].reshape(nf, npt)
    w = uniq[order]
    corner = np.argsort(w == 0, axis=1, kind="stable")[:, :3]  # nonzero corners first, ascending
    rows = np.arange(w.shape[0])
    p = np.zeros((w.shape[0], 3))
    for k in range(3):
        c = corner[:, k]
        wk = w[rows, c]
        p = np.where((wk > 0)[:, None], p + P0[c] * (wk / n)[:, None], p)
    P = np.empty_like(p)
    for r in range(p.shape[0]):
        P[r] = p[r] / np.linalg.norm(p[r])
    loc = []
    for i in range(n):
        for j in range(n - i):
            loc.append((lp[i, j], lp[i + 1, j], lp[i, j + 1]))
            if i + j + 1 < n:
                loc.append((lp[i + 1, j], lp[i + 1, j + 1], lp[i, j + 1]))
    F = ids[:, np.array(loc, np.int64)].reshape(-1, 3).astype(np.int32)
    return P, _orient_outward(P, F)


# --------------------------------------------------------------------------
# cage modifiers
# --------------------------------------------------------------------------

def merge_pairs(faces: np.ndarray, n_merges: int, rng: np.random.Generator):
    """Merge `n_merges` pairs of edge-adjacent triangles into quads.

    Edges are visited in a seeded random permutation of the sorted edge list;
    an edge is merged when both of its triangles are still unmerged. The quad
    replaces the lower-indexed triangle in face order, the other triangle is
    dropped. Triangle (a,b,c) + triangle (b,a,d) -> quad (a,d,b,c), which keeps
    counter-clockwise order. Returns (offsets, verts) in CSC form."""
    F = faces.shape[0]
    nv = int(faces.max()) + 1
    a = faces.reshape(-1).astype(np.int64)
    b = np.roll(faces, -1, axis=1).reshape(-1).astype(np.int64)
    key = a * nv + b                      # directed half-edge a -> b at slot 3f + s
    srt = np.argsort(key)
    edges = _undirected_edges(faces)
    order = rng.permutation(edges.shape[0])
    lo, hi = edges[:, 0].astype(np.int64), edges[:, 1].astype(np.int64)
    h1 = srt[np.searchsorted(key[srt], lo * nv + hi)]  # lo -> hi
    h2 = srt[np.searchsorted(key[srt], hi * nv + lo)]  # hi -> lo
    merged = np.zeros(F, dtype=bool)
    dropped = np.zeros(F, dtype=bool)
    rowsv = np.concatenate([faces, np.full((F, 1), -1, np.int32)], 1)
    done = 0
    for ei in order:
        if done >= n_merges:
            break
        f1, f2 = h1[ei] // 3, h2[ei] // 3
        if merged[f1] or merged[f2]:
            continue
        # f1 holds lo->hi at slot s1: (a=lo, b=hi, c); f2 holds hi->lo: (b, a, d)
        c = faces[f1, (h1[ei] % 3 + 2) % 3]
        d = faces[f2, (h2[ei] % 3 + 2) % 3]
        keep, drop = (f1, f2) if f1 < f2 else (f2, f1)
        rowsv[keep] = (lo[ei], d, hi[ei], c)
        dropped[drop] = True
        merged[f1] = merged[f2] = True
        done += 1
    if done != n_merges:
        raise RuntimeError(f"only {done} of {n_merges} merges possible")
    kept = rowsv[~dropped]
    offsets = np.concatenate([[0], np.cumsum((kept >= 0).sum(1))]).astype(np.int32)
    return offsets, kept[kept >= 0].astype(np.int32)


def cut_holes(faces: np.ndarray, n_remove: int, rng: np.random.Generator) -> np.ndarray:
    """Remove `n_remove` faces chosen by seeded rejection sampling so that no
    two removed faces share a vertex: every hole is one triangle and every
    boundary vertex stays manifold. Returns the remaining faces in order."""
    F = faces.shape[0]
    used = np.zeros(int(faces.max()) + 1, dtype=bool)
    removed = np.zeros(F, dtype=bool)
    count = 0
    for f in rng.permutation(F):
        if count >= n_remove:
            break
        if used[faces[f]].any():
            continue
        used[faces[f]] = True
        removed[f] = True
        count += 1
    if count != n_remove:
        raise RuntimeError(f"only {count} of {n_remove} disjoint holes possible")
    return faces[~removed]


def mesh_edges(offsets: Optional[np.ndarray], verts: np.ndarray, face_order: int = 0) -> np.ndarray:
    """Sorted unique undirected edges (lo, hi) of a CSC face table."""
    if offsets is None:
        return _undirected_edges(verts.reshape(-1, face_order))
    off = offsets.astype(np.int64)
    counts = np.diff(off)
    face_of = np.repeat(np.arange(counts.size), counts)
    start = off[face_of]
    slot = np.arange(verts.size) - start
    nxt = start + (slot + 1) % counts[face_of]
    a, b = verts, verts[nxt]
    pairs = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)
    return np.unique(pairs, axis=0)


def tag_creases(offsets, verts, face_order, n_creases: int, smax: float, rng: np.random.Generator):
    """Tag `n_creases` distinct edges (seeded choice from the sorted edge list)
    with sharpness uniform in [0, smax), float32."""
    edges = mesh_edges(offsets, verts, face_order)
    pick = np.sort(rng.choice(edges.shape[0], size=n_creases, replace=False))
    cv = edges[pick].astype(np.int32)
    cs = rng.uniform(0.0, smax, size=n_creases).astype(np.float32)
    return cv, cs


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def torus_cage(seed: int = 1, n: int = 16, sigma: float = 0.01) -> Mesh:
    """16x16 quad torus (R=1, r=0.3), jitter N(0, sigma), no creases."""
    rng = np.random.default_rng(seed)
    P, F = torus(n, n, 1.0, 0.3)
    return Mesh(positions=_jitter(P, sigma, rng), verts=F.reshape(-1).astype(np.int32),
                offsets=None, face_order=4, name=f"torus{n}x{n}")


def cc_cage(seed: int = 2, level: int = 5, merge_frac: float = 0.30,
            crease_frac: float = 0.03, smax: float = 4.0, sigma: float = 0.01) -> Mesh:
    """Mixed triangle/quad cage: icosphere(level) with round(merge_frac*F/2)
    adjacent triangle pairs merged into quads, jitter N(0, sigma), and
    round(crease_frac*E) edges tagged with sharpness U[0, smax).
    level 5: 14,336 triangles + 3,072 quads, V=10,242, E=27,648, 829 creases."""
    rng = np.random.default_rng(seed)
    P, F = icosphere(level)
    n_merge = int(round(merge_frac * F.shape[0] / 2))
    off, verts = merge_pairs(F, n_merge, rng)
    Pj = _jitter(P, sigma, rng)
    E = mesh_edges(off, verts).shape[0]
    n_cr = int(round(crease_frac * E))
    cv, cs = (None, None)
    if n_cr > 0:
        cv, cs = tag_creases(off, verts, 0, n_cr, smax, rng)
    return Mesh(positions=Pj, verts=verts, offsets=off, crease_verts=cv, crease_sharp=cs,
                name=f"icosphere{level}_merged")


def tri_cage(seed: int = 3, level: int = 6, hole_frac: float = 0.02, sigma: float = 0.005) -> Mesh:
    """Triangle cage with boundaries: icosphere(level), floor(hole_frac*F)
    vertex-disjoint faces removed, jitter N(0, sigma).
    level 6: V=40,962, F=80,282, 4,914 boundary edges, Euler characteristic -1,636."""
    rng = np.random.default_rng(seed)
    P, F = icosphere(level)
    n_rm = int(math.floor(hole_frac * F.shape[0]))
    F = cut_holes(F, n_rm, rng) if n_rm > 0 else F
    return Mesh(positions=_jitter(P, sigma, rng), verts=F.reshape(-1).astype(np.int32),
                offsets=None, face_order=3, name=f"icosphere{level}_holes")


def geodesic_cage(target_faces: int, scheme: str, rng: np.random.Generator,
                  sigma: float = 0.01) -> Mesh:
    """Serving-request cage with about `target_faces` faces: geodesic sphere of
    frequency max(2, round(sqrt(T/20))). A Catmull-Clark cage gets 30% of its
    triangle pairs merged and 3% of its edges creased (sharpness U[0,4)); a
    Loop cage stays an uncreased triangle mesh."""
    freq = max(2, int(round(math.sqrt(target_faces / 20.0))))
    P, F = geodesic_sphere(freq)
    if scheme == "loop":
        return Mesh(positions=_jitter(P, sigma, rng), verts=F.reshape(-1).astype(np.int32),
                    offsets=None, face_order=3, name=f"geodesic{freq}")
    n_merge = int(round(0.30 * F.shape[0] / 2))
    off, verts = merge_pairs(F, n_merge, rng)
    Pj = _jitter(P, sigma, rng)
    E = mesh_edges(off, verts).shape[0]
    n_cr = int(round(0.03 * E))
    cv, cs = tag_creases(off, verts, 0, n_cr, 4.0, rng) if n_cr > 0 else (None, None)
    return Mesh(positions=Pj, verts=verts, offsets=off, crease_verts=cv, crease_sharp=cs,
                name=f"geodesic{freq}_merged")


# --------------------------------------------------------------------------
# tiny hand-built cages for pins
# --------------------------------------------------------------------------

def cube() -> Mesh:
    """Cube [-1,1]^3, 8 vertices, 6 outward quads."""
    P = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], dtype=np.float32)

    def v(x, y, z):
        return ((x > 0) << 2) | ((y > 0) << 1) | (z > 0)

    F = [[v(1, -1, -1), v(1, 1, -1), v(1, 1, 1), v(1, -1, 1)],      # +x
         [v(-1, -1, -1), v(-1, -1, 1), v(-1, 1, 1), v(-1, 1, -1)],  # -x
         [v(-1, 1, -1), v(-1, 1, 1), v(1, 1, 1), v(1, 1, -1)],      # +y
         [v(-1, -1, -1), v(1, -1, -1), v(1, -1, 1), v(-1, -1, 1)],  # -y
         [v(-1, -1, 1), v(1, -1, 1), v(1, 1, 1), v(-1, 1, 1)],      # +z
         [v(-1, -1, -1), v(-1, 1, -1), v(1, 1, -1), v(1, -1, -1)]]  # -z
    return Mesh(positions=P, verts=np.array(F, dtype=np.int32).reshape(-1), face_order=4, name="cube")


def tetrahedron() -> Mesh:
    """Regular tetrahedron with vertices (1,1,1),(1,-1,-1),(-1,1,-1),(-1,-1,1)."""
    P = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    F = _orient_outward(P, np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], dtype=np.int32))
    return Mesh(positions=P.astype(np.float32), verts=F.reshape(-1), face_order=3, name="tetrahedron")


def grid_patch(nx: int, ny: int, tri: bool = False, z_fn=None) -> Mesh:
    """Open planar (nx x ny) grid of quads (or split triangles) in [0,nx]x[0,ny],
    counter-clockwise seen from +z. Optional height function z_fn(x, y)."""
    xs, ys = np.meshgrid(np.arange(nx + 1, dtype=np.float64), np.arange(ny + 1, dtype=np.float64),
                         indexing="ij")
    z = np.zeros_like(xs) if z_fn is None else z_fn(xs, ys)
    P = np.stack([xs, ys, z], -1).reshape(-1, 3).astype(np.float32)

    def vid(i, j):
        return i * (ny + 1) + j

    faces = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if tri:
                faces += [[a, b, c], [a, c, d]]
            else:
                faces.append([a, b, c, d])
    F = np.array(faces, dtype=np.int32)
    return Mesh(positions=P, verts=F.reshape(-1), face_order=F.shape[1], name=f"grid{nx}x{ny}")


def poisson_trace(n_requests: int, qps: float, seed: int):
    """Serving trace: arrival times (s) from seeded exponential gaps, target
    face counts log-uniform in [100, 50k], scheme uniform over {cc, loop},
    levels uniform in 1..4."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    t = np.cumsum(gaps)
    faces = np.exp(rng.uniform(math.log(100.0), math.log(50_000.0), size=n_requests))
    scheme = np.where(rng.integers(0, 2, size=n_requests) == 0, "cc", "loop")
    levels = rng.integers(1, 5, size=n_requests)
    return t, faces, scheme, levels


_SERVING_BASES = {}


def serving_cage(target_faces: float, scheme: str, rng: np.random.Generator, sigma: float = 0.01) -> Mesh:
    """Request cage of the serving trace. The topology of frequency
    nu = max(2, round(sqrt(T/20))) -- the geodesic sphere and, for
    Catmull-Clark, its merged triangle pairs and tagged creases -- is drawn
    once per (nu, scheme) with the seed 1000 + nu and cached; each request
    jitters its own copy of the positions by N(0, sigma)."""
    freq = max(2, int(round(math.sqrt(float(target_faces) / 20.0))))
    key = (freq, scheme)
    base = _SERVING_BASES.get(key)
    if base is None:
        base = geodesic_cage(20 * freq * freq, scheme, np.random.default_rng(1000 + freq), sigma=0.0)
        _SERVING_BASES[key] = base
    return Mesh(positions=_jitter(base.positions, sigma, rng), verts=base.verts, offsets=base.offsets,
                face_order=base.face_order, crease_verts=base.crease_verts, crease_sharp=base.crease_sharp,
                name=base.name)
