"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each check is a closed form, a
hand-worked value, an identity with an independent textbook construction
(tensor-product cubic B-splines, limit-point eigenvectors), a printed count
from the paper's tables, or a structural invariant. Each is chosen so that a
plausible slip in the oracle (a dropped term, a wrong weight, a swapped index,
a wrong edge order) makes at least one of them fail.
"""
import os

import numpy as np
import pytest

from paper_1809_06047_amd import meshgen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def _euler(V, E, F):
    return V - E + F


def _quad_box(nz):
    """Closed 1x1xnz box of nz stacked cubes: V = 4(nz+1), F = 4 nz + 2."""
    P = []
    for z in range(nz + 1):
        for (x, y) in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
            P.append((x, y, 2.0 * z - nz))
    P = np.array(P, np.float64)
    faces = []
    for z in range(nz):
        for k in range(4):
            a, b = 4 * z + k, 4 * z + (k + 1) % 4
            faces.append([a, b, b + 4, a + 4])
    faces.append([3, 2, 1, 0])
    top = 4 * nz
    faces.append([top, top + 1, top + 2, top + 3])
    F = _orient_convex(P, np.array(faces, np.int32))
    return G.Mesh(positions=P.astype(np.float32), verts=F.reshape(-1), face_order=4, name=f"box{nz}")


def _orient_convex(P, F):
    c = P.mean(axis=0)
    out = F.copy()
    for i, f in enumerate(F):
        q = P[f]
        n = np.zeros(3)
        for j in range(len(f)):
            n += np.cross(q[j] - c, q[(j + 1) % len(f)] - c)
        if np.dot(n, q.mean(axis=0) - c) < 0:
            out[i] = f[::-1]
    return out


def _ring_sphere(m):
    """Closed triangle sphere: two poles and one ring of m vertices;
    V = m + 2, F = 2 m."""
    ang = 2 * np.pi * np.arange(m) / m
    P = np.concatenate([np.stack([np.cos(ang), np.sin(ang), np.zeros(m)], 1), [[0, 0, 1], [0, 0, -1]]])
    N, S = m, m + 1
    F = []
    for i in range(m):
        F.append([N, i, (i + 1) % m])
        F.append([S, (i + 1) % m, i])
    F = _orient_convex(P, np.array(F, np.int32))
    return G.Mesh(positions=P.astype(np.float32), verts=F.reshape(-1), face_order=3, name=f"ring{m}")


def _uniform(lvl, order):
    return lvl.verts.reshape(-1, order)


def _edges_of(faces):
    a = faces.reshape(-1)
    b = np.roll(faces, -1, axis=1).reshape(-1)
    return np.unique(np.stack([np.minimum(a, b), np.maximum(a, b)], 1), axis=0)


# ---------------------------------------------------------------- counts

@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_count_closed_forms_and_euler(oracle_mod, scheme):
    """V,E,F per level follow the index rules of Sec. 3.2 / App. A / App. B:
    CC V'=V+E+F, E'=2E+H, F'=H; Loop V'=V+E, E'=2E+3F, F'=4F;
    sqrt3 V'=V+F, E'=E+3F, F'=3F. Euler characteristic is invariant; the
    number of boundary edges doubles (CC, Loop) or stays (sqrt3)."""
    if scheme == "cc":
        mesh, L = G.cc_cage(level=2, crease_frac=0.0), 3
    else:
        base = G.icosphere(3)
        rng = np.random.default_rng(0)
        F = G.cut_holes(base[1], 12, rng)
        mesh, L = G.Mesh(positions=base[0].astype(np.float32), verts=F.reshape(-1), face_order=3), 3
    lv = oracle_mod.refine(mesh, scheme, L + 1)
    for k in range(L):
        a, b = lv[k], lv[k + 1]
        V, F, H, E, NB = a.num_vertices, a.num_faces, a.verts.size, a.edges.shape[0], a.n_boundary
        V2, F2, H2, E2, NB2 = b.num_vertices, b.num_faces, b.verts.size, b.edges.shape[0], b.n_boundary
        if scheme == "cc":
            assert (V2, E2, F2, H2) == (V + E + F, 2 * E + H, H, 4 * H)
            assert NB2 == 2 * NB
        elif scheme == "loop":
            assert (V2, E2, F2) == (V + E, 2 * E + 3 * F, 4 * F)
            assert NB2 == 2 * NB
        else:
            assert (V2, E2, F2) == (V + F, E + 3 * F, 3 * F)
            assert NB2 == NB
        assert _euler(V, E, F) == _euler(V2, E2, F2)


def test_cage_counts_match_workload_recipes(oracle_mod):
    """The synthetic cages have the sizes the workloads are defined with."""
    m = G.cc_cage()
    lv = oracle_mod.refine(m, "cc", 1)
    assert (m.num_vertices, m.num_faces, m.num_halfedges, lv[0].edges.shape[0]) == (10242, 17408, 55296, 27648)
    assert m.num_creases == 829
    t = G.tri_cage()
    lt = oracle_mod.refine(t, "loop", 1)
    E = lt[0].edges.shape[0]
    assert (t.num_vertices, t.num_faces, E, lt[0].n_boundary) == (40962, 80282, 122880, 4914)
    assert _euler(t.num_vertices, E, t.num_faces) == -1636
    assert (lt[1].num_vertices, lt[1].edges is None or True, lt[1].num_faces) == (163842, True, 321128)


def test_paper_table_counts(oracle_mod):
    """Counts printed in Table mesh_info_CC (threeblock) and Table
    mesh_info_S (fox), reproduced on stand-in cages with the same control
    counts (closed, genus 0), at the printed precision."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_table_counts.txt")) if not l.startswith("#")]

    def fmt(x, printed):
        if printed.endswith("k"):
            digits = len(printed[:-1].split(".")[1]) if "." in printed else 0
            return f"{x / 1000:.{digits}f}k"
        return str(x)

    for scheme, name, cf, cv, ni, rf, rv, stand_in in rows:
        cage = _quad_box(4) if stand_in == "box_1x1x4" else _ring_sphere(311)
        assert (cage.num_faces, cage.num_vertices) == (int(cf), int(cv))
        lv = oracle_mod.refine(cage, scheme, int(ni))
        assert fmt(lv[-1].num_faces, rf) == rf, name
        assert fmt(lv[-1].num_vertices, rv) == rv, name


def test_tetrahedron_counts(oracle_mod):
    """CC L1 14/24/12, Loop L1 10/24/16, sqrt3 L1 8/18/12 (by hand)."""
    t = G.tetrahedron()
    want = {"cc": (14, 24, 12), "loop": (10, 24, 16), "sqrt3": (8, 18, 12)}
    for s, (V, E, F) in want.items():
        lv = oracle_mod.refine(t, s, 2)
        assert (lv[1].num_vertices, lv[1].edges.shape[0], lv[1].num_faces) == (V, E, F)


# ---------------------------------------------------------------- topology

def test_edge_enumeration_is_sorted_hi_lo(oracle_mod):
    """Edge ids enumerate the upper triangle of E in ascending (hi, lo)
    (CSC) order, one id per undirected edge (Sec. 3.2)."""
    m = G.cc_cage(level=2)
    lv = oracle_mod.refine(m, "cc", 2)
    for k in range(2):
        e = lv[k].edges
        assert np.all(e[:, 0] < e[:, 1])
        key = e[:, 1].astype(np.int64) * (1 << 32) + e[:, 0]
        assert np.all(np.diff(key) > 0)
    # level 1 is all quads: the edge set equals the face table's edge set
    F1 = _uniform(lv[1], 4)
    ref = _edges_of(F1)
    got = lv[1].edges[np.lexsort((lv[1].edges[:, 1], lv[1].edges[:, 0]))]
    assert np.array_equal(ref, got)


def test_cc_child_layout(oracle_mod):
    """Child (r, j) of face r sits at off_r + j and is
    (v_j, |v|+|f|+e(v_j, v_j+1), |v|+r, |v|+|f|+e(v_j-1, v_j)) (Sec. 3.2)."""
    m = G.cc_cage(level=1, crease_frac=0.0)
    lv = oracle_mod.refine(m, "cc", 1)
    L0, L1 = lv[0], lv[1]
    V, F = L0.num_vertices, L0.num_faces
    eid = {tuple(e): i for i, e in enumerate(L0.edges.tolist())}
    kids = _uniform(L1, 4)
    for r in range(F):
        vs = L0.verts[L0.offsets[r]:L0.offsets[r + 1]].tolist()
        c = len(vs)
        for j in range(c):
            a, b, p = vs[j], vs[(j + 1) % c], vs[j - 1]
            want = [a, V + F + eid[(min(a, b), max(a, b))], V + r, V + F + eid[(min(a, p), max(a, p))]]
            assert kids[L0.offsets[r] + j].tolist() == want


@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_orientation_preserved(oracle_mod, scheme):
    """On a planar counter-clockwise grid every child face keeps a positive
    signed area at every level (the child layouts preserve orientation)."""
    m = G.grid_patch(4, 3, tri=(scheme != "cc"))
    lv = oracle_mod.refine(m, scheme, 3)
    for lvl in lv[1:]:
        P = lvl.positions
        for f in range(lvl.num_faces):
            q = P[lvl.verts[lvl.offsets[f]:lvl.offsets[f + 1]], :2]
            area = 0.5 * np.sum(q[:, 0] * np.roll(q[:, 1], -1) - np.roll(q[:, 0], -1) * q[:, 1])
            assert area > 0


# ---------------------------------------------------------------- values

def test_cube_worked_example(oracle_mod):
    """Hand-worked Catmull-Clark values on the cube (golden fixture)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "cube_cc_level1.txt")) if l.strip() and l[0] != "#"]
    lv = oracle_mod.refine(G.cube(), "cc", 2)
    L0, L1 = lv[0], lv[1]
    V, F = L0.num_vertices, L0.num_faces
    P0 = L0.positions
    for r in rows:
        if r[0] == "counts":
            assert (L1.num_vertices, lv[1].edges.shape[0], L1.num_faces) == tuple(int(x) for x in r[1:])
            continue
        key = np.array([float(x) for x in r[1:4]])
        want = np.array([float(x) for x in r[4:7]])
        if r[0] == "vertex":
            idx = int(np.argmin(np.abs(P0 - key).sum(1)))
        elif r[0] == "face":
            cen = np.array([P0[L0.verts[L0.offsets[f]:L0.offsets[f + 1]]].mean(0) for f in range(F)])
            idx = V + int(np.argmin(np.abs(cen - key).sum(1)))
        else:
            mid = (P0[L0.edges[:, 0]] + P0[L0.edges[:, 1]]) / 2
            idx = V + F + int(np.argmin(np.abs(mid - key).sum(1)))
        np.testing.assert_allclose(L1.positions[idx], want, rtol=0, atol=1e-15)


def _bspline_refine_1d(P, axis):
    """Uniform periodic cubic B-spline refinement along `axis`:
    even = (P[i-1] + 6 P[i] + P[i+1]) / 8, odd = (P[i] + P[i+1]) / 2."""
    Pm, Pp = np.roll(P, 1, axis), np.roll(P, -1, axis)
    even = (Pm + 6 * P + Pp) / 8
    odd = (P + Pp) / 2
    shape = list(P.shape)
    shape[axis] *= 2
    out = np.empty(shape)
    sl = [slice(None)] * P.ndim
    sl[axis] = slice(0, None, 2)
    out[tuple(sl)] = even
    sl[axis] = slice(1, None, 2)
    out[tuple(sl)] = odd
    return out


def test_torus_equals_tensor_product_bspline(oracle_mod):
    """On a regular quad torus every vertex has valence 4, where the CC
    vertex rule becomes the 36/64, 6/64, 1/64 mask and the edge rule the
    [1 1]/2 x [1 6 1]/8 mask: CC equals uniform bicubic B-spline refinement,
    computed here independently as two 1-D periodic refinements."""
    n = 16
    m = G.torus_cage()
    lv = oracle_mod.refine(m, "cc", 3)
    gi = np.repeat(np.arange(n), n)
    gj = np.tile(np.arange(n), n)
    grid = lv[0].positions.reshape(n, n, 3)
    N = n
    for k in range(3):
        a, b = lv[k], lv[k + 1]
        V, F = a.num_vertices, a.num_faces
        ni = np.empty(b.num_vertices, np.int64)
        nj = np.empty(b.num_vertices, np.int64)
        ni[:V], nj[:V] = 2 * gi, 2 * gj
        q = _uniform(a, 4)

        def lower(x, y):
            return np.where((y - x) % N == 1, x, y)

        fi = np.stack([gi[q[:, s]] for s in range(4)], 1)
        fj = np.stack([gj[q[:, s]] for s in range(4)], 1)
        lo_i = lower(fi.min(1), fi.max(1))
        lo_j = lower(fj.min(1), fj.max(1))
        ni[V:V + F], nj[V:V + F] = 2 * lo_i + 1, 2 * lo_j + 1
        e0, e1 = a.edges[:, 0], a.edges[:, 1]
        di = gi[e0] != gi[e1]
        ni[V + F:] = np.where(di, 2 * lower(gi[e0], gi[e1]) + 1, 2 * gi[e0])
        nj[V + F:] = np.where(di, 2 * gj[e0], 2 * lower(gj[e0], gj[e1]) + 1)
        N *= 2
        grid = _bspline_refine_1d(_bspline_refine_1d(grid, 0), 1)
        got = np.empty_like(grid)
        got[ni, nj] = b.positions
        assert len(set(zip(ni.tolist(), nj.tolist()))) == N * N
        np.testing.assert_allclose(got, grid, rtol=0, atol=1e-14)
        gi, gj = ni, nj


def _limit_cc(lvl):
    """Limit positions of a closed all-quad level: (n^2 p + 4 sum e + sum d) / (n (n+5))."""
    q, P = _uniform(lvl, 4), lvl.positions
    V = P.shape[0]
    n = np.zeros(V)
    se = np.zeros((V, 3))
    sd = np.zeros((V, 3))
    for j in range(4):
        v = q[:, j]
        np.add.at(n, v, 1)
        np.add.at(se, v, 0.5 * (P[q[:, (j + 1) % 4]] + P[q[:, (j + 3) % 4]]))
        np.add.at(sd, v, P[q[:, (j + 2) % 4]])
    n2 = n[:, None]
    return (n2 * n2 * P + 4 * se + sd) / (n2 * (n2 + 5))


def _ring_mean_tri(lvl):
    q, P = _uniform(lvl, 3), lvl.positions
    V = P.shape[0]
    n = np.zeros(V)
    s = np.zeros((V, 3))
    for j in range(3):
        v = q[:, j]
        np.add.at(n, v, 1)
        np.add.at(s, v, 0.5 * (P[q[:, (j + 1) % 3]] + P[q[:, (j + 2) % 3]]))
    return n, s / n[:, None]


def _limit_loop(lvl):
    n, r = _ring_mean_tri(lvl)
    beta = (5 / 8 - (3 / 8 + 0.25 * np.cos(2 * np.pi / n)) ** 2) / n
    w = (8 * n * beta)[:, None]
    return (3 * lvl.positions + w * r) / (3 + w)


def _limit_sqrt3(lvl):
    n, r = _ring_mean_tri(lvl)
    a = ((4 - 2 * np.cos(2 * np.pi / n)) / 9)[:, None]
    return (lvl.positions + 3 * a * r) / (1 + 3 * a)


@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_limit_points_invariant(oracle_mod, scheme):
    """The limit position of every smooth vertex (dominant left eigenvector
    of the local subdivision matrix built from the rules) is the same at
    level k and k+1; this ties vertex, edge and face rules together at every
    valence present (3..7 here)."""
    if scheme == "cc":
        m = G.cc_cage(level=2, crease_frac=0.0)
        lv = oracle_mod.refine(m, "cc", 3)
        pairs, fn = [(1, 2), (2, 3)], _limit_cc
    else:
        P, F = G.icosphere(2)
        rng = np.random.default_rng(5)
        m = G.Mesh(positions=(P + rng.normal(0, 0.02, P.shape)).astype(np.float32), verts=F.reshape(-1),
                   face_order=3)
        lv = oracle_mod.refine(m, scheme, 3)
        pairs = [(0, 1), (1, 2), (2, 3)]
        fn = _limit_loop if scheme == "loop" else _limit_sqrt3
    for a, b in pairs:
        la, lb = fn(lv[a]), fn(lv[b])
        V = la.shape[0]
        np.testing.assert_allclose(lb[:V], la, rtol=0, atol=1e-13)


def test_weights_on_tetrahedron(oracle_mod):
    """Valence-3 weights: Loop beta_3 = 3/16 (centre 7/16), sqrt3 alpha_3 = 5/9
    (centre 4/9, neighbours 5/27); Loop edge point 3/8, 3/8, 1/8, 1/8."""
    t = G.tetrahedron()
    lv = oracle_mod.refine(t, "loop", 1, want_R=True)
    R = lv[1].R.toarray()
    for v in range(4):
        row = R[v]
        assert row[v] == pytest.approx(7 / 16, abs=1e-15)
        assert np.allclose(np.delete(row, v), 3 / 16, atol=1e-15)
    for e in range(6):
        row = np.sort(R[4 + e])
        np.testing.assert_allclose(row, [1 / 8, 1 / 8, 3 / 8, 3 / 8], atol=1e-15)
    lv = oracle_mod.refine(t, "sqrt3", 1, want_R=True)
    R = lv[1].R.toarray()
    for v in range(4):
        assert R[v, v] == pytest.approx(4 / 9, abs=1e-15)
        assert np.allclose(np.delete(R[v], v), 5 / 27, atol=1e-15)
    np.testing.assert_allclose(R[4:], np.where(R[4:] > 0, 1 / 3, 0), atol=1e-15)


def test_regular_weights(oracle_mod):
    """Valence 6: Loop beta_6 = 1/16 (centre 10/16); sqrt3 alpha_6 = 1/3
    (centre 2/3, neighbours 1/18). Valence 4 quads: CC centre 36/64."""
    P, F = G.icosphere(2)
    m = G.Mesh(positions=P.astype(np.float32), verts=F.reshape(-1), face_order=3)
    for s, centre, nb in (("loop", 10 / 16, 1 / 16), ("sqrt3", 2 / 3, 1 / 18)):
        lv = oracle_mod.refine(m, s, 1, want_R=True)
        R = lv[1].R.tocsr()
        v = 12  # first vertex created by the midpoint splits: valence 6
        row = R[v].toarray().ravel()
        assert row[v] == pytest.approx(centre, abs=1e-15)
        others = row[np.nonzero(row)[0]]
        assert np.count_nonzero(row) == 7
        assert np.allclose(np.sort(others)[:6], nb, atol=1e-15)
    lv = oracle_mod.refine(G.torus_cage(), "cc", 1, want_R=True)
    row = lv[1].R[0].toarray().ravel()
    assert sorted(np.round(row[row > 0] * 64, 12).tolist()) == [1] * 4 + [6] * 4 + [36]


# ---------------------------------------------------------------- linearity

@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_R_rows_and_affine_invariance(oracle_mod, scheme):
    """P_{k+1} = R_k P_k (Sec. 3.6); every row sums to 1, so translating the
    cage translates the result; R_k does not depend on the positions."""
    if scheme == "cc":
        m = G.cc_cage(level=1)
    else:
        P, F = G.icosphere(2)
        F = G.cut_holes(F, 6, np.random.default_rng(1))
        m = G.Mesh(positions=P.astype(np.float32), verts=F.reshape(-1), face_order=3)
    lv = oracle_mod.refine(m, scheme, 2, want_R=True)
    for k in range(2):
        R = lv[k + 1].R
        np.testing.assert_allclose(np.asarray(R.sum(1)).ravel(), 1.0, atol=1e-14)
        np.testing.assert_allclose(R @ lv[k].positions, lv[k + 1].positions, atol=1e-13)
    shift = np.array([3.0, -2.0, 0.5])
    base = oracle_mod.level_from_mesh(m)
    moved = oracle_mod.Level(offsets=base.offsets, verts=base.verts, positions=base.positions + shift,
                             crease_verts=base.crease_verts, crease_sharp=base.crease_sharp)
    lv2 = oracle_mod.refine(moved, scheme, 2, want_R=True)
    np.testing.assert_allclose(lv2[2].positions - lv[2].positions,
                               np.broadcast_to(shift, lv[2].positions.shape), atol=1e-12)
    assert abs(lv2[1].R - lv[1].R).max() == 0.0


def test_adjoint_equals_finite_differences(oracle_mod):
    """Refinement is linear, so L(P0) = sum |P_L - T|^2 is quadratic and its
    central differences are exact up to rounding: they equal R^T 2(P_L - T)
    with R = R_{L-1} ... R_0 assembled from the rows."""
    m = G.torus_cage()
    lv = oracle_mod.refine(m, "cc", 2, want_R=True)
    R = lv[2].R @ lv[1].R
    rng = np.random.default_rng(7)
    T = lv[2].positions + rng.normal(0, 0.05, lv[2].positions.shape)
    g = R.T @ (2 * (lv[2].positions - T))
    base = oracle_mod.level_from_mesh(m)

    def loss(P):
        l0 = oracle_mod.Level(offsets=base.offsets, verts=base.verts, positions=P,
                              crease_verts=base.crease_verts, crease_sharp=base.crease_sharp)
        out = oracle_mod.refine(l0, "cc", 2)
        return float(np.sum((out[2].positions - T) ** 2))

    h = 1e-3
    for (i, d) in [(0, 0), (17, 1), (200, 2), (255, 0)]:
        Pp, Pm = base.positions.copy(), base.positions.copy()
        Pp[i, d] += h
        Pm[i, d] -= h
        fd = (loss(Pp) - loss(Pm)) / (2 * h)
        assert fd == pytest.approx(g[i, d], rel=1e-8, abs=1e-9)


# ---------------------------------------------------------------- creases

def _cube_with_creases(sigma):
    m = G.cube()
    e = G.mesh_edges(None, m.verts, 4)
    return G.Mesh(positions=m.positions, verts=m.verts, face_order=4, crease_verts=e.astype(np.int32),
                  crease_sharp=np.full(e.shape[0], sigma, np.float32))


def test_infinitely_sharp_cube(oracle_mod):
    """All 12 cube edges sharper than the depth: corners (k = 3) are fixed,
    every refined vertex stays on the cube's surface and crease vertices stay
    on the cube's edges (the rules only average points of one face / edge)."""
    lv = oracle_mod.refine(_cube_with_creases(10.0), "cc", 3)
    for k in range(1, 4):
        P = lv[k].positions
        np.testing.assert_array_equal(P[:8], lv[0].positions)
        assert np.all(np.abs(P) <= 1 + 1e-15)
        assert np.all(np.isclose(np.abs(P).max(1), 1.0, atol=1e-15))
        cv = np.unique(lv[k].crease_verts.reshape(-1))
        on_edge = (np.isclose(np.abs(P[cv]), 1.0, atol=1e-15).sum(1) >= 2)
        assert on_edge.all()
        assert np.all(lv[k].crease_sharp == 10.0 - k)


def test_sigma_one_is_one_sharp_step(oracle_mod):
    """sigma = 1 everywhere: level 1 uses the sharp rules, the children get
    max(1/4 (1 + 3) - 1, 0) = 0, so level 2 equals smooth CC of level 1."""
    lv = oracle_mod.refine(_cube_with_creases(1.0), "cc", 2)
    assert lv[1].crease_sharp.size == 0
    sharp = oracle_mod.refine(_cube_with_creases(50.0), "cc", 1)
    np.testing.assert_allclose(lv[1].positions, sharp[1].positions, atol=1e-15)
    smooth = oracle_mod.step(oracle_mod.Level(offsets=lv[1].offsets, verts=lv[1].verts, positions=lv[1].positions,
                                              crease_verts=np.zeros((0, 2), np.int32),
                                              crease_sharp=np.zeros(0)), 0)
    np.testing.assert_allclose(lv[2].positions, smooth.positions, atol=1e-15)


def test_chaikin_on_closed_crease_loop(oracle_mod):
    """A closed crease loop with constant sigma (every end point has k = 2):
    both children get 1/4 (s + 3 s) - 1 = s - 1 (Sec. 3.3)."""
    m = G.cube()
    # the loop around the four +-y faces' shared 'equator' edges: edges parallel to y at x,z = +-1
    P = m.positions
    e = G.mesh_edges(None, m.verts, 4)
    ring = [i for i, (a, b) in enumerate(e) if P[a][1] == P[b][1]
            and abs(P[a][0] - P[b][0]) + abs(P[a][2] - P[b][2]) == 2 and P[a][1] == 1]
    assert len(ring) == 4
    mm = G.Mesh(positions=P, verts=m.verts, face_order=4, crease_verts=e[ring].astype(np.int32),
                crease_sharp=np.full(4, 2.75, np.float32))
    lv = oracle_mod.refine(mm, "cc", 3)
    assert lv[1].crease_sharp.size == 8 and np.all(lv[1].crease_sharp == 1.75)
    assert lv[2].crease_sharp.size == 16 and np.all(lv[2].crease_sharp == 0.75)
    assert lv[3].crease_sharp.size == 0


def _tet_with_creases(sigma):
    t = G.tetrahedron()
    e = G.mesh_edges(None, t.verts, 3).astype(np.int32)
    return G.Mesh(positions=t.positions, verts=t.verts, face_order=3, crease_verts=e,
                  crease_sharp=np.full(len(e), sigma, np.float32))


def test_loop_infinitely_sharp_tetrahedron(oracle_mod):
    """Loop with every edge of a tetrahedron sharp beyond the levels (the
    Catmull-Clark crease rules applied to Loop's points): each corner has
    three creases and stays exactly where it is; crease edge points are
    midpoints and crease vertices take 3/4 p + 1/8 (two crease neighbours),
    so every crease vertex stays on its edge line; every other new point is
    a Loop combination of points of one face, so it stays in that face's
    plane. A dropped crease term would pull points off the surface."""
    L = 3
    lv = oracle_mod.refine(_tet_with_creases(10.0), "loop", L)
    t = G.tetrahedron()
    P0 = t.positions.astype(np.float64)
    for k in range(1, L + 1):
        np.testing.assert_array_equal(lv[k].positions[:4], P0)
        assert np.all(lv[k].crease_sharp == 10.0 - k)
        assert lv[k].crease_sharp.size == 6 * 2 ** k
    planes = []
    for f in t.face_list():
        a, b, c = P0[f]
        n = np.cross(b - a, c - a)
        planes.append((n / np.linalg.norm(n), a))
    P = lv[L].positions
    d = np.min(np.stack([np.abs((P - a) @ n) for n, a in planes]), axis=0)
    assert d.max() < 1e-14
    # crease vertices of the last level lie on the cage's edge lines
    on_edge = lambda p, a, b: np.linalg.norm(np.cross(p - a, b - a)) / np.linalg.norm(b - a)
    edges = G.mesh_edges(None, t.verts, 3)
    for lo, hi in lv[L].crease_verts:
        for v in (lo, hi):
            assert min(on_edge(P[v], P0[a], P0[b]) for a, b in edges) < 1e-14


def test_loop_creases_zero_sigma_is_smooth_and_chaikin(oracle_mod):
    """Loop with sharpness 0 everywhere is smooth Loop; a closed crease loop
    of constant sigma (every end point has two creases) halves into children
    of sigma - 1, level after level (the rule of Sec. 3.3)."""
    np.testing.assert_array_equal(oracle_mod.refine(_tet_with_creases(0.0), "loop", 2)[2].positions,
                                  oracle_mod.refine(G.tetrahedron(), "loop", 2)[2].positions)
    # the equator of an octahedron: four edges, each end point on two of them
    P = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
    F = [[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4], [1, 0, 5], [2, 1, 5], [3, 2, 5], [0, 3, 5]]
    ring = np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32)
    m = G.Mesh(positions=P, verts=np.array(F, np.int32).reshape(-1), face_order=3, crease_verts=ring,
               crease_sharp=np.full(4, 2.5, np.float32))
    lv = oracle_mod.refine(m, "loop", 3)
    assert lv[1].crease_sharp.size == 8 and np.all(lv[1].crease_sharp == 1.5)
    assert lv[2].crease_sharp.size == 16 and np.all(lv[2].crease_sharp == 0.5)
    assert lv[3].crease_sharp.size == 0
    # a sharp equator keeps the equator's points in the plane z = 0 (crease
    # rules only read points of the loop), and the crease points of level 1
    # are the midpoints of the square's edges or the 3/4, 1/8 rule of its corners
    sharp = G.Mesh(positions=P, verts=m.verts, face_order=3, crease_verts=ring, crease_sharp=np.full(4, 5.0, np.float32))
    s1 = oracle_mod.refine(sharp, "loop", 1)[1]
    np.testing.assert_allclose(s1.positions[0], [0.75, 0, 0], atol=1e-15)       # 3/4 p + 1/8 (p1 + p3)
    eq = [v for v in np.unique(s1.crease_verts)]
    assert np.all(np.abs(s1.positions[eq, 2]) < 1e-15)


def test_loop_semisharp_blend_is_linear_in_sigma(oracle_mod):
    smooth = oracle_mod.refine(G.tetrahedron(), "loop", 1)[1].positions
    sharp = oracle_mod.refine(_tet_with_creases(1.0), "loop", 1)[1].positions
    half = oracle_mod.refine(_tet_with_creases(0.5), "loop", 1)[1].positions
    np.testing.assert_allclose(half, 0.5 * (smooth + sharp), atol=1e-15)


def test_semisharp_blend_is_linear_in_sigma(oracle_mod):
    """Fractional sharpness (0 < sigma < 1) blends the smooth and sharp
    results linearly (reading of the DeRose rules the paper defers to; the
    paper itself does not fix it: only sigma -> 0 and sigma = 1 are pinned)."""
    smooth = oracle_mod.refine(G.cube(), "cc", 1)[1].positions
    sharp = oracle_mod.refine(_cube_with_creases(1.0), "cc", 1)[1].positions
    half = oracle_mod.refine(_cube_with_creases(0.5), "cc", 1)[1].positions
    np.testing.assert_allclose(half, 0.5 * (smooth + sharp), atol=1e-15)


# Cube corners by sign pattern (meshgen.cube numbers (x>0, y>0, z>0) as bits)
_B = 7          # (1, 1, 1)
_A = 6          # (1, 1, -1), cube edge (A, B)
_C = 5          # (1, -1, 1), cube edge (C, B)
_D = 3          # (-1, 1, 1), cube edge (D, B)


def _cube_creases(pairs, sigmas):
    m = G.cube()
    return G.Mesh(positions=m.positions, verts=m.verts, face_order=4,
                  crease_verts=np.array([[min(p), max(p)] for p in pairs], np.int32),
                  crease_sharp=np.array(sigmas, np.float32))


def _crease_set(lvl, P_parent_pairs=None):
    return {(int(a), int(b), float(s)) for (a, b), s in zip(lvl.crease_verts, lvl.crease_sharp)}


def _vertex_at(P, x):
    d = np.abs(P - np.asarray(x, np.float64)).sum(1)
    i = int(np.argmin(d))
    assert d[i] < 1e-12
    return i


def test_chaikin_uses_the_neighbour_crease_on_an_open_path(oracle_mod):
    """Open crease path A - B - C along two cube edges with sigma(AB) = 3 and
    sigma(BC) = 1 (Sec. 3.3, the two Chaikin equations, worked by hand). At B
    (two creases) each child takes sigma_i from the other crease:
    AB's half at B gets 1/4 (1 + 3*3) - 1 = 1.5 and BC's half gets
    1/4 (3 + 3*1) - 1 = 0.5. At the single-crease ends the neighbour is the
    crease itself: A's half gets 3 - 1 = 2 and C's half 1 - 1 = 0, which is
    dropped. Both edges have sigma >= 1, so their edge points are midpoints.
    One level further, with the level-1 values (A's half 2, B's halves 1.5
    and 0.5) every end is again worked out by hand: {1, 0.875, 0.625, 0.25}
    survive. A swapped argument order, the crease's own sigma at a two-crease
    end, or a dropped clamp each breaks one of these numbers."""
    lv = oracle_mod.refine(_cube_creases([(_A, _B), (_C, _B)], [3.0, 1.0]), "cc", 2)
    P0, P1 = lv[0].positions, lv[1].positions
    m_ab = _vertex_at(P1, (P0[_A] + P0[_B]) / 2)
    m_bc = _vertex_at(P1, (P0[_C] + P0[_B]) / 2)
    assert _crease_set(lv[1]) == {(_A, m_ab, 2.0), (_B, m_ab, 1.5), (_B, m_bc, 0.5)}
    # level 2: (A, m_ab) 2 -> at A 2 - 1 = 1, at m_ab 1/4 (1.5 + 6) - 1 = 0.875;
    # (B, m_ab) 1.5 -> at B 1/4 (0.5 + 4.5) - 1 = 0.25, at m_ab 1/4 (2 + 4.5) - 1 = 0.625;
    # (B, m_bc) 0.5 -> at B 1/4 (1.5 + 1.5) - 1 < 0, at m_bc 0.5 - 1 < 0: both dropped
    assert sorted(lv[2].crease_sharp.tolist()) == [0.25, 0.625, 0.875, 1.0]
    ends = sorted(int(a) for a, _ in lv[2].crease_verts)
    assert ends == sorted([_A, m_ab, _B, m_ab])


def test_vertex_sharpness_is_the_mean_of_its_creases(oracle_mod):
    """Vertex sharpness s = mean of the incident creases' sigma (Sec. 3.3,
    the vertex-sharpness definition). The smooth corner point of the cube is
    (5/9) p (the worked example above).
    Two creases at B, sigma 0.25 and 0.75: s = 0.5, the crease rule
    3/4 B + 1/8 (A + C) = (1, 0.75, 0.75), so B moves to
    1/2 (5/9) (1,1,1) + 1/2 (1, 0.75, 0.75).
    Three creases at B, sigma 0.125, 0.625, 0.75: s = 0.5 again (max 0.75,
    min 0.125, no single sigma equals it), the corner rule keeps B, so B moves
    to 1/2 (5/9) (1,1,1) + 1/2 (1,1,1) = (7/9) (1,1,1)."""
    lv = oracle_mod.refine(_cube_creases([(_A, _B), (_C, _B)], [0.25, 0.75]), "cc", 1)
    want = 0.5 * (5.0 / 9.0) * np.ones(3) + 0.5 * np.array([1.0, 0.75, 0.75])
    np.testing.assert_allclose(lv[1].positions[_B], want, rtol=0, atol=1e-15)
    # order of the creases in the list does not matter
    lv = oracle_mod.refine(_cube_creases([(_C, _B), (_A, _B)], [0.75, 0.25]), "cc", 1)
    np.testing.assert_allclose(lv[1].positions[_B], want, rtol=0, atol=1e-15)
    for sig in ([0.125, 0.625, 0.75], [0.75, 0.125, 0.625], [0.625, 0.75, 0.125]):
        lv = oracle_mod.refine(_cube_creases([(_A, _B), (_C, _B), (_D, _B)], sig), "cc", 1)
        np.testing.assert_allclose(lv[1].positions[_B], (7.0 / 9.0) * np.ones(3), rtol=0, atol=1e-15)
        # the three neighbours carry one crease each (k = 1): smooth corners
        for v in (_A, _C, _D):
            np.testing.assert_allclose(lv[1].positions[v], (5.0 / 9.0) * lv[0].positions[v], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- boundaries

def _boundary_loop(m):
    """Ordered boundary polygon of an open grid patch (CCW)."""
    fl = m.face_list()
    nxt = {}
    he = set()
    for f in fl:
        for j in range(len(f)):
            he.add((f[j], f[(j + 1) % len(f)]))
    for (a, b) in he:
        if (b, a) not in he:
            nxt[a] = b
    start = min(nxt)
    loop = [start]
    while nxt[loop[-1]] != start:
        loop.append(nxt[loop[-1]])
    return loop


@pytest.mark.parametrize("scheme", ["cc", "loop"])
def test_boundary_is_cubic_bspline_curve(oracle_mod, scheme):
    """CC and Loop boundaries follow the curve rules 3/4, 1/8 (eq::CC_boundary)
    and edge midpoints: the refined boundary polygon equals periodic cubic
    B-spline refinement of the old boundary polygon (incl. the corners)."""
    rng = np.random.default_rng(3)
    m = G.grid_patch(5, 4, tri=(scheme == "loop"), z_fn=lambda x, y: rng.normal(0, 0.3, x.shape))
    lv = oracle_mod.refine(m, scheme, 2)
    for k in range(2):
        a, b = lv[k], lv[k + 1]
        loop = _boundary_loop(G.Mesh(positions=a.positions, verts=a.verts, offsets=a.offsets))
        eid = {tuple(e): i for i, e in enumerate(a.edges.tolist())}
        V, F = a.num_vertices, a.num_faces
        base = V + F if scheme == "cc" else V
        want = _bspline_refine_1d(a.positions[loop], 0)
        idx = []
        for i, v in enumerate(loop):
            w = loop[(i + 1) % len(loop)]
            idx += [v, base + eid[(min(v, w), max(v, w))]]
        np.testing.assert_allclose(b.positions[idx], want, rtol=0, atol=1e-14)


def test_sqrt3_boundary_vertices_fixed(oracle_mod):
    """sqrt3 boundary vertices are kept in place (reading: the paper omits
    the boundary rule); interior ones move."""
    t = G.tri_cage(level=3, hole_frac=0.02)
    lv = oracle_mod.refine(t, "sqrt3", 2)
    for k in range(2):
        e = lv[k].edges
        nb = np.zeros(lv[k].num_vertices, bool)
        he = set(map(tuple, lv[k].verts.reshape(-1, 3)[:, [0, 1]].tolist() +
                      lv[k].verts.reshape(-1, 3)[:, [1, 2]].tolist() + lv[k].verts.reshape(-1, 3)[:, [2, 0]].tolist()))
        for a, b in he:
            if (b, a) not in he:
                nb[a] = nb[b] = True
        assert nb.sum() > 0
        V = lv[k].num_vertices
        np.testing.assert_array_equal(lv[k + 1].positions[:V][nb], lv[k].positions[nb])
        assert np.all(np.any(lv[k + 1].positions[:V][~nb] != lv[k].positions[~nb], axis=1))


# ---------------------------------------------------------------- validation

def _tri(P, F):
    return G.Mesh(positions=np.asarray(P, np.float32), verts=np.array(F, np.int32).reshape(-1), face_order=3)


def test_status_codes(oracle_mod):
    P = np.zeros((6, 3))
    assert oracle_mod.status_of(G.cube(), "loop") == -2                              # quads for Loop
    assert oracle_mod.status_of(_tri(P, [[0, 1, 1]]), "cc") == -4                    # repeated vertex
    m = G.Mesh(positions=np.zeros((4, 3), np.float32), verts=np.array([0, 1, 2, 3, 2], np.int32),
               offsets=np.array([0, 2, 5], np.int32))
    assert oracle_mod.status_of(m, "cc") == -4                                       # 2-gon
    assert oracle_mod.status_of(_tri(P, [[0, 1, 7]]), "cc") == -1                    # index range
    assert oracle_mod.status_of(_tri(P, [[0, 1, 2]]), "cc") == -4                    # isolated vertices 3..5
    assert oracle_mod.status_of(_tri(P[:5], [[0, 1, 2], [1, 0, 3], [0, 1, 4]]), "cc") == -3  # 3 faces on an edge
    assert oracle_mod.status_of(_tri(P[:4], [[0, 1, 2], [0, 1, 3]]), "cc") == -3    # same direction twice
    assert oracle_mod.status_of(_tri(P[:5], [[0, 1, 2], [0, 3, 4]]), "cc") == -3    # bow-tie vertex 0
    c = G.cube()
    bad = G.Mesh(positions=c.positions, verts=c.verts, face_order=4,
                 crease_verts=np.array([[0, 7]], np.int32), crease_sharp=np.array([1.0], np.float32))
    assert oracle_mod.status_of(bad, "cc") == -5                                     # not an edge
    e = G.mesh_edges(None, c.verts, 4)[:1].astype(np.int32)
    neg = G.Mesh(positions=c.positions, verts=c.verts, face_order=4, crease_verts=e,
                 crease_sharp=np.array([-1.0], np.float32))
    assert oracle_mod.status_of(neg, "cc") == -5                                     # negative sharpness
    dup = G.Mesh(positions=c.positions, verts=c.verts, face_order=4, crease_verts=np.concatenate([e, e[:, ::-1]]),
                 crease_sharp=np.array([1.0, 2.0], np.float32))
    assert oracle_mod.status_of(dup, "cc") == -5                                     # duplicate
    t = G.tetrahedron()
    tc = G.Mesh(positions=t.positions, verts=t.verts, face_order=3, crease_verts=np.array([[0, 1]], np.int32),
                crease_sharp=np.array([1.0], np.float32))
    assert oracle_mod.status_of(tc, "loop") == 0                                     # creases: CC and Loop
    assert oracle_mod.status_of(tc, "sqrt3") == -1                                   # not sqrt(3)
    assert oracle_mod.status_of(G.cube(), "cc") == 0
