"""Pins of the oracle's sqrt(3) boundary cycle (App. A leaves the boundary
to Kobbelt's sqrt(3) paper): the first step of each two-level cycle is the
sqrt(3) step with a fixed boundary, the second trisects every boundary edge.

What fixes it, independently of the oracle's own formulas:
  * counts per step in closed form (V, E, F, boundary edges) and the Euler
    characteristic;
  * regularity: after a cycle, every vertex born in its first step is an
    interior vertex of six faces and every boundary point born in its second
    step has three faces (a wrong link rule leaves 5/7 or 8-valent vertices);
  * the boundary polygon after the second step defines the same uniform cubic
    B-spline curve as before it (evaluated with scipy, knots refined by three):
    the ternary refinement is exact knot insertion;
  * the worked example of one triangle, whose cycle is the 1-to-9 split;
  * a closed surface, which has no boundary, gives the plain sqrt(3) result.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from paper_1809_06047_amd import meshgen as G


def _halfedges(lvl):
    f = lvl.verts.reshape(-1, 3)
    return np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])


def _boundary(lvl):
    """next[u] = w for every boundary half-edge u -> w."""
    he = set(map(tuple, _halfedges(lvl).tolist()))
    return {a: b for (a, b) in he if (b, a) not in he}


def _loops(nxt):
    seen, loops = set(), []
    for s in sorted(nxt):
        if s in seen:
            continue
        loop = [s]
        seen.add(s)
        while nxt[loop[-1]] != s:
            loop.append(nxt[loop[-1]])
            seen.add(loop[-1])
        loops.append(loop)
    return loops


def _faces_per_vertex(lvl):
    return np.bincount(lvl.verts, minlength=lvl.num_vertices)


CAGES = {
    "grid": lambda: G.grid_patch(5, 4, tri=True, z_fn=lambda x, y: 0.2 * np.sin(x) * np.cos(y)),
    "holed": lambda: G.tri_cage(seed=5, level=2, hole_frac=0.05),
    "triangle": lambda: G.Mesh(positions=np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.5]], np.float32),
                               verts=np.array([0, 1, 2], np.int32), face_order=3, name="triangle"),
}


@pytest.mark.parametrize("cage", list(CAGES))
def test_counts_per_step_and_euler(oracle_mod, cage):
    lv = oracle_mod.refine(CAGES[cage](), "sqrt3k", 5)
    oracle_mod.step(lv[5], oracle_mod.SQRT3)  # fills level 5's edge counts (a first step follows)
    for k in range(5):
        V, F, E, B = lv[k].num_vertices, lv[k].num_faces, lv[k].edges.shape[0], lv[k].n_boundary
        V1, F1, E1, B1 = lv[k + 1].num_vertices, lv[k + 1].num_faces, lv[k + 1].edges.shape[0], \
            lv[k + 1].n_boundary
        if k % 2 == 0:  # sqrt(3) step: boundary edges kept
            assert (V1, F1, E1, B1) == (V + F, 3 * F, E + 3 * F, B), k
        else:           # trisection: no face point on the B boundary faces, two points per boundary edge
            assert (V1, F1, E1, B1) == (V + F + B, 3 * F, E + 3 * F + B, 3 * B), k
        assert V1 - E1 + F1 == V - E + F
        assert len(_loops(_boundary(lv[k + 1]))) == len(_loops(_boundary(lv[k])))


@pytest.mark.parametrize("cage", ["grid", "holed"])
def test_cycle_leaves_regular_vertices(oracle_mod, cage):
    m = CAGES[cage]()
    lv = oracle_mod.refine(m, "sqrt3k", 4)
    for c in (0, 2):  # cycles from level 0 and from level 2
        a, mid, b = lv[c], lv[c + 1], lv[c + 2]
        nfaces = _faces_per_vertex(b)
        bnd = np.zeros(b.num_vertices, bool)
        for u, w in _boundary(b).items():
            bnd[u] = bnd[w] = True
        born1 = np.arange(a.num_vertices, mid.num_vertices)      # face points of the cycle's first step
        assert not bnd[born1].any()
        assert np.all(nfaces[born1] == 6), np.unique(nfaces[born1])
        born2b = np.arange(mid.num_vertices + mid.num_faces, b.num_vertices)  # the q points
        p_pts = [mid.num_vertices + r for r in range(mid.num_faces) if bnd[mid.num_vertices + r]]
        assert len(p_pts) == len(born2b) == mid.n_boundary
        assert bnd[born2b].all() and np.all(nfaces[born2b] == 3) and np.all(nfaces[p_pts] == 3)


def _bspline_curve(ctrl, knots_per_unit):
    """Closed uniform cubic B-spline through scipy: control points ctrl (n, 3)
    on knots spaced 1/knots_per_unit, wrapped; returns C(t) for t in [0, n /
    knots_per_unit), with control point i at Greville abscissa i / kpu."""
    n = len(ctrl)
    h = 1.0 / knots_per_unit
    c = np.concatenate([ctrl[-3:], ctrl, ctrl[:3]])   # wrap
    # basis j (0-based in c) spans [t_j, t_j+4]; Greville t_j+2 = (j - 3) h puts ctrl[i] at i h
    t = (np.arange(len(c) + 4) - 5) * h
    spl = BSpline(t, c, 3, extrapolate=False)
    return lambda s: spl(np.mod(s, n * h))


def test_trisection_is_knot_insertion_on_every_boundary_loop(oracle_mod):
    """Boundary polygon of level 2c+1 (control points at spacing 1) and of
    level 2c+2 (spacing 1/3, old vertex i at 3i): the same curve."""
    for cage in ("grid", "holed", "triangle"):
        lv = oracle_mod.refine(CAGES[cage](), "sqrt3k", 4)
        for k in (1, 3):
            a, b = lv[k], lv[k + 1]
            nb = _boundary(b)
            for loop in _loops(_boundary(a)):
                fine = [loop[0]]
                while len(fine) < 3 * len(loop):
                    fine.append(nb[fine[-1]])
                assert fine[3::3] == loop[1:] and nb[fine[-1]] == loop[0]  # old vertices keep their order
                coarse_c = _bspline_curve(a.positions[loop], 1)
                fine_c = _bspline_curve(b.positions[fine], 3)
                s = np.linspace(0.0, len(loop), 12 * len(loop), endpoint=False)
                np.testing.assert_allclose(fine_c(s), coarse_c(s), rtol=0, atol=1e-13)


def test_first_step_keeps_the_boundary(oracle_mod):
    lv = oracle_mod.refine(CAGES["holed"](), "sqrt3k", 3)
    for k in (0, 2):
        nb = _boundary(lv[k])
        v = np.array(sorted(set(nb) | set(nb.values())))
        np.testing.assert_array_equal(lv[k + 1].positions[v], lv[k].positions[v])
        assert _boundary(lv[k + 1]) == nb


def test_one_triangle_becomes_the_one_to_nine_split(oracle_mod):
    """Worked by hand. Triangle a, b, c: level 1 adds the centroid m (three
    faces, each with one boundary edge); level 2 trisects each edge, p near
    its start and q near its end, and keeps m as the centre: the nine
    triangles of the triadic split. Boundary points: p_ab = (c + 16 a + 10 b)
    / 27, q_ab = (10 a + 16 b + c) / 27, corner a -> (4 c + 19 a + 4 b) / 27;
    m -> (1 - alpha_3) m + alpha_3 (a + b + c) / 3 = m (the ring mean is m)."""
    m = CAGES["triangle"]()
    lv = oracle_mod.refine(m, "sqrt3k", 2)
    A, B, C = (lv[0].positions[i] for i in range(3))
    P = lv[2].positions
    assert lv[1].num_vertices == 4 and lv[2].num_vertices == 10 and lv[2].num_faces == 9
    # level-1 faces: 3j + j' ... each child of the triangle is (v_j, v_j+1, m)
    np.testing.assert_array_equal(lv[1].verts.reshape(-1, 3), [[0, 1, 3], [1, 2, 3], [2, 0, 3]])
    # level-1 face r (edge v_r -> v_r+1) gets p at 4 + r and q at 7 + r
    corners = [A, B, C]
    for r in range(3):
        u, w, x = corners[r], corners[(r + 1) % 3], corners[(r + 2) % 3]
        np.testing.assert_allclose(P[4 + r], (x + 16 * u + 10 * w) / 27, rtol=0, atol=1e-15)
        np.testing.assert_allclose(P[7 + r], (10 * u + 16 * w + x) / 27, rtol=0, atol=1e-15)
        np.testing.assert_allclose(P[r], (4 * x + 19 * u + 4 * w) / 27, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P[3], (A + B + C) / 3, rtol=0, atol=1e-15)
    # topology: barycentric labels (3 * weights) of every vertex; the faces
    # must be the nine cells of the triadic grid, all counter-clockwise
    lab = {0: (3, 0, 0), 1: (0, 3, 0), 2: (0, 0, 3), 3: (1, 1, 1)}
    for r in range(3):
        e0, e1 = np.eye(3, dtype=int)[r], np.eye(3, dtype=int)[(r + 1) % 3]
        lab[4 + r] = tuple(2 * e0 + e1)
        lab[7 + r] = tuple(e0 + 2 * e1)
    got = set()
    for f in lv[2].verts.reshape(-1, 3).tolist():
        t = [lab[v] for v in f]
        k = min(range(3), key=lambda i: t[i])
        got.add(tuple(t[k:] + t[:k]))
    want = set()
    for i in range(3):
        for j in range(3 - i):
            for s in (2, 1):  # six upward cells from the points of sum 2, three downward from those of sum 1
                k = s - i - j
                if k < 0:
                    continue
                if s == 2:
                    c = [(i + 1, j, k), (i, j + 1, k), (i, j, k + 1)]
                else:
                    c = [(i, j + 1, k + 1), (i + 1, j, k + 1), (i + 1, j + 1, k)]
                kk = min(range(3), key=lambda x: c[x])
                want.add(tuple(c[kk:] + c[:kk]))
    assert len(want) == 9 and got == want


def test_closed_surface_equals_plain_sqrt3(oracle_mod):
    m = G.tri_cage(seed=8, level=2, hole_frac=0.0)
    a = oracle_mod.refine(m, "sqrt3k", 3)
    b = oracle_mod.refine(m, "sqrt3", 3)
    for k in range(1, 4):
        np.testing.assert_array_equal(a[k].verts, b[k].verts)
        np.testing.assert_array_equal(a[k].positions, b[k].positions)


def test_trisection_rows_are_affine(oracle_mod):
    """Every row of R_k sums to one (translation invariance) on both steps."""
    lv = oracle_mod.refine(CAGES["holed"](), "sqrt3k", 2, want_R=True)
    for k in (1, 2):
        np.testing.assert_allclose(np.asarray(lv[k].R.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-14)


def test_trisection_rejects_two_boundary_edges_per_face(oracle_mod):
    """The trisection step needs at most one boundary edge per face (true
    after a first step); a lone triangle as its input is rejected."""
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.step(oracle_mod.level_from_mesh(CAGES["triangle"]()), oracle_mod.TRISECT_STEP)
