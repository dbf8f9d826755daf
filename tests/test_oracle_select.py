"""Pins of the selective-extraction oracle (Sec. 3.4) against cases counted by
hand and against uniform refinement restricted to the selected region."""
import numpy as np
import pytest

from oracle import refine
from oracle import select as S
from paper_1809_06047_amd import meshgen as G


def _grid(n=4, bumpy=False):
    rng = np.random.default_rng(3)
    return G.grid_patch(n, n, z_fn=(lambda x, y: rng.normal(0, 0.2, x.shape)) if bumpy else None)


def _vid(i, j, n=4):
    return i * (n + 1) + j


def test_everything_seeded_gives_the_cage():
    m = G.cc_cage(seed=24, level=2)
    e = S.extract(m, rings=1, seed=np.ones(m.num_vertices, np.uint8))
    g = m.general()
    np.testing.assert_array_equal(e.offsets, g.offsets)
    np.testing.assert_array_equal(e.verts, g.verts)
    np.testing.assert_array_equal(e.positions, m.positions)
    np.testing.assert_array_equal(e.vertex_map, np.arange(m.num_vertices))
    want = sorted((min(a, b), max(a, b)) for a, b in m.crease_verts)
    assert [tuple(c) for c in e.crease_verts] == want


def test_regular_torus_has_nothing_extraordinary():
    e = S.extract(G.torus_cage(n=8), rings=2)
    assert e.vertex_map.size == 0 and e.face_map.size == 0 and e.verts.size == 0


def test_one_interior_seed_one_and_two_rings():
    m = _grid()
    seed = np.zeros(m.num_vertices, np.uint8)
    seed[_vid(2, 2)] = 1
    e = S.extract(m, rings=1, seed=seed)
    # the four quads around (2, 2) and the 3 x 3 block of their corners
    assert sorted(e.face_map.tolist()) == [1 * 4 + 1, 1 * 4 + 2, 2 * 4 + 1, 2 * 4 + 2]
    assert e.vertex_map.tolist() == sorted(_vid(i, j) for i in (1, 2, 3) for j in (1, 2, 3))
    assert e.offsets.tolist() == [0, 4, 8, 12, 16]
    e2 = S.extract(m, rings=2, seed=seed)
    assert e2.face_map.size == 16 and e2.vertex_map.size == 25


def test_default_seed_on_a_grid_is_the_boundary():
    """Boundary vertices have 1 or 2 incident faces: with one ring the twelve
    faces touching the boundary are kept, and every vertex but the centre."""
    e = S.extract(_grid(), rings=1)
    assert e.face_map.size == 12
    assert e.vertex_map.tolist() == [v for v in range(25) if v != _vid(2, 2)]


def test_creases_follow_the_extracted_edges():
    m = _grid()
    m.crease_verts = np.array([[_vid(2, 2), _vid(2, 3)], [_vid(0, 0), _vid(0, 1)]], np.int32)
    m.crease_sharp = np.array([1.5, 2.0], np.float32)
    seed = np.zeros(m.num_vertices, np.uint8)
    seed[_vid(2, 2)] = 1
    e = S.extract(m, rings=1, seed=seed)
    new = {int(v): i for i, v in enumerate(e.vertex_map)}
    a, b = new[_vid(2, 2)], new[_vid(2, 3)]
    assert [tuple(c) for c in e.crease_verts] == [(min(a, b), max(a, b))]
    assert e.crease_sharp.tolist() == [1.5]


def test_refining_the_extraction_matches_the_uniform_refinement_near_the_seed():
    """With one ring every face around the seed is extracted, so one
    Catmull-Clark level gives the seed's vertex point, its faces' face points
    and its edges' edge points exactly as the whole cage does."""
    m = _grid(bumpy=True)
    s = _vid(2, 2)
    seed = np.zeros(m.num_vertices, np.uint8)
    seed[s] = 1
    e = S.extract(m, rings=1, seed=seed)
    sub = G.Mesh(positions=e.positions, verts=e.verts, offsets=e.offsets, name="extracted")
    full = refine(m, "cc", 1)
    part = refine(sub, "cc", 1)
    V, F = m.num_vertices, m.num_faces
    Vs, Fs = sub.num_vertices, sub.num_faces
    ns = int(np.flatnonzero(e.vertex_map == s)[0])
    np.testing.assert_allclose(part[1].positions[ns], full[1].positions[s], atol=1e-12)
    for k, f in enumerate(e.face_map):
        if s in m.face_list()[f]:
            np.testing.assert_allclose(part[1].positions[Vs + k], full[1].positions[V + f], atol=1e-12)
    # edge points: match the edges at the seed through the two edge lists
    fe = {tuple(x): i for i, x in enumerate(full[0].edges.tolist())}
    for i, (lo, hi) in enumerate(part[0].edges.tolist()):
        a, b = int(e.vertex_map[lo]), int(e.vertex_map[hi])
        if s in (a, b):
            j = fe[(min(a, b), max(a, b))]
            np.testing.assert_allclose(part[1].positions[Vs + Fs + i], full[1].positions[V + F + j], atol=1e-12)


def test_rings_must_be_positive():
    with pytest.raises(ValueError):
        S.extract(_grid(), rings=0)


def _smooth_cage(seed=24, level=2):
    return G.cc_cage(seed=seed, level=level, crease_frac=0.0)


def test_adaptive_with_wide_rings_is_uniform_refinement():
    """Rings wide enough to reach every face: every level's extraction is the
    whole level, so the adaptive chain is the uniform refinement, bit for bit
    in FP64."""
    m = _smooth_cage(level=1)
    ad = S.adaptive(m, 3, rings=50)
    uni = refine(m, "cc", 3)
    assert len(ad) == 3
    for k, a in enumerate(ad):
        assert a.region.vertex_map.tolist() == list(range(uni[k].num_vertices))
        np.testing.assert_array_equal(a.refined.verts, uni[k + 1].verts)
        np.testing.assert_array_equal(a.refined.positions, uni[k + 1].positions)


def _seed_chain(ad, seeds):
    """Ids of the cage's seed vertices on every refined region (old vertices
    keep their ids; the extraction renumbers by rank)."""
    ids, out = np.asarray(seeds), []
    for a in ad:
        vm = a.region.vertex_map
        pos = np.searchsorted(vm, ids)
        assert np.all(vm[pos] == ids), "a seed left the region"
        ids = pos
        out.append(ids.copy())
    return out


@pytest.mark.parametrize("rings", [1, 2])
def test_adaptive_keeps_the_seeds_exact(rings):
    """A seed's vertex point needs only its star, whose faces and corners the
    extraction keeps at every level; refined again and again, the seeds end
    where the uniform refinement puts them (same FP64 stencils). The region
    stays a fraction of the uniform level."""
    m = _smooth_cage()
    L = 3
    ad = S.adaptive(m, L, rings=rings)
    uni = refine(m, "cc", L)
    M = S.mesh_matrix(m)
    seeds = np.flatnonzero(np.asarray(M @ np.ones(M.shape[1])).ravel() != 4)
    assert seeds.size > 0
    for k, ids in enumerate(_seed_chain(ad, seeds)):
        np.testing.assert_allclose(ad[k].refined.positions[ids], uni[k + 1].positions[seeds], rtol=0, atol=1e-12)
        assert ad[k].refined.num_faces <= uni[k + 1].num_faces
    assert ad[-1].refined.num_faces < (0.5 if rings == 1 else 1.0) * uni[L].num_faces


def test_adaptive_seed_flags_follow_the_old_vertices():
    m = _smooth_cage()
    ad = S.adaptive(m, 2, rings=1)
    for a in ad:
        nv = a.region.vertex_map.size
        assert not a.seed[nv:].any()  # new points never seed
    M = S.mesh_matrix(m)
    n0 = int((np.asarray(M @ np.ones(M.shape[1])).ravel() != 4).sum())
    assert int(ad[0].seed.sum()) == n0 and int(ad[1].seed.sum()) == n0


def test_pinch_closing_joins_regions_touching_at_a_vertex():
    """Two seeds on a grid diagonal two apart: their one-ring regions meet
    at one vertex only, which the plain extraction leaves with two fans; the
    closed selection adds that vertex's whole star, and the two regions
    become one manifold patch."""
    m = _grid()
    seed = np.zeros(m.num_vertices, np.uint8)
    seed[_vid(1, 1)] = 1
    seed[_vid(3, 3)] = 1
    x, q = S.select(m, 1, seed)
    assert q.sum() == 8  # two 2 x 2 blocks of quads sharing the vertex (2, 2)
    xc, qc = S.select(m, 1, seed, close=True)
    assert qc.sum() == 10 and qc[1 * 4 + 2] and qc[2 * 4 + 1]  # the two faces around (2, 2) between the blocks
    assert xc.sum() == x.sum() + 2
    faces = m.face_list()
    star = [[f for f, c in enumerate(faces) if v in c] for v in range(m.num_vertices)]
    assert not any(S._pinched(faces, star, qc, v) for v in np.flatnonzero(xc))
