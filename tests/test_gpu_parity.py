"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Topology (face tables, edge enumeration, crease sharpness) must be bit-exact;
positions within 1e-5 normwise relative error at every level.
"""
import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, crease_table, level_edges, normwise_err

pytestmark = pytest.mark.gpu


def _gpu(mesh, scheme, levels, flags=0):
    outs, r = api.refine(mesh, scheme, levels, flags=flags, keep="all", edges=True, creases=True)
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs], r


def _compare(mesh, scheme, levels, oracle_mod, flags=0, label=""):
    print(f"[parity] {label} {mesh.name} scheme={scheme} levels={levels} flags={flags}", flush=True)
    ref = oracle_mod.refine(mesh, scheme, levels)
    got, r = _gpu(mesh, scheme, levels, flags)
    order = 4 if scheme == "cc" else 3
    errs = []
    for k in range(1, levels + 1):
        g, o = got[k], ref[k]
        info = r.level_info(k)
        assert (info["V"], info["F"], info["H"]) == (o.num_vertices, o.num_faces, o.verts.size), k
        np.testing.assert_array_equal(g["face_verts"], o.verts, err_msg=f"{label} topology level {k}")
        np.testing.assert_array_equal(g["edge_verts"], ref[k - 1].edges, err_msg=f"{label} edges of level {k-1}")
        e = normwise_err(g["positions"], o.positions)
        errs.append(e)
        assert e <= POS_TOL, f"{label} level {k}: positions err {e:.3e}"
        if "crease_sharpness" in g:
            sig = crease_table(o, level_edges(o.verts, order))
            np.testing.assert_array_equal(g["crease_sharpness"], sig, err_msg=f"{label} creases level {k}")
    print(f"[parity] {label} errors per level: " + " ".join(f"{x:.2e}" for x in errs), flush=True)
    return got


def test_cc_torus_levels_1_to_4(oracle_mod):
    _compare(G.torus_cage(), "cc", 4, oracle_mod, label="torus")


def test_cc_mixed_cage_with_creases(oracle_mod):
    m = G.cc_cage(seed=11, level=3)
    assert m.num_creases > 0
    _compare(m, "cc", 4, oracle_mod, label="mixed+creases")


@pytest.mark.parametrize("cage", ["mixed", "holes"])
def test_cc_creases_alive_on_deep_levels(oracle_mod, cage):
    """Sharpness up to 7 keeps creases alive past level 3, so the
    corner-class kernels of levels >= 3 apply the crease rules at interior,
    boundary, dart, crease and corner vertices."""
    rng = np.random.default_rng(16)
    if cage == "mixed":
        m = G.cc_cage(seed=16, level=2, crease_frac=0.2, smax=7.0)
    else:
        m = G.tri_cage(seed=17, level=2, hole_frac=0.05)
        m.crease_verts, m.crease_sharp = G.tag_creases(m.offsets, m.verts, m.face_order, 90, 7.0, rng)
    ref = oracle_mod.refine(m, "cc", 4)
    alive = crease_table(ref[4], level_edges(ref[4].verts, 4))
    assert (alive > 0).sum() > 0, "the cage must still carry creases at level 4"
    _compare(m, "cc", 5, oracle_mod, label=f"deep-creases-{cage}")


@pytest.mark.parametrize("cage", ["mixed", "holes"])
def test_cc_rebuild_each_level_matches_carried_adjacency(oracle_mod, cage):
    """The paper's per-level mapped M M^T build (explicit kernels on every
    level) and the closed-form carry-over from the parent level give the same
    canonical ids: topology, edge enumeration and crease sharpness agree bit
    for bit; positions differ only by summation order."""
    if cage == "mixed":
        m = G.cc_cage(seed=12, level=2)
    else:
        m = G.tri_cage(seed=15, level=2, hole_frac=0.05)
    _compare(m, "cc", 4, oracle_mod, flags=_lib.FLAG_REBUILD_EACH_LEVEL, label="rebuild")
    a, _ = _gpu(m, "cc", 4)
    b, _ = _gpu(m, "cc", 4, flags=_lib.FLAG_REBUILD_EACH_LEVEL)
    for k in range(1, 5):
        for key in a[k]:
            if key == "positions":
                assert normwise_err(a[k][key], b[k][key]) <= POS_TOL
            else:
                np.testing.assert_array_equal(a[k][key], b[k][key], err_msg=f"level {k} {key}")


@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
@pytest.mark.parametrize("cage", ["icosphere", "holes", "fan"])
def test_triangle_carried_adjacency_matches_rebuild(oracle_mod, cage, scheme):
    """Loop and sqrt(3) levels carried over in closed form (counts, one scan,
    twins and ids per face) against the per-level mapped M M^T build:
    topology, edge enumeration and positions agree bit for bit (the carried
    ring starts are the canonical ones the build picks)."""
    m = {"icosphere": lambda: G.tri_cage(seed=18, level=2, hole_frac=0.0),
         "holes": lambda: G.tri_cage(seed=19, level=2, hole_frac=0.08),
         "fan": lambda: _bipyramid(12, closed=False)}[cage]()
    _compare(m, scheme, 4, oracle_mod, label=f"{scheme}-carried-{cage}")
    a, _ = _gpu(m, scheme, 4)
    b, _ = _gpu(m, scheme, 4, flags=_lib.FLAG_REBUILD_EACH_LEVEL)
    for k in range(1, 5):
        for key in a[k]:
            np.testing.assert_array_equal(a[k][key], b[k][key], err_msg=f"level {k} {key}")


def _pillow():
    """Two triangles on the same three vertices, opposite orientations: every
    edge is shared by the same two faces."""
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    return G.Mesh(positions=P, verts=np.array([0, 1, 2, 0, 2, 1], np.int32), face_order=3, name="pillow")


@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_two_faces_sharing_every_edge(oracle_mod, scheme):
    """A pillow refines under Catmull-Clark at any depth; under Loop and
    sqrt(3) its first level has edges on four faces, so only one level is
    valid and the plan rejects deeper refinement as the oracle does."""
    assert oracle_mod.status_of(_pillow(), scheme) == 0
    if scheme == "cc":
        _compare(_pillow(), scheme, 3, oracle_mod, label="pillow-cc")
        return
    _compare(_pillow(), scheme, 1, oracle_mod, label=f"pillow-{scheme}")
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.refine(_pillow(), scheme, 2)
    assert api.plan_status(_pillow(), scheme, levels=2) == _lib.NONMANIFOLD


@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
def test_triangle_schemes_with_holes(oracle_mod, scheme):
    m = G.tri_cage(seed=13, level=3, hole_frac=0.02)
    _compare(m, scheme, 3, oracle_mod, label="holes")


@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_open_grid_patches(oracle_mod, scheme):
    rng = np.random.default_rng(4)
    m = G.grid_patch(7, 5, tri=(scheme != "cc"), z_fn=lambda x, y: rng.normal(0, 0.2, x.shape))
    _compare(m, scheme, 3, oracle_mod, label="grid")
    if scheme == "cc":
        t = G.grid_patch(6, 4, tri=True, z_fn=lambda x, y: rng.normal(0, 0.2, x.shape))
        _compare(t, "cc", 3, oracle_mod, label="tri-grid-cc")


def _prism(n, h=1.0):
    """Closed n-gon prism: two n-gons and n quads (general polygon cage)."""
    a = 2 * np.pi * np.arange(n) / n
    P = np.concatenate([np.stack([np.cos(a), np.sin(a), np.zeros(n)], 1),
                        np.stack([np.cos(a), np.sin(a), np.full(n, h)], 1)]).astype(np.float32)
    faces = [list(range(n - 1, -1, -1)), list(range(n, 2 * n))]
    for i in range(n):
        j = (i + 1) % n
        faces.append([i, j, n + j, n + i])
    off = np.cumsum([0] + [len(f) for f in faces]).astype(np.int32)
    return G.Mesh(positions=P, verts=np.array(sum(faces, []), np.int32), offsets=off, name=f"prism{n}")


@pytest.mark.parametrize("n", [3, 5, 6, 9])
def test_general_polygon_cages(oracle_mod, n):
    _compare(_prism(n), "cc", 3, oracle_mod, label=f"prism{n}")


def _bipyramid(n, closed=True):
    """Two apexes over an n-gon ring (valence n at the apexes); the open
    variant keeps only the upper fan, so its apex has valence n and the ring
    is a boundary."""
    a = 2 * np.pi * np.arange(n) / n
    ring = np.stack([np.cos(a), np.sin(a), 0.1 * np.sin(3 * a)], 1)
    P = np.concatenate([ring, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]]).astype(np.float32)
    top, bot = n, n + 1
    faces = [[i, (i + 1) % n, top] for i in range(n)]
    if closed:
        faces += [[(i + 1) % n, i, bot] for i in range(n)]
    else:
        P = P[:n + 1]
    return G.Mesh(positions=P, verts=np.array(faces, np.int32).reshape(-1), face_order=3,
                  name=f"bipyramid{n}" if closed else f"fan{n}")


@pytest.mark.parametrize("scheme", ["cc", "loop", "sqrt3"])
def test_high_valence_vertices(oracle_mod, scheme):
    """Valence 12 at the apexes takes the general (memory) row path of the
    cage build; the ring vertices (valence 4 or 3) take the register path."""
    _compare(_bipyramid(12), scheme, 3, oracle_mod, label=f"bipyramid12-{scheme}")
    _compare(_bipyramid(12, closed=False), scheme, 3, oracle_mod, label=f"fan12-{scheme}")


def test_single_faces(oracle_mod):
    quad = G.Mesh(positions=np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0.5], [0, 1, 0]], np.float32),
                  verts=np.arange(4, dtype=np.int32), face_order=4, name="quad")
    tri = G.Mesh(positions=np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.5]], np.float32),
                 verts=np.arange(3, dtype=np.int32), face_order=3, name="tri")
    _compare(quad, "cc", 3, oracle_mod, label="one-quad")
    for s in ("cc", "loop", "sqrt3"):
        _compare(tri, s, 3, oracle_mod, label="one-tri")


def test_deterministic_repeat():
    m = G.cc_cage(seed=14, level=3)
    a, _ = _gpu(m, "cc", 4)
    b, _ = _gpu(m, "cc", 4)
    for k in range(1, 5):
        for key in a[k]:
            np.testing.assert_array_equal(a[k][key], b[k][key])


def _tri(P, F):
    return G.Mesh(positions=np.asarray(P, np.float32), verts=np.array(F, np.int32).reshape(-1), face_order=3)


def test_status_codes_match_oracle(oracle_mod):
    P = np.zeros((6, 3))
    c = G.cube()
    e = G.mesh_edges(None, c.verts, 4)[:1].astype(np.int32)
    cases = [
        (G.cube(), "loop"),
        (_tri(P, [[0, 1, 1]]), "cc"),
        (G.Mesh(positions=np.zeros((4, 3), np.float32), verts=np.array([0, 1, 2, 3, 2], np.int32),
                offsets=np.array([0, 2, 5], np.int32)), "cc"),
        (_tri(P, [[0, 1, 7]]), "cc"),
        (_tri(P, [[0, 1, 2]]), "cc"),
        (_tri(P[:5], [[0, 1, 2], [1, 0, 3], [0, 1, 4]]), "cc"),
        (_tri(P[:4], [[0, 1, 2], [0, 1, 3]]), "cc"),
        (_tri(P[:5], [[0, 1, 2], [0, 3, 4]]), "cc"),
        (G.Mesh(positions=c.positions, verts=c.verts, face_order=4, crease_verts=np.array([[0, 7]], np.int32),
                crease_sharp=np.array([1.0], np.float32)), "cc"),
        (G.Mesh(positions=c.positions, verts=c.verts, face_order=4, crease_verts=e,
                crease_sharp=np.array([-1.0], np.float32)), "cc"),
        (G.Mesh(positions=c.positions, verts=c.verts, face_order=4, crease_verts=np.concatenate([e, e[:, ::-1]]),
                crease_sharp=np.array([1.0, 2.0], np.float32)), "cc"),
        (G.cube(), "cc"),
    ]
    for i, (m, s) in enumerate(cases):
        want = oracle_mod.status_of(m, s)
        got = api.plan_status(m, s)
        assert got == want, f"case {i}: gpu {got} oracle {want}"
        if i < len(cases) - 1:
            assert got != 0


@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
def test_final_buffer_shared_with_level_L_minus_2(scheme):
    """The step before the last also writes the final points of its level's
    newest vertices (they lie in the lanes that form their rings). A caller may
    hand level L-2's positions the same buffer as the final level's (level L-2
    is not read by the last step): the library then leaves those points to
    the last step, and the final level is the same bit for bit."""
    m = G.tri_cage(seed=19, level=2, hole_frac=0.08)
    L = 4
    print(f"[parity] {scheme} final buffer shared with level {L - 2}: {m.name} L={L}", flush=True)
    want, _ = api.refine(m, scheme, L)
    r = api.Refiner(m, scheme, L)
    r.plan()
    r._outs_struct[L - 2].positions = r.outs[L]["positions"].data_ptr()
    r.run()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(r.outs[L]["face_verts"].cpu().numpy(), want[L]["face_verts"].cpu().numpy())
    np.testing.assert_array_equal(r.outs[L]["positions"].cpu().numpy(), want[L]["positions"].cpu().numpy())


@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
@pytest.mark.parametrize("cage,levels", [(c, L) for c in ("icosphere", "holes", "fan", "bipyramid", "grid")
                                         for L in (3, 4)] + [("holes", 5), ("fan", 5), ("tri", 4), ("tri", 5)])
def test_last_step_from_two_levels_down(oracle_mod, cage, levels, scheme):
    """The last Loop or sqrt(3) step runs from level L-2 (the level L-1 was
    refined from) and level L-1's adjacency is never built. The final level
    equals the per-level path (the per-level build) bit for bit and the
    oracle within tolerance; asking for every level's face table as well
    changes nothing; the last step also writes level L-1's edge list."""
    rng = np.random.default_rng(21)
    m = {"icosphere": lambda: G.tri_cage(seed=18, level=2, hole_frac=0.0),
         "holes": lambda: G.tri_cage(seed=19, level=2, hole_frac=0.08),
         "fan": lambda: _bipyramid(12, closed=False),
         "bipyramid": lambda: _bipyramid(9),
         "grid": lambda: G.grid_patch(7, 5, tri=True, z_fn=lambda x, y: rng.normal(0, 0.2, x.shape)),
         # one triangle: every level-(L-3) wave of the steps from below is a partial one
         "tri": lambda: G.Mesh(positions=np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.5]], np.float32),
                               verts=np.arange(3, dtype=np.int32), face_order=3, name="tri")}[cage]()
    L = levels
    print(f"[parity] {scheme} last step from level {L - 2}: {m.name} L={L}", flush=True)
    outs, _ = api.refine(m, scheme, L)
    lag = {k: v.cpu().numpy() for k, v in outs[L].items()}
    per, _ = api.refine(m, scheme, L, flags=_lib.FLAG_REBUILD_EACH_LEVEL)
    np.testing.assert_array_equal(lag["face_verts"], per[L]["face_verts"].cpu().numpy())
    np.testing.assert_array_equal(lag["positions"], per[L]["positions"].cpu().numpy())
    ref = oracle_mod.refine(m, scheme, L)
    np.testing.assert_array_equal(lag["face_verts"], ref[L].verts)
    assert normwise_err(lag["positions"], ref[L].positions) <= POS_TOL
    every, _ = api.refine(m, scheme, L, keep="all")
    for k in range(1, L + 1):
        np.testing.assert_array_equal(every[k]["face_verts"].cpu().numpy(), ref[k].verts, err_msg=f"level {k}")
        assert normwise_err(every[k]["positions"].cpu().numpy(), ref[k].positions) <= POS_TOL
    np.testing.assert_array_equal(every[L]["positions"].cpu().numpy(), lag["positions"])
    with_edges, _ = api.refine(m, scheme, L, edges=True)
    np.testing.assert_array_equal(with_edges[L]["edge_verts"].cpu().numpy(), ref[L - 1].edges)
    np.testing.assert_array_equal(with_edges[L]["positions"].cpu().numpy(), lag["positions"])
