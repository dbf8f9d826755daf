"""Loop with creases (the Catmull-Clark crease rules of Sec. 3.3 on Loop's
points) through the C ABI against the FP64 oracle: topology, edge
enumeration and inherited sharpness bit for bit, positions within the
tolerance, at every level; the last step from two levels down where the
creases have died out by then; the per-level build gives the same bits."""
import numpy as np
import pytest

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err
from tests.test_gpu_parity import _compare, _gpu

pytestmark = pytest.mark.gpu


def _creased(m, n, smax, seed):
    rng = np.random.default_rng(seed)
    cv, cs = G.tag_creases(m.offsets, m.verts, m.face_order, n, smax, rng)
    return G.Mesh(positions=m.positions, verts=m.verts, face_order=3, crease_verts=cv, crease_sharp=cs,
                  name=m.name + "-creased")


def _all_sharp(m, sigma):
    e = G.mesh_edges(None, m.verts, 3).astype(np.int32)
    return G.Mesh(positions=m.positions, verts=m.verts, face_order=3, crease_verts=e,
                  crease_sharp=np.full(len(e), sigma, np.float32), name=m.name + "-sharp")


def _octahedron_equator(sigma):
    P = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
    F = [[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4], [1, 0, 5], [2, 1, 5], [3, 2, 5], [0, 3, 5]]
    ring = np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32)
    return G.Mesh(positions=P, verts=np.array(F, np.int32).reshape(-1), face_order=3, crease_verts=ring,
                  crease_sharp=np.full(4, sigma, np.float32), name="octahedron-equator")


CAGES = {
    "closed_deep": lambda: _creased(G.tri_cage(seed=18, level=2, hole_frac=0.0), 120, 7.0, 41),
    "holes_deep": lambda: _creased(G.tri_cage(seed=19, level=2, hole_frac=0.08), 120, 7.0, 42),
    "grid": lambda: _creased(G.grid_patch(7, 5, tri=True), 30, 3.0, 43),
    "tet_sharp": lambda: _all_sharp(G.tetrahedron(), 10.0),
    "tet_semisharp": lambda: _all_sharp(G.tetrahedron(), 0.6),
    "equator": lambda: _octahedron_equator(2.5),
}


@pytest.mark.parametrize("cage", list(CAGES))
def test_loop_creases_every_level(oracle_mod, cage):
    _compare(CAGES[cage](), "loop", 4, oracle_mod, label=f"loop-creases-{cage}")


@pytest.mark.parametrize("cage", ["closed_deep", "holes_deep", "grid"])
def test_loop_creases_final_level_only(oracle_mod, cage):
    """Only the last level asked for: with sharpness below L-1 everywhere the
    last step runs from two levels down; the result still matches."""
    m = CAGES[cage]()
    L = 5 if cage == "grid" else 4
    print(f"[loop creases] {cage} final level {L}", flush=True)
    outs, _ = api.refine(m, "loop", L)
    ref = oracle_mod.refine(m, "loop", L)[L]
    np.testing.assert_array_equal(outs[L]["face_verts"].cpu().numpy(), ref.verts)
    assert normwise_err(outs[L]["positions"].cpu().numpy(), ref.positions) <= POS_TOL


@pytest.mark.parametrize("cage", ["holes_deep", "equator"])
def test_loop_creases_rebuild_matches_carried(oracle_mod, cage):
    m = CAGES[cage]()
    a, _ = _gpu(m, "loop", 3)
    b, _ = _gpu(m, "loop", 3, flags=_lib.FLAG_REBUILD_EACH_LEVEL)
    for k in range(1, 4):
        for key in a[k]:
            np.testing.assert_array_equal(a[k][key], b[k][key], err_msg=f"level {k} {key}")


def test_sqrt3_creases_rejected():
    m = _all_sharp(G.tetrahedron(), 1.0)
    assert api.plan_status(m, "sqrt3", levels=1) == _lib.INVALID_ARG
