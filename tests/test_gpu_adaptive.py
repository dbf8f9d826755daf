"""Feature-adaptive refinement on the GPU (Sec. 3.4 level after level:
select around the seeds with pinches closed, extract, refine the region one
Catmull-Clark level, carry the seeds) against the oracle's adaptive loop:
maps and topology bit for bit, positions within tolerance, at every level;
the seeds end where the uniform refinement puts them."""
import numpy as np
import pytest
import torch

from oracle import select as S
from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu

CAGES = {
    "mixed": lambda: G.cc_cage(seed=24, level=2, crease_frac=0.0),
    "cube": lambda: G.cube(),
    "grid": lambda: G.grid_patch(6, 5, z_fn=lambda x, y: 0.2 * np.sin(x) * np.cos(y)),
}


@pytest.mark.parametrize("cage,levels,rings", [("mixed", 4, 1), ("mixed", 3, 2), ("cube", 4, 1), ("grid", 3, 1)])
def test_adaptive_matches_oracle(cage, levels, rings):
    m = CAGES[cage]()
    print(f"[adaptive] {m.name} L={levels} rings={rings}", flush=True)
    got = api.adaptive_refine(m, levels, rings)
    torch.cuda.synchronize()
    ref = S.adaptive(m, levels, rings)
    assert len(got) == len(ref)
    for k, (g, o) in enumerate(zip(got, ref)):
        np.testing.assert_array_equal(g["vertex_map"].cpu().numpy(), o.region.vertex_map, err_msg=f"level {k}")
        np.testing.assert_array_equal(g["face_map"].cpu().numpy(), o.region.face_map, err_msg=f"level {k}")
        np.testing.assert_array_equal(g["region"].verts.cpu().numpy(), o.region.verts, err_msg=f"level {k}")
        fin = g["mesh"]
        np.testing.assert_array_equal(fin.verts.cpu().numpy(), o.refined.verts, err_msg=f"level {k + 1}")
        err = normwise_err(fin.positions.cpu().numpy(), o.refined.positions)
        assert err <= POS_TOL, f"level {k + 1}: {err:.2e}"


def test_adaptive_seeds_match_uniform_refinement():
    m = CAGES["mixed"]()
    L = 4
    got = api.adaptive_refine(m, L, 1)
    uni, _ = api.refine(m, "cc", L, keep="all")
    M = S.mesh_matrix(m)
    seeds = np.flatnonzero(np.asarray(M @ np.ones(M.shape[1])).ravel() != 4)
    ids = seeds
    for k, g in enumerate(got):
        vm = g["vertex_map"].cpu().numpy()
        ids = np.searchsorted(vm, ids)
        a = g["mesh"].positions.cpu().numpy()[ids]
        b = uni[k + 1]["positions"].cpu().numpy()[seeds]
        scale = np.abs(uni[k + 1]["positions"].cpu().numpy()).max()
        assert np.abs(a - b).max() / scale <= POS_TOL, k


def test_pinch_closing_on_the_gpu():
    """The grid case of the oracle pin: two regions touching at one vertex are
    joined by that vertex's star, and the extraction is planned (manifold)."""
    m = G.grid_patch(4, 4)
    seed = np.zeros(m.num_vertices, np.uint8)
    seed[1 * 5 + 1] = 1
    seed[3 * 5 + 3] = 1
    r = api.Refiner(m, "cc", 1)
    r.plan()
    ds = torch.from_numpy(seed).cuda()
    plain = api.extract_region(r, ds, 1)
    assert plain["face_map"].numel() == 8
    with pytest.raises(_lib.SubdivError) as e:  # the plain extraction is pinched
        api.Refiner(plain["mesh"], "cc", 1).plan()
    assert e.value.status == _lib.NONMANIFOLD
    closed = api.extract_region(r, ds, 1, close_pinches=True)
    ref = S.extract(m, 1, seed, close=True)
    np.testing.assert_array_equal(closed["face_map"].cpu().numpy(), ref.face_map)
    np.testing.assert_array_equal(closed["vertex_map"].cpu().numpy(), ref.vertex_map)
    np.testing.assert_array_equal(closed["seed_flags"].cpu().numpy(), seed[ref.vertex_map])
    api.Refiner(closed["mesh"], "cc", 1).plan()
