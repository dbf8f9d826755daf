"""The library's reverse Cuthill-McKee reordering (a host routine of the C ABI,
so these run without a GPU) against the oracle, permutation for permutation."""
import numpy as np
import pytest

from oracle import rcm as R
from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.test_oracle_rcm import _shuffled, _strip


def _two_components():
    a, b = _strip(2), _strip(1)
    faces = a.face_list() + [[v + a.num_vertices for v in f] for f in b.face_list()]
    return G.Mesh(positions=np.concatenate([a.positions, b.positions]),
                  verts=np.array(faces, np.int32).reshape(-1), face_order=4, name="two")


CASES = {
    "strip": lambda: _strip(5),
    "shuffled_grid": lambda: _shuffled(G.grid_patch(12, 9), seed=3),
    "mixed_cage": lambda: G.cc_cage(seed=24, level=2),
    "tri_holes": lambda: G.tri_cage(seed=19, level=2, hole_frac=0.08),
    "two_components": _two_components,
}


@pytest.mark.parametrize("case", list(CASES))
def test_rcm_equals_oracle(case):
    m = CASES[case]()
    got, vperm, fperm = api.rcm_reorder(m)
    wv, wf = R.rcm_order(m)
    np.testing.assert_array_equal(vperm, wv)
    np.testing.assert_array_equal(fperm, wf)
    # the reordered cage is the same surface: positions and faces permuted
    newid = np.empty(m.num_vertices, np.int64)
    newid[vperm] = np.arange(m.num_vertices)
    faces = m.face_list()
    assert got.face_list() == [[int(newid[v]) for v in faces[f]] for f in fperm]
    np.testing.assert_array_equal(got.positions, np.asarray(m.positions)[vperm])
    assert R.bandwidth(got) == R.bandwidth(m, vperm)


def test_rcm_rejects_bad_indices():
    m = _strip(2)
    bad = G.Mesh(positions=m.positions, verts=np.where(m.verts == 3, 99, m.verts).astype(np.int32),
                 face_order=4, name="bad")
    with pytest.raises(_lib.SubdivError) as e:
        api.rcm_reorder(bad)
    assert e.value.status == _lib.INVALID_ARG
