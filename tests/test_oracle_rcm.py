"""Pins of the reverse Cuthill-McKee oracle (Sec. 4.5)."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from oracle import rcm as R
from paper_1809_06047_amd import meshgen as G


def _strip(n):
    """A 1 x n strip of quads: vertices (i, 0) = i, (i, 1) = n + 1 + i."""
    faces = [[i, i + 1, n + 2 + i, n + 1 + i] for i in range(n)]
    P = np.array([[i, j, 0] for j in range(2) for i in range(n + 1)], np.float32)
    return G.Mesh(positions=P, verts=np.array(faces, np.int32).reshape(-1), face_order=4, name="strip")


def _shuffled(m, seed):
    rng = np.random.default_rng(seed)
    p = rng.permutation(m.num_vertices)          # old -> new
    inv = np.argsort(p)
    faces = [[int(p[v]) for v in f] for f in m.face_list()]
    order = rng.permutation(len(faces))
    faces = [faces[i] for i in order]
    return G.Mesh(positions=np.asarray(m.positions)[inv], verts=np.array(faces, np.int32).reshape(-1),
                  face_order=len(faces[0]), name=m.name + "-shuffled")


def test_strip_by_hand():
    """Corner 0 has degree 2 (the smallest id among the four corners); BFS
    from it visits 1 and 4 (degree 3 and 2: 4 first), then ... ; reversed,
    the strip is numbered column by column from the far end."""
    m = _strip(3)  # vertices 0..3 bottom, 4..7 top
    vperm, fperm = R.rcm_order(m)
    # Cuthill-McKee from 0: 0, then its neighbours 4 (deg 2) and 1 (deg 3): 0 4 1, then 1's 5 and 2 ...
    assert list(vperm[::-1]) == [0, 4, 1, 5, 2, 6, 3, 7]
    # faces by their smallest new corner: the far face first
    assert list(fperm) == [2, 1, 0]


def test_is_a_permutation_and_lowers_the_bandwidth():
    m = _shuffled(G.grid_patch(12, 9), seed=3)
    vperm, fperm = R.rcm_order(m)
    assert sorted(vperm.tolist()) == list(range(m.num_vertices))
    assert sorted(fperm.tolist()) == list(range(m.num_faces))
    b0, b1 = R.bandwidth(m), R.bandwidth(m, vperm)
    assert b1 < b0 / 4
    # the grid's best ordering (row by row along the short side) has bandwidth 11;
    # RCM stays within a small factor, like scipy's independent implementation
    V = m.num_vertices
    rows, cols = [], []
    for f in m.face_list():
        for j in range(len(f)):
            rows += [f[j], f[(j + 1) % len(f)]]
            cols += [f[(j + 1) % len(f)], f[j]]
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(V, V))
    ref = reverse_cuthill_mckee(A, symmetric_mode=True)
    assert b1 <= 2 * R.bandwidth(m, np.asarray(ref))


def test_disconnected_components_each_start_at_their_smallest_degree():
    a = _strip(2)
    b = _strip(1)
    faces = a.face_list() + [[v + a.num_vertices for v in f] for f in b.face_list()]
    P = np.concatenate([a.positions, b.positions])
    m = G.Mesh(positions=P, verts=np.array(faces, np.int32).reshape(-1), face_order=4, name="two")
    vperm, _ = R.rcm_order(m)
    cm = list(vperm[::-1])
    # degrees: every corner of the single quad has degree 2; the strip's ends too.
    # The first start is vertex 0 (degree 2, smallest id); its component comes first.
    assert cm[:6] == [0, 3, 1, 4, 2, 5]
    assert sorted(cm[6:]) == list(range(6, 10))
