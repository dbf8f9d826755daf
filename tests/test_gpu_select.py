"""Selective subdivision's extraction step (Sec. 3.4) through the C ABI,
against the oracle's M' = X M X-ring and P' = X P: integer outputs and copied
positions bit for bit, creases as a set; then the extracted cage refined on
the GPU against the oracle refining the oracle's extraction."""
import numpy as np
import pytest
import torch

from oracle import refine as oracle_refine
from oracle import select as S
from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err
from tests.test_gpu_adjoint import _grid_with_creases

pytestmark = pytest.mark.gpu


def _quad_level1():
    """Level 1 of a creased mixed cage: a uniform quad cage with creases."""
    lv = oracle_refine(G.cc_cage(seed=24, level=2), "cc", 1)[1]
    return G.Mesh(positions=lv.positions.astype(np.float32), verts=lv.verts, face_order=4,
                  crease_verts=lv.crease_verts, crease_sharp=lv.crease_sharp.astype(np.float32), name="quad-l1")


CAGES = {
    "mixed_creases": lambda: G.cc_cage(seed=24, level=2),
    "quads_creases": _quad_level1,
    "tri_holes": lambda: G.tri_cage(seed=19, level=2, hole_frac=0.08),
    "grid_creases": lambda: _grid_with_creases(23),
}


def _seed(kind, V):
    if kind == "extraordinary":
        return None
    rng = np.random.default_rng(7)
    if kind == "sparse":
        return (rng.random(V) < 0.03).astype(np.uint8)
    if kind == "all":
        return np.ones(V, np.uint8)
    return np.zeros(V, np.uint8)


def _run(m, seed, rings):
    r = api.Refiner(m, "cc" if m.face_order != 3 or m.offsets is not None else "loop", 1)
    r.plan()
    t = None if seed is None else torch.from_numpy(seed).cuda()
    return api.extract_region(r, t, rings)


@pytest.mark.parametrize("rings", [1, 2, 3])
@pytest.mark.parametrize("seed_kind", ["extraordinary", "sparse", "all", "none"])
@pytest.mark.parametrize("cage", list(CAGES))
def test_extraction_equals_oracle(cage, seed_kind, rings):
    m = CAGES[cage]()
    seed = _seed(seed_kind, m.num_vertices)
    print(f"[select] {cage} seed={seed_kind} rings={rings}", flush=True)
    got = _run(m, seed, rings)
    torch.cuda.synchronize()
    want = S.extract(m, rings=rings, seed=seed)
    np.testing.assert_array_equal(got["vertex_map"].cpu().numpy(), want.vertex_map)
    np.testing.assert_array_equal(got["face_map"].cpu().numpy(), want.face_map)
    np.testing.assert_array_equal(got["face_verts"].cpu().numpy(), want.verts)
    if got["face_offsets"] is not None:
        np.testing.assert_array_equal(got["face_offsets"].cpu().numpy(), want.offsets)
    else:
        order = m.face_order
        np.testing.assert_array_equal(want.offsets, np.arange(want.face_map.size + 1) * order)
    np.testing.assert_array_equal(got["positions"].cpu().numpy(), want.positions)
    if got["crease_verts"] is None:
        assert want.crease_verts.shape[0] == 0
    else:
        cv = np.sort(got["crease_verts"].cpu().numpy(), axis=1)
        cs = got["crease_sharpness"].cpu().numpy()
        order = np.lexsort((cv[:, 1], cv[:, 0]))
        np.testing.assert_array_equal(cv[order], want.crease_verts)
        np.testing.assert_array_equal(cs[order], want.crease_sharp)
    if seed_kind == "none":
        assert got["mesh"] is None and want.vertex_map.size == 0


@pytest.mark.parametrize("cage", ["mixed_creases", "quads_creases", "grid_creases"])
def test_refining_the_extraction(oracle_mod, cage):
    """The extracted cage is a cage like any other: planned and refined on the
    GPU it matches the oracle refining the oracle's extraction. Where two
    selected regions touch at a single vertex the extraction is not manifold
    there; then both sides reject it with the same status."""
    m = CAGES[cage]()
    got = _run(m, None, 1)
    want = S.extract(m, rings=1)
    sub = G.Mesh(positions=want.positions, verts=want.verts, offsets=want.offsets,
                 crease_verts=want.crease_verts if want.crease_verts.shape[0] else None,
                 crease_sharp=want.crease_sharp if want.crease_verts.shape[0] else None, name="region")
    L = 3
    status = oracle_mod.status_of(sub, "cc")
    print(f"[select] refine the {cage} extraction: oracle status {status}", flush=True)
    if status != 0:
        assert api.plan_status(got["mesh"], "cc", levels=L) == status
        return
    r = api.Refiner(got["mesh"], "cc", L)
    r.plan()
    outs = r.run()
    torch.cuda.synchronize()
    ref = oracle_mod.refine(sub, "cc", L)
    np.testing.assert_array_equal(outs[L]["face_verts"].cpu().numpy(), ref[L].verts)
    assert normwise_err(outs[L]["positions"].cpu().numpy(), ref[L].positions) <= POS_TOL


def test_selection_needs_the_plan():
    m = G.cc_cage(seed=24, level=2)
    r = api.Refiner(m, "cc", 1)
    with pytest.raises(_lib.SubdivError) as e:
        api.extract_region(r, None, 1)  # not planned yet
    assert e.value.status == _lib.STATE
    r.plan()
    with pytest.raises(_lib.SubdivError) as e:
        api.extract_region(r, None, 0)
    assert e.value.status == _lib.INVALID_ARG
