"""Batched refinement: every mesh of a batch equals the same mesh refined
alone (bit for bit) and the oracle (within tolerance)."""
import numpy as np
import pytest
import torch

from paper_1809_06047_amd import api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu


def _solo(mesh, scheme, L):
    outs, _ = api.refine(mesh, scheme, L)
    return {k: v.cpu().numpy() for k, v in outs[L].items()}


def _check_batch(oracle_mod, meshes, scheme, L, label):
    b = api.BatchRefiner(meshes, scheme, L)
    b.plan()
    outs = b.run()
    torch.cuda.synchronize()
    print(f"[batch] {label}: {len(meshes)} meshes, {b.output_faces()} faces", flush=True)
    for i, m in enumerate(meshes):
        got = {k: v.cpu().numpy() for k, v in outs[i].items()}
        solo = _solo(m, scheme, L)
        np.testing.assert_array_equal(got["face_verts"], solo["face_verts"], err_msg=f"{label} mesh {i}")
        np.testing.assert_array_equal(got["positions"], solo["positions"], err_msg=f"{label} mesh {i}")
        if i % 3 == 0:
            ref = oracle_mod.refine(m, scheme, L)[L]
            np.testing.assert_array_equal(got["face_verts"], ref.verts)
            assert normwise_err(got["positions"], ref.positions) <= POS_TOL


def test_cc_batch_uneven_meshes(oracle_mod):
    rng = np.random.default_rng(9)
    meshes = [G.geodesic_cage(int(t), "cc", rng) for t in (100, 400, 1500, 90, 3000)]
    meshes += [G.torus_cage(n=8), G.cube(), G.grid_patch(3, 2)]
    _check_batch(oracle_mod, meshes, "cc", 3, "cc")


def test_cc_batch_deep_levels_fast_path(oracle_mod):
    rng = np.random.default_rng(10)
    meshes = [G.geodesic_cage(int(t), "cc", rng) for t in (120, 300)] + [G.torus_cage(n=4)]
    _check_batch(oracle_mod, meshes, "cc", 4, "cc-deep")


@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
def test_triangle_batch(oracle_mod, scheme):
    rng = np.random.default_rng(11)
    meshes = [G.geodesic_cage(int(t), "loop", rng) for t in (100, 700, 2000)]
    meshes += [G.tri_cage(seed=4, level=2, hole_frac=0.05), G.tetrahedron()]
    _check_batch(oracle_mod, meshes, scheme, 3, scheme)


def test_batch_of_one_equals_solo(oracle_mod):
    m = G.cc_cage(seed=3, level=3)
    _check_batch(oracle_mod, [m], "cc", 3, "single")
