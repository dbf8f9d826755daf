"""Batched refinement: every mesh of a batch equals the same mesh refined
alone (bit for bit) and the oracle (within tolerance). Batches may mix
schemes and level counts; the library groups them by (scheme, levels)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu


def _solo(mesh, scheme, L):
    outs, _ = api.refine(mesh, scheme, L)
    return {k: v.cpu().numpy() for k, v in outs[L].items()}


def _check_batch(oracle_mod, meshes, schemes, levels, label, oracle_every=3, plans=None, host=None):
    n = len(meshes)
    schemes = schemes if isinstance(schemes, list) else [schemes] * n
    levels = levels if isinstance(levels, list) else [levels] * n
    b = api.BatchRefiner(meshes, schemes, levels, plans=plans)
    if plans is None:
        b.plan()
    outs = b.run()
    torch.cuda.synchronize()
    print(f"[batch] {label}: {n} meshes, {b.output_faces()} faces", flush=True)
    for i, m in enumerate(meshes):
        got = {k: v.cpu().numpy() for k, v in outs[i].items()}
        solo = _solo(m, schemes[i], levels[i])
        np.testing.assert_array_equal(got["face_verts"], solo["face_verts"], err_msg=f"{label} mesh {i}")
        np.testing.assert_array_equal(got["positions"], solo["positions"], err_msg=f"{label} mesh {i}")
        if i % oracle_every == 0:
            ref = oracle_mod.refine(host[i] if host else m, schemes[i], levels[i])[levels[i]]
            np.testing.assert_array_equal(got["face_verts"], ref.verts, err_msg=f"{label} mesh {i}")
            assert normwise_err(got["positions"], ref.positions) <= POS_TOL, f"{label} mesh {i}"
    return b


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
@pytest.mark.parametrize("L", [3, 4])
def test_triangle_batch(oracle_mod, scheme, L):
    """Level 4 runs the last two steps from the level below them on a
    disjoint union with holes, a tetrahedron and small components."""
    rng = np.random.default_rng(11)
    meshes = [G.geodesic_cage(int(t), "loop", rng) for t in (100, 700, 2000)]
    meshes += [G.tri_cage(seed=4, level=2, hole_frac=0.05), G.tetrahedron()]
    _check_batch(oracle_mod, meshes, scheme, L, f"{scheme}-L{L}")


def test_batch_of_one_equals_solo(oracle_mod):
    m = G.cc_cage(seed=3, level=3)
    _check_batch(oracle_mod, [m], "cc", 3, "single")


def test_mixed_schemes_and_levels(oracle_mod):
    """One call with Catmull-Clark, Loop and sqrt(3) meshes at levels 1-4 in
    an interleaved order (groups of one and of several); every mesh against
    its solo refinement and the oracle."""
    rng = np.random.default_rng(12)
    spec = [("cc", 2, 300), ("loop", 4, 200), ("cc", 2, 900), ("sqrt3", 3, 500), ("loop", 1, 100),
            ("cc", 4, 150), ("loop", 4, 600), ("sqrt3", 3, 80), ("cc", 1, 2000), ("loop", 1, 400),
            ("cc", 2, 100)]
    meshes = [G.geodesic_cage(t, "cc" if s == "cc" else "loop", rng) for s, _, t in spec]
    meshes[3] = G.tri_cage(seed=5, level=2, hole_frac=0.05)   # a holed cage in a sqrt(3) group
    _check_batch(oracle_mod, meshes, [s for s, _, _ in spec], [l for _, l, _ in spec], "mixed", oracle_every=1)


def test_member_plans_skip_the_batch_plan(oracle_mod):
    """Plans kept from solo subdiv_plan calls (with more levels than asked)
    serve the batch directly: no subdiv_plan_batch, same bits."""
    rng = np.random.default_rng(13)
    spec = [("cc", 3, 400), ("loop", 2, 300), ("cc", 3, 120), ("loop", 4, 800)]
    meshes = [G.geodesic_cage(t, s, rng) for s, _, t in spec]
    dms = [api.DeviceMesh(m) for m in meshes]
    plans = []
    for dm, (s, _, _) in zip(dms, spec):
        r = api.Refiner(dm, s, 4)
        r.plan()
        plans.append(r.plan_info)
    _check_batch(oracle_mod, dms, [s for s, _, _ in spec], [l for _, l, _ in spec], "member-plans", oracle_every=1,
                 plans=plans, host=meshes)
    # the batch plan's own plans are plans of each mesh: subdiv_refine takes them
    b = api.BatchRefiner(dms, [s for s, _, _ in spec], [l for _, l, _ in spec])
    b.plan()
    lib = _lib.load()
    for i, (dm, (s, l, _)) in enumerate(zip(dms, spec)):
        p = b.plans[i]
        ws = torch.empty(int(p.workspace_bytes), dtype=torch.uint8, device="cuda")
        outs = (_lib.subdiv_level_out * (l + 1))()
        fv = torch.empty(p.level[l].num_halfedges, dtype=torch.int32, device="cuda")
        P = torch.empty((p.level[l].num_vertices, 3), dtype=torch.float32, device="cuda")
        outs[l].face_verts, outs[l].positions = fv.data_ptr(), P.data_ptr()
        _lib.check(lib.subdiv_refine(ctypes.byref(dm.struct), ctypes.byref(p), outs, ctypes.c_void_p(ws.data_ptr()),
                                     int(p.workspace_bytes), ctypes.c_void_p(api.current_stream_handle())),
                   "subdiv_refine")
        torch.cuda.synchronize()
        solo = _solo(dm, s, l)
        np.testing.assert_array_equal(fv.cpu().numpy(), solo["face_verts"])
        np.testing.assert_array_equal(P.cpu().numpy(), solo["positions"])
