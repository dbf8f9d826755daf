"""GPU adjoint (transposed gathers through the C ABI) against the oracle's
R^T and against finite differences."""
import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu


def _oracle_RT(oracle_mod, mesh, levels, g):
    lv = oracle_mod.refine(mesh, "cc", levels, want_R=True)
    for k in range(levels, 0, -1):
        g = lv[k].R.T @ g
    return g, lv


def _grid_with_creases(seed):
    """Open quad grid with creases tagged on interior and boundary edges."""
    rng = np.random.default_rng(seed)
    m = G.grid_patch(6, 5, z_fn=lambda x, y: rng.normal(0, 0.3, x.shape))
    cv, cs = G.tag_creases(None, m.verts, 4, 14, 4.0, rng)
    m.crease_verts, m.crease_sharp = cv, cs
    return m


@pytest.mark.parametrize("case", ["mixed_creases", "deep_creases", "grid_creases", "torus", "grid_boundary", "prism"])
def test_adjoint_equals_oracle_transpose(oracle_mod, case):
    """Levels k >= 2 take the corner-class coefficient and face-point paths
    (creases on the halves of edge points, boundary edge points); the cases
    with four levels carry creases through two such levels."""
    if case == "mixed_creases":
        m, L = G.cc_cage(seed=21, level=2), 3
    elif case == "deep_creases":
        m, L = G.cc_cage(seed=24, level=2), 4
    elif case == "grid_creases":
        m, L = _grid_with_creases(23), 4
    elif case == "torus":
        m, L = G.torus_cage(n=8), 3
    elif case == "grid_boundary":
        rng = np.random.default_rng(2)
        m, L = G.grid_patch(5, 4, z_fn=lambda x, y: rng.normal(0, 0.3, x.shape)), 3
    else:
        from tests.test_gpu_parity import _prism
        m, L = _prism(5), 3
    print(f"[adjoint] {case} levels={L}", flush=True)
    r = api.differentiable_refiner(m, L)
    r.run()
    VL = r.level_info(L)["V"]
    rng = np.random.default_rng(5)
    g = rng.normal(0, 1, (VL, 3)).astype(np.float32)
    got = r.backward(torch.from_numpy(g).cuda()).cpu().numpy()
    want, lv = _oracle_RT(oracle_mod, m, L, g.astype(np.float64))
    err = normwise_err(got, want)
    print(f"[adjoint] {case}: normwise err {err:.2e}", flush=True)
    assert err <= POS_TOL
    # the forward of the keep-state path is the same refinement
    assert normwise_err(r.final["positions"].cpu().numpy(), lv[L].positions) <= POS_TOL
    np.testing.assert_array_equal(r.final["face_verts"].cpu().numpy(), lv[L].verts)


def test_autograd_matches_finite_differences():
    """L(P0) = sum |P_2 - T|^2 on the torus: quadratic, so central
    differences in FP32 with h = 1e-2 agree with the adjoint to ~1e-3."""
    m = G.torus_cage()
    r = api.differentiable_refiner(m, 2)
    P0 = torch.from_numpy(m.positions.copy()).cuda().requires_grad_(True)
    with torch.no_grad():
        base = api.SubdivFunction.apply(P0, r)
    T = base + 0.05 * torch.randn_like(base)
    loss = ((api.SubdivFunction.apply(P0, r) - T) ** 2).sum()
    loss.backward()
    grad = P0.grad.detach().cpu().numpy()
    h = 1e-2
    for (i, d) in [(0, 0), (37, 1), (128, 2), (255, 0)]:
        vals = []
        for sgn in (1, -1):
            Q = P0.detach().clone()
            Q[i, d] += sgn * h
            with torch.no_grad():
                vals.append(float(((api.SubdivFunction.apply(Q, r) - T) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(grad[i, d], rel=2e-3, abs=2e-3), (i, d, fd, grad[i, d])


def test_backward_without_keep_state_is_rejected():
    r = api.Refiner(G.torus_cage(), "cc", 2)
    r.plan()
    r.run()
    with pytest.raises(_lib.SubdivError) as e:
        r.backward(torch.zeros((r.level_info(2)["V"], 3), device="cuda"))
    assert e.value.status == _lib.STATE


@pytest.mark.parametrize("cage", ["mixed_creases", "holes"])
def test_refine_positions_equals_full_refine(oracle_mod, cage):
    """Static topology: with the state kept, new cage positions refined by
    subdiv_refine_positions (positions only) give bit for bit the positions
    of a full subdiv_refine of the moved cage, at every level, and match the
    oracle."""
    if cage == "mixed_creases":
        m = G.cc_cage(seed=31, level=2, crease_frac=0.1, smax=6.0)
    else:
        m = G.tri_cage(seed=32, level=2, hole_frac=0.06)
    L = 4
    r = api.Refiner(m, "cc", L, flags=_lib.FLAG_KEEP_STATE, keep="all")
    r.plan()
    r.run()
    rng = np.random.default_rng(33)
    moved = G.Mesh(**{**m.__dict__, "positions": (m.positions + rng.normal(0, 0.05, m.positions.shape)).astype(
        np.float32)})
    r.dmesh.set_positions(torch.from_numpy(moved.positions.copy()).cuda())
    outs = r.run_positions()
    torch.cuda.synchronize()
    got = [None] + [outs[k]["positions"].cpu().numpy() for k in range(1, L + 1)]
    full, _ = api.refine(moved, "cc", L, keep="all")
    ref = oracle_mod.refine(moved, "cc", L)
    for k in range(1, L + 1):
        np.testing.assert_array_equal(got[k], full[k]["positions"].cpu().numpy(), err_msg=f"level {k}")
        assert normwise_err(got[k], ref[k].positions) <= POS_TOL


def test_backward_coefficients_once_per_plan():
    """The adjoint's vertex-rule coefficients are written by the first
    backward after a keep-state refinement and reused after it: the gradient
    is the same bits after a positions-only forward, after a second full
    refinement (which clears them) and after a new plan of another cage in
    the same refiner slot."""
    import torch
    m = G.cc_cage(seed=24, level=2)
    r = api.differentiable_refiner(m, 3)
    r.run()
    g = torch.from_numpy(np.random.default_rng(8).normal(0, 1, (r.level_info(3)["V"], 3)).astype(np.float32)).cuda()
    a = r.backward(g).cpu().numpy()
    b = r.backward(g).cpu().numpy()
    r.run_positions()
    c = r.backward(g).cpu().numpy()
    r.run()
    d = r.backward(g).cpu().numpy()
    for x in (b, c, d):
        np.testing.assert_array_equal(a, x)
    # a new plan (another cage with the same counts would reuse nothing): the
    # coefficients are computed again for it
    m2 = _grid_with_creases(23)
    r2 = api.differentiable_refiner(m2, 3)
    r2.run()
    g2 = torch.ones((r2.level_info(3)["V"], 3), dtype=torch.float32, device="cuda")
    e = r2.backward(g2).cpu().numpy()
    r2.plan()
    r2.run()
    f = r2.backward(g2).cpu().numpy()
    np.testing.assert_array_equal(e, f)
    # every row of R sums to one, so a gradient of ones sums to the refined vertex count
    assert abs(float(e.sum()) - 3 * r2.level_info(3)["V"]) <= 1e-3 * 3 * r2.level_info(3)["V"]


def test_state_calls_follow_the_workspace_record():
    """The order plan -> backward (no refinement yet) is refused with
    SUBDIV_STATE before any device work; after a run the state calls work;
    after subdiv_state_destroy (Refiner.release) they are refused again, and
    a new run brings the state back with the same gradient bits."""
    m = G.cc_cage(seed=2, level=2)
    r = api.Refiner(m, "cc", 2, flags=_lib.FLAG_KEEP_STATE)
    r.plan()
    V2 = r.plan_info.level[2].num_vertices
    g = torch.linspace(-1, 1, V2 * 3, device="cuda").reshape(V2, 3)
    for call in (lambda: r.backward(g), r.run_positions,
                 lambda: r.run_vertex_data(torch.ones((m.num_vertices, 2), device="cuda"))):
        with pytest.raises(_lib.SubdivError) as e:
            call()
        assert e.value.status == _lib.STATE
    r.run()
    g1 = r.backward(g).clone()
    torch.cuda.synchronize()
    assert r.release()
    with pytest.raises(_lib.SubdivError) as e:
        r.backward(g)
    assert e.value.status == _lib.STATE
    assert not r.release()
    r.run()
    g2 = r.backward(g)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
