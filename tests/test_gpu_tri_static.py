"""Static topology and general vertex data for Loop and sqrt(3) (Sec. 3.6:
refinement is linear in the vertex data, P_L = R_{L-1} ... R_0 P_0 with every
R_k fixed by topology and creases). A plan with FLAG_KEEP_STATE keeps every
level's face table and adjacency; subdiv_refine_positions then re-evaluates
moved cage positions through the same point kernels with every topology
output off, and subdiv_refine_vertex_data does so three channels at a time.
Checked bit for bit against full refinements of the moved cage and against
the oracle, through the C ABI."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu


def _creased(m, n, smax, seed):
    cv, cs = G.tag_creases(m.offsets, m.verts, m.face_order, n, smax, np.random.default_rng(seed))
    return dataclasses.replace(m, crease_verts=cv, crease_sharp=cs, name=m.name + "-creased")


CAGES = {
    "holes": lambda: G.tri_cage(seed=61, level=2, hole_frac=0.06),
    "closed": lambda: G.tri_cage(seed=62, level=2, hole_frac=0.0),
    "loop_creases": lambda: _creased(G.tri_cage(seed=63, level=2, hole_frac=0.06), 60, 5.0, 64),
}


def _kept(m, scheme, L):
    r = api.Refiner(m, scheme, L, flags=_lib.FLAG_KEEP_STATE, keep="all")
    r.plan()
    r.run()
    return r


@pytest.mark.parametrize("scheme,cage", [("loop", "holes"), ("loop", "closed"), ("loop", "loop_creases"),
                                         ("sqrt3", "holes"), ("sqrt3", "closed")])
def test_triangle_positions_equal_full_refine(oracle_mod, scheme, cage):
    """Moved cage positions re-evaluated from the kept state equal, bit for
    bit and at every level, a full refinement of the moved cage (which runs
    the last steps from two levels down), and the oracle within tolerance."""
    m, L = CAGES[cage](), 4
    print(f"[static] {scheme} {m.name} L={L}", flush=True)
    r = _kept(m, scheme, L)
    first = [None] + [r.outs[k]["positions"].cpu().numpy().copy() for k in range(1, L + 1)]
    plain, _ = api.refine(m, scheme, L, keep="all")
    for k in range(1, L + 1):  # the kept-state refinement itself is the ordinary one
        np.testing.assert_array_equal(first[k], plain[k]["positions"].cpu().numpy(), err_msg=f"level {k}")
        np.testing.assert_array_equal(r.outs[k]["face_verts"].cpu().numpy(), plain[k]["face_verts"].cpu().numpy())
    moved = dataclasses.replace(m, positions=(m.positions + np.random.default_rng(65).normal(
        0, 0.05, m.positions.shape)).astype(np.float32))
    r.dmesh.set_positions(torch.from_numpy(moved.positions.copy()).cuda())
    outs = r.run_positions()
    torch.cuda.synchronize()
    full, _ = api.refine(moved, scheme, L, keep="all")
    ref = oracle_mod.refine(moved, scheme, L)
    for k in range(1, L + 1):
        got = outs[k]["positions"].cpu().numpy()
        np.testing.assert_array_equal(got, full[k]["positions"].cpu().numpy(), err_msg=f"level {k}")
        err = normwise_err(got, ref[k].positions)
        assert err <= POS_TOL, f"level {k}: {err:.2e}"


@pytest.mark.parametrize("dim", [1, 5, 7])
@pytest.mark.parametrize("scheme", ["loop", "sqrt3"])
def test_triangle_vertex_data_equals_oracle(oracle_mod, scheme, dim):
    """Every group of three channels against the oracle refining those
    channels as positions, on the holed cage at level 4; positions as
    channels 0-2 give the refined positions bit for bit."""
    m, L = CAGES["holes"](), 4
    print(f"[vertex data] {scheme} dim={dim}", flush=True)
    r = _kept(m, scheme, L)
    data = np.random.default_rng(66 + dim).normal(0, 1, (m.num_vertices, dim)).astype(np.float32)
    got = r.run_vertex_data(torch.from_numpy(data).cuda()).cpu().numpy()
    assert got.shape == (r.level_info(L)["V"], dim)
    for c0 in range(0, dim, 3):
        w = min(3, dim - c0)
        sl = np.zeros((m.num_vertices, 3), np.float32)
        sl[:, :w] = data[:, c0:c0 + w]
        ref = oracle_mod.refine(dataclasses.replace(m, positions=sl), scheme, L)[L].positions
        assert normwise_err(got[:, c0:c0 + w], ref[:, :w]) <= POS_TOL
    P = torch.from_numpy(m.positions).cuda()
    pos = r.run_vertex_data(torch.cat([P, 2 * P], 1))
    torch.cuda.synchronize()
    assert torch.equal(pos[:, 0:3], r.final["positions"])
    assert torch.equal(pos[:, 3:6], 2 * r.final["positions"])


def test_triangle_state_calls():
    """Without the kept state the calls are refused; the adjoint stays
    Catmull-Clark only."""
    m = CAGES["holes"]()
    plain = api.Refiner(m, "loop", 3)
    plain.plan()
    plain.run()
    with pytest.raises(_lib.SubdivError) as e:
        plain.run_positions()
    assert e.value.status == _lib.STATE
    r = _kept(m, "loop", 3)
    with pytest.raises(_lib.SubdivError) as e:
        r.backward(torch.zeros((r.level_info(3)["V"], 3), device="cuda"))
    assert e.value.status == _lib.STATE
