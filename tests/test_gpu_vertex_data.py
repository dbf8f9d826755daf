"""General vertex data (any number of channels: UVs, colours) refined with the
kept Catmull-Clark state, through the C ABI. Refinement is linear in the
vertex data with the same operators for every channel (Sec. 3.6), so the
oracle refining three channels at a time as positions is the reference."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err
from tests.test_gpu_adjoint import _grid_with_creases

pytestmark = pytest.mark.gpu


def _kept(m, L):
    r = api.Refiner(m, "cc", L, flags=_lib.FLAG_KEEP_STATE)
    r.plan()
    r.run()
    return r


@pytest.mark.parametrize("dim", [1, 5, 7])
@pytest.mark.parametrize("cage", ["mixed_creases", "grid_creases"])
def test_vertex_data_equals_oracle_per_channel_group(oracle_mod, cage, dim):
    m, L = (G.cc_cage(seed=24, level=2), 4) if cage == "mixed_creases" else (_grid_with_creases(23), 4)
    print(f"[vertex data] {cage} dim={dim} levels={L}", flush=True)
    r = _kept(m, L)
    data = np.random.default_rng(dim).normal(0, 1, (m.num_vertices, dim)).astype(np.float32)
    got = r.run_vertex_data(torch.from_numpy(data).cuda()).cpu().numpy()
    assert got.shape == (r.level_info(L)["V"], dim)
    for c0 in range(0, dim, 3):
        w = min(3, dim - c0)
        sl = np.zeros((m.num_vertices, 3), np.float32)
        sl[:, :w] = data[:, c0:c0 + w]
        ref = oracle_mod.refine(dataclasses.replace(m, positions=sl), "cc", L)[L].positions
        err = normwise_err(got[:, c0:c0 + w], ref[:, :w])
        print(f"[vertex data] channels {c0}..{c0 + w - 1}: normwise err {err:.2e}", flush=True)
        assert err <= POS_TOL


def test_vertex_data_routes_every_channel():
    """Positions as channels 0-2 give subdiv_refine's positions bit for bit;
    twice the positions (an exact scaling) in channels 3-5 give exactly twice
    them; a constant channel stays constant (every stencil sums to one)."""
    m = G.cc_cage(seed=24, level=2)
    r = _kept(m, 4)
    P = torch.from_numpy(m.positions).cuda()
    data = torch.cat([P, 2 * P, torch.ones((m.num_vertices, 1), device="cuda")], 1)
    got = r.run_vertex_data(data)
    torch.cuda.synchronize()
    ref = r.final["positions"]
    assert torch.equal(got[:, 0:3], ref)
    assert torch.equal(got[:, 3:6], 2 * ref)
    assert torch.max(torch.abs(got[:, 6] - 1.0)).item() <= 2e-6


def test_vertex_data_rejects_bad_calls():
    m = G.cc_cage(seed=24, level=2)
    r = _kept(m, 2)
    with pytest.raises(_lib.SubdivError) as e:
        r.run_vertex_data(torch.zeros((m.num_vertices, 0), device="cuda"))
    assert e.value.status == _lib.INVALID_ARG
    plain = api.Refiner(m, "cc", 2)
    plain.plan()
    plain.run()
    with pytest.raises(_lib.SubdivError) as e:
        plain.run_vertex_data(torch.zeros((m.num_vertices, 2), device="cuda"))
    assert e.value.status == _lib.STATE


@pytest.mark.parametrize("dim", [1, 2, 3, 4, 6, 8, 13])
def test_vertex_data_every_group_width(dim):
    """Channel j holds position coordinate j mod 3 scaled by 2^(j div 3), an
    exact scaling: every output column is that coordinate of the refined
    positions, scaled the same way, bit for bit. The dims cover the last
    group of one to six channels."""
    m = G.cc_cage(seed=24, level=2)
    r = _kept(m, 3)
    P = torch.from_numpy(m.positions).cuda()
    data = torch.stack([P[:, j % 3] * 2.0 ** (j // 3) for j in range(dim)], 1).contiguous()
    print(f"[vertex data] group widths, dim={dim}", flush=True)
    got = r.run_vertex_data(data)
    torch.cuda.synchronize()
    ref = r.final["positions"]
    for j in range(dim):
        assert torch.equal(got[:, j], ref[:, j % 3] * 2.0 ** (j // 3)), j
