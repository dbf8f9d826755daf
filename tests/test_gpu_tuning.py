"""The launch-shape table moves time only: the same refinements and the same
adjoint under two different tables (every kernel at 64 lanes per workgroup,
then every kernel at 512) are bit for bit equal, and equal to the oracle
within tolerance."""
import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G
from tests.parity_util import POS_TOL, normwise_err

pytestmark = pytest.mark.gpu


@pytest.fixture
def restore_table():
    src = _lib.tuning_source()
    yield
    _lib.tuning_load(src if src.startswith("/") else None)


def _run(mesh, scheme, L, block):
    _lib.tuning_set("*", block)
    outs, _ = api.refine(mesh, scheme, L, keep="all")
    torch.cuda.synchronize()
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]


@pytest.mark.parametrize("scheme,L", [("cc", 5), ("loop", 5), ("sqrt3", 5), ("loop", 3)])
def test_outputs_independent_of_the_table(oracle_mod, restore_table, scheme, L):
    m = G.cc_cage(seed=51, level=2, crease_frac=0.1, smax=6.0) if scheme == "cc" else \
        G.tri_cage(seed=52, level=2, hole_frac=0.06)
    print(f"[tuning] {scheme} L={L} {m.name}: blocks 64 vs 512", flush=True)
    a = _run(m, scheme, L, 64)
    b = _run(m, scheme, L, 512)
    ref = oracle_mod.refine(m, scheme, L)
    for k in range(1, L + 1):
        for key in a[k]:
            np.testing.assert_array_equal(a[k][key], b[k][key], err_msg=f"level {k} {key}")
        np.testing.assert_array_equal(a[k]["face_verts"], ref[k].verts)
        assert normwise_err(a[k]["positions"], ref[k].positions) <= POS_TOL


def test_adjoint_independent_of_the_table(restore_table):
    m = G.cc_cage(seed=53, level=2, crease_frac=0.1, smax=6.0)
    grads = []
    for block in (64, 512):
        _lib.tuning_set("*", block)
        r = api.Refiner(m, "cc", 4, flags=_lib.FLAG_KEEP_STATE)
        r.plan()
        outs = r.run()
        g = torch.from_numpy(np.random.default_rng(54).normal(size=tuple(outs[4]["positions"].shape)).astype(
            np.float32)).cuda()
        grads.append(r.backward(g).cpu().numpy())
        grads.append(r.run_positions()[4]["positions"].cpu().numpy())
    np.testing.assert_array_equal(grads[0], grads[2])
    np.testing.assert_array_equal(grads[1], grads[3])


def test_timing_names_the_tuned_kernel(restore_table):
    _lib.tuning_set("*", 128)
    r = api.Refiner(G.cc_cage(seed=55, level=2), "cc", 4)
    r.plan()
    _lib.timing_enable(True)
    _lib.timing_read_kernels()
    r.run()
    torch.cuda.synchronize()
    recs = _lib.timing_read_kernels()
    _lib.timing_enable(False)
    kern = {(s, lv): (k, n, b) for s, lv, k, n, b, _, _ in recs}
    assert kern[("cc_group", 3)] == ("lag2_group", r.level_info(2)["F"], 128)
    assert kern[("cc_edge_group", 3)] == ("lag_edge", r.level_info(2)["E"], 128)
    assert kern[("cc_group", 1)][0] == "lag_group"
