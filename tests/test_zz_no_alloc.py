"""subdiv_refine_static: the refinement in the library's own device array,
for callers that cannot allocate. Its outputs equal subdiv_refine's with a
caller workspace bit for bit (the same kernels), on calls in a row whose
sizes shrink, so the array's leftovers from a larger call never leak into a
smaller one."""
import numpy as np
import pytest
import torch

from paper_1809_06047_amd import _lib, api
from paper_1809_06047_amd import meshgen as G

pytestmark = pytest.mark.gpu


def _snapshot(outs):
    return [{k: v.cpu().numpy().copy() for k, v in o.items()} for o in outs]


def _check_static(mesh, scheme, levels, label):
    r = api.Refiner(mesh, scheme, levels, keep="all")
    r.plan()
    assert r.plan_info.workspace_bytes <= _lib.STATIC_WORKSPACE_BYTES, label
    ref = _snapshot(r.run())
    for o in r.outs:  # the static call must write every output again
        for v in o.values():
            v.fill_(-7)
    print(f"[no-alloc] {label}: {mesh.name} {scheme} L={levels} ws={r.plan_info.workspace_bytes}", flush=True)
    got = _snapshot(r.run_static())
    torch.cuda.synchronize()
    for k in range(1, levels + 1):
        for key in ref[k]:
            np.testing.assert_array_equal(got[k][key], ref[k][key], err_msg=f"{label} level {k} {key}")
    return r


def test_static_workspace_equals_caller_workspace():
    big = G.cc_cage(seed=3, level=3)  # 642 vertices, creases
    small = G.torus_cage(seed=4, n=8)
    _check_static(big, "cc", 4, "first call")
    _check_static(small, "cc", 3, "second call, smaller")
    _check_static(G.tri_cage(seed=5, level=2, hole_frac=0.05), "loop", 4, "third call, Loop")
    _check_static(small, "cc", 2, "fourth call, smaller again")


def test_static_workspace_limits():
    r = api.Refiner(G.cc_cage(seed=3, level=3), "cc", 6)
    r.plan()
    assert r.plan_info.workspace_bytes > _lib.STATIC_WORKSPACE_BYTES
    with pytest.raises(_lib.SubdivError) as e:
        r.run_static()
    assert e.value.status == _lib.WORKSPACE
    k = api.Refiner(G.torus_cage(seed=4, n=8), "cc", 2, flags=_lib.FLAG_KEEP_STATE)
    k.plan()
    with pytest.raises(_lib.SubdivError) as e:
        k.run_static()
    assert e.value.status == _lib.INVALID_ARG
