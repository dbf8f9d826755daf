"""Serving scheduler on the CPU: a fake executor (simulated clock, injectable
delay and out-of-memory, results from the oracle) drives the same Server the
GPU uses, and the host-side level sizes are pinned to the oracle's counts."""
import numpy as np
import pytest

from paper_1809_06047_amd import meshgen as G
from paper_1809_06047_amd import serve as S


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


_SIZES = {}


def _sizes(oracle_mod, mesh, scheme, levels):
    """(io bytes, final faces) of a request from the oracle's counts: cage
    positions in, final face table and positions out."""
    key = (id(mesh.verts), scheme, levels)
    if key not in _SIZES:
        lv = oracle_mod.refine(mesh, scheme, levels)[levels]
        _SIZES[key] = (12 * mesh.num_vertices + 4 * lv.verts.size + 12 * lv.num_vertices, lv.num_faces, mesh.verts)
    return _SIZES[key][:2]


class FakeExecutor:
    """Batches take `delay(reqs)` simulated seconds; the footprint of a batch
    is the sum of its requests' io bytes + `fixed`; launches of more than
    `oom_above` requests raise ExecutorOOM; sizes and results come from the
    oracle."""

    def __init__(self, clock, oracle_mod, delay=lambda reqs: 2e-3, fixed=1000, oom_above=None, slots=2):
        self.clock, self.oracle = clock, oracle_mod
        self.delay, self.fixed, self.oom_above = delay, fixed, oom_above
        self.busy = [False] * slots
        self.inflight_bytes = 0
        self.max_inflight_bytes = 0
        self.launches = []   # (time, [rid...])

    def prepare(self, reqs):
        for r in reqs:
            r.footprint, r.final_faces = _sizes(self.oracle, r.mesh, r.scheme, r.levels)
            r.meta["prepared"] = True

    def footprint_fn(self, reqs):
        cum = np.cumsum([r.footprint for r in reqs])
        return lambda k: int(cum[k - 1]) + self.fixed

    def launch(self, reqs, slot):
        assert not self.busy[slot], "launch on a busy slot"
        assert all(r.meta.get("prepared") for r in reqs)
        if self.oom_above is not None and len(reqs) > self.oom_above:
            raise S.ExecutorOOM("simulated")
        self.busy[slot] = True
        fp = self.footprint_fn(reqs)(len(reqs))
        self.inflight_bytes += fp
        self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight_bytes)
        self.launches.append((self.clock(), [r.rid for r in reqs]))
        return dict(slot=slot, t=self.clock() + self.delay(reqs), reqs=list(reqs), fp=fp)

    def done(self, h):
        return self.clock() >= h["t"]

    def results(self, h):
        return [dict(rid=r.rid, level=self.oracle.refine(r.mesh, r.scheme, r.levels)[-1]) for r in h["reqs"]]

    def retire(self, h):
        self.busy[h["slot"]] = False
        self.inflight_bytes -= h["fp"]


def _small_requests(n, seed=0, spacing=1e-3):
    rng = np.random.default_rng(seed)
    cages = [("cc", G.cube()), ("cc", G.cc_cage(seed=5, level=0)), ("loop", G.tetrahedron()),
             ("loop", G.grid_patch(2, 3, tri=True)), ("sqrt3", G.tetrahedron()), ("cc", G.grid_patch(3, 2))]
    out = []
    for k in range(n):
        sc, m = cages[int(rng.integers(len(cages)))]
        out.append(S.Request(rid=k, arrival=k * spacing, mesh=m, scheme=sc, levels=int(rng.integers(1, 3))))
    return out


def _server(ex, clock, budget=10**9, slots=2, max_batch=256, keep=True):
    return S.Server(ex, budget, slots=slots, max_batch=max_batch, clock=clock, sleep=clock.sleep,
                    keep_results=keep)


def test_every_request_served_with_its_own_result(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod)
    reqs = _small_requests(40, spacing=2e-4)
    st = _server(ex, clock).run(reqs)
    assert st["rejected"] == 0 and sum(st["batch_sizes"]) == 40
    for r in reqs:
        assert r.error is None and r.done >= r.arrival
        assert r.result["rid"] == r.rid
        ref = oracle_mod.refine(r.mesh, r.scheme, r.levels)[-1]
        np.testing.assert_array_equal(r.result["level"].verts, ref.verts)
        assert r.final_faces == ref.num_faces


def test_batches_are_fifo_prefixes_and_within_budget(oracle_mod):
    """Batches mix schemes and level counts (the library groups them) and
    are prefixes of the queue: over all launches, requests leave in arrival
    order."""
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, delay=lambda reqs: 1e-3 + 1e-4 * len(reqs))
    reqs = _small_requests(120, seed=3, spacing=5e-5)
    budget = 6 * max(_sizes(oracle_mod, r.mesh, r.scheme, r.levels)[0] for r in reqs) + 2000
    srv = _server(ex, clock, budget=budget)
    st = srv.run(reqs)
    assert st["rejected"] == 0
    assert ex.max_inflight_bytes <= budget
    assert st["peak_admitted_bytes"] <= budget
    order = [i for _, ids in ex.launches for i in ids]
    assert order == sorted(order) == [r.rid for r in sorted(reqs, key=lambda r: r.arrival)]
    # more than one request per batch on average under this load, and mixed batches
    assert np.mean(st["batch_sizes"]) > 1.5
    by_id = {r.rid: r for r in reqs}
    assert any(len({(by_id[i].scheme, by_id[i].levels) for i in ids}) > 1 for _, ids in ex.launches)


def test_latency_is_the_service_time_without_contention(oracle_mod):
    clock = FakeClock()
    d = 2e-3
    ex = FakeExecutor(clock, oracle_mod, delay=lambda reqs: d)
    reqs = _small_requests(12, spacing=10e-3)
    _server(ex, clock, keep=False).run(reqs)
    lat = np.array([r.latency for r in reqs])
    assert np.all(lat >= d - 1e-12) and np.all(lat <= d + 2e-4), lat


def test_burst_joins_the_next_batch(oracle_mod):
    """Continuous batching: requests that arrive while the only slot is busy
    are all admitted together as soon as it frees."""
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, delay=lambda reqs: 5e-3, slots=1)
    m = G.cube()
    reqs = [S.Request(rid=0, arrival=0.0, mesh=m, scheme="cc", levels=2)]
    reqs += [S.Request(rid=k, arrival=1e-3 + k * 1e-4, mesh=m, scheme="cc", levels=2) for k in range(1, 11)]
    st = _server(ex, clock, slots=1).run(reqs)
    assert st["batch_sizes"] == [1, 10]


def test_budget_caps_batch_size(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, delay=lambda reqs: 3e-3)
    m = G.cube()
    one = _sizes(oracle_mod, m, "cc", 2)[0]
    reqs = [S.Request(rid=k, arrival=0.0, mesh=m, scheme="cc", levels=2) for k in range(20)]
    budget = 1000 + 3 * one
    st = _server(ex, clock, budget=budget).run(reqs)
    assert max(st["batch_sizes"]) == 3 and sum(st["batch_sizes"]) == 20
    assert ex.max_inflight_bytes <= budget


def test_oversized_request_is_rejected_and_others_served(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod)
    small, big = G.cube(), G.cc_cage(seed=5, level=1)
    reqs = [S.Request(rid=0, arrival=0.0, mesh=small, scheme="cc", levels=1),
            S.Request(rid=1, arrival=0.0, mesh=big, scheme="cc", levels=2),
            S.Request(rid=2, arrival=1e-4, mesh=small, scheme="cc", levels=1)]
    budget = 1000 + 4 * _sizes(oracle_mod, small, "cc", 1)[0]
    assert 1000 + _sizes(oracle_mod, big, "cc", 2)[0] > budget
    st = _server(ex, clock, budget=budget).run(reqs)
    assert st["rejected"] == 1 and reqs[1].error is not None
    assert reqs[0].error is None and reqs[2].error is None
    s = S.summarize(reqs, st["makespan"])
    assert s["served"] == 2 and s["rejected"] == 1


def test_face_cap_splits_batches(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, slots=1)
    m = G.cube()
    reqs = [S.Request(rid=k, arrival=0.0, mesh=m, scheme="cc", levels=2) for k in range(10)]
    faces = _sizes(oracle_mod, m, "cc", 2)[1]  # 96 faces per request
    srv = S.Server(ex, 10**9, slots=1, clock=clock, sleep=clock.sleep, max_batch_faces=3 * faces + 1)
    st = srv.run(reqs)
    assert st["batch_sizes"] == [3, 3, 3, 1]
    srv = S.Server(ex, 10**9, slots=1, clock=clock, sleep=clock.sleep, max_batch_faces=1)
    assert srv.run([S.Request(rid=0, arrival=0.0, mesh=m, scheme="cc", levels=2)])["batch_sizes"] == [1]


def test_out_of_memory_halves_the_batch(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, oom_above=4, slots=1)
    m = G.tetrahedron()
    reqs = [S.Request(rid=k, arrival=0.0, mesh=m, scheme="loop", levels=1) for k in range(13)]
    st = _server(ex, clock, slots=1).run(reqs)
    assert st["oom_retries"] >= 1 and st["rejected"] == 0
    assert max(st["batch_sizes"]) <= 4 and sum(st["batch_sizes"]) == 13
    assert all(r.error is None for r in reqs)


def test_single_request_oom_with_nothing_in_flight_is_rejected(oracle_mod):
    clock = FakeClock()
    ex = FakeExecutor(clock, oracle_mod, oom_above=0, slots=1)
    reqs = [S.Request(rid=0, arrival=0.0, mesh=G.cube(), scheme="cc", levels=1)]
    st = _server(ex, clock, slots=1).run(reqs)
    assert st["rejected"] == 1 and reqs[0].error == "out of device memory"


def test_trace_recipe():
    reqs = S.make_trace(64, seed=9, qps=100.0)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) >= 0) and abs(t[-1] - 64 / 100.0) < 0.5
    assert {r.scheme for r in reqs} <= {"cc", "loop"}
    assert {r.levels for r in reqs} <= {1, 2, 3, 4}
    for r in reqs:
        F = r.mesh.num_faces
        assert 60 <= F <= 50_000
        if r.scheme == "loop":
            assert r.mesh.offsets is None and r.mesh.face_order == 3 and r.mesh.num_creases == 0
        else:
            assert r.mesh.offsets is not None and r.mesh.num_creases > 0
    again = S.make_trace(64, seed=9, qps=100.0)
    assert all(np.array_equal(a.mesh.positions, b.mesh.positions) and a.arrival == b.arrival
               for a, b in zip(reqs, again))
