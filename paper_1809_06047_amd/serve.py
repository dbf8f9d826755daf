"""Continuous-batching serving of refinement requests on one GPU.

A request is a cage (a meshgen.Mesh), a scheme and a level count; its result
is the final level's face table and positions, left resident on the device.

Scheduler (`Server`, host logic only):
  * arrivals join a first-in first-out queue (the executor prepares them:
    on the GPU, a cage topology seen for the first time is uploaded and
    planned once, and every request takes its level sizes from that plan);
  * whenever an execution slot is free, the longest prefix of the queue, at
    most `max_batch` requests and `max_batch_faces` output faces, whose
    device footprint fits the part of the HBM budget not held by batches in
    flight, is admitted as one batch -- requests of every scheme and level
    count together, strictly in arrival order;
  * a batch is one subdiv_refine_batch on the executor's stream: the library
    groups it by (scheme, levels), every group runs one launch per stage,
    and every mesh's output is bitwise the one it gets when refined alone;
  * its requests complete when the batch's completion event has fired;
  * a request whose footprint alone exceeds the whole budget is rejected; a
    launch that runs out of device memory puts its requests back and retries
    with half the batch once memory has been released.
Latency = completion - arrival, on the host clock.

Footprint of a batch = the library's exact workspace size for it (from the
members' plans) + the device copy of its positions + every request's
final-level face table and positions (level sizes from the plans); 0 for a
single request replayed from its captured graph, whose buffers exist.

Baseline (`serve_per_mesh`): the same trace served first-in first-out with
one plan + refine per request on one stream.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

INF = float("inf")


def poll_sleep(dt: float) -> None:
    """The servers' wait: time.sleep for a positive gap; a zero gap ("poll
    again") returns at once. A zero-length time.sleep is still a system call,
    which the kernel's timer slack can hold for tens of microseconds: every
    completion or arrival seen through it would be seen that much late."""
    if dt > 0.0:
        time.sleep(dt)


# ---------------------------------------------------------------------------
# requests and their sizes
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival: float                  # seconds after the start of the trace
    mesh: object                    # meshgen.Mesh (host arrays)
    scheme: str                     # "cc" | "loop" | "sqrt3"
    levels: int
    done: float = math.nan          # completion time (same clock as arrival)
    error: Optional[str] = None     # set when the request was rejected
    batch: int = -1                 # index of the batch that served it
    final_faces: int = 0
    footprint: int = 0              # io bytes: cage in + final level out
    result: Optional[Dict] = None   # final level (device tensors) when kept
    meta: Dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


# ---------------------------------------------------------------------------
# the scheduler
# ---------------------------------------------------------------------------

class ExecutorOOM(MemoryError):
    """A batch could not get its device memory."""


@dataclass
class _Inflight:
    reqs: List[Request]
    handle: object
    nbytes: int
    index: int


class Server:
    """Continuous batching over an executor with the interface
    prepare(reqs) (sets r.footprint and r.final_faces of newly arrived
    requests), footprint_fn(reqs) -> f(k) (bytes of the batch reqs[:k],
    non-decreasing in k, INF when it cannot be planned), launch(reqs, slot)
    -> handle (may raise ExecutorOOM), done(handle) -> bool,
    results(handle) -> list of per-request outputs (called only when
    results are kept), retire(handle) (the batch's memory may be released
    once the outputs taken from it are dropped)."""

    def __init__(self, executor, hbm_budget: int, slots: int = 1, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = poll_sleep,
                 keep_results: bool = False, spin_window: float = 200e-6, max_batch_faces: int = 16 << 20):
        if slots < 1 or max_batch < 1 or hbm_budget <= 0:
            raise ValueError("slots, max_batch and hbm_budget must be positive")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.slots = int(slots)
        self.max_batch = int(max_batch)
        self.max_batch_faces = int(max_batch_faces)  # larger batches gain nothing: the GPU is busy anyway
        self.clock = clock
        self.sleep = sleep
        self.keep_results = keep_results
        self.spin_window = spin_window  # the last part of an idle gap is spent polling, not sleeping
        self.on_complete: Optional[Callable[[Request], None]] = None
        self.stats: Dict = {}

    # the longest admissible prefix of the queue
    def _form(self, queue: deque, avail: int):
        cands = []
        faces = 0
        for r in queue:
            if len(cands) == self._cap or (cands and faces + r.final_faces > self.max_batch_faces):
                break
            cands.append(r)
            faces += r.final_faces
        f = self.ex.footprint_fn(cands)
        if f(1) > avail:
            return None, f(1)
        lo, hi = 1, len(cands)  # f(lo) <= avail
        if f(hi) <= avail:
            return cands, f(hi)
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if f(mid) <= avail:
                lo = mid
            else:
                hi = mid - 1
        return cands[:lo], f(lo)

    def run(self, requests: List[Request]) -> Dict:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        n = len(reqs)
        i = 0
        queue: deque = deque()
        inflight: List[Optional[_Inflight]] = [None] * self.slots
        used = 0
        self._cap = self.max_batch
        hold = False            # after an OOM: no launch until a batch retires
        nbatch = 0
        st = dict(batches=0, batch_sizes=[], max_queue=0, peak_admitted_bytes=0, rejected=0, oom_retries=0)
        t0 = self.clock()
        while i < n or queue or any(b is not None for b in inflight):
            now = self.clock() - t0
            j = i
            while j < n and reqs[j].arrival <= now:
                j += 1
            if j > i:
                self.ex.prepare(reqs[i:j])
                queue.extend(reqs[i:j])
                i = j
            st["max_queue"] = max(st["max_queue"], len(queue))
            progressed = False
            # retire finished batches
            for s, b in enumerate(inflight):
                if b is not None and self.ex.done(b.handle):
                    t = self.clock() - t0
                    outs = self.ex.results(b.handle) if self.keep_results else [None] * len(b.reqs)
                    self.ex.retire(b.handle)
                    for r, o in zip(b.reqs, outs):
                        r.done = t
                        r.result = o
                        if self.on_complete is not None:
                            self.on_complete(r)
                    used -= b.nbytes
                    inflight[s] = None
                    hold = False
                    self._cap = self.max_batch
                    progressed = True
            # admit
            while queue and not hold:
                free = [s for s in range(self.slots) if inflight[s] is None]
                if not free:
                    break
                batch, fp = self._form(queue, self.budget - used)
                if batch is None:
                    if fp > self.budget:
                        r = queue.popleft()  # can never fit: reject
                        r.error = "footprint exceeds the HBM budget"
                        r.done = self.clock() - t0
                        st["rejected"] += 1
                        progressed = True
                        continue
                    break  # wait for memory
                try:
                    h = self.ex.launch(batch, free[0])
                except ExecutorOOM:
                    st["oom_retries"] += 1
                    if any(b is not None for b in inflight):
                        hold = True
                    elif len(batch) > 1:
                        self._cap = max(1, len(batch) // 2)
                    else:
                        r = queue.popleft()
                        r.error = "out of device memory"
                        r.done = self.clock() - t0
                        st["rejected"] += 1
                    progressed = True
                    continue
                for _ in range(len(batch)):  # the batch is a prefix of the queue
                    queue.popleft()
                for r in batch:
                    r.batch = nbatch
                inflight[free[0]] = _Inflight(batch, h, int(fp), nbatch)
                nbatch += 1
                used += int(fp)
                st["batches"] += 1
                st["batch_sizes"].append(len(batch))
                st["peak_admitted_bytes"] = max(st["peak_admitted_bytes"], used)
                progressed = True
            if not progressed:
                if i < n and not queue and all(b is None for b in inflight):
                    # idle until the next arrival: sleep most of the gap, then spin
                    gap = reqs[i].arrival - (self.clock() - t0)
                    self.sleep(min(gap - self.spin_window, 1e-3) if gap > self.spin_window else 0.0)
                else:
                    self.sleep(0.0)  # poll the in-flight batches again right away
        st["makespan"] = self.clock() - t0
        self.stats = st
        return st


def summarize(requests: List[Request], makespan: float) -> Dict:
    ok = [r for r in requests if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    faces = sum(r.final_faces for r in ok)
    return dict(requests=len(requests), served=len(ok), rejected=len(requests) - len(ok),
                p50_ms=float(np.percentile(lat, 50)) if lat.size else None,
                p99_ms=float(np.percentile(lat, 99)) if lat.size else None,
                mean_ms=float(lat.mean()) if lat.size else None,
                makespan_s=float(makespan),
                requests_per_s=len(ok) / makespan if makespan > 0 else None,
                faces_per_s=faces / makespan if makespan > 0 else None)


# ---------------------------------------------------------------------------
# the GPU executor and the per-mesh baseline
# ---------------------------------------------------------------------------

def reserve(device, nbytes: int, stream=None):
    """Grow torch's caching allocator by one segment of `nbytes` for
    `stream`, so that later workspaces and outputs are carved from it instead
    of each new size reaching the device allocator mid-trace."""
    import torch
    if nbytes <= 0:
        return
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(device)):
        x = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        del x


class _Cage:
    """A cage topology the executor has seen: its device arrays (face table,
    column pointer, creases; the positions of the request that brought it)
    and the library's plan of it for `levels` levels, whose counts size every
    level of every later request with this topology."""

    def __init__(self, dmesh, plan, levels: int):
        self.dmesh = dmesh
        self.plan = plan
        self.levels = levels


class GpuBatchExecutor:
    """Runs each batch as one subdiv_refine_batch on one stream (default
    priority); batches in flight queue behind each other on it, so the host
    forms and enqueues the next batch while the previous one runs.

    Cages are keyed by their host face-table object and scheme. A topology
    seen for the first time is uploaded and planned once (subdiv_plan_batch
    over every new cage of an arrival burst: one read-back for all of them,
    on a stream of its own); the plans then give every later request its
    level sizes and let subdiv_refine_batch run without any host round
    trip. A batch uploads only its positions (one pinned copy) and allocates
    one workspace and one output block per kind, released after it retires."""

    def __init__(self, device="cuda", reserve_bytes: int = 0, plan_levels: int = 4, graph_max_faces: int = 0):
        import torch
        from . import _lib, api
        self.torch, self._lib, self.api = torch, _lib, api
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.reg_stream = torch.cuda.Stream(self.device)
        self.plan_levels = int(plan_levels)
        self.cages: Dict[tuple, _Cage] = {}
        self._keep_alive: Dict[tuple, object] = {}
        self.registered = 0
        # single-request refinements captured as HIP graphs (see precapture)
        self.graph_max_faces = int(graph_max_faces)
        self.graphs: Dict[tuple, dict] = {}
        self.graph_stream = torch.cuda.Stream(self.device)
        self.graph_launches = 0
        reserve(self.device, reserve_bytes, self.stream)

    @staticmethod
    def _key(r):
        return (id(r.mesh.verts), r.scheme)

    def _register(self, reqs):
        torch, L, api = self.torch, self._lib, self.api
        new, seen = [], set()
        for r in reqs:
            k = self._key(r)
            c = self.cages.get(k)
            if (c is None or c.levels < r.levels) and k not in seen:
                seen.add(k)
                new.append(r)
        if not new:
            return
        levels = [max(self.plan_levels, r.levels) for r in new]
        with torch.cuda.stream(self.reg_stream):
            dms = [api.DeviceMesh(r.mesh, self.device) for r in new]
            b = api.BatchRefiner(dms, [r.scheme for r in new], levels)
            b.plan(stream=self.reg_stream.cuda_stream)
        for r, dm, lv, k in zip(new, dms, levels, range(len(new))):
            p = L.subdiv_plan_info()
            ctypes_copy(p, b.plans[k])
            self.cages[self._key(r)] = _Cage(dm, p, lv)
            self._keep_alive[self._key(r)] = r.mesh.verts  # the key's id stays this array's
        self.registered += len(new)

    def prepare(self, reqs):
        self._register(reqs)
        for r in reqs:
            c = self.cages[self._key(r)]
            li = c.plan.level[r.levels]
            r.meta["cage"] = c
            r.final_faces = int(li.num_faces)
            # positions in, final face table and positions out
            r.footprint = 12 * r.mesh.num_vertices + 4 * int(li.num_halfedges) + 12 * int(li.num_vertices)

    def _arrays(self, reqs):
        L = self._lib
        n = len(reqs)
        structs = (L.subdiv_mesh * n)(*[r.meta["cage"].dmesh.struct for r in reqs])
        sc = (ctypes.c_int * n)(*[L.SCHEMES[r.scheme] for r in reqs])
        lv = (ctypes.c_int * n)(*[r.levels for r in reqs])
        plans = (L.subdiv_plan_info * n)(*[r.meta["cage"].plan for r in reqs])
        return structs, sc, lv, plans

    def footprint_fn(self, reqs):
        if len(reqs) == 1:
            e = self.graphs.get(self._graph_key(reqs[0]))
            if e is not None and not e["busy"]:
                return lambda k: 0  # launch() replays the graph: its buffers exist already
        structs, sc, lv, plans = self._arrays(reqs)
        io = np.cumsum([r.footprint for r in reqs])
        lib = self.lib

        def f(k: int):
            ws = int(lib.subdiv_batch_workspace_bound(structs, sc, lv, k, plans, 0))
            return INF if ws == 0 else ws + int(io[k - 1])
        return f

    # ---- single requests replayed from HIP graphs --------------------------
    # At low load almost every batch holds one request, and its time goes to
    # launching some thirty small kernels from the host. A request whose
    # (cage topology, level count) was captured runs as one graph launch: its
    # positions go into the graph's static input, the graph replays the
    # library's refinement of that mesh alone (the kernels only: a batch of
    # one enqueues no copies and no memsets), and the result is the graph's
    # static output, which stays the request's until it retires (a second
    # request with the same key meanwhile runs eagerly).

    def _graph_key(self, r):
        return (self._key(r), r.levels)

    def precapture(self, reqs):
        """Capture one graph per (topology, level count) among `reqs` whose
        final level has at most graph_max_faces faces."""
        torch, L, lib = self.torch, self._lib, self.lib
        self.prepare(reqs)
        for r in reqs:
            key = self._graph_key(r)
            if key in self.graphs:
                continue
            c = self.cages[self._key(r)]
            li = c.plan.level[r.levels]
            if int(li.num_faces) > self.graph_max_faces:
                continue
            structs, sc, lv, plans = self._arrays([r])
            V = r.mesh.num_vertices
            P_in = torch.empty((V, 3), dtype=torch.float32, device=self.device)
            P_in.copy_(torch.from_numpy(np.ascontiguousarray(r.mesh.positions, np.float32)))
            structs[0].positions = P_in.data_ptr()
            ws_bytes = int(lib.subdiv_batch_workspace_bound(structs, sc, lv, 1, plans, 0))
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
            fv = torch.empty(int(li.num_halfedges), dtype=torch.int32, device=self.device)
            P = torch.empty((int(li.num_vertices), 3), dtype=torch.float32, device=self.device)
            outs = (L.subdiv_level_out * 1)()
            outs[0].face_verts = fv.data_ptr()
            outs[0].positions = P.data_ptr()
            gs = self.graph_stream

            def call():
                L.check(lib.subdiv_refine_batch(structs, sc, lv, 1, plans, outs, ctypes.c_void_p(ws.data_ptr()),
                                                ws_bytes, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
                        "subdiv_refine_batch")
            torch.cuda.synchronize(self.device)
            with torch.cuda.stream(gs):
                call()  # eager once: the same enqueues the capture records
            gs.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=gs):
                call()
            # a pinned staging buffer and a completion event of the graph's own:
            # a replay reuses them only after the previous one has retired
            host = torch.empty((V, 3), dtype=torch.float32, pin_memory=True)
            self.graphs[key] = dict(g=g, P_in=P_in, ws=ws, fv=fv, P=P, args=(structs, sc, lv, plans, outs),
                                    busy=False, H=int(li.num_halfedges), host=host, host_np=host.numpy(),
                                    ev=torch.cuda.Event())

    def _launch_graph(self, r, e):
        torch = self.torch
        e["host_np"][...] = r.mesh.positions  # (the graph is not busy: its last copy has completed)
        with torch.cuda.stream(self.stream):
            e["P_in"].copy_(e["host"], non_blocking=True)
            e["g"].replay()
            e["ev"].record(self.stream)
        e["busy"] = True
        self.graph_launches += 1
        return dict(ev=e["ev"], keep=(), graph=e, hofs=np.array([0, e["H"]]), hs=[e["H"]],
                    pofs=np.array([0, e["P"].shape[0]]))

    def launch(self, reqs, slot):
        torch, L, lib = self.torch, self._lib, self.lib
        n = len(reqs)
        if n == 1:
            e = self.graphs.get(self._graph_key(reqs[0]))
            if e is not None and not e["busy"]:
                return self._launch_graph(reqs[0], e)
        structs, sc, lv, plans = self._arrays(reqs)
        try:
            with torch.cuda.stream(self.stream):
                nv = [r.mesh.num_vertices for r in reqs]
                vofs = np.concatenate([[0], np.cumsum(nv)])
                host = torch.empty(3 * int(vofs[-1]), dtype=torch.float32, pin_memory=True)
                hn = host.numpy()
                for k, r in enumerate(reqs):
                    hn[3 * int(vofs[k]):3 * int(vofs[k + 1])] = np.asarray(r.mesh.positions, np.float32).reshape(-1)
                dev = torch.empty(hn.size, dtype=torch.float32, device=self.device)
                dev.copy_(host, non_blocking=True)
                base = dev.data_ptr()
                for k in range(n):
                    structs[k].positions = base + 12 * int(vofs[k])
                ws_bytes = int(lib.subdiv_batch_workspace_bound(structs, sc, lv, n, plans, 0))
                if ws_bytes == 0:
                    raise L.SubdivError(L.INVALID_ARG, "subdiv_batch_workspace_bound")
                ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
                # outputs: one int32 and one float32 allocation, every face table 16-byte aligned
                hs = [int(plans[k].level[reqs[k].levels].num_halfedges) for k in range(n)]
                vs = [int(plans[k].level[reqs[k].levels].num_vertices) for k in range(n)]
                hofs = np.concatenate([[0], np.cumsum([(h + 3) // 4 * 4 for h in hs])])
                pofs = np.concatenate([[0], np.cumsum(vs)])
                fv = torch.empty(int(hofs[-1]), dtype=torch.int32, device=self.device)
                P = torch.empty((int(pofs[-1]), 3), dtype=torch.float32, device=self.device)
                outs = (L.subdiv_level_out * n)()
                for k in range(n):
                    outs[k].face_verts = fv.data_ptr() + 4 * int(hofs[k])
                    outs[k].positions = P.data_ptr() + 12 * int(pofs[k])
                L.check(lib.subdiv_refine_batch(structs, sc, lv, n, plans, outs, ctypes.c_void_p(ws.data_ptr()),
                                                ws_bytes, ctypes.c_void_p(self.stream.cuda_stream)),
                        "subdiv_refine_batch")
                ev = torch.cuda.Event()
                ev.record(self.stream)
        except torch.cuda.OutOfMemoryError as e:
            raise ExecutorOOM(str(e)) from e
        return dict(ev=ev, keep=(dev, ws, fv, P, host), hofs=hofs, hs=hs, pofs=pofs)

    def done(self, h) -> bool:
        return h["ev"].query()

    def results(self, h):
        if "graph" in h:  # the graph's static outputs are reused by its next replay
            e = h["graph"]
            torch = self.torch
            # copied on the replay stream, so the next replay comes after the copy;
            # the caller's stream waits for it
            with torch.cuda.stream(self.stream):
                out = {"face_verts": e["fv"].clone(), "positions": e["P"].clone()}
            torch.cuda.current_stream(self.device).wait_stream(self.stream)
            return [out]
        fv, P = h["keep"][2], h["keep"][3]
        return [{"face_verts": fv[int(h["hofs"][k]):int(h["hofs"][k]) + h["hs"][k]],
                 "positions": P[int(h["pofs"][k]):int(h["pofs"][k + 1])]} for k in range(len(h["hs"]))]

    def retire(self, h):
        if "graph" in h:
            h["graph"]["busy"] = False
        h.clear()


def ctypes_copy(dst, src):
    """Byte copy of one ctypes structure into another of the same type."""
    ctypes.memmove(ctypes.addressof(dst), ctypes.addressof(src), ctypes.sizeof(dst))


def serve_per_mesh(requests: List[Request], device="cuda", clock=time.perf_counter, sleep=poll_sleep,
                   keep_results: bool = False) -> Dict:
    """Baseline: first-in first-out, one plan + refine per request on one
    stream, the host waiting for each before taking the next."""
    import torch
    from .api import refine
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = clock()
    for r in reqs:
        while clock() - t0 < r.arrival:  # same idle policy as the server: sleep, then spin
            gap = r.arrival - (clock() - t0)
            sleep(min(gap - 200e-6, 1e-3) if gap > 200e-6 else 0.0)
        outs, rf = refine(r.mesh, r.scheme, r.levels, device=device)
        r.final_faces = int(rf.plan_info.level[r.levels].num_faces)
        r.done = clock() - t0
        r.result = outs[r.levels] if keep_results else None
    torch.cuda.synchronize(device)
    return dict(makespan=clock() - t0)


def serve_per_mesh_cached(requests: List[Request], executor: "GpuBatchExecutor", clock=time.perf_counter,
                          sleep=poll_sleep) -> Dict:
    """Baseline with the batched server's topology cache: first-in first-out,
    one request at a time through the same executor (its kept plan, one
    positions upload, one refinement of that mesh alone), the host waiting
    for each before taking the next. No plan read-back per request."""
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    executor.prepare(reqs)
    t0 = clock()
    for r in reqs:
        while clock() - t0 < r.arrival:
            gap = r.arrival - (clock() - t0)
            sleep(min(gap - 200e-6, 1e-3) if gap > 200e-6 else 0.0)
        h = executor.launch([r], 0)
        h["ev"].synchronize()
        r.done = clock() - t0
        executor.retire(h)
    return dict(makespan=clock() - t0)


# ---------------------------------------------------------------------------
# traces and the QPS sweep
# ---------------------------------------------------------------------------

def make_trace(n_requests: int, seed: int = 4, qps: float = 1.0, schemes=("cc", "loop")) -> List[Request]:
    """Poisson arrivals at `qps`; target faces log-uniform in [100, 50k];
    scheme uniform over `schemes`; levels uniform in 1..4."""
    from . import meshgen as G
    t, faces, scheme, levels = G.poisson_trace(n_requests, qps, seed)
    rng = np.random.default_rng(seed + 1)
    out = []
    for k in range(n_requests):
        sc = str(scheme[k]) if str(scheme[k]) in schemes else schemes[0]
        out.append(Request(rid=k, arrival=float(t[k]), mesh=G.serving_cage(faces[k], sc, rng), scheme=sc,
                           levels=int(levels[k])))
    return out


def _retime(reqs: List[Request], base_times: np.ndarray, qps: float) -> List[Request]:
    return [Request(rid=r.rid, arrival=float(t / qps), mesh=r.mesh, scheme=r.scheme, levels=r.levels)
            for r, t in zip(reqs, base_times)]


def sweep(n_requests: int = 4096, factors=(0.5, 0.8, 1.0, 1.2, 1.5, 2.0, 3.0), seed: int = 4, budget_gib: float = 64.0,
          slots: int = 2, max_batch: int = 256, device="cuda", sat_requests: Optional[int] = None,
          log=print, cold_factor: Optional[float] = 1.0, graph_max_faces: int = 1 << 18) -> Dict:
    """Measure the per-mesh-launch saturation rate, then serve the trace at
    each factor x that rate with the batched server and the baseline.

    The batched server's topology cache is warm for the timed points: a
    warm-up serves one request of every (scheme, levels) group, the head of
    the trace, and one request of every cage topology the trace holds, so
    every later request is refined from its topology's kept plan. At
    `cold_factor` (if not None) the trace is served once more by a server
    whose cache starts empty: there the first request of each topology pays
    its registration plan (one read-back) inside its latency."""
    import torch
    trace = make_trace(n_requests, seed=seed, qps=1.0)
    base_t = np.array([r.arrival for r in trace])
    # both servers start from an allocator that already holds the memory a
    # large request needs
    reserve_bytes = int(min(budget_gib, 8.0) * 2**30)
    reserve(device, reserve_bytes)
    budget = int(budget_gib * 2**30)
    ex = GpuBatchExecutor(device, reserve_bytes, graph_max_faces=graph_max_faces)
    # warm-up of both paths: one request of every (scheme, levels) group, the
    # head of the trace, and (batched server) every topology, all at t = 0
    seen, warm, topo = set(), [], set()
    for r in trace:
        if (r.scheme, r.levels) not in seen:
            seen.add((r.scheme, r.levels))
            warm.append(r)
    warm += trace[:min(64, n_requests)]
    for r in trace:
        if (id(r.mesh.verts), r.scheme) not in topo:
            topo.add((id(r.mesh.verts), r.scheme))
            warm.append(r)
    Server(ex, budget, slots, max_batch).run(_retime(warm, np.zeros(len(warm)), 1.0))
    # every (topology, level count) of the trace with a small final level gets
    # its single-request graph before the timed runs
    t0 = time.perf_counter()
    ex.precapture(trace)
    log(f"[serve] {len(ex.graphs)} single-request graphs captured in {time.perf_counter() - t0:.2f} s")
    serve_per_mesh(_retime(warm[:64], np.zeros(min(64, len(warm))), 1.0), device)
    # saturation of the baseline: everything arrives at t = 0
    ns = min(n_requests, sat_requests or n_requests)
    sat_reqs = _retime(trace[:ns], np.zeros(ns), 1.0)
    sat = serve_per_mesh(sat_reqs, device)
    sat_qps = ns / sat["makespan"]
    log(f"[serve] per-mesh saturation {sat_qps:.1f} req/s over {ns} requests; {len(topo)} cage topologies")

    def batched(qps, executor):
        rb = _retime(trace, base_t, qps)
        srv = Server(executor, budget, slots, max_batch)
        torch.cuda.reset_peak_memory_stats(device)
        st = srv.run(rb)
        b = summarize(rb, st["makespan"])
        b.update(batches=st["batches"], mean_batch=float(np.mean(st["batch_sizes"])) if st["batch_sizes"] else 0.0,
                 max_queue=st["max_queue"], peak_admitted_gib=st["peak_admitted_bytes"] / 2**30,
                 peak_allocated_gib=torch.cuda.max_memory_allocated(device) / 2**30)
        return b

    points = []
    for fac in factors:
        qps = fac * sat_qps
        b = batched(qps, ex)
        rp = _retime(trace, base_t, qps)
        sp = serve_per_mesh(rp, device)
        p = summarize(rp, sp["makespan"])
        rc = _retime(trace, base_t, qps)
        sc = serve_per_mesh_cached(rc, ex)
        c = summarize(rc, sc["makespan"])
        points.append(dict(factor=fac, qps=qps, batched=b, per_mesh=p, per_mesh_cached=c))
        log(f"[serve] x{fac}: {qps:.0f} req/s batched p50 {b['p50_ms']:.3f} p99 {b['p99_ms']:.3f} ms "
            f"(mean batch {b['mean_batch']:.1f}) | per-mesh p50 {p['p50_ms']:.3f} p99 {p['p99_ms']:.3f} ms "
            f"| per-mesh, cached plans p50 {c['p50_ms']:.3f} p99 {c['p99_ms']:.3f} ms")
    cold = None
    if cold_factor is not None:
        cex = GpuBatchExecutor(device, 0)
        cold = dict(factor=cold_factor, batched=batched(cold_factor * sat_qps, cex), registered=cex.registered)
        log(f"[serve] x{cold_factor} cold cache: p50 {cold['batched']['p50_ms']:.3f} "
            f"p99 {cold['batched']['p99_ms']:.3f} ms ({cex.registered} topologies registered in the trace)")
    return dict(requests=n_requests, seed=seed, budget_gib=budget_gib, slots=slots, max_batch=max_batch,
                topologies=len(topo), per_mesh_saturation_qps=sat_qps, points=points, cold_cache=cold,
                graphs=len(ex.graphs), graph_max_faces=graph_max_faces, graph_launches=ex.graph_launches)


def main(argv=None):
    ap = argparse.ArgumentParser(description="continuous-batching refinement server: QPS sweep")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--factors", default="0.5,0.8,1.0,1.2,1.5,2,3")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=2, help="batches in flight at once (queued on one stream)")
    ap.add_argument("--max-batch", type=int, default=256)
    ap.add_argument("--graph-max-faces", type=int, default=1 << 18,
                    help="single requests with at most this many final faces replay a captured graph (0: none)")
    a = ap.parse_args(argv)
    res = sweep(a.requests, tuple(float(x) for x in a.factors.split(",")), a.seed, a.budget_gib, a.slots,
                a.max_batch, graph_max_faces=a.graph_max_faces)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
