"""Continuous-batching serving of refinement requests on one GPU.

A request is a cage (a meshgen.Mesh), a scheme and a level count; its result
is the final level's face table and positions, left resident on the device.

Scheduler (`Server`, host logic only):
  * arrivals join a first-in first-out queue;
  * whenever an execution slot is free, the oldest queued request picks the
    group (scheme, levels); the longest run of that group's queued requests,
    in arrival order and at most `max_batch` long, whose device footprint
    fits the part of the HBM budget not held by batches in flight, is
    admitted as one batch;
  * a batch is one subdiv_plan_batch + subdiv_refine_batch on the slot's
    stream: every stage is one launch over all of its meshes, and every
    mesh's output is bitwise the one it gets when refined alone;
  * its requests complete when the batch's completion event has fired;
  * a request whose footprint alone exceeds the whole budget is rejected; a
    launch that runs out of device memory puts its requests back and retries
    with half the batch once memory has been released.
Latency = completion - arrival, on the host clock.

Footprint of a batch = the library's workspace bound for the union of its
cages + the device copy of the cages + every request's final-level face
table and positions (exact level sizes from the cage's edge count).

Baseline (`serve_per_mesh`): the same trace served first-in first-out with
one plan + refine per request on one stream.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

INF = float("inf")


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


_EDGE_CACHE: Dict[int, tuple] = {}


def edge_count(mesh) -> int:
    """Undirected edges of a cage (cached per face table object: the
    serving cages of one frequency share their topology arrays)."""
    key = id(mesh.verts)
    hit = _EDGE_CACHE.get(key)
    if hit is not None and hit[0] is mesh.verts:
        return hit[1]
    v = np.asarray(mesh.verts, np.int64)
    if mesh.offsets is None:
        f = v.reshape(-1, int(mesh.face_order))
        nxt = np.roll(f, -1, axis=1).reshape(-1)
    else:
        off = np.asarray(mesh.offsets, np.int64)
        cnt = np.diff(off)
        face = np.repeat(np.arange(cnt.size), cnt)
        slot = np.arange(v.size) - off[face]
        nxt = v[off[face] + (slot + 1) % cnt[face]]
    lo, hi = np.minimum(v, nxt), np.maximum(v, nxt)
    E = int(np.unique(hi * (int(v.max()) + 1) + lo).size)
    _EDGE_CACHE[key] = (mesh.verts, E)
    return E


def final_sizes(V: int, F: int, H: int, E: int, scheme: str, levels: int):
    """(V, F, H, E) of the refined level `levels` from the cage's counts.
    Catmull-Clark: one vertex per vertex, face and edge; one quad per
    half-edge; every edge splits in two and every half-edge adds one edge
    inside its face. Loop: one vertex per vertex and edge; four triangles per
    triangle; 2E + 3F edges. sqrt(3): one vertex per vertex and face; three
    triangles per triangle; every edge stays (flipped or on the boundary) and
    every face adds three."""
    for _ in range(levels):
        if scheme == "cc":
            V, F, H, E = V + F + E, H, 4 * H, 2 * E + H
        elif scheme == "loop":
            V, F, E = V + E, 4 * F, 2 * E + 3 * F
            H = 3 * F
        elif scheme == "sqrt3":
            V, F, E = V + F, 3 * F, E + 3 * F
            H = 3 * F
        else:
            raise ValueError(scheme)
    return V, F, H, E


def request_bytes(mesh, scheme: str, levels: int) -> tuple:
    """(io bytes, final faces): cage arrays in, final face table + positions out."""
    V, F, H, C = mesh.num_vertices, mesh.num_faces, mesh.num_halfedges, mesh.num_creases
    VL, FL, HL, _ = final_sizes(V, F, H, edge_count(mesh), scheme, levels)
    cage = 4 * H + 12 * V + 12 * C + (4 * (F + 1) if mesh.offsets is not None else 0)
    return cage + 4 * HL + 12 * VL, FL


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
    prepare(req), footprint_fn(reqs, scheme, levels) -> f(k) (bytes of the
    batch reqs[:k], non-decreasing in k, INF when it cannot be planned),
    launch(reqs, scheme, levels, slot) -> handle (may raise ExecutorOOM),
    done(handle) -> bool, results(handle) -> list of per-request outputs
    (called only when results are kept), retire(handle) (the batch's memory
    may be released once the outputs taken from it are dropped)."""

    def __init__(self, executor, hbm_budget: int, slots: int = 1, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
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

    # the longest admissible run of the head request's group
    def _form(self, queue: deque, avail: int):
        head = queue[0]
        key = (head.scheme, head.levels)
        cands = [r for r in queue if (r.scheme, r.levels) == key][: self._cap]
        faces = np.cumsum([r.final_faces for r in cands])
        cands = cands[: max(1, int(np.searchsorted(faces, self.max_batch_faces, side="right")))]
        f = self.ex.footprint_fn(cands, head.scheme, head.levels)
        if f(1) > avail:
            return None, f(1)
        lo, hi = 1, len(cands)  # f(lo) <= avail
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
            while i < n and reqs[i].arrival <= now:
                r = reqs[i]
                r.footprint, r.final_faces = request_bytes(r.mesh, r.scheme, r.levels)
                self.ex.prepare(r)
                queue.append(r)
                i += 1
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
                    h = self.ex.launch(batch, batch[0].scheme, batch[0].levels, free[0])
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
                ids = {id(r) for r in batch}
                queue = deque(r for r in queue if id(r) not in ids)
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


def _packed(mesh) -> tuple:
    """One int32 array holding a cage's face table, column pointer, crease
    pairs, positions and sharpness (float bits), every part starting on a
    16-byte boundary; returns (array, part offsets in ints)."""
    parts = [np.ascontiguousarray(mesh.verts, np.int32).reshape(-1)]
    parts.append(None if mesh.offsets is None else np.ascontiguousarray(mesh.offsets, np.int32).reshape(-1))
    parts.append(np.ascontiguousarray(mesh.crease_verts, np.int32).reshape(-1) if mesh.num_creases else None)
    parts.append(np.ascontiguousarray(mesh.positions, np.float32).reshape(-1).view(np.int32))
    parts.append(np.ascontiguousarray(mesh.crease_sharp, np.float32).reshape(-1).view(np.int32)
                 if mesh.num_creases else None)
    offs, chunks, at = [], [], 0
    for x in parts:
        if x is None:
            offs.append(-1)
            continue
        offs.append(at)
        pad = (-x.size) % 4
        chunks.append(x)
        if pad:
            chunks.append(np.zeros(pad, np.int32))
        at += x.size + pad
    return np.concatenate(chunks), offs


class GpuBatchExecutor:
    """Runs each batch through the library's batch entry points (all streams
    at the default priority): one upload of the packed cages, one workspace,
    one allocation per output kind.

    one_refine_stream=False: every slot plans and refines on its own stream.
    one_refine_stream=True: plans go to a plan stream and every refinement to
    one refine stream, so with two slots the next batch is uploaded and
    planned while the previous one refines, and its refinement queues behind
    it instead of running beside it. A batch's cage upload and workspace are
    allocated for the plan stream and its outputs for the refine stream; all
    of them are released only after the batch has retired."""

    def __init__(self, device="cuda", slots: int = 1, reserve_bytes: int = 0, one_refine_stream: bool = False):
        import torch
        from . import _lib
        self.torch = torch
        self._lib = _lib
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.one_refine_stream = one_refine_stream
        if one_refine_stream:
            self.plan_stream = torch.cuda.Stream(self.device)
            self.refine_stream = torch.cuda.Stream(self.device)
            for s in (self.plan_stream, self.refine_stream):
                reserve(self.device, reserve_bytes, s)
        else:
            self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
            for s in self.streams:
                reserve(self.device, reserve_bytes, s)

    def prepare(self, r: Request):
        m = r.mesh
        r.meta["packed"] = _packed(m)
        s = self._lib.subdiv_mesh()
        s.num_vertices, s.num_faces, s.num_halfedges = m.num_vertices, m.num_faces, m.num_halfedges
        s.face_order = 0 if m.offsets is not None else m.face_order
        s.face_offsets = 16 if m.offsets is not None else None  # sizes only: never dereferenced
        s.face_verts = s.positions = 16
        s.num_creases = m.num_creases
        if m.num_creases:
            s.crease_verts = s.crease_sharpness = 16
        r.meta["shape"] = s

    def footprint_fn(self, reqs, scheme, levels):
        structs = (self._lib.subdiv_mesh * len(reqs))(*[r.meta["shape"] for r in reqs])
        io = np.cumsum([r.footprint for r in reqs])
        sid = self._lib.SCHEMES[scheme]
        lib = self.lib

        def f(k: int):
            ws = int(lib.subdiv_batch_workspace_bound(structs, k, sid, levels, 0))
            return INF if ws == 0 else ws + int(io[k - 1])
        return f

    def launch(self, reqs, scheme, levels, slot):
        import ctypes
        torch, L, lib = self.torch, self._lib, self.lib
        if self.one_refine_stream:
            s, rs = self.plan_stream, self.refine_stream
        else:
            s = rs = self.streams[slot]
        n = len(reqs)
        sid = L.SCHEMES[scheme]
        try:
            with torch.cuda.stream(s):
                host = np.concatenate([r.meta["packed"][0] for r in reqs])
                dev = torch.from_numpy(host).to(self.device)
                base = dev.data_ptr()
                structs = (L.subdiv_mesh * n)()
                at = 0
                for k, r in enumerate(reqs):
                    arr, offs = r.meta["packed"]
                    structs[k] = r.meta["shape"]
                    st = structs[k]  # a view into the array
                    st.face_verts = base + 4 * (at + offs[0])
                    st.face_offsets = None if offs[1] < 0 else base + 4 * (at + offs[1])
                    st.crease_verts = None if offs[2] < 0 else base + 4 * (at + offs[2])
                    st.positions = base + 4 * (at + offs[3])
                    st.crease_sharpness = None if offs[4] < 0 else base + 4 * (at + offs[4])
                    at += arr.size
                ws_bytes = int(lib.subdiv_batch_workspace_bound(structs, n, sid, levels, 0))
                if ws_bytes == 0:
                    raise L.SubdivError(L.INVALID_ARG, "subdiv_batch_workspace_bound")
                ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
                bplan = L.subdiv_batch_plan()
                plans = (L.subdiv_plan_info * n)()
                L.check(lib.subdiv_plan_batch(structs, n, sid, levels, 0, ctypes.c_void_p(ws.data_ptr()), ws_bytes,
                                              ctypes.byref(bplan), plans, ctypes.c_void_p(s.cuda_stream)),
                        "subdiv_plan_batch")
            # (the plan read back on s: its work is done before the refinement below starts)
            with torch.cuda.stream(rs):
                # outputs: one int32 and one float32 allocation, every face table 16-byte aligned
                hs = [int(plans[k].level[levels].num_halfedges) for k in range(n)]
                vs = [int(plans[k].level[levels].num_vertices) for k in range(n)]
                hofs = np.concatenate([[0], np.cumsum([(h + 3) // 4 * 4 for h in hs])])
                vofs = np.concatenate([[0], np.cumsum(vs)])
                fv = torch.empty(int(hofs[-1]), dtype=torch.int32, device=self.device)
                P = torch.empty((int(vofs[-1]), 3), dtype=torch.float32, device=self.device)
                outs = (L.subdiv_level_out * n)()
                for k in range(n):
                    outs[k].face_verts = fv.data_ptr() + 4 * int(hofs[k])
                    outs[k].positions = P.data_ptr() + 12 * int(vofs[k])
                L.check(lib.subdiv_refine_batch(structs, n, ctypes.byref(bplan), outs, ctypes.c_void_p(ws.data_ptr()),
                                                ws_bytes, ctypes.c_void_p(rs.cuda_stream)), "subdiv_refine_batch")
                ev = torch.cuda.Event()
                ev.record(rs)
        except torch.cuda.OutOfMemoryError as e:
            raise ExecutorOOM(str(e)) from e
        return dict(ev=ev, keep=(dev, ws, fv, P), hofs=hofs, hs=hs, vofs=vofs)

    def done(self, h) -> bool:
        return h["ev"].query()

    def results(self, h):
        fv, P = h["keep"][2], h["keep"][3]
        return [{"face_verts": fv[int(h["hofs"][k]):int(h["hofs"][k]) + h["hs"][k]],
                 "positions": P[int(h["vofs"][k]):int(h["vofs"][k + 1])]} for k in range(len(h["hs"]))]

    def retire(self, h):
        h.clear()


def serve_per_mesh(requests: List[Request], device="cuda", clock=time.perf_counter, sleep=time.sleep,
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
        r.footprint, r.final_faces = request_bytes(r.mesh, r.scheme, r.levels)
        outs, _ = refine(r.mesh, r.scheme, r.levels, device=device)
        r.done = clock() - t0
        r.result = outs[r.levels] if keep_results else None
    torch.cuda.synchronize(device)
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
          log=print, one_refine_stream: bool = True) -> Dict:
    """Measure the per-mesh-launch saturation rate, then serve the trace at
    each factor x that rate with the batched server and the baseline. By
    default two batches are in flight: the next one is uploaded and planned
    while the previous one refines, and refinements run one after the other
    on one stream."""
    import torch
    trace = make_trace(n_requests, seed=seed, qps=1.0)
    base_t = np.array([r.arrival for r in trace])
    # both servers start from an allocator that already holds the memory a
    # large request needs (one segment per stream they use)
    reserve_bytes = int(min(budget_gib, 8.0) * 2**30) // max(1, slots)
    reserve(device, reserve_bytes)
    ex = GpuBatchExecutor(device, slots, reserve_bytes, one_refine_stream=one_refine_stream)
    # warm-up of both paths: one request of every (scheme, levels) group and
    # the head of the trace, all arriving at once
    seen, warm = set(), []
    for r in trace:
        if (r.scheme, r.levels) not in seen:
            seen.add((r.scheme, r.levels))
            warm.append(r)
    warm += trace[:min(64, n_requests)]
    Server(ex, int(budget_gib * 2**30), slots, max_batch).run(_retime(warm, np.zeros(len(warm)), 1.0))
    serve_per_mesh(_retime(warm, np.zeros(len(warm)), 1.0), device)
    # saturation of the baseline: everything arrives at t = 0
    ns = min(n_requests, sat_requests or n_requests)
    sat_reqs = _retime(trace[:ns], np.zeros(ns), 1.0)
    sat = serve_per_mesh(sat_reqs, device)
    sat_qps = ns / sat["makespan"]
    log(f"[serve] per-mesh saturation {sat_qps:.1f} req/s over {ns} requests")
    points = []
    for fac in factors:
        qps = fac * sat_qps
        rb = _retime(trace, base_t, qps)
        srv = Server(ex, int(budget_gib * 2**30), slots, max_batch)
        torch.cuda.reset_peak_memory_stats(device)
        st = srv.run(rb)
        b = summarize(rb, st["makespan"])
        b.update(batches=st["batches"], mean_batch=float(np.mean(st["batch_sizes"])) if st["batch_sizes"] else 0.0,
                 max_queue=st["max_queue"], peak_admitted_gib=st["peak_admitted_bytes"] / 2**30,
                 peak_allocated_gib=torch.cuda.max_memory_allocated(device) / 2**30)
        rp = _retime(trace, base_t, qps)
        sp = serve_per_mesh(rp, device)
        p = summarize(rp, sp["makespan"])
        points.append(dict(factor=fac, qps=qps, batched=b, per_mesh=p))
        log(f"[serve] x{fac}: {qps:.0f} req/s batched p50 {b['p50_ms']:.2f} p99 {b['p99_ms']:.2f} ms "
            f"(mean batch {b['mean_batch']:.1f}) | per-mesh p50 {p['p50_ms']:.2f} p99 {p['p99_ms']:.2f} ms")
    return dict(requests=n_requests, seed=seed, budget_gib=budget_gib, slots=slots, max_batch=max_batch,
                per_mesh_saturation_qps=sat_qps, points=points)


def main(argv=None):
    ap = argparse.ArgumentParser(description="continuous-batching refinement server: QPS sweep")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--factors", default="0.5,0.8,1.0,1.2,1.5,2,3")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=1,
                    help="batches in flight at once (one: a second concurrent batch only slows the first)")
    ap.add_argument("--max-batch", type=int, default=256)
    a = ap.parse_args(argv)
    res = sweep(a.requests, tuple(float(x) for x in a.factors.split(",")), a.seed, a.budget_gib, a.slots,
                a.max_batch)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
