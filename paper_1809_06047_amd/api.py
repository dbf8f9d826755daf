"""Python surface over the C ABI: device uploads, workspace and output
allocation with torch (device memory and streams only), plan + refine.

Every step of the refinement runs in libsubdiv's HIP kernels; this module
only allocates buffers and passes pointers.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _lib
from ._lib import check, load


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def current_stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class DeviceMesh:
    """A cage uploaded to the device; keeps its tensors alive."""

    def __init__(self, mesh, device="cuda"):
        dev = torch.device(device)
        self.device = dev
        self.name = getattr(mesh, "name", "")
        self.verts = torch.from_numpy(np.ascontiguousarray(mesh.verts, np.int32)).to(dev)
        self.offsets = None if mesh.offsets is None else torch.from_numpy(
            np.ascontiguousarray(mesh.offsets, np.int32)).to(dev)
        self.positions = torch.from_numpy(np.ascontiguousarray(mesh.positions, np.float32)).to(dev)
        C = mesh.num_creases
        self.crease_verts = torch.from_numpy(np.ascontiguousarray(mesh.crease_verts, np.int32)).to(dev) if C else None
        self.crease_sharp = torch.from_numpy(np.ascontiguousarray(mesh.crease_sharp, np.float32)).to(dev) if C \
            else None
        self.V = int(mesh.num_vertices)
        self.F = int(mesh.num_faces)
        self.H = int(mesh.num_halfedges)
        self.C = int(C)
        self.order = 0 if mesh.offsets is not None else int(mesh.face_order)
        self.struct = self._make_struct()

    @classmethod
    def from_tensors(cls, verts, offsets, positions, crease_verts, crease_sharp, face_order: int, name: str = ""):
        """A cage whose arrays already live on the device (e.g. views into one
        packed upload); offsets None means uniform `face_order`."""
        self = cls.__new__(cls)
        self.device = verts.device
        self.name = name
        self.verts, self.offsets, self.positions = verts, offsets, positions
        self.crease_verts, self.crease_sharp = crease_verts, crease_sharp
        self.V = int(positions.shape[0])
        self.F = int(offsets.shape[0] - 1) if offsets is not None else int(verts.shape[0]) // int(face_order)
        self.H = int(verts.shape[0])
        self.C = 0 if crease_verts is None else int(crease_verts.shape[0])
        self.order = 0 if offsets is not None else int(face_order)
        self.struct = self._make_struct()
        return self

    def _make_struct(self):
        m = _lib.subdiv_mesh()
        m.num_vertices = self.V
        m.num_faces = self.F
        m.face_order = self.order
        m.num_halfedges = self.H
        m.face_offsets = None if self.offsets is None else self.offsets.data_ptr()
        m.face_verts = self.verts.data_ptr()
        m.positions = self.positions.data_ptr()
        m.num_creases = self.C
        m.crease_verts = None if self.crease_verts is None else self.crease_verts.data_ptr()
        m.crease_sharpness = None if self.crease_sharp is None else self.crease_sharp.data_ptr()
        return m

    def set_positions(self, P: torch.Tensor):
        """Point the cage at other positions (same topology), e.g. for autograd."""
        assert P.shape == (self.V, 3) and P.dtype == torch.float32 and P.is_contiguous()
        self.positions = P
        self.struct.positions = P.data_ptr()


class Refiner:
    """Plan + refine of one cage. `keep` selects the levels whose meshes are
    kept as outputs (the final level always is)."""

    def __init__(self, mesh, scheme, levels: int, flags: int = 0, keep: str = "final", edges: bool = False,
                 creases: bool = False, device="cuda"):
        load()
        self.dmesh = mesh if isinstance(mesh, DeviceMesh) else DeviceMesh(mesh, device)
        self.scheme = _lib.SCHEMES.get(scheme, scheme)
        self.levels = int(levels)
        self.flags = int(flags)
        self.keep = keep
        self.want_edges = edges
        self.want_creases = creases
        lib = load()
        d = self.dmesh
        self.ws_bytes = int(lib.subdiv_workspace_bound(d.V, d.F, d.H, d.C, self.scheme, self.levels, self.flags))
        if self.ws_bytes == 0:
            raise _lib.SubdivError(_lib.INVALID_ARG, "subdiv_workspace_bound")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=d.device)
        self.plan_info = _lib.subdiv_plan_info()
        self.outs: List[Dict[str, torch.Tensor]] = []
        self._outs_struct = None

    def plan(self, stream=None):
        lib = load()
        s = current_stream_handle(self.dmesh.device) if stream is None else stream
        st = lib.subdiv_plan(ctypes.byref(self.dmesh.struct), self.scheme, self.levels, self.flags,
                             ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.byref(self.plan_info),
                             ctypes.c_void_p(s))
        check(st, "subdiv_plan")
        if self.plan_info.workspace_bytes > self.ws_bytes:
            raise _lib.SubdivError(_lib.WORKSPACE, "workspace bound below the planned size")
        self._alloc_outputs()
        self._state_ready = False  # a new plan: the next run rebuilds the kept state
        return self.plan_info

    def level_info(self, k):
        li = self.plan_info.level[k]
        return dict(V=li.num_vertices, E=li.num_edges, F=li.num_faces, H=li.num_halfedges,
                    B=li.num_boundary_edges, order=li.face_order, max_creases=li.max_creases)

    def _alloc_outputs(self):
        dev = self.dmesh.device
        L = self.levels
        arr = (_lib.subdiv_level_out * (L + 1))()
        self.outs = [dict() for _ in range(L + 1)]
        for k in range(1, L + 1):
            if self.keep != "all" and k != L:
                continue
            li = self.plan_info.level[k]
            o = self.outs[k]
            o["face_verts"] = torch.empty(li.num_halfedges, dtype=torch.int32, device=dev)
            o["positions"] = torch.empty((li.num_vertices, 3), dtype=torch.float32, device=dev)
            if self.want_edges:
                o["edge_verts"] = torch.empty((self.plan_info.level[k - 1].num_edges, 2), dtype=torch.int32,
                                              device=dev)
            if self.want_creases and li.max_creases > 0:
                o["crease_sharpness"] = torch.zeros(li.num_edges, dtype=torch.float64, device=dev)
            arr[k].face_verts = o["face_verts"].data_ptr()
            arr[k].positions = o["positions"].data_ptr()
            if "edge_verts" in o:
                arr[k].edge_verts = o["edge_verts"].data_ptr()
            if "crease_sharpness" in o:
                arr[k].crease_sharpness = o["crease_sharpness"].data_ptr()
        self._outs_struct = arr

    def run(self, stream=None):
        """Enqueue the refinement (no host synchronisation)."""
        lib = load()
        s = current_stream_handle(self.dmesh.device) if stream is None else stream
        st = lib.subdiv_refine(ctypes.byref(self.dmesh.struct), ctypes.byref(self.plan_info), self._outs_struct,
                               ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.c_void_p(s))
        check(st, "subdiv_refine")
        return self.outs

    def run_static(self, stream=None):
        """The refinement in the library's own device workspace
        (subdiv_refine_static): same outputs as run(), nothing allocated by the
        call; the plan may come from any workspace."""
        lib = load()
        s = current_stream_handle(self.dmesh.device) if stream is None else stream
        st = lib.subdiv_refine_static(ctypes.byref(self.dmesh.struct), ctypes.byref(self.plan_info),
                                      self._outs_struct, ctypes.c_void_p(s))
        check(st, "subdiv_refine_static")
        return self.outs

    def run_positions(self, stream=None):
        """Static topology: refine the cage's current positions again with the
        kept state of the last run (plan with FLAG_KEEP_STATE, Catmull-Clark);
        only the position outputs are written. Enqueues work only."""
        lib = load()
        s = current_stream_handle(self.dmesh.device) if stream is None else stream
        st = lib.subdiv_refine_positions(ctypes.byref(self.dmesh.struct), ctypes.byref(self.plan_info),
                                         self._outs_struct, ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                         ctypes.c_void_p(s))
        check(st, "subdiv_refine_positions")
        return self.outs

    def run_vertex_data(self, data: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """General vertex data ([V_0, dim] float32 on the device, any dim >= 1:
        UVs, colours, ...) refined with the kept state of the last run, like
        run_positions (plan with FLAG_KEEP_STATE, Catmull-Clark); returns
        [V_L, dim]. Enqueues work only."""
        lib = load()
        d = self.dmesh
        dev = torch.device(d.device)
        same_dev = data.device.type == dev.type and (dev.index is None or data.device.index == dev.index)
        if data.dim() != 2 or data.shape[0] != d.V or data.dtype != torch.float32 or not same_dev:
            raise ValueError(f"vertex data must be a [{d.V}, dim] float32 tensor on {d.device}")
        data = data.contiguous()
        dim = int(data.shape[1])
        VL = self.plan_info.level[self.levels].num_vertices
        if out is None:
            out = torch.empty((VL, dim), dtype=torch.float32, device=d.device)
        elif tuple(out.shape) != (VL, dim) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous [{VL}, {dim}] float32 tensor")
        s = current_stream_handle(d.device) if stream is None else stream
        st = lib.subdiv_refine_vertex_data(ctypes.byref(d.struct), ctypes.byref(self.plan_info),
                                           ctypes.c_void_p(data.data_ptr()), dim, ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.c_void_p(s))
        check(st, "subdiv_refine_vertex_data")
        return out

    @property
    def final(self):
        return self.outs[self.levels]

    def release(self):
        """Drop the library's record of the state this refiner's plan keeps in
        its workspace (subdiv_state_destroy); later state calls on it fail
        until the next plan and run. Returns True when a state was dropped."""
        st = load().subdiv_state_destroy(ctypes.byref(self.plan_info), ctypes.c_void_p(self.ws.data_ptr()))
        self._state_ready = False
        return st == _lib.OK

    def backward(self, grad_out: torch.Tensor, grad_in: Optional[torch.Tensor] = None, stream=None):
        """grad_in = R^T grad_out for the last run (needs flags with
        FLAG_KEEP_STATE). Enqueues work only."""
        lib = load()
        d = self.dmesh
        g = grad_out.contiguous()
        assert g.dtype == torch.float32 and g.shape == (self.plan_info.level[self.levels].num_vertices, 3)
        if grad_in is None:
            grad_in = torch.empty((d.V, 3), dtype=torch.float32, device=d.device)
        s = current_stream_handle(d.device) if stream is None else stream
        st = lib.subdiv_backward(ctypes.byref(d.struct), ctypes.byref(self.plan_info), ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(grad_in.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                 self.ws_bytes, ctypes.c_void_p(s))
        check(st, "subdiv_backward")
        return grad_in


class SubdivFunction(torch.autograd.Function):
    """P_L = refine(P_0) with the hand-written adjoint as its backward.
    `refiner` must be planned with FLAG_KEEP_STATE; the topology (and
    creases) are the refiner's, the positions the differentiable input."""

    @staticmethod
    def forward(ctx, P0: torch.Tensor, refiner: "Refiner"):
        P0c = P0.detach().contiguous()
        refiner.dmesh.set_positions(P0c)
        # the topology is fixed: after the first run only positions are recomputed
        outs = refiner.run_positions() if getattr(refiner, "_state_ready", False) else refiner.run()
        refiner._state_ready = True
        ctx.refiner = refiner
        ctx.keep = P0c
        return outs[refiner.levels]["positions"].clone()

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.refiner.backward(grad_out.float())
        return g, None


def differentiable_refiner(mesh, levels: int, device="cuda") -> "Refiner":
    """A planned Catmull-Clark refiner whose runs can be differentiated."""
    r = Refiner(mesh, "cc", levels, flags=_lib.FLAG_KEEP_STATE, device=device)
    r.plan()
    return r


def refine(mesh, scheme, levels: int, flags: int = 0, keep: str = "final", edges: bool = False,
           creases: bool = False, device="cuda"):
    """Refine `mesh` (a meshgen.Mesh or DeviceMesh) `levels` times; returns
    the list of per-level output dicts (index 0 empty) after synchronising."""
    r = Refiner(mesh, scheme, levels, flags, keep, edges, creases, device)
    r.plan()
    outs = r.run()
    torch.cuda.synchronize(r.dmesh.device)
    return outs, r


def extract_region(r: "Refiner", seed: Optional[torch.Tensor] = None, rings: int = 1, stream=None,
                   close_pinches: bool = False) -> Dict:
    """Selective subdivision (Sec. 3.4): the region around the seed vertices
    of `r`'s cage (planned with r.plan()), `rings` face rings deep, as a cage
    of its own. seed: [V] uint8/bool device mask, or None for the
    extraordinary vertices (valence != 4). Returns the extracted arrays, the
    maps back to the cage and a DeviceMesh of the extraction ("mesh", None
    when nothing is selected). Synchronises once (the sizes)."""
    lib = load()
    d = r.dmesh
    s = current_stream_handle(d.device) if stream is None else stream
    seed_ptr = None
    if seed is not None:
        if seed.shape != (d.V,) or seed.dtype not in (torch.uint8, torch.bool) or not seed.is_cuda:
            raise ValueError(f"seed must be a [{d.V}] uint8 or bool device tensor")
        seed = seed.to(torch.uint8).contiguous()
        seed_ptr = ctypes.c_void_p(seed.data_ptr())
    sel = _lib.subdiv_selection()
    check(lib.subdiv_select_ex(ctypes.byref(d.struct), ctypes.byref(r.plan_info), seed_ptr, int(rings),
                               _lib.SELECT_CLOSE_PINCHES if close_pinches else 0, ctypes.c_void_p(r.ws.data_ptr()),
                               r.ws_bytes, ctypes.byref(sel), ctypes.c_void_p(s)), "subdiv_select_ex")
    V1, F1, H1, C1, order = sel.num_vertices, sel.num_faces, sel.num_halfedges, sel.num_creases, sel.face_order
    dev = d.device
    out = {"positions": torch.empty((V1, 3), dtype=torch.float32, device=dev),
           "face_verts": torch.empty(H1, dtype=torch.int32, device=dev),
           "face_offsets": (torch.empty if F1 else torch.zeros)(F1 + 1, dtype=torch.int32, device=dev)
           if order == 0 else None,
           "crease_verts": torch.empty((C1, 2), dtype=torch.int32, device=dev) if C1 else None,
           "crease_sharpness": torch.empty(C1, dtype=torch.float32, device=dev) if C1 else None,
           "vertex_map": torch.empty(V1, dtype=torch.int32, device=dev),
           "face_map": torch.empty(F1, dtype=torch.int32, device=dev),
           "seed_flags": torch.empty(V1, dtype=torch.uint8, device=dev)}
    e = _lib.subdiv_extraction()
    for k in ("positions", "face_verts", "face_offsets", "crease_verts", "vertex_map", "face_map", "seed_flags"):
        if out[k] is not None and out[k].numel():
            setattr(e, k, out[k].data_ptr())
    if out["crease_sharpness"] is not None:
        e.crease_sharpness = out["crease_sharpness"].data_ptr()
    check(lib.subdiv_extract(ctypes.byref(d.struct), ctypes.byref(r.plan_info), ctypes.byref(sel), ctypes.byref(e),
                             ctypes.c_void_p(r.ws.data_ptr()), r.ws_bytes, ctypes.c_void_p(s)), "subdiv_extract")
    out["mesh"] = None if V1 == 0 else DeviceMesh.from_tensors(
        out["face_verts"], out["face_offsets"], out["positions"], out["crease_verts"], out["crease_sharpness"],
        order if order else 0, name=f"{d.name}-region")
    return out


def adaptive_refine(mesh, levels: int, rings: int = 1, seed: Optional[torch.Tensor] = None, device="cuda",
                    stream=None) -> List[Dict]:
    """Feature-adaptive Catmull-Clark refinement (Sec. 3.4, level after
    level): on every level the region `rings` face rings around the seeds is
    selected and extracted (subdiv_select, subdiv_extract), and only that
    region is refined one level (subdiv_plan, subdiv_refine); the seeds - the
    cage's extraordinary vertices (valence != 4) unless `seed` is given - keep
    their ids through the refinement and are carried into every extraction
    (the extraction's seed flags), while the extraction's own boundary never
    seeds; pinches (regions touching at one vertex) are closed
    (SUBDIV_SELECT_CLOSE_PINCHES). Returns, per level k = 0 .. levels-1
    (fewer when a selection comes out empty), the extraction of level k
    ("region": DeviceMesh, with vertex_map / face_map into level k's mesh)
    and the refined region of level k + 1 ("mesh": DeviceMesh, whose first
    region-vertex-count vertices are the region's vertices). Cages with creases are refused (the
    refined region's sharpness would have to become a crease list again).
    Each level synchronises on the plans and the selection (sizes)."""
    dm = mesh if isinstance(mesh, DeviceMesh) else DeviceMesh(mesh, device)
    if dm.C:
        raise ValueError("adaptive_refine takes cages without creases")
    out = []
    cur = Refiner(dm, "cc", 1)
    cur.plan(stream)
    for k in range(int(levels)):
        reg = extract_region(cur, seed, rings, stream, close_pinches=True)
        if reg["mesh"] is None:
            break
        rr = Refiner(reg["mesh"], "cc", 1)
        rr.plan(stream)
        fin = rr.run(stream)[1]
        V1 = rr.level_info(1)["V"]
        nxt = DeviceMesh.from_tensors(fin["face_verts"], None, fin["positions"], None, None, 4,
                                      name=f"{dm.name}-adaptive{k + 1}")
        out.append({"level": k, "region": reg["mesh"], "vertex_map": reg["vertex_map"], "face_map": reg["face_map"],
                    "mesh": nxt})
        # the region's vertices keep their ids in its refinement; the new
        # points never seed
        seed = torch.zeros(V1, dtype=torch.uint8, device=dm.device)
        seed[:reg["mesh"].V].copy_(reg["seed_flags"])
        if k + 1 < levels:
            cur = Refiner(nxt, "cc", 1)
            cur.plan(stream)
    return out


def rcm_reorder(mesh):
    """Mesh reordering (Sec. 4.5) of a host cage (meshgen.Mesh): the library's
    reverse Cuthill-McKee permutations applied to it. Returns (reordered
    mesh, vertex_perm, face_perm), perms mapping new id -> old id."""
    from . import meshgen
    lib = load()
    V, F = mesh.num_vertices, mesh.num_faces
    verts = np.ascontiguousarray(mesh.verts, np.int32)
    offs = None if mesh.offsets is None else np.ascontiguousarray(mesh.offsets, np.int32)
    vperm = np.empty(V, np.int32)
    fperm = np.empty(F, np.int32)
    ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    check(lib.subdiv_rcm_order(V, F, ptr(offs), 0 if offs is not None else int(mesh.face_order), ptr(verts),
                               ptr(vperm), ptr(fperm)), "subdiv_rcm_order")
    newid = np.empty(V, np.int32)
    newid[vperm] = np.arange(V, dtype=np.int32)
    if offs is None:
        k = int(mesh.face_order)
        nverts = newid[verts.reshape(F, k)[fperm]].reshape(-1)
        noffs = None
    else:
        sizes = np.diff(offs)[fperm]
        noffs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        idx = np.concatenate([np.arange(offs[f], offs[f + 1]) for f in fperm])
        nverts = newid[verts[idx]]
    cv = None if mesh.crease_verts is None else newid[np.asarray(mesh.crease_verts, np.int32)]
    out = meshgen.Mesh(positions=np.asarray(mesh.positions)[vperm], verts=nverts.astype(np.int32), offsets=noffs,
                       face_order=mesh.face_order if offs is None else 0, crease_verts=cv,
                       crease_sharp=mesh.crease_sharp, name=f"{mesh.name}-rcm")
    return out, vperm, fperm


def plan_status(mesh, scheme, levels: int = 1, device="cuda") -> int:
    """Status subdiv_plan reports for this cage (0 = accepted)."""
    try:
        Refiner(mesh, scheme, levels, device=device).plan()
        return 0
    except _lib.SubdivError as e:
        return e.status


class StreamingRefiner:
    """Cages with changing topology, refined one after the other, `depth`
    deep (default two): the plan of cage i (into its own workspace, on a plan
    stream) overlaps the refinement of cage i-1, so the GPU does not idle
    while the host waits for a plan's read-back. Each slot (workspace,
    outputs) has its own refine stream, so cage i's refinement also runs
    beside the ones before it: the launch-bound small levels of one fill the
    gaps of another's HBM-bound last level. Every cage is still validated, built and refined
    in full. step() returns the cage's output dicts (as Refiner.run) and an
    event recorded after its refinement; the tensors are ready once the
    event has completed. A slot's refiner is reused while the cage is the
    same DeviceMesh, its plan waits for the refinement that last used its
    workspace, and its refinements run in order on its stream. All streams
    have the default priority."""

    def __init__(self, scheme, levels: int, flags: int = 0, keep: str = "final", device="cuda", depth: int = 2):
        self.scheme, self.levels, self.flags, self.keep = scheme, int(levels), int(flags), keep
        if int(depth) < 1:
            raise ValueError("depth must be at least 1")
        self.depth = int(depth)
        dev = torch.device(device)
        self.plan_stream = torch.cuda.Stream(dev)
        self.refine_streams = [torch.cuda.Stream(dev) for _ in range(self.depth)]
        self.slots: List[Optional[Refiner]] = [None] * self.depth
        self.done: List[Optional[torch.cuda.Event]] = [None] * self.depth
        self.i = 0

    def refiner(self, slot: int) -> Optional[Refiner]:
        """The slot's refiner. Its last refinement may still run on the slot's
        stream (non-blocking): wait for it (the event step() returned, or a
        device synchronisation) before planning or refining with it on another
        stream, since a plan rewrites the workspace that refinement reads."""
        return self.slots[slot]

    def step(self, dmesh: "DeviceMesh"):
        j = self.i % self.depth
        r = self.slots[j]
        rs = self.refine_streams[j]
        if self.done[j] is not None:
            self.plan_stream.wait_event(self.done[j])
        if r is None or r.dmesh is not dmesh:
            with torch.cuda.stream(rs):
                r = Refiner(dmesh, self.scheme, self.levels, self.flags, self.keep)
            self.slots[j] = r
        with torch.cuda.stream(rs):  # the slot's outputs are allocated for, and written on, its stream
            r.plan(stream=self.plan_stream.cuda_stream)
            outs = r.run(stream=rs.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(rs)
        self.done[j] = ev
        self.i += 1
        return outs, ev


def _per_mesh(x, n, conv=int):
    if isinstance(x, (list, tuple, np.ndarray)):
        if len(x) != n:
            raise ValueError(f"expected {n} values, got {len(x)}")
        return [conv(v) for v in x]
    return [conv(x)] * n


def mesh_shape_struct(m) -> "_lib.subdiv_mesh":
    """A subdiv_mesh carrying a host cage's sizes only (for the host-only
    size queries; its pointers are placeholders that are never read)."""
    s = _lib.subdiv_mesh()
    s.num_vertices, s.num_faces, s.num_halfedges = m.num_vertices, m.num_faces, m.num_halfedges
    s.face_order = 0 if m.offsets is not None else m.face_order
    s.face_offsets = 16 if m.offsets is not None else None
    s.face_verts = s.positions = 16
    s.num_creases = m.num_creases
    if m.num_creases:
        s.crease_verts = s.crease_sharpness = 16
    return s


class BatchRefiner:
    """A batch of uneven meshes, each with its own scheme and level count
    (`schemes` / `levels`: one value for every mesh, or one per mesh). The
    library groups the meshes by (scheme, levels) and refines each group
    with one launch per stage; every mesh's final level lands in its own
    tensors. Meshes are meshgen.Mesh or DeviceMesh.

    plan() runs subdiv_plan_batch: one read-back for the whole batch, one
    plan per mesh. `plans` (one subdiv_plan_info per mesh, e.g. kept from
    earlier plans of the same device cages) skips it. run() enqueues
    subdiv_refine_batch, which never waits for the device."""

    def __init__(self, meshes, schemes, levels, flags: int = 0, device="cuda", ws: Optional[torch.Tensor] = None,
                 plans=None):
        load()
        self.dmeshes = [m if isinstance(m, DeviceMesh) else DeviceMesh(m, device) for m in meshes]
        self.n = len(self.dmeshes)
        self.schemes = _per_mesh(schemes, self.n, lambda v: _lib.SCHEMES.get(v, v))
        self.levels = _per_mesh(levels, self.n)
        self.flags = int(flags)
        self.device = self.dmeshes[0].device
        self.structs = (_lib.subdiv_mesh * self.n)(*[d.struct for d in self.dmeshes])
        self.c_schemes = (ctypes.c_int * self.n)(*self.schemes)
        self.c_levels = (ctypes.c_int * self.n)(*self.levels)
        self.plans = (_lib.subdiv_plan_info * self.n)()
        self.outs: List[Dict[str, torch.Tensor]] = []
        self._ws_arg = ws
        self.ws = None
        self.ws_bytes = 0
        if plans is not None:
            for i, p in enumerate(plans):
                self.plans[i] = p
            self._alloc()

    @staticmethod
    def footprint(meshes, schemes, levels, flags: int = 0, plans=None) -> int:
        """Workspace bytes of a batch of host cages (host-only): exact for the
        refinement when `plans` are given, an upper bound otherwise."""
        n = len(meshes)
        structs = (_lib.subdiv_mesh * n)(*[mesh_shape_struct(m) for m in meshes])
        sc = (ctypes.c_int * n)(*_per_mesh(schemes, n, lambda v: _lib.SCHEMES.get(v, v)))
        lv = (ctypes.c_int * n)(*_per_mesh(levels, n))
        pl = None
        if plans is not None:
            pl = (_lib.subdiv_plan_info * n)(*plans)
        return int(load().subdiv_batch_workspace_bound(structs, sc, lv, n, pl, flags))

    def _ensure_ws(self, with_plans: bool):
        lib = load()
        need = int(lib.subdiv_batch_workspace_bound(self.structs, self.c_schemes, self.c_levels, self.n,
                                                    self.plans if with_plans else None, self.flags))
        if need == 0:
            raise _lib.SubdivError(_lib.INVALID_ARG, "subdiv_batch_workspace_bound")
        if self.ws is None or self.ws_bytes < need:
            if self._ws_arg is not None and self._ws_arg.numel() >= need:
                self.ws = self._ws_arg
            else:
                self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.ws_bytes = int(self.ws.numel())

    def plan(self, stream=None):
        lib = load()
        self._ensure_ws(False)
        s = current_stream_handle(self.device) if stream is None else stream
        st = lib.subdiv_plan_batch(self.structs, self.c_schemes, self.c_levels, self.n, self.flags,
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.plans, ctypes.c_void_p(s))
        check(st, "subdiv_plan_batch")
        self._alloc()
        return self.plans

    def _alloc(self):
        arr = (_lib.subdiv_level_out * self.n)()
        self.outs = []
        for i in range(self.n):
            li = self.plans[i].level[self.levels[i]]
            fv = torch.empty(li.num_halfedges, dtype=torch.int32, device=self.device)
            P = torch.empty((li.num_vertices, 3), dtype=torch.float32, device=self.device)
            arr[i].face_verts = fv.data_ptr()
            arr[i].positions = P.data_ptr()
            self.outs.append({"face_verts": fv, "positions": P})
        self._outs_struct = arr

    def output_faces(self) -> int:
        return sum(int(self.plans[i].level[self.levels[i]].num_faces) for i in range(self.n))

    def run(self, stream=None):
        lib = load()
        self._ensure_ws(True)
        s = current_stream_handle(self.device) if stream is None else stream
        st = lib.subdiv_refine_batch(self.structs, self.c_schemes, self.c_levels, self.n, self.plans,
                                     self._outs_struct, ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                     ctypes.c_void_p(s))
        check(st, "subdiv_refine_batch")
        return self.outs
