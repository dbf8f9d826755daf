#!/usr/bin/env python3
"""Benchmark: Catmull-Clark refined faces/s at level 6 on the 10k-vertex
mixed triangle/quad cage (icosphere level 5, 30% of adjacent triangle pairs
merged into quads, 3% of edges creased with sharpness U[0,4), jitter
N(0, 0.01)), one MI355X.

One step = subdiv_plan (cage validation + adjacency, the symbolic pass, with
its host read-back) + subdiv_refine levels 0 -> 6 (build and eval at every
level, dynamic topology: nothing is precomputed across steps). The cage is
resident in HBM before the timed region; outputs are written to preallocated
device buffers.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (timed live with HIP events on the library's stream) and the FP64
oracle timed on one host core over a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CC refined faces/s at level 6 (10k cage); batched p99 ms vs per-mesh launch"
HBM_PEAK_GBS = 8000.0

# Algorithmic (compulsory) bytes of the kernels of the last Catmull-Clark step
# (level k -> k+1, refined from the parent level m = k-1, no adjacency
# emitted), 3 x fp32 positions and int32 indices. The step's compulsory
# traffic -- read M_k and P_k once, write M_{k+1} and P_{k+1} once -- is split
# over the kernel that owns each part:
#   cc_group      per parent face   : read M_k rows 4x16 + write M_{k+1} 16x16 + write 4 face points 48
#                                     + read and write the face-point vertex 12 + 12         = 392 B
#   cc_old_vertex per parent vertex : read p 12 + write its vertex point 12                  = 24 B
#   cc_edge_group per parent edge   : write 4 edge points 48 + read and write the edge-point
#                                     vertex 12 + 12                                         = 72 B
# Per parent quad (V ~ F, E ~ 2F): 392 + 24 + 144 = 560 B = 35 B per refined face.
BYTES_PER_UNIT = {"cc_group": lambda m: 392 * m["F"], "cc_old_vertex": lambda m: 24 * m["V"],
                  "cc_edge_group": lambda m: 72 * m["E"]}

# HBM bytes per launch of the dominant kernel from the committed rocprofv3
# counter passes (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's
# readings); reported only while the kernel sources are the ones measured.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "cc_group_L5to6_mixed10k_traffic.json")


def measured_traffic(stage, level):
    import hashlib
    try:
        t = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if (t.get("stage"), t.get("level")) != (stage, level):
        return None
    h = hashlib.sha256()
    for src in t["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["sources_sha256"]:
        return None
    return int(t["fetch_bytes"]) + int(t["write_bytes"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-levels", type=int, default=5, help="levels of the oracle sample (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving trace (Poisson arrivals; 0 = skip the serving leg)")
    ap.add_argument("--serve-factors", default="0.5,0.8,1.0,1.2,1.5,2,3",
                    help="arrival rates as multiples of the per-mesh-launch saturation rate")
    ap.add_argument("--adjoint-levels", type=int, default=4,
                    help="levels of the adjoint leg on the same cage (0 = skip)")
    ap.add_argument("--tri-levels", type=int, default=5,
                    help="levels of the Loop and sqrt(3) legs on the holed triangle cage (0 = skip)")
    ap.add_argument("--depth", type=int, default=2, help="steps in flight in the timed loop (refine streams)")
    ap.add_argument("--no-side-legs", action="store_true",
                    help="skip the static-topology, selective, reorder and adjoint legs (for kernel profiles: "
                         "the Catmull-Clark kernels then come from full refinements of the headline workload only)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (counter calibration) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: under rocprofv3 --pmc its FETCH_SIZE /
    WRITE_SIZE per dispatch give the factor between counter units and bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "dispatches": 5}))


def cpu_baseline(mesh, levels):
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    lv = oracle.refine(mesh, "cc", levels)
    dt = time.perf_counter() - t0
    faces = lv[-1].num_faces
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": faces / dt, "unit": "refined faces/s", "cores": 1, "kind": "oracle",
            "sample": f"same cage refined to level {levels} ({faces} faces) by the serial FP64 oracle, "
                      f"{dt:.1f} s on one host core",
            "host_cpu": model, "host_logical_cpus": os.cpu_count(),
            "host_cpus_usable": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


class TwoDeep:
    """Steps two deep through api.StreamingRefiner: step i is planned on a
    third stream, into the second of two workspaces, while step i-1 still
    refines, and refines on its slot's stream beside step i-1; every step
    validates, builds and refines its cage in full."""

    def __init__(self, dmesh, levels, scheme="cc", depth=2):
        import torch
        from paper_1809_06047_amd import api
        self.dmesh = dmesh
        self.sr = api.StreamingRefiner(scheme, levels, depth=depth)
        for _ in range(depth):  # every slot's refiner exists from the start
            self.sr.step(dmesh)
        self.rs = [self.sr.refiner(j) for j in range(depth)]
        # the slots' refinements run on non-blocking streams: they must be done
        # before a caller plans or refines with these refiners on another
        # stream (a plan rewrites the workspace a refinement still reads)
        torch.cuda.synchronize()

    def step(self):
        self.sr.step(self.dmesh)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported: the refinement of one cage "
              "is a single-GPU workload (several GPUs would each refine a block of the cage's faces with a ghost "
              "ring, or serve their own requests)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch
    from paper_1809_06047_amd import _lib, api
    from paper_1809_06047_amd import meshgen as G

    mesh = G.cc_cage(seed=args.seed)
    dmesh = api.DeviceMesh(mesh, "cuda")
    pipe = TwoDeep(dmesh, args.levels, depth=args.depth)
    r = pipe.rs[0]
    r.plan()
    torch.cuda.synchronize()
    L = args.levels
    info = [r.level_info(k) for k in range(L + 1)]
    faces_out = info[L]["F"]

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()

    # stage breakdown (untimed calibration steps, an event pair around every
    # stage): it names the dominant kernel, the largest total device time
    calib = max(3, args.steps // 4)
    _lib.timing_enable(True)
    _lib.timing_read()
    for _ in range(calib):
        r.plan()
        r.run()
    torch.cuda.synchronize()
    krecs = _lib.timing_read_kernels()
    _lib.timing_enable(False)
    all_stages = {}
    for stage, level, _, _, _, n, ms in krecs:
        n0, t0 = all_stages.get((stage, level), (0, 0.0))
        all_stages[(stage, level)] = (n0 + n, t0 + ms)
    cand = {k: v for k, v in all_stages.items() if k[0] in BYTES_PER_UNIT}
    dname, dlevel = max(cand.items(), key=lambda kv: kv[1][1])[0]
    dkern = [(kern, items, block) for stage, level, kern, items, block, _, _ in krecs
             if (stage, level) == (dname, dlevel)]
    device_ms = sum(v[1] for v in all_stages.values()) / calib

    # the same steps one after the other on one stream (reported beside the
    # timed figure): the GPU idles while the host waits for each plan
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.plan()
        r.run()
    torch.cuda.synchronize()
    ms_serial = (time.perf_counter() - t0) * 1000.0 / args.steps

    # timed region: steps two deep (TwoDeep); events around the dominant kernel
    # only, so that the event pairs of the other stages do not sit between the
    # kernels of the step
    for _ in range(args.depth):  # every refiner's outputs allocated for its slot's stream again
        pipe.step()
    _lib.timing_select(dname, dlevel)
    _lib.timing_enable(True)
    _lib.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    _lib.timing_select(None)

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = faces_out / (ms_per_step / 1000.0)

    launches, total_ms = stages[(dname, dlevel)]
    nbytes = BYTES_PER_UNIT[dname](info[dlevel - 1])  # one thread per element of the parent level
    avg_ms = total_ms / launches
    achieved = nbytes / (avg_ms / 1000.0) / 1e9
    alone_ms = all_stages[(dname, dlevel)][1] / all_stages[(dname, dlevel)][0]
    alone_gbs = nbytes / (alone_ms / 1000.0) / 1e9
    # the whole last step (every stage of level L-1 -> L) against the step's
    # compulsory bytes: read M_{L-1} and P_{L-1}, write M_L and P_L
    k_info = info[L - 1]
    step_bytes = 16 * k_info["F"] + 12 * k_info["V"] + 16 * info[L]["F"] + 12 * info[L]["V"]
    step_ms = sum(v[1] for kk, v in all_stages.items() if kk[1] == L - 1) / calib
    step_gbs = step_bytes / (step_ms / 1000.0) / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "refined faces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"Catmull-Clark levels 0->{L} of a mixed tri/quad cage: icosphere level 5 "
                        f"(V={info[0]['V']}, F={info[0]['F']}, H={info[0]['H']}), 30% of triangle pairs merged, "
                        f"{mesh.num_creases} creases sharpness U[0,4), seed {args.seed}",
            "faces_out": faces_out,
            "vertices_out": info[L]["V"],
            "step": "subdiv_plan + subdiv_refine (dynamic topology), steps two deep: the plan of a step "
                    "and its refinement (on its slot's stream) overlap the refinement of the one before",
            "ms_per_step_one_at_a_time": round(ms_serial, 4),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dname} (level {dlevel} -> {dlevel + 1})",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dname, dlevel),
            "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": nbytes,
            # the timed steps run two deep, so the other slot's small levels and
            # plan share the GPU with this kernel; the same kernel in the
            # calibration steps, one step at a time on one stream:
            "alone": {"avg_launch_ms": round(alone_ms, 5), "achieved": round(alone_gbs, 1),
                      "frac": round(alone_gbs / HBM_PEAK_GBS, 4)},
        },
        "tuning": {"table": os.path.relpath(_lib.tuning_source(), ROOT) if os.path.isabs(_lib.tuning_source())
                   else _lib.tuning_source(),
                   "dominant_kernel": [{"kernel": k, "items": n, "block": b} for k, n, b in dkern]},
        "last_step": {"levels": f"{L - 1} -> {L}", "device_ms": round(step_ms, 5), "compulsory_bytes": step_bytes,
                      "achieved_GBs": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                      "note": "every stage of the last step (calibration steps, one at a time) against reading "
                              "M and P of level L-1 once and writing M and P of level L once"},
        "device_ms_per_step": round(device_ms, 4),
        "stages_ms_per_step": {f"{k[0]}@{k[1]}": round(v[1] / calib, 4) for k, v in sorted(all_stages.items())},
        "stages_note": "stage times from untimed calibration steps with an event pair around every stage; "
                       "the timed steps carry events around the dominant kernel only",
    }
    if not args.no_side_legs:
        out["static_topology"] = static_leg(mesh, args.levels, max(5, args.steps // 2))
        out["selective"] = selective_leg(mesh, 4, 2, 2, max(3, args.steps // 4))
        out["reorder"] = reorder_leg(mesh, args.levels, max(5, args.steps // 2))
        out["adaptive"] = adaptive_leg(args.seed, args.levels, 1, max(3, args.steps // 4))
    if args.adjoint_levels > 0 and not args.no_side_legs:
        out["adjoint"] = adjoint_leg(mesh, args.adjoint_levels, max(3, args.steps // 4))
    if args.tri_levels > 0:
        out["triangle_schemes"] = {sc: scheme_leg(G.tri_cage(), sc, args.tri_levels, max(3, args.steps // 4))
                                   for sc in ("loop", "sqrt3", "sqrt3k")}
    if args.serve_requests > 0:
        out["serving"] = serving(args)
    if args.cpu_levels > 0:
        out["cpu_baseline"] = cpu_baseline(mesh, args.cpu_levels)
    print(json.dumps(out), flush=True)


# algorithmic bytes of the last step's triangle-scheme kernels (no adjacency
# carried), from the sizes of level k = L-1 and of level m = L-2:
#   Loop (computed from level m): the face kernel reads a level-m face's
#   vertex and edge rows (24 B) and writes its 16 grandchildren (192 B); the
#   edge kernel reads the edge's half-edge (4 B), reads and writes the vertex
#   point of its edge point (24 B) and writes the edge points of level k's
#   edges (12 B each); the vertex kernel reads and writes the positions of
#   level m's vertices (24 B), of level m-1's only when the step before also
#   ran from two levels down (L >= 4: it wrote the final points of level m's
#   edge points);
#   sqrt(3) (computed from level m): the face kernel reads a level-m face's
#   vertex and twin rows (24 B), writes its 9 grandchildren (108 B) and the
#   face points of its 3 children (36 B), and reads and writes the vertex
#   point of its face point (24 B); the vertex kernel reads and writes the
#   positions of level m's vertices, of level m-1's when the step before ran
#   from two levels down (it wrote the final points of level m's face points
#   away from the boundary; those few next to it are left out of the count).
TRI_BYTES = {"loop_face": lambda k, m, g: 216 * m["F"], "loop_edge": lambda k, m, g: 12 * k["E"] + 28 * m["E"],
             "loop_vertex": lambda k, m, g: 24 * (g or m)["V"],
             "sqrt3_face": lambda k, m, g: 192 * m["F"], "sqrt3_vertex": lambda k, m, g: 24 * (g or m)["V"]}


def scheme_leg(mesh, scheme, levels, steps):
    """Loop / sqrt(3) on the holed triangle cage (icosphere level 6, 2% of the
    faces removed as vertex-disjoint holes): plan + refine per step, two deep
    like the main workload; refined faces/s and the per-stage device time."""
    import torch
    from paper_1809_06047_amd import _lib, api
    pipe = TwoDeep(api.DeviceMesh(mesh, "cuda"), levels, scheme)
    r = pipe.rs[0]
    r.plan()
    r.run()
    torch.cuda.synchronize()
    faces = r.level_info(levels)["F"]
    _lib.timing_enable(True)  # stage breakdown from calibration steps
    _lib.timing_read()
    for _ in range(steps):
        r.plan()
        r.run()
    torch.cuda.synchronize()
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    for _ in range(2):  # both refiners' outputs allocated for stream R before the timed steps
        pipe.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()  # timed steps, two deep: no events
    for _ in range(steps):
        pipe.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / steps
    per_stage = {}
    for (name, lvl), (_, tot) in stages.items():
        per_stage[name] = per_stage.get(name, 0.0) + tot / steps
    last = levels - 1  # the last step: level L-1 -> L
    roof = {}
    for (name, lvl), (n, tot) in stages.items():
        # (the byte counts are those of the last step from two levels down,
        # which sqrt(3) with the boundary cycle does not take)
        if lvl != last or name not in TRI_BYTES or scheme == "sqrt3k":
            continue
        g = r.level_info(last - 2) if levels >= 4 else None
        nbytes = TRI_BYTES[name](r.level_info(last), r.level_info(last - 1), g)
        avg = tot / n
        gbs = nbytes / (avg / 1000.0) / 1e9
        roof[name] = {"avg_launch_ms": round(avg, 5), "algorithmic_bytes_per_launch": nbytes,
                      "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return {"workload": f"{scheme} levels 0->{levels} of the holed triangle cage (F={mesh.num_faces})",
            "faces_out": faces, "ms_per_step": round(ms, 4), "refined_faces_per_s": round(faces / (ms / 1000.0), 1),
            "device_ms_per_step": round(sum(per_stage.values()), 4),
            "stages_ms_per_step": {k: round(v, 4) for k, v in sorted(per_stage.items(), key=lambda kv: -kv[1])},
            f"last_step_roofline (level {last} -> {levels})": roof}


def static_leg(mesh, levels, steps):
    """Static topology on the main workload: the plan keeps every level's
    state; after one full subdiv_refine, subdiv_refine_positions re-evaluates
    P_6 = R_5 ... R_0 P_0 for moved cage positions, writing positions only."""
    import torch
    from paper_1809_06047_amd import _lib, api
    r = api.Refiner(mesh, "cc", levels, flags=_lib.FLAG_KEEP_STATE)
    r.plan()
    r.run()
    r.run_positions()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.run_positions()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        r.run()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # general vertex data: five channels (a UV pair and an RGB colour), three
    # channels per pass through the same kernels
    data = torch.rand((mesh.num_vertices, 5), device="cuda")
    out = r.run_vertex_data(data)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(steps):
        r.run_vertex_data(data, out=out)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    faces = r.level_info(levels)["F"]
    ms_pos = (t1 - t0) * 1000.0 / steps
    return {"workload": f"Catmull-Clark levels 0->{levels}, positions only with the topology kept",
            "ms_per_eval": round(ms_pos, 4), "refined_faces_per_s": round(faces / (ms_pos / 1000.0), 1),
            "ms_per_full_refine_same_plan": round((t2 - t1) * 1000.0 / steps, 4),
            "ms_per_vertex_data_eval_5_channels": round((t4 - t3) * 1000.0 / steps, 4)}


def reorder_leg(mesh, levels, steps, seed=5):
    """Mesh reordering (Sec. 4.5): the main cage with its vertices and faces
    in a seeded random order, and that cage after reverse Cuthill-McKee,
    refined to `levels` (plan + refine per step, one at a time), beside the
    cage in its generated order."""
    import torch
    from paper_1809_06047_amd import api
    from paper_1809_06047_amd import meshgen as G
    rng = np.random.default_rng(seed)
    p = rng.permutation(mesh.num_vertices)  # old -> new
    inv = np.argsort(p)
    faces = [[int(p[v]) for v in f] for f in mesh.face_list()]
    faces = [faces[i] for i in rng.permutation(len(faces))]
    offs = np.concatenate([[0], np.cumsum([len(f) for f in faces])]).astype(np.int32)
    shuffled = G.Mesh(positions=np.asarray(mesh.positions)[inv], verts=np.array([v for f in faces for v in f], np.int32),
                      offsets=offs, crease_verts=p[np.asarray(mesh.crease_verts)].astype(np.int32),
                      crease_sharp=mesh.crease_sharp, name="shuffled")
    t0 = time.perf_counter()
    rcm, _, _ = api.rcm_reorder(shuffled)
    ms_rcm_host = (time.perf_counter() - t0) * 1000.0
    out = {"workload": f"Catmull-Clark levels 0->{levels}: the 10k cage as generated, with vertices and faces "
                       f"shuffled (seed {seed}), and the shuffled cage after reverse Cuthill-McKee",
           "ms_rcm_order_host": round(ms_rcm_host, 3)}
    for name, m in (("generated", mesh), ("shuffled", shuffled), ("rcm_of_shuffled", rcm)):
        r = api.Refiner(api.DeviceMesh(m, "cuda"), "cc", levels)
        r.plan()
        r.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r.plan()
            r.run()
        torch.cuda.synchronize()
        out[f"ms_per_step_{name}"] = round((time.perf_counter() - t0) * 1000.0 / steps, 4)
    return out


def selective_leg(mesh, base_level, rings, extra_levels, steps):
    """Selective subdivision (Sec. 3.4) on the main cage refined to
    `base_level` (all quads, 3.5 M faces at level 4): the region `rings`
    face rings around its extraordinary vertices (valence != 4) is extracted
    and refined `extra_levels` further, against refining the whole level."""
    import torch
    from paper_1809_06047_amd import api
    outs, _ = api.refine(mesh, "cc", base_level)
    fv, P = outs[base_level]["face_verts"], outs[base_level]["positions"]
    dm = api.DeviceMesh.from_tensors(fv, None, P, None, None, 4, name=f"cc-l{base_level}")
    whole = api.Refiner(dm, "cc", extra_levels)
    whole.plan()
    reg = api.extract_region(whole, None, rings)
    part = api.Refiner(reg["mesh"], "cc", extra_levels)
    part.plan()
    torch.cuda.synchronize()

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / steps

    ms_extract = timed(lambda: api.extract_region(whole, None, rings))  # select (one read-back) + extract
    ms_region = timed(lambda: (part.plan(), part.run()))
    ms_whole = timed(lambda: (whole.plan(), whole.run()))
    return {"workload": f"Catmull-Clark level {base_level} of the 10k cage ({dm.F} quads), region {rings} rings "
                        f"around the extraordinary vertices, refined {extra_levels} more levels",
            "region_faces": reg["mesh"].F, "region_vertices": reg["mesh"].V, "whole_faces": dm.F,
            "ms_select_and_extract": round(ms_extract, 4), "ms_region_plan_refine": round(ms_region, 4),
            "ms_whole_plan_refine": round(ms_whole, 4),
            "region_faces_out": part.level_info(extra_levels)["F"],
            "whole_faces_out": whole.level_info(extra_levels)["F"]}


def adaptive_leg(seed, levels, rings, steps):
    """Feature-adaptive refinement (Sec. 3.4 level after level) of the 10k
    cage's topology without creases: on every level the region `rings` rings
    around the cage's extraordinary vertices (pinches closed) is extracted and
    refined one level; against the uniform refinement of the same cage. Every
    adaptive level synchronises on its plans and its selection."""
    import torch
    from paper_1809_06047_amd import api
    from paper_1809_06047_amd import meshgen as G
    mesh = G.cc_cage(seed=seed, crease_frac=0.0)
    dm = api.DeviceMesh(mesh, "cuda")
    res = api.adaptive_refine(dm, levels, rings)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.adaptive_refine(dm, levels, rings)
    torch.cuda.synchronize()
    ms_adaptive = (time.perf_counter() - t0) * 1000.0 / steps
    r = api.Refiner(dm, "cc", levels)
    r.plan()
    r.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.plan()
        r.run()
    torch.cuda.synchronize()
    ms_uniform = (time.perf_counter() - t0) * 1000.0 / steps
    return {"workload": f"Catmull-Clark levels 0->{levels} of the 10k cage without creases, {rings} ring(s) around "
                        "the extraordinary vertices (valence != 4) on every level",
            "region_faces_per_level": [g["mesh"].F for g in res],
            "uniform_faces_per_level": [r.level_info(k + 1)["F"] for k in range(levels)],
            "ms_adaptive": round(ms_adaptive, 4), "ms_uniform_plan_refine": round(ms_uniform, 4)}


def adjoint_leg(mesh, levels, steps):
    """Cage-fitting gradient: Catmull-Clark level 4 of the 10k cage with its
    state kept, then subdiv_backward (g_k = R_k^T g_{k+1}, level by level).
    A fitting loop refines once (building the state) and then runs the
    positions-only forward and the backward per step, as SubdivFunction
    does; both are timed, and the full refinement beside them. Per level the
    adjoint must read g_{k+1} and write g_k once: 12 (V_{k+1} + V_k) bytes,
    reported for the largest level."""
    import torch
    from paper_1809_06047_amd import _lib, api
    r = api.Refiner(mesh, "cc", levels, flags=_lib.FLAG_KEEP_STATE)
    r.plan()
    outs = r.run()
    g = torch.randn_like(outs[levels]["positions"])
    r.backward(g)
    torch.cuda.synchronize()
    _lib.timing_enable(True)  # stage breakdown from calibration steps
    _lib.timing_read()
    for _ in range(steps):
        r.run_positions()
        r.backward(g)
    torch.cuda.synchronize()
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    tf = tb = tr = 0.0
    for _ in range(steps):  # timed steps: no events
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.run_positions()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r.backward(g)
        torch.cuda.synchronize()
        tf += t1 - t0
        tb += time.perf_counter() - t1
    for _ in range(steps):  # the full refinement (which the fitting loop runs once)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r.run()
        torch.cuda.synchronize()
        tr += time.perf_counter() - t2
    k = levels - 1
    bw = sum(tot for (name, lvl), (_, tot) in stages.items() if name.startswith("bw_") and lvl == k) / steps
    nbytes = 12 * (r.level_info(levels)["V"] + r.level_info(k)["V"])
    gbs = nbytes / (bw / 1000.0) / 1e9
    return {"workload": f"Catmull-Clark level {levels} of the 10k-vertex mixed cage, gradient w.r.t. the cage "
                        f"(V_{levels}={r.level_info(levels)['V']})",
            "ms_forward": round(tf * 1000.0 / steps, 4), "ms_backward": round(tb * 1000.0 / steps, 4),
            "ms_refine_building_the_state": round(tr * 1000.0 / steps, 4),
            f"backward_level_{levels}_to_{k}": {"device_ms": round(bw, 5), "algorithmic_bytes": nbytes,
                                                 "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def serving(args):
    """Continuous-batching server against one plan + refine per request on the
    same Poisson trace (cages of 100..50k faces, Catmull-Clark or Loop, levels
    1..4), at multiples of the per-mesh-launch saturation rate."""
    from paper_1809_06047_amd import serve as S
    res = S.sweep(n_requests=args.serve_requests, factors=tuple(float(x) for x in args.serve_factors.split(",")),
                  log=lambda m: print(m, file=sys.stderr, flush=True))

    def side(d, keys):
        return {k: (round(d[k], 3) if isinstance(d[k], float) else d[k]) for k in keys}
    pts = []
    for p in res["points"]:
        pts.append({"factor": p["factor"], "qps": round(p["qps"], 1),
                    "batched": side(p["batched"], ("p50_ms", "p99_ms", "faces_per_s", "mean_batch", "max_queue")),
                    "per_mesh": side(p["per_mesh"], ("p50_ms", "p99_ms", "faces_per_s")),
                    "per_mesh_cached_plans": side(p["per_mesh_cached"], ("p50_ms", "p99_ms", "faces_per_s"))})
    cold = res.get("cold_cache")
    if cold:
        cold = {"factor": cold["factor"], "registered": cold["registered"],
                "batched": side(cold["batched"], ("p50_ms", "p99_ms", "faces_per_s", "mean_batch"))}
    return {"requests": res["requests"], "topologies": res["topologies"],
            "single_request_graphs": {"captured": res["graphs"], "max_final_faces": res["graph_max_faces"],
                                      "replays": res["graph_launches"]},
            "per_mesh_saturation_qps": round(res["per_mesh_saturation_qps"], 1),
            "budget_gib": res["budget_gib"], "slots": res["slots"], "max_batch": res["max_batch"],
            "batched_server": "FIFO prefixes of the queue, any schemes and level counts; one subdiv_refine_batch "
                              "per batch, no host round trip; topology cache warm (every cage topology of the "
                              "trace planned once before the timed runs); a batch of one whose final level is "
                              "small replays its (topology, levels) HIP graph",
            "per_mesh_server": "one subdiv_plan (with its read-back) + subdiv_refine per request, FIFO, one stream",
            "per_mesh_cached_plans_server": "one request at a time through the batched server's executor and topology "
                                            "cache (kept plan, one positions upload, the mesh refined alone, the "
                                            "same graphs), FIFO",
            "points": pts, "cold_cache": cold}


if __name__ == "__main__":
    main()
