"""Launch-shape tuner: measures every tunable kernel of the refinement and
adjoint steps at each candidate workgroup size on the benchmark workloads,
and writes the table the library loads (tuning_gfx950.json beside
libsubdiv.so).

For each candidate size B the whole table is set to B and the workloads run
with the library's stage timing on; every tuned launch is recorded with its
kernel, element count and B (subdiv_timing_read_kernels). Per kernel and
element count the fastest B wins (mean over the repetitions); size buckets
are cut at the geometric mean of neighbouring measured counts, and
neighbouring buckets with the same B are merged. Outputs do not depend on
the workgroup size, so the table only moves time.

    python -m paper_1809_06047_amd.tune [--reps 5] [--out PATH]
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CANDIDATES = (64, 128, 256, 512)
DEFAULT_OUT = os.path.join(HERE, "tuning_gfx950.json")


def workloads():
    """(label, callable that enqueues one step) on the benchmark cages: the
    mixed 10k cage to CC level 6 and level 4 (the smaller levels' buckets),
    the holed triangle cage to Loop and sqrt(3) levels 5 and 4, and the
    adjoint of CC level 4 (positions-only forward and backward)."""
    import torch
    from . import _lib, api
    from . import meshgen as G
    cc, tri = G.cc_cage(), G.tri_cage()
    out = []
    for scheme, mesh, L in (("cc", cc, 6), ("cc", cc, 4), ("loop", tri, 5), ("loop", tri, 4), ("sqrt3", tri, 5),
                            ("sqrt3", tri, 4)):
        r = api.Refiner(api.DeviceMesh(mesh, "cuda"), scheme, L)
        r.plan()
        out.append((f"{scheme} L{L}", lambda r=r: (r.plan(), r.run())))
    a = api.Refiner(api.DeviceMesh(cc, "cuda"), "cc", 4, flags=_lib.FLAG_KEEP_STATE)
    a.plan()
    outs = a.run()
    g = torch.randn_like(outs[4]["positions"])
    a.backward(g)
    out.append(("adjoint cc L4", lambda: (a.run_positions(), a.backward(g))))
    return out


def measure(steps, reps, log):
    """{(kernel, items): {B: mean ms per launch}} and {label: {B: device ms per step}}"""
    import torch
    from . import _lib
    per = {}
    totals = {}
    for b in CANDIDATES:
        _lib.tuning_set("*", b)
        for label, step in steps:
            step()  # warm-up at this size
            torch.cuda.synchronize()
            _lib.timing_enable(True)
            _lib.timing_read_kernels()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            recs = _lib.timing_read_kernels()
            _lib.timing_enable(False)
            tot = 0.0
            for stage, level, kernel, items, block, launches, ms in recs:
                tot += ms
                if not kernel:
                    continue
                assert block == b, (kernel, block, b)
                d = per.setdefault((kernel, items), {})
                n0, t0 = d.get(b, (0, 0.0))
                d[b] = (n0 + launches, t0 + ms)
            totals.setdefault(label, {})[b] = tot / reps
        log(f"[tune] B={b}: " + ", ".join(f"{k} {v[b]:.3f} ms" for k, v in totals.items()))
    return {k: {b: t / n for b, (n, t) in d.items()} for k, d in per.items()}, totals


def table_from(per):
    """kernel -> [[max_items, block], ...] (last bound -1)."""
    by_kernel = {}
    for (kernel, items), times in per.items():
        by_kernel.setdefault(kernel, []).append((items, min(times, key=times.get)))
    table = {}
    for kernel, rows in sorted(by_kernel.items()):
        rows.sort()
        entries = []
        for i, (items, best) in enumerate(rows):
            bound = -1 if i + 1 == len(rows) else int(math.sqrt(items * rows[i + 1][0]))
            if entries and entries[-1][1] == best:
                entries[-1][0] = bound
            else:
                entries.append([bound, best])
        table[kernel] = entries
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)
    import torch
    from . import _lib
    assert torch.cuda.is_available(), "the tuner measures on the GPU"

    def log(m):
        print(m, file=sys.stderr, flush=True)
    steps = workloads()
    t0 = time.time()
    per, totals = measure(steps, args.reps, log)
    table = table_from(per)
    # the tuned table against each single size, per workload
    _lib.tuning_load(None)
    tmp = args.out + ".tmp"
    doc = {"device": torch.cuda.get_device_name(0), "arch": "gfx950",
           "generated_by": "python -m paper_1809_06047_amd.tune", "candidates": list(CANDIDATES), "reps": args.reps,
           "kernels": table,
           "measured_ms_per_launch": {f"{k} n={n}": {str(b): round(t, 5) for b, t in sorted(v.items())}
                                      for (k, n), v in sorted(per.items())},
           "device_ms_per_step_single_block": {w: {str(b): round(t, 4) for b, t in v.items()}
                                               for w, v in totals.items()}}
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    _lib.tuning_load(tmp)
    tuned = {}
    for label, step in steps:
        step()
        torch.cuda.synchronize()
        _lib.timing_enable(True)
        _lib.timing_read_kernels()
        for _ in range(args.reps):
            step()
        torch.cuda.synchronize()
        tuned[label] = sum(r[6] for r in _lib.timing_read_kernels()) / args.reps
        _lib.timing_enable(False)
    doc["device_ms_per_step_tuned"] = {w: round(t, 4) for w, t in tuned.items()}
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, args.out)
    _lib.tuning_load(args.out)
    log(f"[tune] wrote {args.out} in {time.time() - t0:.1f} s; tuned device ms per step: "
        + ", ".join(f"{k} {v:.3f}" for k, v in tuned.items()))
    print(json.dumps({"table": args.out, "tuned": doc["device_ms_per_step_tuned"],
                      "single_block": doc["device_ms_per_step_single_block"]}))


if __name__ == "__main__":
    main()
