#!/usr/bin/env python
"""Benchmark of the ESES hot path on one MI355X.

A step is one pass of the whole path over one batch of molecules (by default
256 seeded globules of 200-20,000 atoms at 0.5 A spacing) whose inputs are
already in HBM: eses_build_candidates (cell binning, SAS pairs and circles,
concave probe positions, exposure flags, tile lists), eses_classify (every grid
point) and eses_edge_intersections (every crossing edge, roots and normals).

Prints one JSON line.  The timed steps run the certified FP32 classification
with FP64 recheck (and exact arbitration of the FP64-uncertain points); `value`
is grid points through the whole path per second in that form.  The same steps
in plain FP64 are timed after it and reported beside (`fp64`), with the ratio of
the two; the classification and intersection rates of the metric, a roofline
entry for the dominant kernel and the FP64 CPU oracle timed on a bounded sample
of the same workload complete the line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid points classified/s + edge intersections/s; batched FP32+FP64-recheck vs FP64"
DEFAULT_WORKLOAD = "batch256_h0.5"

# MI355X FP64 vector peak: 256 CUs x 128 FP64 flop/clock (64 FMA lanes) x 2.4 GHz.
PEAK_FP64_TFLOPS = 78.6

# FP64 flops of one test of the classification decision (an FMA counts 2):
#   atom: c - x (3), |.|^2 (5), r^2, r + rho, s^2 (3)                      = 11
#   vertex: x - p (3), |.|^2 (5)                                           = 8
#   face reach: x - c (3), |.|^2 (5), r + 2 rho (2), square (1)            = 11
#   face or circle half-space: dot (5), |.| tau (1)                        = 6
#   circle reach: w (3), w.n (5), |w|^2 (5), b^2 (2), sqrt (1), R^2 (1),
#                 |w|^2 + R^2 - rho^2 (2), 2 b R (2)                       = 21
FLOPS_PER_TEST = {"tests_atom": 11, "tests_vertex": 8, "tests_face": 11, "tests_face_cut": 6,
                  "tests_circle": 21, "tests_circle_cut": 6}

# FP64 flops of the edge-root kernels' work items (from their statistics pass):
#   sphere reach (van der Waals or probe): mid - c (3), |.|^2 (5), bounds (4)   = 12
#   torus reach: mid - o (3), t (5), |.|^2 (5), b (3), (b-R)^2 + t^2 (4),
#                bounds (3)                                                   = 23
#   quadratic: coefficients (9), discriminant (3), sqrt, two roots (5)        = 18
#   quartic set-up: |w|^2, t, a/b coefficients, g coefficients                 = 35
#   half-space test of a root: dot (5), |.| tau (1)                           = 6
#   cone test of a cut against an edge's direction cone: |v| (6), cos phi (6),
#     sin phi (3), |v| cos(phi + theta) (4), threshold (1)                    = 20
#   per edge: coordinates, normal and its norm                                = 30
# plus the solver's polynomial evaluations (counted in flops) and the label
# evaluations between roots (classification constants above).
FLOPS_EDGE = {"reach_sphere": 12, "reach_torus": 23, "quad_solves": 18, "quartic_solves": 35,
              "horner_flops": 1, "cut_tests": 6, "n_edges": 30,
              "label_tests_atom": 11, "label_tests_vertex": 8, "label_tests_face": 11,
              "label_tests_face_cut": 6, "label_tests_circle": 21, "label_tests_circle_cut": 6,
              "cone_tests": 20}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--prec", choices=["both", "fp64", "fp32"], default="both",
                    help="both: timed FP32+recheck steps (value), then FP64 steps beside")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=40.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--stream", type=int, default=0, metavar="PLANES",
                    help="time the out-of-core form instead (one molecule's grid in z-slabs of "
                         "PLANES planes, labels and records to host memory) beside the in-HBM step")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (a known-size "
                         "reference for HBM byte counters)")
    return ap.parse_args()


def cpu_sample(o, m, budget_s, orc):
    """Labels and crossing-edge records of the oracle `o` on evenly spaced
    z-slice pairs of molecule m, about budget_s seconds of CPU work.  Returns
    (points, label seconds, edges, edge seconds, slice pairs)."""
    import numpy as np
    nx, ny, nz = m.dims
    mid = max(0, nz // 2 - 1)
    t0 = time.perf_counter()
    L = o.labels_grid(m.lo, m.spacing, m.dims, mid, mid + 2)
    t_pair_lab = time.perf_counter() - t0
    keys = orc.crossing_keys(L)
    keys = keys[(keys // 3) < nx * ny] + 3 * mid * nx * ny  # edges whose s is in slice mid
    t0 = time.perf_counter()
    o.edges(m.lo, m.spacing, m.dims, keys)
    t_pair_edge = time.perf_counter() - t0
    per_pair = max(t_pair_lab + t_pair_edge, 1e-4)
    n_pairs = int(max(1, min(nz // 2, budget_s / per_pair)))
    ks = np.linspace(0, nz - 2, n_pairs).astype(int)
    t_lab = t_edge = 0.0
    pts = edges = 0
    for k in ks:
        t0 = time.perf_counter()
        L = o.labels_grid(m.lo, m.spacing, m.dims, int(k), int(k) + 2)
        t_lab += time.perf_counter() - t0
        pts += 2 * nx * ny
        kk = orc.crossing_keys(L)
        kk = kk[(kk // 3) < nx * ny]
        # keys of the two-slice sub-grid mapped to the full grid
        kk_full = kk + 3 * int(k) * nx * ny
        t0 = time.perf_counter()
        o.edges(m.lo, m.spacing, m.dims, kk_full)
        t_edge += time.perf_counter() - t0
        edges += len(kk)
    return pts, t_lab, edges, t_edge, len(ks)


def cpu_baseline(mols_np, counts, target_s):
    """The FP64 oracle on a bounded sample of the same workload, extrapolated
    to all of it: for a batch, 24 molecules at evenly spaced ranks of size
    (smallest to largest), each built whole (probe enumeration) and labelled,
    with its crossing edges solved, on evenly spaced z-slice pairs; the time
    per atom of the builds, per point of the labels and per crossing of the
    edges, pooled over the sample, times the workload's atoms, points and
    crossings."""
    import platform

    import numpy as np
    from oracle import oracle as orc

    orc.build(force=False)
    order = np.argsort([m.n_atoms for m in mols_np], kind="stable")
    pick = sorted(set(int(order[int(round(f * (len(order) - 1)))])
                      for f in np.linspace(0.0, 1.0, 24)))
    t_create = t_lab = t_edge = 0.0
    atoms = pts = edges = pairs = 0
    per_mol = target_s / len(pick)
    for q in pick:
        m = mols_np[q]
        t0 = time.perf_counter()
        o = orc.Oracle(m.centres, m.radii, m.probe)
        tc = time.perf_counter() - t0
        p, tl, e, te, npair = cpu_sample(o, m, max(per_mol - tc, 0.05), orc)
        del o
        t_create += tc
        atoms += m.n_atoms
        t_lab += tl
        pts += p
        t_edge += te
        edges += e
        pairs += npair
    n_atoms = sum(m.n_atoms for m in mols_np)
    n_points = sum(m.n_points for m in mols_np)
    n_cross = sum(counts)
    t_full = (t_create / atoms * n_atoms + t_lab / pts * n_points
              + (t_edge / max(edges, 1)) * n_cross)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        cpu = platform.processor() or cpu
    what = (f"molecules {pick} of {len(mols_np)}" if len(mols_np) > 1 else "the molecule")
    return {
        "value": n_points / t_full,
        "unit": "grid points/s",
        "cores": orc.threads(),
        "cpu_model": cpu,
        "kind": "oracle",
        "sample": (f"{what} ({atoms} atoms): whole-molecule probe enumeration "
                   f"({t_create:.2f} s) + labels of {pts} points in {pairs} evenly spaced slice "
                   f"pairs ({t_lab:.2f} s) + {edges} crossing edges there ({t_edge:.2f} s); "
                   f"per-atom, per-point and per-crossing times extrapolated to {n_atoms} atoms, "
                   f"{n_points} points and {n_cross} crossings"),
        "seconds": t_create + t_lab + t_edge,
        "extrapolated_seconds": t_full,
        "classify_pts_per_s": pts / t_lab,
        "isect_per_s": edges / max(t_edge, 1e-9),
    }


def load_workload(name):
    from eses_inputs import workload, batch
    if name.startswith("batch"):
        # batch<count>_h<spacing>
        count = int(name[5:].split("_")[0])
        h = float(name.split("_h")[1])
        return batch(count, h)
    return [workload(name)]


PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (packed instructions)
PEAK_HBM_GBS = 8000.0


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by molecule or z-slab with no exchange step; only the "
              "one-GPU share is measured)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1809_04352_amd import eses

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    eses.load()
    if args.stream:
        bench_stream(args, eses)
        return
    precs = {"both": [eses.ESES_FP32_RECHECK, eses.ESES_FP64],
             "fp32": [eses.ESES_FP32_RECHECK], "fp64": [eses.ESES_FP64]}[args.prec]
    pname = {eses.ESES_FP32_RECHECK: "fp32", eses.ESES_FP64: "fp64"}
    mols_np = load_workload(args.workload)
    dev = torch.device("cuda:0")
    tens = [(torch.as_tensor(m.centres, device=dev), torch.as_tensor(m.radii, device=dev))
            for m in mols_np]
    mols = [eses.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
            for (c, r), m in zip(tens, mols_np)]
    dims = [eses.grid_dims(m) for m in mols]
    npts = sum(d[0] * d[1] * d[2] for d in dims)
    labels = [torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device=dev) for d in dims]

    # launch configuration: the autotuner's choice for these molecules and the
    # timed precision (outside the timed region)
    from paper_1809_04352_amd import autotune
    tuned, tune_ms = autotune.tune(mols, precs[0], use_cache=False)
    knobs = dict(tile=tuned.get("tile", 0), blocks_per_cu=tuned.get("blocks_per_cu", 0),
                 unit_order=tuned.get("unit_order", 0))
    # sizing pass (outside the timed region): output capacities and work counts
    cand = eses.build_candidates(mols, **knobs)
    infos = [cand.info(q) for q in range(len(mols))]
    work = eses.classify(cand, eses.ESES_FP64, labels, stats=True)
    work32 = eses.classify(cand, eses.ESES_FP32_RECHECK, labels, stats=True)
    probe_out = [eses.alloc_isect(1) for _ in mols]
    _, counts = eses.edge_intersections(cand, labels, probe_out)
    ework = eses.edge_work(cand, labels)
    cand.close()
    outs = [eses.alloc_isect(max(k, 1)) for k in counts]
    n_cross = sum(counts)

    def total(dicts, key):
        return sum(d[key] for d in dicts)

    flops_classify = sum(FLOPS_PER_TEST[k] * total(work, k) for k in FLOPS_PER_TEST)
    flops_atom = FLOPS_PER_TEST["tests_atom"] * total(work, "tests_atom")
    flops_edges = sum(FLOPS_EDGE[k] * total(ework, k) for k in FLOPS_EDGE)

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def measure(prec):
        stage = {"build": [], "classify": [], "edges": []}
        kern = {"classify_ms": [], "edge_detect_ms": [], "edge_roots_ms": []}

        def step(record):
            if record:
                ev[0].record(stream)
            c = eses.build_candidates(mols, **knobs)
            if record:
                ev[1].record(stream)
            eses.classify(c, prec, labels)
            if record:
                ev[2].record(stream)
            st, cnt = eses.edge_intersections(c, labels, outs)
            if record:
                ev[3].record(stream)
                kt = eses.kernel_times(c)
            c.close()
            if st != eses.ESES_OK or sum(cnt) != n_cross:
                raise RuntimeError("unexpected edge count")
            if record:
                torch.cuda.synchronize()
                stage["build"].append(ev[0].elapsed_time(ev[1]))
                stage["classify"].append(ev[1].elapsed_time(ev[2]))
                stage["edges"].append(ev[2].elapsed_time(ev[3]))
                for k in kern:
                    kern[k].append(kt[k])

        for _ in range(args.warmup):
            step(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = 1e3 * wall / args.steps
        # per-stage and per-kernel HIP-event timing in separate steps, so the
        # event reads do not disturb the timed loop
        eses.set_timing(True)
        for _ in range(max(3, min(args.steps, 10))):
            step(True)
        eses.set_timing(False)
        med = {k: float(np.median(v)) for k, v in stage.items()}
        kmed = {k: float(np.median(v)) for k, v in kern.items()}
        return {"ms_per_step": ms, "value": npts / (ms * 1e-3),
                "classify_pts_per_s": npts / (kmed["classify_ms"] * 1e-3),
                "isect_per_s": n_cross / (med["edges"] * 1e-3),
                "stages_ms": med, "kernels_ms": kmed}

    runs = {}
    for p in precs:
        runs[pname[p]] = measure(p)
    main_p = pname[precs[0]]
    R = runs[main_p]
    kmed = R["kernels_ms"]
    batch = len(mols) > 1
    rl = {}
    for name, fl, t in (("classify", flops_classify, kmed["classify_ms"]),
                        ("edge_roots", flops_edges, kmed["edge_roots_ms"])):
        a = fl / (t * 1e-3) / 1e12
        kname = "k_classify" if name == "classify" else "k_edge_chunks"
        if batch:
            kname += "_batch"  # the fused launches of a batch
        peak = PEAK_FP64_TFLOPS
        if name == "classify" and main_p == "fp32":
            # phase-1 ball tests in FP32, the rest in FP64: the peak of this
            # mix is the rate at which the vector units could retire it
            f32, f64 = flops_atom, fl - flops_atom
            peak = fl / (f32 / PEAK_FP32_TFLOPS + f64 / PEAK_FP64_TFLOPS)
        rl[name] = {"kernel": kname, "bound": "alu", "achieved": a, "peak": peak,
                    "unit": "TFLOP/s", "frac": a / peak, "traffic": None,
                    "algorithmic_flops": fl, "ms": t}
    for v in rl.values():
        prof = profiled_counters(v["kernel"], args.workload, main_p)
        if prof:
            v["traffic"] = prof.get("HBM bytes per launch")
            if v["traffic"]:
                gbs = v["traffic"] / (v["ms"] * 1e-3) / 1e9
                v["hbm_gbs"] = gbs
                v["hbm_frac"] = gbs / PEAK_HBM_GBS
            for k in ("measured FP32 flops per launch", "measured FP64 flops per launch"):
                if prof.get(k) is not None:
                    v[k.replace(" ", "_")] = prof[k]
            f32 = prof.get("measured FP32 flops per launch")
            f64 = prof.get("measured FP64 flops per launch")
            if f32 is not None and f64 is not None:
                t = v["ms"] * 1e-3
                v["mixed_precision_frac"] = (f32 / (PEAK_FP32_TFLOPS * 1e12)
                                             + f64 / (PEAK_FP64_TFLOPS * 1e12)) / t
                v["wasted_work_ratio"] = (f32 + f64) / v["algorithmic_flops"]
    dominant = max(rl, key=lambda k: rl[k]["ms"])
    roof = dict(rl[dominant])
    m0 = mols_np[0]
    config = {"workload": args.workload, "molecules": len(mols_np),
              "atoms": sum(m.n_atoms for m in mols_np), "probe": m0.probe,
              "spacing": m0.spacing, "points": npts, "precision": main_p,
              "tile": knobs["tile"] or 8, "blocks_per_cu": knobs["blocks_per_cu"],
              "unit_order": knobs["unit_order"], "autotune_classify_ms": tune_ms}
    if not batch:
        config["dims"] = list(dims[0])
    res = {
        "metric": METRIC,
        "value": R["value"],
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": config,
        "classify_pts_per_s": R["classify_pts_per_s"],
        "isect_per_s": R["isect_per_s"],
        "crossings": n_cross,
        "stages_ms": R["stages_ms"],
        "kernels_ms": kmed,
        "rechecked_points": total(work32, "n_rechecked"),
        "exact_points": {"fp32": total(work32, "n_exact"), "fp64": total(work, "n_exact")},
        "classify_work": {k: total(work, k) for k in work[0]},
        "edge_work": {k: total(ework, k) for k in ework[0]},
        "roofline": roof,
        "roofline_other": {k: v for k, v in rl.items() if k != dominant},
    }
    if "fp64" in runs and main_p != "fp64":
        F = runs["fp64"]
        res["fp64"] = F
        res["fp32_vs_fp64"] = {
            "step": F["ms_per_step"] / R["ms_per_step"],
            "classify": F["kernels_ms"]["classify_ms"] / kmed["classify_ms"]}
    if not batch:
        res["candidates"] = {k: (list(v) if isinstance(v, tuple) else v)
                             for k, v in infos[0].items()}
    res["ses"] = ses_per_atom(mols_np, work, outs, counts)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calibrate_copy_bytes"] = nbytes
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(mols_np, counts, args.cpu_seconds)
    print(json.dumps(res))


def bench_stream(args, eses):
    """The out-of-core form on one molecule: a step is eses_build_candidates
    plus eses_stream_slabs (labels and records into pinned host memory, slabs
    of args.stream planes), timed beside the in-HBM step (build, classify,
    edges into device memory) of the same molecule and precision (FP32 +
    FP64 recheck)."""
    import numpy as np
    import torch
    mols_np = load_workload(args.workload)
    if len(mols_np) != 1:
        sys.exit("--stream takes a one-molecule workload")
    m = mols_np[0]
    dev = torch.device("cuda:0")
    c = torch.as_tensor(m.centres, device=dev)
    r = torch.as_tensor(m.radii, device=dev)
    mol = eses.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
    prec = eses.ESES_FP32_RECHECK
    nx, ny, nz = eses.grid_dims(mol)
    npts = nx * ny * nz
    cand = eses.build_candidates([mol])
    labels_dev = torch.empty(npts, dtype=torch.uint8, device=dev)
    eses.classify(cand, prec, [labels_dev])
    _, counts = eses.edge_intersections(cand, [labels_dev], [eses.alloc_isect(1)])
    cand.close()
    n_cross = counts[0]
    out_dev = eses.alloc_isect(n_cross)
    labels_host = torch.empty(npts, dtype=torch.uint8).pin_memory()
    from paper_1809_04352_amd.eses import IsectBuffers
    cap = max(n_cross, 1)
    out_host = IsectBuffers(torch.empty(cap, dtype=torch.int64).pin_memory(),
                            torch.empty(cap, dtype=torch.float64).pin_memory(),
                            torch.empty((cap, 3), dtype=torch.float64).pin_memory(),
                            torch.empty(cap, dtype=torch.uint8).pin_memory(),
                            torch.empty((cap, 3), dtype=torch.int32).pin_memory())

    def step_stream():
        h = eses.build_candidates([mol])
        st, k = eses.stream_slabs(h, prec, args.stream, labels_host, out_host)
        h.close()
        if st != eses.ESES_OK or k != n_cross:
            raise RuntimeError("unexpected edge count")

    def step_hbm():
        h = eses.build_candidates([mol])
        eses.classify(h, prec, [labels_dev])
        st, k = eses.edge_intersections(h, [labels_dev], [out_dev])
        h.close()
        if st != eses.ESES_OK or k[0] != n_cross:
            raise RuntimeError("unexpected edge count")

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps

    ms_stream = timed(step_stream)
    ms_hbm = timed(step_hbm)
    planes = min(args.stream, nz)
    res = {
        "metric": METRIC + " (out-of-core form)",
        "value": npts / (ms_stream * 1e-3),
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_stream,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": m.n_atoms, "dims": [nx, ny, nz],
                   "points": npts, "slab_planes": planes,
                   "slabs": (nz + planes - 1) // planes, "precision": "fp32"},
        "crossings": n_cross,
        "isect_per_s": n_cross / (ms_stream * 1e-3),
        "in_hbm_ms_per_step": ms_hbm,
        "stream_vs_in_hbm": ms_hbm / ms_stream,
        "slab_label_bytes": 2 * nx * ny * (planes + 1),
        "whole_grid_label_bytes": npts,
    }
    print(json.dumps(res))


def ses_per_atom(mols_np, work, outs, counts):
    """SES volume and area per atom from the timed path's own outputs (outside
    the timed region), beside the paper's per-atom ranges (appendix table):
    volume = inside points x h^3; area = h^2 x sum over crossings of |n_a|, the
    normal's component along the crossing's axis a (a crossing of an axis-a
    grid line stands for h^2 / |n_a| of surface; weighted by n_a^2, whose sum
    over the three axes is 1, that is h^2 |n_a|)."""
    vol = area = 0.0
    for m, w, o, k in zip(mols_np, work, outs, counts):
        h = m.spacing
        vol += w["n_inside"] * h ** 3
        if k:
            axis = (o.key[:k] % 3).view(-1, 1)
            area += float(o.normal[:k].gather(1, axis).abs().sum()) * h * h
    n = sum(m.n_atoms for m in mols_np)
    return {"volume_per_atom_A3": vol / n, "area_per_atom_A2": area / n,
            "paper_range_volume_A3": [8.8, 9.3], "paper_range_area_A2": [2.0, 3.2]}


def kernel_sources_digest(kernel):
    """Digest of the sources a kernel is built from (to match a profile)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1809_04352_amd", "csrc")
    files = ["eses_device.h", "eses_internal.h",
             "classify.hip" if kernel.startswith("k_classify") else "edges.hip"]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_counters(kernel, workload, prec):
    """Figures of a committed PMC summary of this exact kernel source
    (profiles/pmc_<kernel>_<workload>_<prec>.md: lines "- name: value"),
    or None when there is none or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload}_{prec}.md")
    if not os.path.exists(path):
        return None
    digest = kernel_sources_digest(kernel)
    vals = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources digest") != digest:
        return None
    out = {}
    for k, v in vals.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


if __name__ == "__main__":
    main()
