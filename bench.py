#!/usr/bin/env python
"""Benchmark of the ESES hot path on one MI355X.

A step is one pass of the whole path over one molecule whose inputs are
already in HBM: eses_build_candidates (cell binning, SAS pairs and circles,
concave probe positions, exposure flags, tile lists), eses_classify (every grid
point) and eses_edge_intersections (every crossing edge, roots and normals).

Prints one JSON line.  `value` is grid points through the whole path per
second; the classification and intersection rates of the metric are reported
beside it, with a roofline entry for the dominant kernel and the FP64 CPU
oracle timed on a bounded sample of the same workload.
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
DEFAULT_WORKLOAD = "globule5000_h0.25"

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
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB (a known-size "
                         "reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(m, n_crossings, target_s):
    """The FP64 oracle on a bounded, evenly strided sample of z-slices."""
    import numpy as np
    from oracle import oracle as orc

    orc.build(force=False)
    nx, ny, nz = m.dims
    t0 = time.perf_counter()
    o = orc.Oracle(m.centres, m.radii, m.probe)
    t_create = time.perf_counter() - t0
    # time one pair of middle slices to pick the stride
    mid = nz // 2
    t0 = time.perf_counter()
    L = o.labels_grid(m.lo, m.spacing, m.dims, mid, mid + 2)
    t_pair_lab = time.perf_counter() - t0
    keys = orc.crossing_keys(L)
    keys = keys[(keys // 3) < nx * ny] + 3 * mid * nx * ny  # edges whose s is in slice mid
    t0 = time.perf_counter()
    o.edges(m.lo, m.spacing, m.dims, keys)
    t_pair_edge = time.perf_counter() - t0
    per_pair = max(t_pair_lab + t_pair_edge, 1e-3)
    n_pairs = int(max(1, min(nz // 2, target_s / per_pair)))
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
    t_full = t_create + t_lab / pts * m.n_points + (t_edge / max(edges, 1)) * n_crossings
    return {
        "value": m.n_points / t_full,
        "unit": "grid points/s",
        "cores": orc.threads(),
        "kind": "oracle",
        "sample": (f"whole-molecule probe enumeration ({t_create:.2f} s) + labels of {pts} points "
                   f"in {len(ks)} evenly spaced slice pairs ({t_lab:.2f} s) + {edges} crossing "
                   f"edges there ({t_edge:.2f} s), extrapolated to {m.n_points} points and "
                   f"{n_crossings} crossings"),
        "seconds": t_create + t_lab + t_edge,
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
    prec = eses.ESES_FP64 if args.prec == "fp64" else eses.ESES_FP32_RECHECK
    mols_np = load_workload(args.workload)
    dev = torch.device("cuda:0")
    tens = [(torch.as_tensor(m.centres, device=dev), torch.as_tensor(m.radii, device=dev))
            for m in mols_np]
    mols = [eses.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
            for (c, r), m in zip(tens, mols_np)]
    dims = [eses.grid_dims(m) for m in mols]
    npts = sum(d[0] * d[1] * d[2] for d in dims)
    labels = [torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device=dev) for d in dims]

    # sizing pass (outside the timed region): output capacities and work counts
    cand = eses.build_candidates(mols)
    infos = [cand.info(q) for q in range(len(mols))]
    work = eses.classify(cand, prec, labels, stats=True)
    probe_out = [eses.alloc_isect(1) for _ in mols]
    _, counts = eses.edge_intersections(cand, labels, probe_out)
    ework = eses.edge_work(cand, labels)
    cand.close()
    outs = [eses.alloc_isect(max(k, 1)) for k in counts]
    n_cross = sum(counts)

    def total(dicts, key):
        return sum(d[key] for d in dicts)

    flops_classify = sum(FLOPS_PER_TEST[k] * total(work, k) for k in FLOPS_PER_TEST)
    flops_edges = sum(FLOPS_EDGE[k] * total(ework, k) for k in FLOPS_EDGE)

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    stage = {"build": [], "classify": [], "edges": []}
    kern = {"classify_ms": [], "edge_detect_ms": [], "edge_roots_ms": []}

    def step(record):
        if record:
            ev[0].record(stream)
        c = eses.build_candidates(mols)
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

    rl = {}
    for name, fl, t in (("classify", flops_classify, kmed["classify_ms"]),
                        ("edge_roots", flops_edges, kmed["edge_roots_ms"])):
        a = fl / (t * 1e-3) / 1e12
        kname = "k_classify" if name == "classify" else "k_edge_chunks"
        if len(mols) > 1:
            kname += "_batch"  # the fused launches of a batch
        rl[name] = {"kernel": kname,
                    "bound": "alu", "achieved": a, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": a / PEAK_FP64_TFLOPS, "traffic": None, "algorithmic_flops": fl,
                    "ms": t}
    for v in rl.values():
        v["traffic"] = profiled_traffic(v["kernel"], args.workload, args.prec)
    dominant = max(rl, key=lambda k: rl[k]["ms"])
    roof = dict(rl[dominant])
    single = len(mols_np) == 1
    m0 = mols_np[0]
    config = {"workload": args.workload, "molecules": len(mols_np),
              "atoms": sum(m.n_atoms for m in mols_np), "probe": m0.probe,
              "spacing": m0.spacing, "points": npts, "precision": args.prec, "tile": 8}
    if single:
        config["dims"] = list(dims[0])
    res = {
        "metric": METRIC,
        "value": npts / (ms * 1e-3),
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": config,
        "classify_pts_per_s": npts / (kmed["classify_ms"] * 1e-3),
        "isect_per_s": n_cross / (med["edges"] * 1e-3),
        "crossings": n_cross,
        "stages_ms": med,
        "kernels_ms": kmed,
        "classify_work": {k: total(work, k) for k in work[0]},
        "edge_work": {k: total(ework, k) for k in ework[0]},
        "roofline": roof,
        "roofline_other": {k: v for k, v in rl.items() if k != dominant},
    }
    if single:
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
    if not args.no_cpu_baseline and single:
        res["cpu_baseline"] = cpu_baseline(m0, n_cross, args.cpu_seconds)
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


def profiled_traffic(kernel, workload, prec):
    """HBM bytes per launch from a committed PMC summary of this exact kernel
    source (profiles/pmc_<kernel>_<workload>_<prec>.md), else None."""
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
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


if __name__ == "__main__":
    main()
