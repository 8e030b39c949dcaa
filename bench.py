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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by molecule or z-slab with no exchange step; only the "
              "one-GPU share is measured)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from eses_inputs import workload
    from paper_1809_04352_amd import eses

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    eses.load()
    prec = eses.ESES_FP64 if args.prec == "fp64" else eses.ESES_FP32_RECHECK
    m = workload(args.workload)
    dev = torch.device("cuda:0")
    ct = torch.as_tensor(m.centres, device=dev)
    rt = torch.as_tensor(m.radii, device=dev)
    mol = eses.make_molecule(ct, rt, m.probe, m.spacing, m.lo, m.hi)
    dims = eses.grid_dims(mol)
    npts = dims[0] * dims[1] * dims[2]
    labels = torch.empty(npts, dtype=torch.uint8, device=dev)

    # sizing pass (outside the timed region): output capacity and work counts
    cand = eses.build_candidates([mol])
    info = cand.info(0)
    work = eses.classify(cand, prec, [labels], stats=True)[0]
    probe_out = eses.alloc_isect(1)
    _, counts = eses.edge_intersections(cand, [labels], [probe_out])
    cand.close()
    out = eses.alloc_isect(counts[0])
    n_cross = counts[0]
    flops_classify = sum(FLOPS_PER_TEST[k] * work[k] for k in FLOPS_PER_TEST)

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    stage = {"build": [], "classify": [], "edges": []}

    def step(record):
        if record:
            ev[0].record(stream)
        c = eses.build_candidates([mol])
        if record:
            ev[1].record(stream)
        eses.classify(c, prec, [labels])
        if record:
            ev[2].record(stream)
        st, cnt = eses.edge_intersections(c, [labels], [out])
        if record:
            ev[3].record(stream)
        c.close()
        if st != eses.ESES_OK or cnt[0] != n_cross:
            raise RuntimeError("unexpected edge count")
        if record:
            torch.cuda.synchronize()
            stage["build"].append(ev[0].elapsed_time(ev[1]))
            stage["classify"].append(ev[1].elapsed_time(ev[2]))
            stage["edges"].append(ev[2].elapsed_time(ev[3]))

    for _ in range(args.warmup):
        step(True)
    stage = {k: [] for k in stage}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    # per-stage event timing in separate steps (the synchronising reads of
    # the timed loop are not disturbed)
    for _ in range(max(3, min(args.steps, 10))):
        step(True)
    med = {k: float(np.median(v)) for k, v in stage.items()}

    t_cls = med["classify"] * 1e-3
    achieved = flops_classify / t_cls / 1e12
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
        "config": {"workload": args.workload, "atoms": m.n_atoms, "probe": m.probe,
                   "spacing": m.spacing, "dims": list(dims), "points": npts,
                   "precision": args.prec, "tile": 8},
        "classify_pts_per_s": npts / t_cls,
        "isect_per_s": n_cross / (med["edges"] * 1e-3),
        "crossings": n_cross,
        "stages_ms": med,
        "candidates": {k: (list(v) if isinstance(v, tuple) else v) for k, v in info.items()},
        "classify_work": work,
        "roofline": {
            "kernel": "k_classify_fp64",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": None,
            "algorithmic_flops": flops_classify,
            "flops_per_point": flops_classify / npts,
        },
    }
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calibrate_copy_bytes"] = nbytes
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(m, n_cross, args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
