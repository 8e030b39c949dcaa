"""Parity at the workloads' full sizes.

globule5000_h0.25 is compared over the whole grid.  For the 100,000-atom
(h = 0.2 A) and 20,000-atom (h = 0.1 A) globules the HIP path runs on the
whole grid, in the configuration the benchmark times, and is compared with
the oracle on evenly spaced pairs of z-slices (labels of both slices, every
edge leaving the first) plus the whole set of concave probe positions; the
FP32+recheck labels are compared with the FP64 labels over the whole grid.
"""
import numpy as np
import pytest

from tests.parity import POS_TOL, compare_edges, compare_labels, compare_vertices

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def test_globule5000_full(E, oracle_mod):
    from eses_inputs import workload
    m = workload("globule5000_h0.25")
    print("case: globule5000_h0.25 full", m.dims, flush=True)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    ref = o.labels_grid(m.lo, m.spacing, m.dims)
    for prec in (E.ESES_FP64, E.ESES_FP32_RECHECK):
        res = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, prec=prec)
        compare_labels(res["labels"], ref)
        compare_edges(res, o, m.lo, m.spacing, m.dims, ref)
    assert compare_vertices(res["vertices"], o) > 1000


def sampled_parity(E, oracle_mod, name, n_pairs):
    import torch
    from eses_inputs import workload
    m = workload(name)
    nx, ny, nz = m.dims
    print(f"case: {name} sampled, dims {m.dims}", flush=True)
    r64 = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, prec=E.ESES_FP64)
    r32 = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi,
                    prec=E.ESES_FP32_RECHECK, stats=True)
    assert np.array_equal(r64["labels"], r32["labels"])
    for k in ("key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(r64[k], r32[k]), k
    print("rechecked", r32["classify_stats"]["n_rechecked"], "of", m.n_points, flush=True)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    assert compare_vertices(r64["vertices"], o) > 1000
    key = r64["key"]
    slab = (key // 3) // (nx * ny)
    ks = np.linspace(1, nz - 3, n_pairs).astype(int)
    checked = 0
    for k in ks:
        ref = o.labels_grid(m.lo, m.spacing, m.dims, int(k), int(k) + 2)
        compare_labels(r64["labels"][k:k + 2], ref)
        sel = slab == k
        want = oracle_mod.crossing_keys(ref)
        want = want[(want // 3) < nx * ny] + 3 * int(k) * nx * ny
        assert np.array_equal(key[sel], want)
        sub = {q: r64[q][sel] for q in ("key", "lam", "normal", "patch_type", "atoms")}
        compare_edges(sub, o, m.lo, m.spacing, m.dims)
        checked += int(sel.sum())
    assert checked > 10000
    return m, r64


def test_globule100k_sampled(E, oracle_mod):
    sampled_parity(E, oracle_mod, "globule100k_h0.2", 10)


def test_globule20k_fine_sampled(E, oracle_mod):
    sampled_parity(E, oracle_mod, "globule20k_h0.1", 10)
