"""GPU parity on inputs full of exact ties, through the C-ABI.

Grid points exactly on van der Waals and SAS spheres, exactly rho from probe
positions and on the axes of circles (dyadic lattices), and points within
rounding of spheres (a chain on a decimal lattice): the classification
certifies each FP64 decision against a bound on its rounding error and the
host re-decides the rest exactly, so the labels equal the oracle's exact labels
bit for bit -- in both precisions, whichever FP64 evaluation order either side
uses.  Edges as in the other parity tests.
"""
import math

import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels, compare_vertices
from tests.test_oracle_exact_pins import decimal_chain, dyadic_lattice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def tie_case(case):
    h = 0.25
    if case == "chain":
        c, r, rho = decimal_chain()
        lo = np.array([-4.1, -3.0, -3.0])  # points at offsets 0.9, 1.2, -0.8 ... from centres
        hi = (c + r[:, None]).max(axis=0) + 1.0
    elif case == "lattice":
        c, r, rho = dyadic_lattice()
        lo = (c - r[:, None]).min(axis=0) - 1.0
        hi = (c + r[:, None]).max(axis=0) + 1.0
    elif case == "lattice_rho":
        # probe 1.25, atoms 1.0 on a 2.5 A lattice: SAS radius 2.25 (9 + 12 = 15^2 / 4
        # ... 1.35^2 + 1.8^2 = 2.25^2 on the grid)
        g = np.array([[x, y, z] for z in (0.0, 2.5) for y in (0.0, 2.5, 5.0) for x in (0.0, 2.5)])
        c, r, rho = g, np.full(len(g), 1.0), 1.25
        h = 0.125
        lo = (c - r[:, None]).min(axis=0) - 1.5
        hi = (c + r[:, None]).max(axis=0) + 1.5
    dims = tuple(int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    return c, r, rho, h, lo, hi, dims


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("case", ["lattice", "chain", "lattice_rho"])
def test_tie_lattices_bit_exact(E, oracle_mod, case, prec):
    c, r, rho, h, lo, hi, dims = tie_case(case)
    print(f"case: {case} prec={prec} dims={dims}", flush=True)
    res = E.surface(c, r, rho, h, lo, hi, prec=prec, stats=True)
    assert res["dims"] == dims
    o = oracle_mod.Oracle(c, r, rho)
    ref = o.labels_grid(lo, h, dims)
    assert o.last_undecided > 0
    compare_labels(res["labels"], ref)
    st = res["classify_stats"]
    print(f"exact re-decisions: GPU {st['n_exact']}, oracle {o.last_undecided}", flush=True)
    assert st["n_exact"] > 0
    compare_vertices(res["vertices"], o)
    compare_edges(res, o, lo, h, dims, ref)


def test_uncertain_queue_overflow(E, oracle_mod):
    """A queue of 8 entries for the uncertain points: it overflows, is grown
    and the molecule is classified again; the labels do not change."""
    c, r, rho, h, lo, hi, dims = tie_case("lattice")
    res = E.surface(c, r, rho, h, lo, hi, stats=True, unc_queue=8)
    assert res["classify_stats"]["n_exact"] > 8
    o = oracle_mod.Oracle(c, r, rho)
    compare_labels(res["labels"], o.labels_grid(lo, h, dims))


def test_tie_lattice_batch(E, oracle_mod):
    """The tie lattices as molecules of one batch (fused classification under
    a HIP graph, uncertain points gathered per molecule and re-decided)."""
    import torch
    cases = [tie_case(k) for k in ("lattice", "chain", "lattice_rho")]
    dev = "cuda"
    tens = [(torch.as_tensor(c, device=dev), torch.as_tensor(r, device=dev))
            for c, r, *_ in cases]
    mols = [E.make_molecule(ct, rt, rho, h, lo, hi)
            for (ct, rt), (_, _, rho, h, lo, hi, _) in zip(tens, cases)]
    labels = [torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device=dev)
              for *_, d in cases]
    cand = E.build_candidates(mols)
    try:
        for prec in (E.ESES_FP32_RECHECK, E.ESES_FP64):
            st = E.classify(cand, prec, labels, stats=True)
            assert all(s["n_exact"] > 0 for s in st)
            for (c, r, rho, h, lo, hi, dims), L in zip(cases, labels):
                o = oracle_mod.Oracle(c, r, rho)
                compare_labels(L.cpu().numpy().reshape(dims[2], dims[1], dims[0]),
                               o.labels_grid(lo, h, dims))
    finally:
        cand.close()
