"""Parity at full size: globule5000_h0.25 over the whole grid, in both
precisions (the larger workloads are compared whole in test_gpu_whole.py)."""
import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels, compare_vertices

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
