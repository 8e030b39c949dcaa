"""GPU parity of the out-of-core form (eses_stream_slabs, through the C-ABI):
labels and records streamed slab by slab into host memory equal, bit for bit,
those of the whole-grid calls (eses_classify + eses_edge_intersections) for
slab sizes from one tile layer to more than the grid, a ragged last slab and
both precisions; on the small molecule they are also compared with the
oracle directly.  Capacity and argument errors are reported as documented."""
import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels

pytestmark = pytest.mark.gpu

FIELDS = ("key", "lam", "normal", "patch_type", "atoms")


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def host_isect(cap):
    import torch
    from paper_1809_04352_amd.eses import IsectBuffers
    cap = max(int(cap), 1)
    pin = torch.cuda.is_available()
    return IsectBuffers(torch.empty(cap, dtype=torch.int64, pin_memory=pin),
                        torch.empty(cap, dtype=torch.float64, pin_memory=pin),
                        torch.empty((cap, 3), dtype=torch.float64, pin_memory=pin),
                        torch.empty(cap, dtype=torch.uint8, pin_memory=pin),
                        torch.empty((cap, 3), dtype=torch.int32, pin_memory=pin))


def whole(E, cand, m, prec):
    import torch
    labels = torch.empty(m.n_points, dtype=torch.uint8, device="cuda")
    E.classify(cand, prec, [labels])
    _, counts = E.edge_intersections(cand, [labels], [E.alloc_isect(1)])
    out = E.alloc_isect(counts[0])
    st, counts = E.edge_intersections(cand, [labels], [out])
    assert st == E.ESES_OK
    k = counts[0]
    return labels.cpu().numpy(), {f: getattr(out, f)[:k].cpu().numpy() for f in FIELDS}


def streamed(E, cand, m, prec, planes, cap):
    import torch
    labels = torch.full((m.n_points,), 7, dtype=torch.uint8).pin_memory()
    out = host_isect(cap)
    st, k = E.stream_slabs(cand, prec, planes, labels, out)
    torch.cuda.synchronize()
    return st, k, labels.numpy().copy(), {f: getattr(out, f)[:min(k, cap)].numpy().copy()
                                          for f in FIELDS}


def handle(E, m):
    import torch
    c = torch.as_tensor(m.centres, device="cuda")
    r = torch.as_tensor(m.radii, device="cuda")
    mol = E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
    return (c, r), E.build_candidates([mol])


def same(ref_lab, ref, lab, res):
    assert np.array_equal(lab, ref_lab), int(np.count_nonzero(lab != ref_lab))
    for f in FIELDS:
        assert np.array_equal(res[f], ref[f]), f


@pytest.mark.parametrize("name", ["globule500_h0.5", "globule5000_h0.25"])
def test_stream_equals_whole_grid(E, name):
    from eses_inputs import workload
    m = workload(name)
    keep, cand = handle(E, m)
    try:
        nz = m.dims[2]
        for prec in (E.ESES_FP32_RECHECK, E.ESES_FP64):
            ref_lab, ref = whole(E, cand, m, prec)
            for planes in (8, 24, 64, 8 * (nz // 8 + 2)):
                print("case:", name, "prec", prec, "slab planes", planes, "nz", nz, flush=True)
                st, k, lab, res = streamed(E, cand, m, prec, planes, len(ref["key"]) + 5)
                assert st == E.ESES_OK and k == len(ref["key"])
                same(ref_lab, ref, lab, res)
    finally:
        cand.close()


def test_stream_against_oracle(E, oracle_mod):
    """The streamed outputs of a molecule whose grid height is not a multiple
    of the slab, against the oracle's labels and records."""
    from eses_inputs import molecule
    m = molecule(400, 11, 0.45)
    keep, cand = handle(E, m)
    try:
        print("case: oracle, dims", m.dims, flush=True)
        _, k0, _, _ = streamed(E, cand, m, E.ESES_FP32_RECHECK, 16, 1)
        st, k, lab, res = streamed(E, cand, m, E.ESES_FP32_RECHECK, 16, k0)
        assert st == E.ESES_OK and k == k0
        o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
        ref = o.labels_grid(m.lo, m.spacing, m.dims)
        compare_labels(lab.reshape(ref.shape), ref)
        compare_edges(res, o, m.lo, m.spacing, m.dims, ref)
    finally:
        cand.close()


def test_stream_capacity_and_arguments(E):
    import torch
    from eses_inputs import molecule
    m = molecule(200, 12, 0.5)
    keep, cand = handle(E, m)
    try:
        ref_lab, ref = whole(E, cand, m, E.ESES_FP64)
        n = len(ref["key"])
        st, k, lab, res = streamed(E, cand, m, E.ESES_FP64, 8, n // 3)
        assert st == E.ESES_ECAPACITY and k == n
        assert np.array_equal(lab, ref_lab)  # the labels are complete all the same
        for f in FIELDS:
            assert np.array_equal(res[f], ref[f][:n // 3]), f
        labels = torch.empty(m.n_points, dtype=torch.uint8).pin_memory()
        for bad in (0, 4, 12, -8):
            with pytest.raises(E.EsesError):
                E.stream_slabs(cand, E.ESES_FP64, bad, labels, host_isect(n))
    finally:
        cand.close()
    m2 = molecule(150, 13, 0.5)
    # a handle of two molecules is refused
    t = [(torch.as_tensor(x.centres, device="cuda"), torch.as_tensor(x.radii, device="cuda"))
         for x in (m, m2)]
    mols = [E.make_molecule(c, r, x.probe, x.spacing, x.lo, x.hi) for (c, r), x in zip(t, (m, m2))]
    cand2 = E.build_candidates(mols)
    try:
        labels = torch.empty(m.n_points, dtype=torch.uint8).pin_memory()
        with pytest.raises(E.EsesError):
            E.stream_slabs(cand2, E.ESES_FP64, 8, labels, host_isect(10))
    finally:
        cand2.close()
