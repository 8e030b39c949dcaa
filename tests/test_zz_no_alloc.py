"""The allocation-free edge entry point (eses_edge_intersections_noalloc)
against eses_edge_intersections, through the C-ABI: two calls in a row, the
second on a smaller molecule, each with records identical to the allocating
form's; while it runs a caller allocator installed with eses_set_allocator is
never asked for memory (the allocating form asks it for every temporary)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def run_pair(E, n, seed, h):
    import torch
    from eses_inputs import molecule
    m = molecule(n, seed, h)
    print(f"case: n={n} seed={seed} h={h} dims={m.dims}", flush=True)
    c = torch.as_tensor(m.centres, device="cuda")
    r = torch.as_tensor(m.radii, device="cuda")
    mol = E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
    d = E.grid_dims(mol)
    labels = torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device="cuda")
    cand = E.build_candidates([mol])
    try:
        E.classify(cand, E.ESES_FP64, [labels])
        _, counts = E.edge_intersections(cand, [labels], [E.alloc_isect(1)])
        ref = E.alloc_isect(counts[0])
        st, _ = E.edge_intersections(cand, [labels], [ref])
        assert st == E.ESES_OK
        out = E.alloc_isect(counts[0])
        calls = []
        E.set_allocator(lambda nbytes, stream: calls.append(nbytes) or 0,
                        lambda ptr, stream: calls.append(-1))
        try:
            st, k = E.edge_intersections_noalloc(cand, labels, out)
        finally:
            E.set_allocator()
        assert st == E.ESES_OK and k == counts[0]
        assert calls == [], calls
        torch.cuda.synchronize()
        for f in ("key", "lam", "normal", "patch_type", "atoms"):
            a, b = getattr(out, f)[:k].cpu().numpy(), getattr(ref, f)[:k].cpu().numpy()
            assert np.array_equal(a, b), f
        return k
    finally:
        cand.close()


def test_noalloc_two_calls_smaller_second(E):
    k1 = run_pair(E, 400, 11, 0.35)
    k2 = run_pair(E, 60, 12, 0.4)
    assert k1 > k2 > 0


def test_noalloc_rejects_batches(E):
    import torch
    from eses_inputs import molecule
    ms = [molecule(30, 20 + q, 0.5) for q in range(2)]
    tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
            for m in ms]
    mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi) for (c, r), m in zip(tens, ms)]
    cand = E.build_candidates(mols)
    try:
        d = E.grid_dims(mols[0])
        labels = torch.zeros(d[0] * d[1] * d[2], dtype=torch.uint8, device="cuda")
        with pytest.raises(E.EsesError) as ei:
            E.edge_intersections_noalloc(cand, labels, E.alloc_isect(8))
        assert ei.value.status == E.ESES_EINVAL
    finally:
        cand.close()
