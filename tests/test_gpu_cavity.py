"""GPU parity of the cavity-filled variant (eses_fill_cavities, through the
C-ABI): filled labels bit-exact against the oracle's fill of its exact labels,
the crossing records of the filled grid against the oracle's; a hollow shell
with an enclosed cavity, a globule without one, and both in one batch."""
import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels
from tests.test_oracle_cavity_pins import shell

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def cases():
    from eses_inputs import Molecule, grid_dims, molecule
    c, r = shell()
    lo, hi = np.full(3, -12.0), np.full(3, 12.0)
    sh = Molecule(c, r, 1.4, 0.5, lo, hi, grid_dims(lo, hi, 0.5))
    c2, r2 = shell(n=90, R=6.0, r=1.6)
    lo2, hi2 = np.array([-9.7, -9.1, -9.3]), np.array([9.2, 9.8, 9.4])
    sh2 = Molecule(c2 + 0.123, r2, 1.4, 0.3, lo2, hi2, grid_dims(lo2, hi2, 0.3))
    return [sh, molecule(300, 5, 0.5), sh2]


def check(E, oracle_mod, cand, mols_np, labels, filled):
    import torch
    _, counts = E.edge_intersections(cand, labels, [E.alloc_isect(1) for _ in labels])
    outs = [E.alloc_isect(max(k, 1)) for k in counts]
    st, counts = E.edge_intersections(cand, labels, outs)
    assert st == E.ESES_OK
    torch.cuda.synchronize()
    for m, L, n, out, k in zip(mols_np, labels, filled, outs, counts):
        o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
        ref, nref = oracle_mod.fill_cavities(o.labels_grid(m.lo, m.spacing, m.dims))
        compare_labels(L.cpu().numpy().reshape(ref.shape), ref)
        assert n == nref
        res = {f: getattr(out, f)[:k].cpu().numpy() for f in ("key", "lam", "normal",
                                                              "patch_type", "atoms")}
        compare_edges(res, o, m.lo, m.spacing, m.dims, ref)


@pytest.mark.parametrize("batch", [False, True])
def test_fill_cavities(E, oracle_mod, batch):
    import torch
    mols_np = cases()
    groups = [mols_np] if batch else [[m] for m in mols_np]
    for g in groups:
        print("case: fill", "batch" if batch else "single", [m.dims for m in g], flush=True)
        tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
                for m in g]
        mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi) for (c, r), m in zip(tens, g)]
        cand = E.build_candidates(mols)
        try:
            labels = [torch.empty(m.n_points, dtype=torch.uint8, device="cuda") for m in g]
            E.classify(cand, E.ESES_FP32_RECHECK, labels)
            filled = E.fill_cavities(cand, labels)
            if g[0].n_atoms == 140:
                assert filled[0] > 1000
            check(E, oracle_mod, cand, g, labels, filled)
        finally:
            cand.close()
