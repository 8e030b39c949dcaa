"""GPU parity of the marching-cubes mesh (eses_mesh, through the C-ABI):
the triangles (record-index triples) identical to the oracle's mesh of the
same labels and records, area and volume within 1e-11 relative of the oracle's
sums over the same mesh and within 1e-6 of the oracle's mesh on its own
records; one sphere against its closed forms; a batch."""
import math

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


def gpu_mesh(E, mols_np):
    import torch
    tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
            for m in mols_np]
    mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi) for (c, r), m in zip(tens, mols_np)]
    cand = E.build_candidates(mols)
    try:
        labels = [torch.empty(m.n_points, dtype=torch.uint8, device="cuda") for m in mols_np]
        E.classify(cand, E.ESES_FP64, labels)
        _, counts = E.edge_intersections(cand, labels, [E.alloc_isect(1) for _ in mols])
        outs = [E.alloc_isect(max(k, 1)) for k in counts]
        E.edge_intersections(cand, labels, outs)
        st = E.mesh(cand, labels, outs, counts)
        tris = [torch.empty((max(s["n_triangles"], 1), 3), dtype=torch.int32, device="cuda")
                for s in st]
        st2 = E.mesh(cand, labels, outs, counts, triangles=tris)
        torch.cuda.synchronize()
        assert st2 == st
        res = []
        for m, L, o, k, s, t in zip(mols_np, labels, outs, counts, st, tris):
            res.append(dict(labels=L.cpu().numpy().reshape(m.dims[2], m.dims[1], m.dims[0]),
                            key=o.key[:k].cpu().numpy(), lam=o.lam[:k].cpu().numpy(),
                            tri=t[:s["n_triangles"]].cpu().numpy(), **s))
        return res
    finally:
        cand.close()


def check(oracle_mod, m, g):
    from oracle import mesh as M
    tri, V = M.mesh(g["labels"], m.lo, m.spacing, g["key"], g["lam"])
    assert np.array_equal(g["tri"], tri)
    assert M.closed_and_oriented(tri)
    A, Vol = M.area_volume(tri, V)
    assert abs(g["area"] / A - 1) < 1e-11 and abs(g["volume"] / Vol - 1) < 1e-11
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    rec = o.edges(m.lo, m.spacing, m.dims, g["key"])
    tri_o, V_o = M.mesh(g["labels"], m.lo, m.spacing, g["key"], rec["lam"])
    A_o, Vol_o = M.area_volume(tri_o, V_o)
    assert abs(g["area"] / A_o - 1) < 1e-6 and abs(g["volume"] / Vol_o - 1) < 1e-6
    print(f"mesh: {len(tri)} triangles, area {g['area']:.4f}, volume {g['volume']:.4f}", flush=True)


def test_mesh_sphere_and_globule(E, oracle_mod):
    from eses_inputs import Molecule, grid_dims, molecule
    c = np.array([[0.031, -0.017, 0.011]])
    lo, hi = np.full(3, -2.5), np.full(3, 2.5)
    sphere = Molecule(c, np.array([1.7]), 1.4, 0.1, lo, hi, grid_dims(lo, hi, 0.1))
    mols = [sphere, molecule(300, 5, 0.4)]
    for m in mols:
        print("case: mesh", m.n_atoms, m.dims, flush=True)
        g = gpu_mesh(E, [m])[0]
        check(oracle_mod, m, g)
    g = gpu_mesh(E, [sphere])[0]
    assert abs(g["area"] / (4 * math.pi * 1.7 ** 2) - 1) < 0.015
    assert abs(g["volume"] / (4 / 3 * math.pi * 1.7 ** 3) - 1) < 0.015


def test_mesh_batch(E, oracle_mod):
    from eses_inputs import molecule
    mols = [molecule(n, 50 + n, h) for n, h in ((40, 0.35), (200, 0.5), (90, 0.3))]
    print("case: mesh batch", [m.dims for m in mols], flush=True)
    for m, g in zip(mols, gpu_mesh(E, mols)):
        check(oracle_mod, m, g)
