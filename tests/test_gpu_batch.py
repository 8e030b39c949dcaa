"""The batched form: one persistent fused classification launch over many
molecules (recorded as a HIP graph and replayed), against per-molecule
results and the oracle."""
import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def run_batch(E, mols_np, prec, reps=2, blocks_per_cu=0, tile=0, unit_order=0,
              edges_per_molecule=False, partial=False):
    import torch
    tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
            for m in mols_np]
    mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
            for (c, r), m in zip(tens, mols_np)]
    cand = E.build_candidates(mols, tile=tile, blocks_per_cu=blocks_per_cu,
                              unit_order=unit_order, edges_per_molecule=edges_per_molecule)
    dims = [E.grid_dims(m) for m in mols]
    out = []
    for rep in range(reps):
        labels = [torch.full((d[0] * d[1] * d[2],), 7, dtype=torch.uint8, device="cuda")
                  for d in dims]
        E.classify(cand, prec, labels)
        torch.cuda.synchronize()
        # eager work between replays
        _ = torch.arange(1000, device="cuda").sum().item()
        out.append([l.cpu().numpy().reshape(d[2], d[1], d[0]) for l, d in zip(labels, dims)])
    for rep in range(1, reps):
        for a, b in zip(out[0], out[rep]):
            assert np.array_equal(a, b), "replay differs"
    edges = []
    isect = [E.alloc_isect(1) for _ in mols]
    st, counts = E.edge_intersections(cand, labels, isect)
    if partial:
        # every molecule's output a third of what it needs (one molecule none):
        # the counts are complete, the records written are the first ones
        caps = [k // 3 for k in counts]
        caps[0] = 0
        full = counts
        isect = [E.alloc_isect(max(k, 1)) for k in caps]
        isect = [E.IsectBuffers(o.key[:k], o.lam[:k], o.normal[:k], o.patch_type[:k],
                                o.atoms[:k]) for o, k in zip(isect, caps)]
        st, counts = E.edge_intersections(cand, labels, isect)
        assert st == E.ESES_ECAPACITY and list(counts) == list(full)
        counts = caps
    else:
        isect = [E.alloc_isect(max(k, 1)) for k in counts]
        st, counts = E.edge_intersections(cand, labels, isect)
        assert st == E.ESES_OK
    torch.cuda.synchronize()
    for o, k in zip(isect, counts):
        edges.append(dict(key=o.key[:k].cpu().numpy(), lam=o.lam[:k].cpu().numpy(),
                          normal=o.normal[:k].cpu().numpy(),
                          patch_type=o.patch_type[:k].cpu().numpy(),
                          atoms=o.atoms[:k].cpu().numpy()))
    cand.close()
    return out[0], edges


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_matches_single(E, oracle_mod, prec):
    from eses_inputs import molecule
    spec = [(1, 1, 0.4), (2, 2, 0.5), (40, 3, 0.35), (300, 4, 0.5), (120, 5, 0.25), (60, 6, 0.45),
            (800, 7, 0.5), (3, 8, 0.3)]
    mols = [molecule(n, s, h) for n, s, h in spec]
    print("case: batch of", len(mols), "prec", prec, flush=True)
    labels, edges = run_batch(E, mols, prec, reps=3)
    for m, lab, ed in zip(mols, labels, edges):
        single = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, prec=prec)
        assert np.array_equal(single["labels"], lab)
        for k in ("key", "lam", "normal", "patch_type", "atoms"):
            assert np.array_equal(single[k], ed[k]), k
        o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
        ref = o.labels_grid(m.lo, m.spacing, m.dims)
        compare_labels(lab, ref)
        compare_edges(ed, o, m.lo, m.spacing, m.dims, ref)


def test_batch_with_empty_surfaces(E, oracle_mod):
    """Molecules whose grids hold no crossing edge (a box away from the atoms:
    every point outside; a box inside one atom: every point inside) batched
    with ordinary ones."""
    from eses_inputs import Molecule, grid_dims, molecule
    c1 = np.array([[0.0, 0.0, 0.0], [2.9, 0.3, 0.1]])
    r1 = np.array([1.7, 1.5])
    far_lo, far_hi = np.array([10.0, 10.0, 10.0]), np.array([14.1, 12.3, 13.2])
    in_lo, in_hi = np.array([-0.6, -0.5, -0.55]), np.array([0.6, 0.45, 0.5])
    mols = [Molecule(c1, r1, 1.4, 0.3, far_lo, far_hi, grid_dims(far_lo, far_hi, 0.3)),
            molecule(90, 41, 0.4),
            Molecule(c1, r1, 1.4, 0.1, in_lo, in_hi, grid_dims(in_lo, in_hi, 0.1)),
            molecule(30, 42, 0.3)]
    print("case: batch with empty surfaces", flush=True)
    labels, edges = run_batch(E, mols, 0, reps=2)
    assert labels[0].sum() == 0 and len(edges[0]["key"]) == 0
    assert labels[2].all() and len(edges[2]["key"]) == 0
    for m, lab, ed in zip(mols, labels, edges):
        o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
        ref = o.labels_grid(m.lo, m.spacing, m.dims)
        compare_labels(lab, ref)
        compare_edges(ed, o, m.lo, m.spacing, m.dims, ref)


def test_launch_knobs_do_not_change_results(E):
    """Unit order, workgroups per CU, tile edge and the per-molecule
    crossing-edge passes change the launch only: labels and records equal
    those of the default configuration; with outputs too small, the counts
    are complete and the records written are the first ones."""
    from eses_inputs import molecule
    mols = [molecule(n, 60 + n, h) for n, h in ((150, 0.5), (700, 0.4), (40, 0.3))]
    base_l, base_e = run_batch(E, mols, 1, reps=1)
    for knobs in (dict(unit_order=1), dict(blocks_per_cu=2), dict(tile=4, unit_order=1),
                  dict(edges_per_molecule=True), dict(partial=True),
                  dict(partial=True, edges_per_molecule=True)):
        print("case: knobs", knobs, flush=True)
        lab, ed = run_batch(E, mols, 1, reps=2, **knobs)
        for a, b in zip(base_l, lab):
            assert np.array_equal(a, b)
        for a, b in zip(base_e, ed):
            for k in a:
                assert np.array_equal(a[k][:len(b[k])], b[k]), k
                assert knobs.get("partial") or len(a[k]) == len(b[k]), k


def test_autotune(E, tmp_path, monkeypatch):
    from eses_inputs import molecule
    from paper_1809_04352_amd import autotune
    import torch
    monkeypatch.setenv("ESES_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    mols_np = [molecule(n, 30 + n, 0.5) for n in (100, 400, 900)]
    tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
            for m in mols_np]
    mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)
            for (c, r), m in zip(tens, mols_np)]
    best, times = autotune.tune(mols, E.ESES_FP32_RECHECK, reps=2)
    assert len(times) == len(autotune.CANDIDATES_BATCH)
    assert best in autotune.CANDIDATES_BATCH
    best2, times2 = autotune.tune(mols, E.ESES_FP32_RECHECK, reps=2)
    assert best2 == best and times2 == times  # cached
