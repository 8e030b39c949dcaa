"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Labels bit-exact, the crossing-edge set identical, intersection positions
within 1e-6 A and normals within 1e-6, concave probe positions identical as
a set (triple + side) and within 1e-9 A.
"""
import math

import numpy as np
import pytest

from tests.parity import compare_edges, compare_labels, compare_vertices

pytestmark = pytest.mark.gpu

RHO = 1.4


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def run_and_compare(E, oracle_mod, c, r, probe, h, lo, hi, prec, tile=0):
    from eses_inputs import grid_dims
    dims = grid_dims(lo, hi, h)
    print(f"case: n={len(r)} h={h} dims={dims} prec={prec} tile={tile}", flush=True)
    res = E.surface(c, r, probe, h, lo, hi, prec=prec, tile=tile)
    assert res["dims"] == dims
    o = oracle_mod.Oracle(c, r, probe)
    ref = o.labels_grid(lo, h, dims)
    compare_labels(res["labels"], ref)
    nv = compare_vertices(res["vertices"], o)
    ne, ties = compare_edges(res, o, lo, h, dims, ref)
    return res, nv, ne


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,seed,h,tile", [
    (1, 1, 0.25, 8), (2, 2, 0.3, 8), (40, 3, 0.35, 8), (120, 4, 0.5, 4), (120, 4, 0.5, 8),
    (300, 5, 0.45, 8),
])
def test_small_molecules(E, oracle_mod, prec, n, seed, h, tile):
    from eses_inputs import molecule
    m = molecule(n, seed, h)
    run_and_compare(E, oracle_mod, m.centres, m.radii, m.probe, h, m.lo, m.hi, prec, tile)


@pytest.mark.parametrize("probe,prec", [(0.6, 0), (2.2, 0), (2.2, 1)])
def test_probe_radii(E, oracle_mod, probe, prec):
    """A small and a large probe (more and fewer concave patches, spindle
    tori with the large one) on a 120-atom globule."""
    from eses_inputs import molecule
    m = molecule(120, 4, 0.4)
    run_and_compare(E, oracle_mod, m.centres, m.radii, probe, 0.4, m.lo, m.hi, prec)


@pytest.mark.parametrize("h,lo,hi", [
    (2.0, (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)),      # 2 x 2 x 2 points
    (0.9, (-1.3, -0.4, -2.2), (1.1, 0.5, 2.0)),      # 4 x 2 x 6
    (0.35, (-2.0, -0.1, -0.1), (2.1, 0.2, 0.2)),     # one line of points along x
])
def test_tiny_grids(E, oracle_mod, h, lo, hi):
    """Grids of a few points (smaller than one tile and than a label word)
    cutting through two atoms."""
    c = np.array([[0.05, 0.02, -0.03], [1.9, 0.1, 0.4]])
    r = np.array([1.6, 1.2])
    run_and_compare(E, oracle_mod, c, r, RHO, h, np.array(lo), np.array(hi), 0)


@pytest.mark.parametrize("probe", [0.1, 5.0])
def test_extreme_probe_radii(E, oracle_mod, probe):
    """A probe far smaller than an atom (the surface close to the van der
    Waals surface, thin saddles) and far larger (wide tori and probe spheres,
    long reaches in the tile lists)."""
    from eses_inputs import molecule
    m = molecule(50, 5, 0.4)
    run_and_compare(E, oracle_mod, m.centres, m.radii, probe, 0.4, m.lo, m.hi, 0)


@pytest.mark.parametrize("prec", [0, 1])
def test_far_from_origin(E, oracle_mod, prec):
    """A molecule thousands of angstroms from the origin (tile-local FP32
    offsets, large FP64 coordinates)."""
    from eses_inputs import bbox_from_atoms, molecule
    m = molecule(80, 6, 0.4)
    c = m.centres + np.array([5321.37, -2987.11, 1234.56])
    lo, hi = bbox_from_atoms(c, m.radii, 4.0)
    run_and_compare(E, oracle_mod, c, m.radii, RHO, 0.4, lo, hi, prec)


def test_scaled_molecule(E, oracle_mod):
    """Every length doubled (radii 2.4-3.6 A, probe 2.8 A, spacing 0.8 A): a
    power-of-two scaling leaves every label unchanged."""
    from eses_inputs import molecule
    m = molecule(60, 8, 0.4)
    base = E.surface(m.centres, m.radii, RHO, 0.4, m.lo, m.hi)
    res, _, _ = run_and_compare(E, oracle_mod, 2 * m.centres, 2 * m.radii, 2 * RHO, 0.8,
                                2 * m.lo, 2 * m.hi, 0)
    assert np.array_equal(res["labels"], base["labels"])


@pytest.mark.parametrize("rotate", [False, True])
def test_collinear_chain(E, oracle_mod, rotate):
    """Atoms on one line: every triple is collinear (no three-sphere point)
    and all tori share one axis, parallel to x with rotate=False.  Lengths
    are chosen so that no grid point lies within rounding of a sphere, where
    two FP64 evaluations in different operation orders may disagree (decimal
    lattices make such exact ties: a chain at 2.6 A spacing on this grid puts
    three points exactly on van der Waals spheres)."""
    from eses_inputs import bbox_from_atoms
    c = np.stack([np.arange(6) * 2.6137, np.zeros(6), np.zeros(6)], axis=1) + np.array(
        [0.0, 0.0313, -0.0271])
    if rotate:
        q, _ = np.linalg.qr(np.random.default_rng(3).normal(size=(3, 3)))
        c = c @ q.T + np.array([0.3, -0.2, 0.1])
    r = np.array([1.7, 1.5, 1.8, 1.55, 1.7, 1.2])
    lo, hi = bbox_from_atoms(c, r, 2.0)
    res, nv, ne = run_and_compare(E, oracle_mod, c, r, RHO, 0.25, lo, hi, 0)
    assert nv == 0 and ne > 1000


def test_contained_atoms(E, oracle_mod):
    """Atoms whose balls lie inside another's, beside ordinary neighbours:
    they add nothing to the surface (lengths chosen away from exact ties)."""
    from eses_inputs import bbox_from_atoms
    c = np.array([[0.0137, -0.0219, 0.0071], [0.3121, 0.2093, -0.1187], [-0.2113, 0.1171, 0.2534],
                  [3.2173, 0.4129, 0.1063], [1.5191, 2.7137, -0.3119]])
    r = np.array([1.8113, 1.2071, 1.1937, 1.6129, 1.5083])
    lo, hi = bbox_from_atoms(c, r, 2.0)
    res, _, _ = run_and_compare(E, oracle_mod, c, r, RHO, 0.2, lo, hi, 0)
    keep = [0, 3, 4]
    ref = E.surface(c[keep], r[keep], RHO, 0.2, lo, hi)
    assert np.array_equal(res["labels"], ref["labels"])


@pytest.mark.parametrize("prec", [0, 1])
def test_globule500(E, oracle_mod, prec):
    from eses_inputs import workload
    m = workload("globule500_h0.5")
    res, nv, ne = run_and_compare(E, oracle_mod, m.centres, m.radii, m.probe, m.spacing, m.lo,
                                  m.hi, prec)
    assert nv > 100 and ne > 1000


def test_dyadic_single_sphere_ties(E, oracle_mod):
    """Grid points exactly on the sphere (dyadic inputs) are inside."""
    c = np.array([[0.25, -0.5, 0.125]])
    r = np.array([1.5])
    lo = np.array([-4.0, -4.0, -4.0])
    hi = np.array([4.0, 4.0, 4.0])
    res, _, ne = run_and_compare(E, oracle_mod, c, r, RHO, 0.125, lo, hi, 0)
    assert res["labels"].sum() > 0


def test_two_atoms_on_grid_axis(E, oracle_mod):
    """Atoms on a grid line: points on the circle's axis see every circle point
    at the same distance (the degenerate nearest point)."""
    c = np.array([[0.0, 0.0, 0.0], [5.6, 0.0, 0.0]])
    r = np.array([1.5, 1.5])
    lo = np.array([-4.0, -4.0, -4.0])
    hi = np.array([9.6, 4.0, 4.0])
    run_and_compare(E, oracle_mod, c, r, RHO, 0.2, lo, hi, 0)


def test_sparse_atoms_far_apart(E, oracle_mod):
    """Isolated atoms far apart (empty cells, tiles with no candidates)."""
    c = np.array([[0.0, 0.0, 0.0], [30.0, 1.0, -2.0], [3.1, 0.2, 0.1]])
    r = np.array([1.7, 1.2, 1.55])
    from eses_inputs import bbox_from_atoms
    lo, hi = bbox_from_atoms(c, r, 2.0)
    run_and_compare(E, oracle_mod, c, r, RHO, 0.4, lo, hi, 0)


@pytest.mark.parametrize("motion,prec", [(0, 0), (1, 0), (1, 1), (2, 0)])
def test_cospherical_lattice(E, oracle_mod, motion, prec):
    """Equal atoms (r 1.7 A) on a 4x4x3 simple cubic lattice at 3.0 A: every
    lattice square is a cospherical quadruple whose probe touches four atoms
    and is reported by all four triples on both sides.  Motion 0 keeps the
    lattice on the grid's axes (circle axes along grid lines), the others
    move it rigidly."""
    from eses_inputs import bbox_from_atoms
    g = np.array([[i, j, k] for k in range(3) for j in range(4) for i in range(4)], float)
    c = g * 3.0
    if motion:
        rng = np.random.default_rng(motion)
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        c = c @ q.T + rng.uniform(-5.0, 5.0, 3)
    r = np.full(len(c), 1.7)
    lo, hi = bbox_from_atoms(c, r, 3.0)
    if motion == 0:
        lo = np.floor(lo)  # whole angstroms: grid points on the lattice planes
    res, nv, ne = run_and_compare(E, oracle_mod, c, r, RHO, 0.25, lo, hi, prec)
    # 42 lattice squares on the outer faces, four triples each, outer side only
    assert nv == 168
    assert ne > 1000


def test_capacity_and_counts(E, oracle_mod):
    import torch
    from eses_inputs import molecule
    m = molecule(80, 9, 0.5)
    ct = torch.as_tensor(m.centres, device="cuda")
    rt = torch.as_tensor(m.radii, device="cuda")
    mol = E.make_molecule(ct, rt, m.probe, m.spacing, m.lo, m.hi)
    cand = E.build_candidates([mol])
    dims = E.grid_dims(mol)
    lab = torch.empty(dims[0] * dims[1] * dims[2], dtype=torch.uint8, device="cuda")
    E.classify(cand, 0, [lab])
    small = E.alloc_isect(10)
    st, counts = E.edge_intersections(cand, [lab], [small])
    assert st == E.ESES_ECAPACITY and counts[0] > 10
    full = E.alloc_isect(counts[0])
    st, counts2 = E.edge_intersections(cand, [lab], [full])
    assert st == E.ESES_OK and counts2 == counts
    torch.cuda.synchronize()
    assert np.array_equal(small.key.cpu().numpy(), full.key[:10].cpu().numpy())
    assert np.array_equal(small.lam.cpu().numpy(), full.lam[:10].cpu().numpy())
    stats = E.classify(cand, 0, [lab], stats=True)
    assert stats[0]["n_inside"] == int(lab.sum().item())
    cand.close()


def test_invalid_device_input(E):
    import torch
    c = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    r = torch.tensor([1.5, -1.0], dtype=torch.float64, device="cuda")
    mol = E.make_molecule(c, r, 1.4, 0.5, [-5, -5, -5], [5, 5, 5])
    with pytest.raises(E.EsesError) as ei:
        E.build_candidates([mol])
    assert ei.value.status == E.ESES_EINVAL


@pytest.mark.parametrize("radii", [(1.5, 1.5), (1.7, 1.2)])
def test_coincident_centres_rejected(E, oracle_mod, radii):
    """Two atoms sharing a centre (a duplicate or a concentric pair) are
    rejected by both the library and the oracle; a valid molecule built right
    after still matches the oracle."""
    import torch
    c = np.array([[0.0, 0.0, 0.0], [3.0, 0.5, 0.2], [0.0, 0.0, 0.0]])
    r = np.array([radii[0], 1.5, radii[1]])
    mol = E.make_molecule(torch.as_tensor(c, device="cuda"), torch.as_tensor(r, device="cuda"),
                          RHO, 0.5, [-5, -5, -5], [7, 5, 5])
    with pytest.raises(E.EsesError) as ei:
        E.build_candidates([mol])
    assert ei.value.status == E.ESES_EINVAL
    assert "distinct" in str(ei.value)
    with pytest.raises(ValueError):
        oracle_mod.Oracle(c, r, RHO)
    lo, hi = np.array([-5.0, -5.0, -5.0]), np.array([7.0, 5.0, 5.0])
    run_and_compare(E, oracle_mod, c[:2], r[:2], RHO, 0.25, lo, hi, 0)


def test_repeat_is_deterministic(E):
    from eses_inputs import molecule
    m = molecule(150, 12, 0.4)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(a["vertices"], b["vertices"]):
        assert np.array_equal(x, y)


def test_repeated_classification_of_one_handle(E, oracle_mod):
    """Regression: one handle classified eight times in a row (both
    precisions) gives the oracle's labels every time.  A molecule whose tiles
    stage circles with short cut lists: their direction cones were once read
    from LDS before the threads staging the circles had written them, which
    changed labels from call to call."""
    import torch
    from eses_inputs import molecule
    m = molecule(120, 5, 0.25)
    c = torch.as_tensor(m.centres, device="cuda")
    r = torch.as_tensor(m.radii, device="cuda")
    cand = E.build_candidates([E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi)])
    try:
        ref = oracle_mod.Oracle(m.centres, m.radii, m.probe).labels_grid(m.lo, m.spacing, m.dims)
        for call in range(8):
            prec = call % 2
            print("case: repeated classification, call", call, flush=True)
            lab = torch.empty(m.n_points, dtype=torch.uint8, device="cuda")
            E.classify(cand, prec, [lab])
            compare_labels(lab.cpu().numpy().reshape(ref.shape), ref)
    finally:
        cand.close()


def test_tile_shape_invariance(E):
    from eses_inputs import molecule
    m = molecule(200, 13, 0.3)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, tile=8)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, tile=4)
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k


def test_fp32_recheck_matches_fp64_and_counts(E):
    """FP32 certified decisions plus FP64 recheck give the FP64 labels; forcing
    every point through the recheck path gives them too."""
    from eses_inputs import molecule
    m = molecule(400, 21, 0.3)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, prec=E.ESES_FP64,
                  stats=True)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi,
                  prec=E.ESES_FP32_RECHECK, stats=True)
    c = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi,
                  prec=E.ESES_FP32_RECHECK, force_recheck=True, stats=True)
    for r in (b, c):
        for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
            assert np.array_equal(a[k], r[k]), k
    assert a["classify_stats"]["n_rechecked"] == 0
    n = a["labels"].size
    assert c["classify_stats"]["n_rechecked"] == n
    assert b["classify_stats"]["n_rechecked"] < 1e-3 * n
    print("rechecked", b["classify_stats"]["n_rechecked"], "of", n)


def test_kernel_timing_and_edge_work(E):
    """Library-side HIP-event timing and the edge statistics pass."""
    import torch
    from eses_inputs import molecule
    m = molecule(300, 31, 0.4)
    ct = torch.as_tensor(m.centres, device="cuda")
    rt = torch.as_tensor(m.radii, device="cuda")
    mol = E.make_molecule(ct, rt, m.probe, m.spacing, m.lo, m.hi)
    cand = E.build_candidates([mol])
    dims = E.grid_dims(mol)
    lab = torch.empty(dims[0] * dims[1] * dims[2], dtype=torch.uint8, device="cuda")
    E.set_timing(True)
    try:
        E.classify(cand, 0, [lab])
        out = E.alloc_isect(1)
        _, counts = E.edge_intersections(cand, [lab], [out])
        out = E.alloc_isect(counts[0])
        E.edge_intersections(cand, [lab], [out])
        t = E.kernel_times(cand)
    finally:
        E.set_timing(False)
    assert t["classify_ms"] > 0 and t["edge_roots_ms"] > 0 and t["edge_detect_ms"] > 0
    w = E.edge_work(cand, [lab])[0]
    assert w["n_edges"] == counts[0]
    assert w["quad_solves"] > 0 and w["reach_sphere"] >= w["quad_solves"]
    assert w["label_evals"] <= 8 * counts[0]
    # the statistics pass leaves the records untouched
    st, c2 = E.edge_intersections(cand, [lab], [out])
    assert c2 == counts
    cand.close()


@pytest.mark.parametrize("n,seed,h", [(120, 4, 0.5), (300, 5, 0.45), (500, 1, 0.5)])
def test_edge_fallback_path(E, oracle_mod, n, seed, h):
    """The one-wavefront-per-edge root kernel (taken by edges of tiles whose
    root lists overflow) gives the chunk path's records bit for bit, and the
    oracle's."""
    from eses_inputs import molecule
    m = molecule(n, seed, h)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, edge_fallback=True)
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    ref = o.labels_grid(m.lo, m.spacing, m.dims)
    compare_edges(b, o, m.lo, m.spacing, m.dims, ref)


def test_workspace_cache_reuse_and_trim(E):
    """Workspace blocks reused from the cache, and freed by eses_trim_cache,
    leave the results unchanged."""
    from eses_inputs import molecule
    m = molecule(150, 12, 0.4)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    E.trim_cache()
    c = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k


@pytest.mark.parametrize("pool", [1, 16])
def test_vertex_pool_overflow(E, oracle_mod, pool):
    """Probe positions recomputed by the fill pass when the count pass's pool
    overflows (a pool of one or 16 entries) come out in the same order as
    the pooled ones, with identical labels and records, and match the
    oracle's positions."""
    from eses_inputs import molecule
    m = molecule(500, 1, 0.5)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, vertex_pool=pool)
    assert a["info"]["n_vertices"] > pool
    for q in range(3):
        assert np.array_equal(a["vertices"][q], b["vertices"][q])
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    assert compare_vertices(b["vertices"], o) > 10


@pytest.mark.parametrize("pool", [1, 16])
def test_tile_pool_overflow(E, oracle_mod, pool):
    """Tile candidate lists rebuilt by the fill pass for the tiles with more
    entries than the count pass keeps (one: every non-trivial tile; 16: a mix)
    give the same labels and records as the kept lists, and the oracle's
    labels."""
    from eses_inputs import molecule
    m = molecule(400, 6, 0.45)
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi, tile_pool=pool)
    assert a["info"]["tile_list_entries"] == b["info"]["tile_list_entries"] > 0
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    compare_labels(b["labels"], o.labels_grid(m.lo, m.spacing, m.dims))


def test_caller_allocator(E):
    """Workspace taken from the caller's allocator (torch's caching allocator
    through eses_set_allocator) gives the same records as the library's own
    cache, for one molecule and for a batch, and every block is handed back."""
    import torch
    from eses_inputs import molecule
    live = {}

    def alloc(n, stream):
        p = torch.cuda.caching_allocator_alloc(n, stream=stream)
        live[p] = n
        return p

    def release(p, stream):
        assert p in live
        del live[p]
        torch.cuda.caching_allocator_delete(p)

    ms = [molecule(n, s, 0.45) for n, s in ((150, 21), (260, 22), (90, 23))]

    def run_batch():
        mols, labs = [], []
        for m in ms:
            c = torch.as_tensor(m.centres, device="cuda")
            r = torch.as_tensor(m.radii, device="cuda")
            mols.append((E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi), c, r))
        cand = E.build_candidates([x[0] for x in mols])
        dims = [E.grid_dims(x[0]) for x in mols]
        labs = [torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device="cuda") for d in dims]
        E.classify(cand, 0, labs)
        outs = [E.alloc_isect(1) for _ in ms]
        _, counts = E.edge_intersections(cand, labs, outs)
        outs = [E.alloc_isect(k) for k in counts]
        E.edge_intersections(cand, labs, outs)
        torch.cuda.synchronize()
        cand.close()
        return [l.cpu().numpy() for l in labs], [o.lam[:k].cpu().numpy() for o, k in zip(outs, counts)]

    m = ms[0]
    a = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
    la, ra = run_batch()
    E.set_allocator(alloc, release)
    try:
        b = E.surface(m.centres, m.radii, m.probe, m.spacing, m.lo, m.hi)
        lb, rb = run_batch()
    finally:
        E.set_allocator()
    torch.cuda.synchronize()
    for k in ("labels", "key", "lam", "normal", "patch_type", "atoms"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(la + ra, lb + rb):
        assert np.array_equal(x, y)
    assert not live, f"{len(live)} blocks not handed back"


@pytest.mark.parametrize("batch", [False, True])
def test_caller_allocator_out_of_memory(E, batch):
    """A caller allocator that has no memory: eses_build_candidates returns
    ESES_ENOMEM (with the bytes asked for in the message), for one molecule
    and for a batch (the failure comes from a worker thread), and the library
    works again once its own cache is restored."""
    import torch
    from eses_inputs import molecule
    ms = [molecule(60, 31 + q, 0.5) for q in range(3 if batch else 1)]
    tens = [(torch.as_tensor(m.centres, device="cuda"), torch.as_tensor(m.radii, device="cuda"))
            for m in ms]
    mols = [E.make_molecule(c, r, m.probe, m.spacing, m.lo, m.hi) for (c, r), m in zip(tens, ms)]
    asked = []
    E.set_allocator(lambda n, stream: asked.append(n) or 0, lambda p, stream: None)
    try:
        with pytest.raises(E.EsesError) as ei:
            E.build_candidates(mols)
    finally:
        E.set_allocator()
    assert ei.value.status == E.ESES_ENOMEM
    assert "no memory" in str(ei.value) and asked
    cand = E.build_candidates(mols)
    cand.close()
