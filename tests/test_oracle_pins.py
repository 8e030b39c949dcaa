"""Pins of the FP64 oracle against facts the mathematics fixes independently.

Each test checks the oracle against something other than itself: closed forms
of the solvent-excluded surface for one and two atoms and for the concave
probe position of three equal atoms, brute force on tiny inputs (all-triples
probe enumeration, dense sampling of the admissible probe set), invariances of
the definition, and integrals whose values are known.

The definition pinned (section 1 and eq. 2 of the paper): with SAS radii
s = r + rho, U the union of open SAS balls and A its complement, a point is
inside iff its distance to A is at least rho.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

RHO = 1.4


def rot(seed):
    q = np.random.default_rng(seed).normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


# ---------------------------------------------------------------- one atom

def test_single_sphere_labels_closed_form(oracle_mod):
    """One atom: M is the closed van der Waals ball (the probe rolls freely)."""
    c = np.array([[0.25, -0.5, 0.125]])
    r = np.array([1.5])
    o = oracle_mod.Oracle(c, r, RHO)
    lo = np.array([-4.0, -4.0, -4.0])
    h = 0.125  # dyadic: grid coordinates and squared distances are exact
    dims = (65, 65, 65)
    L = o.labels_grid(lo, h, dims)
    g = lo[0] + np.arange(65) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    ref = ((X - c[0, 0]) ** 2 + (Y - c[0, 1]) ** 2 + (Z - c[0, 2]) ** 2) <= 1.5 ** 2
    assert np.array_equal(L.astype(bool), ref)
    # a grid point exactly on the surface is inside (M is closed)
    tie = np.array([[0.25 + 1.5, -0.5, 0.125]])
    assert o.labels_points(tie)[0] == 1
    assert o.labels_points(tie + [[2.0 ** -40, 0, 0]])[0] == 0


def test_single_sphere_distance_closed_form(oracle_mod):
    o = oracle_mod.Oracle([[0.0, 0.0, 0.0]], [1.7], RHO)
    rng = np.random.default_rng(3)
    x = rng.uniform(-3.0, 3.0, size=(2000, 3))
    d = np.linalg.norm(x, axis=1)
    dist, typ = o.dist_points(x, 10.0)
    inU = d < 1.7 + RHO
    assert np.allclose(dist[inU], (1.7 + RHO) - d[inU], atol=1e-12)
    assert np.all(dist[~inU] == 0)
    assert np.all(typ[inU] == 1)


# ---------------------------------------------------------------- two atoms

def two_atom_label(x, c1, c2, r1, r2, rho):
    """Closed form in profile coordinates (xi along c1->c2, eta >= 0).

    Inside iff in a van der Waals ball, or inside the triangle c1, P, c2
    (P = (a, R) the circle's profile point) and at least rho from P; the two
    radial projections are buried there, so the nearest admissible probe
    centre is the circle point of the same azimuth.  Elsewhere in U the
    radial projection onto a sphere is exposed and closer than rho.
    Returns (label, margin) where margin bounds the distance to a decision
    boundary of this formula.
    """
    s1, s2 = r1 + rho, r2 + rho
    v = c2 - c1
    d = np.linalg.norm(v)
    e = v / d
    w = x - c1
    xi = w @ e
    eta = np.linalg.norm(w - np.outer(xi, e), axis=1)
    d1 = np.linalg.norm(x - c1, axis=1)
    d2 = np.linalg.norm(x - c2, axis=1)
    a = (s1 * s1 - s2 * s2 + d * d) / (2 * d)
    R = math.sqrt(s1 * s1 - a * a)
    vdw = (d1 <= r1) | (d2 <= r2)
    inU = (d1 < s1) | (d2 < s2)
    # triangle (0,0), (d,0), (a,R), counter-clockwise
    def cross(ax, ay, bx, by):
        return ax * by - ay * bx
    t1 = cross(d, 0.0, xi, eta)
    t2 = cross(a - d, R, xi - d, eta)
    t3 = cross(-a, -R, xi - a, eta - R)
    tri = (t1 >= 0) & (t2 >= 0) & (t3 >= 0)
    dP = np.hypot(xi - a, eta - R)
    lab = np.where(vdw, 1, np.where(~inU, 0, np.where(tri, dP >= rho, 0))).astype(np.uint8)
    margin = np.minimum.reduce([np.abs(d1 - r1), np.abs(d2 - r2), np.abs(d1 - s1),
                                np.abs(d2 - s2), np.where(tri, np.abs(dP - rho), np.inf)])
    return lab, margin


@pytest.mark.parametrize("r1,r2,d", [
    (1.7, 1.7, 3.2),     # ordinary saddle, R > rho
    (1.5, 1.5, 5.6),     # spindle torus, R < rho: the neck is open
    (1.2, 1.8, 1.0),     # circle centre behind c1 (a < 0)
    (1.52, 1.2, 2.4),
    (1.8, 1.55, 4.9),
])
def test_two_atoms_closed_form(oracle_mod, r1, r2, d):
    R = rot(int(r1 * 100 + r2 * 10 + d * 7))
    c1 = np.array([0.3, -0.2, 0.1])
    c2 = c1 + R @ np.array([d, 0.0, 0.0])
    o = oracle_mod.Oracle(np.stack([c1, c2]), [r1, r2], RHO)
    rng = np.random.default_rng(11)
    lo = np.minimum(c1, c2) - 5.0
    hi = np.maximum(c1, c2) + 5.0
    x = rng.uniform(lo, hi, size=(60000, 3))
    ref, margin = two_atom_label(x, c1, c2, r1, r2, RHO)
    got = o.labels_points(x)
    keep = margin > 1e-9
    assert keep.mean() > 0.999
    assert np.array_equal(got[keep], ref[keep])
    assert ref.min() == 0 and ref.max() == 1


def test_two_atoms_axis_points(oracle_mod):
    """Points on the axis are equidistant from every circle point (degenerate nearest point)."""
    r1, r2, d = 1.5, 1.5, 5.6
    c1 = np.zeros(3)
    c2 = np.array([d, 0.0, 0.0])
    o = oracle_mod.Oracle(np.stack([c1, c2]), [r1, r2], RHO)
    xi = np.linspace(-0.5, d + 0.5, 1201)
    x = np.stack([xi, np.zeros_like(xi), np.zeros_like(xi)], axis=1)
    ref, margin = two_atom_label(x, c1, c2, r1, r2, RHO)
    got = o.labels_points(x)
    keep = margin > 1e-9
    assert np.array_equal(got[keep], ref[keep])
    assert got.min() == 0  # the open neck


# ---------------------------------------------------------------- vertices

def test_equilateral_vertex_closed_form(oracle_mod):
    """Three equal SAS spheres on an equilateral triangle of side L: the two
    probe positions sit on the normal through the centroid at height
    sqrt(s^2 - L^2/3)."""
    r, L = 1.7, 3.6
    s = r + RHO
    ang = np.array([0.0, 2 * math.pi / 3, 4 * math.pi / 3])
    base = np.stack([L / math.sqrt(3) * np.cos(ang), L / math.sqrt(3) * np.sin(ang),
                     np.zeros(3)], axis=1)
    Rm = rot(5)
    c = base @ Rm.T + np.array([1.0, 2.0, -0.5])
    o = oracle_mod.Oracle(c, [r] * 3, RHO)
    p, atoms, sign = o.vertices()
    assert p.shape == (2, 3)
    assert np.array_equal(atoms, [[0, 1, 2], [0, 1, 2]])
    hgt = math.sqrt(s * s - L * L / 3)
    nrm = Rm @ np.array([0.0, 0.0, 1.0])
    cen = c.mean(axis=0)
    want = {1: cen + hgt * nrm, -1: cen - hgt * nrm}
    # sign convention: + has (p - c_i) . ((c_j - c_i) x (c_k - c_i)) > 0
    for q in range(2):
        assert np.allclose(p[q], want[int(sign[q])], atol=1e-12)
    # probe balls are outside, the three van der Waals balls inside
    for q in range(2):
        pts = p[q] + rng_ball(200, RHO * 0.999, 17 + q)
        assert np.all(o.labels_points(pts) == 0)
    pts = np.concatenate([c[m] + rng_ball(200, r, 30 + m) for m in range(3)])
    assert np.all(o.labels_points(pts) == 1)


def test_concave_cap_flips_at_probe_radius(oracle_mod):
    """Three atoms and one of their probes p: inside the cone spanned from p
    by the directions to the three centres, p is the nearest admissible point,
    so dist(x, A) = |x - p| and the label flips exactly at |x - p| = rho along
    every ray of the cone (the concave patch is the probe sphere there)."""
    r, L = np.array([1.7, 1.55, 1.52]), 3.4
    s = r + RHO
    ang = np.array([0.0, 2.1, 4.3])
    base = np.stack([L / math.sqrt(3) * np.cos(ang), L / math.sqrt(3) * np.sin(ang),
                     np.array([0.0, 0.3, -0.2])], axis=1)
    Rm = rot(11)
    c = base @ Rm.T + np.array([-0.7, 1.3, 2.1])
    o = oracle_mod.Oracle(c, r, RHO)
    p, atoms, sign = o.vertices()
    assert p.shape == (2, 3)
    rng = np.random.default_rng(3)
    for q in range(2):
        pq = p[q]
        assert np.allclose(np.linalg.norm(c - pq, axis=1), s, atol=1e-12)
        dirs = (c - pq) / np.linalg.norm(c - pq, axis=1, keepdims=True)
        wts = rng.dirichlet(np.ones(3), size=200)
        u = wts @ dirs
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        for f, want in ((1 - 1e-9, 0), (1 + 1e-9, 1)):
            assert np.all(o.labels_points(pq + f * RHO * u) == want)
        d, typ = o.dist_points(pq + 0.5 * RHO * u, 50.0)
        assert np.allclose(d, 0.5 * RHO, atol=1e-12)
        assert np.all(typ == 3)


def test_cospherical_square_every_triple(oracle_mod):
    """Four equal atoms on a square of half-side a: the probe above (and below)
    the centre touches all four at height sqrt(s^2 - 2 a^2), so each of the four
    triples reports it on both sides, at that closed-form position, under any
    rigid motion (the rounding of the point must not drop a triple)."""
    r, a = 1.7, 1.5
    s = r + RHO
    base = np.array([[a, a, 0.0], [-a, a, 0.0], [-a, -a, 0.0], [a, -a, 0.0]])
    hgt = math.sqrt(s * s - 2 * a * a)
    triples = {t for t in itertools.combinations(range(4), 3)}
    for seed in range(60):
        Rm = rot(100 + seed)
        shift = np.random.default_rng(seed).uniform(-20.0, 20.0, 3)
        c = base @ Rm.T + shift
        o = oracle_mod.Oracle(c, [r] * 4, RHO)
        p, atoms, sign = o.vertices()
        assert p.shape == (8, 3)
        got = {(tuple(int(v) for v in t), int(sg)) for t, sg in zip(atoms, sign)}
        assert got == {(t, sg) for t in triples for sg in (1, -1)}
        nrm = Rm @ np.array([0.0, 0.0, 1.0])
        tops = (shift + hgt * nrm, shift - hgt * nrm)
        for q in range(8):
            assert min(np.linalg.norm(p[q] - t) for t in tops) < 1e-12 * (1 + np.abs(shift).max())
        # the concave region under each probe is outside, the atoms inside
        for top in (shift + hgt * nrm, shift - hgt * nrm):
            pts = top + rng_ball(100, RHO * 0.999, seed)
            assert np.all(o.labels_points(pts) == 0)


def rng_ball(n, radius, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * radius * rng.uniform(0, 1, size=(n, 1)) ** (1 / 3)


def brute_vertices(c, r, rho):
    """All triples, all atoms: the two points on three SAS spheres from the
    two radical planes and one sphere, kept if no other open SAS ball holds
    them."""
    s = r + rho
    n = len(r)
    out = {}
    for i, j, k in itertools.combinations(range(n), 3):
        A = np.stack([c[j] - c[i], c[k] - c[i]])
        b = 0.5 * np.array([s[i] ** 2 - s[j] ** 2 + c[j] @ c[j] - c[i] @ c[i],
                            s[i] ** 2 - s[k] ** 2 + c[k] @ c[k] - c[i] @ c[i]])
        m = np.cross(A[0], A[1])
        if np.linalg.norm(m) < 1e-9:
            continue
        p0 = np.linalg.lstsq(A, b, rcond=None)[0]
        w = p0 - c[i]
        qa, qb, qc = m @ m, 2 * (w @ m), w @ w - s[i] ** 2
        disc = qb * qb - 4 * qa * qc
        if disc < 0:
            continue
        for t in ((-qb + math.sqrt(disc)) / (2 * qa), (-qb - math.sqrt(disc)) / (2 * qa)):
            p = p0 + t * m
            others = [l for l in range(n) if l not in (i, j, k)]
            # admissible up to a relative 1e-9 of s_l^2 (a probe touching a
            # fourth atom exactly stays admissible under rounding)
            if others and np.any(np.sum((c[others] - p) ** 2, axis=1)
                                 < s[others] ** 2 * (1 - 1e-9)):
                continue
            sg = 1 if (p - c[i]) @ m > 0 else -1
            out[(i, j, k, sg)] = p
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_vertices_brute_force(oracle_mod, seed):
    from eses_inputs import globule
    c, r = globule(24, 100 + seed)
    o = oracle_mod.Oracle(c, r, RHO)
    p, atoms, sign = o.vertices()
    got = {(int(a[0]), int(a[1]), int(a[2]), int(s)): pp for pp, a, s in zip(p, atoms, sign)}
    want = brute_vertices(c, r, RHO)
    assert set(got) == set(want)
    assert len(want) > 0
    for key in want:
        assert np.allclose(got[key], want[key], atol=1e-10)
    # residuals on the three spheres
    s = r + RHO
    for key, pp in got.items():
        for m in key[:3]:
            assert abs(np.linalg.norm(pp - c[m]) - s[m]) < 1e-12


# ---------------------------------------------------------------- brute force distance

def fib_sphere(n):
    k = np.arange(n) + 0.5
    z = 1 - 2 * k / n
    phi = math.pi * (1 + math.sqrt(5)) * k
    rr = np.sqrt(1 - z * z)
    return np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)


def exposed_samples(c, r, rho, per_sphere):
    s = r + rho
    unit = fib_sphere(per_sphere)
    pts = []
    for i in range(len(r)):
        y = c[i] + s[i] * unit
        ok = np.ones(len(y), bool)
        for k in range(len(r)):
            if k != i:
                ok &= np.sum((y - c[k]) ** 2, axis=1) >= s[k] ** 2
        pts.append(y[ok])
    return np.concatenate(pts)


def test_coincident_centres_rejected(oracle_mod):
    """Atoms are distinct balls: two atoms sharing a centre (duplicate or
    concentric) are rejected rather than given a rounding-dependent surface."""
    c = np.array([[0.0, 0.0, 0.0], [3.0, 0.5, 0.2], [0.0, 0.0, 0.0]])
    for r in ([1.7, 1.5, 1.7], [1.7, 1.5, 1.2]):
        with pytest.raises(ValueError):
            oracle_mod.Oracle(c, r, RHO)
    oracle_mod.Oracle(c[:2], [1.7, 1.5], RHO)


def lattice(nx, ny, nz, step, seed):
    """Equal-radius atoms on a simple cubic lattice, rigidly moved by seed
    (seed 0: axis-aligned, unmoved).  Every lattice square is a cospherical
    quadruple: the probe above its centre touches four atoms."""
    g = np.array([[i, j, k] for k in range(nz) for j in range(ny) for i in range(nx)], float)
    c = g * step
    if seed:
        c = c @ rot(200 + seed).T + np.random.default_rng(seed).uniform(-5.0, 5.0, 3)
    return c, np.full(len(c), 1.7)


@pytest.mark.parametrize("seed,rho", [(7, RHO), (8, RHO), ("lattice", RHO), (11, 0.6), (12, 2.2)])
def test_distance_brute_force(oracle_mod, seed, rho):
    """dist(x, A) from the oracle against the nearest of ~1e6 admissible
    points sampled on the exposed parts of the SAS spheres (the boundary of
    A): the sample set lies in A, so the oracle may never exceed it, and it
    is dense, so the oracle may not fall below it by more than its spacing.
    The lattice case is a 3x3 slab of equal atoms at 3.0 A, whose concave
    probes each touch four atoms; two cases use a small and a large probe."""
    from eses_inputs import globule
    if seed == "lattice":
        c, r = lattice(3, 3, 1, 3.0, 3)
        seed = 9
    else:
        c, r = globule(10, seed)
    s = r + rho
    per = 120000
    samp = exposed_samples(c, r, rho, per)
    tree = cKDTree(samp)
    o = oracle_mod.Oracle(c, r, rho)
    rng = np.random.default_rng(seed)
    lo = c.min(axis=0) - 3.5
    hi = c.max(axis=0) + 3.5
    x = rng.uniform(lo, hi, size=(40000, 3))
    d2 = np.sum((x[:, None, :] - c[None]) ** 2, axis=2)
    inU = np.any(d2 < s ** 2, axis=1)
    x = x[inU]
    dist_bf = tree.query(x)[0]
    dist, typ = o.dist_points(x, 50.0)
    # nearest-sample gap on the largest sphere of the Fibonacci sampling
    spacing = 1.1 * math.sqrt(4 * math.pi * s.max() ** 2 / per)
    assert np.all(dist <= dist_bf + 1e-9)
    assert np.all(dist >= dist_bf - spacing)
    assert set(np.unique(typ)) >= {1, 2}
    # labels from the definition where the brute force is decisive
    vdw = np.any(d2[inU] <= r ** 2, axis=1)
    lab_bf = np.where(vdw, 1, dist_bf >= rho).astype(np.uint8)
    keep = vdw | (np.abs(dist_bf - rho) > spacing)
    got = o.labels_points(x)
    assert np.array_equal(got[keep], lab_bf[keep])
    assert keep.mean() > 0.95


# ---------------------------------------------------------------- invariances

def _small_case(n=60, seed=9, h=0.5):
    from eses_inputs import globule, bbox_from_atoms, grid_dims
    c, r = globule(n, seed)
    # snap the box corner to the grid spacing so dyadic moves keep it exact
    lo, hi = bbox_from_atoms(c, r, 4.0)
    lo = np.floor(lo / h) * h
    dims = grid_dims(lo, hi, h)
    return c, r, lo, h, dims


def test_invariance_permutation_translation(oracle_mod):
    c, r, lo, h, dims = _small_case()
    base = oracle_mod.Oracle(c, r, RHO).labels_grid(lo, h, dims)
    assert 0.05 < base.mean() < 0.6
    perm = np.random.default_rng(1).permutation(len(r))
    L2 = oracle_mod.Oracle(c[perm], r[perm], RHO).labels_grid(lo, h, dims)
    assert np.array_equal(base, L2)
    shift = np.array([8.0, -4.0, 2.0])  # multiples of h = 0.5: exact in binary
    L3 = oracle_mod.Oracle(c + shift, r, RHO).labels_grid(lo + shift, h, dims)
    assert np.array_equal(base, L3)


def test_invariance_reflection_axis_permutation(oracle_mod):
    c, r, lo, h, dims = _small_case(seed=10)
    nx, ny, nz = dims
    hi = lo + (np.array(dims) - 1) * h
    base = oracle_mod.Oracle(c, r, RHO).labels_grid(lo, h, dims)  # [z, y, x]
    # reflect x -> -x: grid point i maps to nx-1-i
    cr = c.copy()
    cr[:, 0] = -cr[:, 0]
    lor = lo.copy()
    lor[0] = -hi[0]
    L = oracle_mod.Oracle(cr, r, RHO).labels_grid(lor, h, dims)
    assert np.array_equal(base[:, :, ::-1], L)
    # axis permutation (x, y, z) -> (y, z, x)
    cp = c[:, [1, 2, 0]]
    lop = lo[[1, 2, 0]]
    dp = (ny, nz, nx)
    L = oracle_mod.Oracle(cp, r, RHO).labels_grid(lop, h, dp)  # [x, z, y]
    assert np.array_equal(base.transpose(2, 0, 1), L)


def test_vdw_inside_and_outside_sas(oracle_mod):
    c, r, lo, h, dims = _small_case(seed=12)
    o = oracle_mod.Oracle(c, r, RHO)
    L = o.labels_grid(lo, h, dims).reshape(-1)
    g = [lo[a] + np.arange(dims[a]) * h for a in range(3)]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    x = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    d2 = np.min(np.sum((x[:, None, :] - c[None]) ** 2, axis=2) - r ** 2, axis=1)
    s2 = np.min(np.sum((x[:, None, :] - c[None]) ** 2, axis=2) - (r + RHO) ** 2, axis=1)
    assert np.all(L[d2 <= 0] == 1)
    assert np.all(L[s2 >= 0] == 0)
    # and strictly between the two bounds for some points
    mid = (d2 > 0) & (s2 < 0)
    assert 0 < L[mid].mean() < 1
