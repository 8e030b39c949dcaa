"""Pins of the oracle's edge intersections (eq. 3-4 of the paper).

For an axis edge st with Inside[s] != Inside[t] the record holds
lambda = 1 - u*, where u* is the first parameter along s + u (t - s) at which
the label changes, the outward unit normal there and the patch that carries
it.  Checked against: closed-form roots for one sphere and for the saddle of
two atoms, the label function alone (bisection, no surfaces involved), the
gradient of the distance to the admissible probe set, and volume and area
integrals.
"""
import math

import numpy as np
import pytest

RHO = 1.4


def grid_axes(lo, h, dims):
    return [lo[a] + np.arange(dims[a]) * h for a in range(3)]


def key_to_points(keys, lo, h, dims):
    nx, ny, nz = dims
    axis = keys % 3
    idx = keys // 3
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    s = np.stack([lo[0] + i * h, lo[1] + j * h, lo[2] + k * h], axis=1)
    e = np.eye(3)[axis]
    return s, e, axis


def test_single_sphere_roots_and_normals(oracle_mod):
    c = np.array([0.1, -0.23, 0.37])
    r = 1.6
    o = oracle_mod.Oracle(c[None], [r], RHO)
    lo = np.array([-4.0, -4.0, -4.0])
    h = 0.2
    dims = (41, 41, 41)
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(lo, h, dims, keys)
    assert np.all(rec["status"] == 1) and np.all(rec["type"] == 1)
    s, e, axis = key_to_points(keys, lo, h, dims)
    w = s - c
    # |w + u h e|^2 = r^2; the root inside [0, 1]
    b = 2 * h * np.sum(w * e, axis=1)
    cc = np.sum(w * w, axis=1) - r * r
    disc = b * b - 4 * h * h * cc
    u1 = (-b - np.sqrt(disc)) / (2 * h * h)
    u2 = (-b + np.sqrt(disc)) / (2 * h * h)
    u = np.where((u1 >= 0) & (u1 <= 1), u1, u2)
    assert np.allclose(1 - rec["lam"], u, atol=1e-12)
    p = s + (u * h)[:, None] * e
    assert np.allclose(rec["normal"], (p - c) / r, atol=1e-12)
    assert np.all(rec["atoms"][:, 0] == 0)


def test_two_atom_saddle_roots_closed_form(oracle_mod):
    """Atoms on the x axis: on an x-edge that meets the saddle, the root lies
    on the profile circle of radius rho around (a, R):
    xi = a -+ sqrt(rho^2 - (eta - R)^2)."""
    r1, r2, d = 1.7, 1.55, 3.9
    s1, s2 = r1 + RHO, r2 + RHO
    c = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    o = oracle_mod.Oracle(c, [r1, r2], RHO)
    a = (s1 * s1 - s2 * s2 + d * d) / (2 * d)
    R = math.sqrt(s1 * s1 - a * a)
    lo = np.array([-4.0, -4.03, -4.07])
    h = 0.1
    dims = (int(round((d + 8) / h)) + 1, 82, 82)
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(lo, h, dims, keys)
    sad = (rec["type"] == 2) & (keys % 3 == 0)
    assert sad.sum() > 50
    s, e, _ = key_to_points(keys[sad], lo, h, dims)
    eta = np.hypot(s[:, 1], s[:, 2])
    u = 1 - rec["lam"][sad]
    xi = s[:, 0] + u * h
    off = np.sqrt(RHO * RHO - (eta - R) ** 2)
    err = np.minimum(np.abs(xi - (a - off)), np.abs(xi - (a + off)))
    assert np.max(err) < 1e-9
    # normal towards the probe centre on the circle
    p = s + (u * h)[:, None] * e
    q = np.stack([np.full(len(p), a), R * p[:, 1] / eta, R * p[:, 2] / eta], axis=1)
    want = (q - p) / np.linalg.norm(q - p, axis=1, keepdims=True)
    assert np.allclose(rec["normal"][sad], want, atol=1e-9)


def _molecule(n, seed, h):
    from eses_inputs import molecule
    return molecule(n, seed, h)


@pytest.mark.parametrize("n,seed,h", [(40, 21, 0.35), (120, 22, 0.5)])
def test_edges_against_label_bisection(oracle_mod, n, seed, h):
    """u* from bisection of the label function alone (no surface enumeration)."""
    m = _molecule(n, seed, h)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    L = o.labels_grid(m.lo, m.spacing, m.dims)
    keys = oracle_mod.crossing_keys(L)
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(len(keys), size=min(800, len(keys)), replace=False))
    keys = keys[pick]
    rec = o.edges(m.lo, m.spacing, m.dims, keys)
    assert np.all(rec["status"] == 1)
    assert set(np.unique(rec["type"])) == {1, 2, 3}
    s, e, _ = key_to_points(keys, m.lo, m.spacing, m.dims)
    K = 256
    us = np.linspace(0.0, 1.0, K + 1)
    pts = s[:, None, :] + (us[None, :, None] * m.spacing) * e[:, None, :]
    # the bisection closes in on the surface to within rounding, so it runs on
    # the FP64 label function as computed (the crossing records are FP64 too)
    lab = o.labels_points_fp64(pts.reshape(-1, 3)).reshape(len(keys), K + 1)
    first = np.argmax(lab != lab[:, :1], axis=1)
    assert np.all(lab[np.arange(len(keys)), first] != lab[:, 0])
    lo_u = us[first - 1]
    hi_u = us[first]
    L0 = lab[:, 0]
    for _ in range(48):
        mid = 0.5 * (lo_u + hi_u)
        lm = o.labels_points_fp64(s + (mid * m.spacing)[:, None] * e)
        same = lm == L0
        lo_u = np.where(same, mid, lo_u)
        hi_u = np.where(same, hi_u, mid)
    ustar = 1 - rec["lam"]
    # an interval of 1/256 can hide two crossings; the oracle reports the first
    # change, so it may only be at or before the sampled one
    close = np.abs(ustar - 0.5 * (lo_u + hi_u)) * m.spacing < 1e-9
    assert close.mean() > 0.995
    assert np.all(ustar <= hi_u + 1e-12)


def test_normals_are_distance_gradients(oracle_mod):
    """At a surface point the outward normal is -grad dist(x, A)."""
    m = _molecule(80, 31, 0.45)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    L = o.labels_grid(m.lo, m.spacing, m.dims)
    keys = oracle_mod.crossing_keys(L)
    rng = np.random.default_rng(2)
    keys = np.sort(rng.choice(keys, size=600, replace=False))
    rec = o.edges(m.lo, m.spacing, m.dims, keys)
    s, e, _ = key_to_points(keys, m.lo, m.spacing, m.dims)
    p = s + ((1 - rec["lam"]) * m.spacing)[:, None] * e
    eps = 1e-6
    grad = np.zeros_like(p)
    for a in range(3):
        dp = np.zeros(3)
        dp[a] = eps
        fp, _ = o.dist_points(p + dp, 10.0)
        fm, _ = o.dist_points(p - dp, 10.0)
        grad[:, a] = (fp - fm) / (2 * eps)
    dist, _ = o.dist_points(p, 10.0)
    on = np.abs(dist - RHO) < 1e-9
    assert on.mean() > 0.99
    smooth = on & (np.abs(np.linalg.norm(grad, axis=1) - 1) < 1e-3)
    assert smooth.mean() > 0.95
    assert np.allclose(rec["normal"][smooth], -grad[smooth], atol=2e-4)
    assert np.allclose(np.linalg.norm(rec["normal"], axis=1), 1.0, atol=1e-12)
    # leaving M along the edge (s inside) the outward normal points forward
    comp = rec["normal"][np.arange(len(keys)), keys % 3]
    inside_s = L.reshape(-1)[keys // 3] == 1
    assert np.all(np.where(inside_s, comp > -1e-12, comp < 1e-12))


def line_volume(L, keys, lam, h, axis):
    """Volume from crossings along lines of one axis: h^2 * sum of inside lengths."""
    nz, ny, nx = L.shape
    A = np.moveaxis(L, 2 - axis, -1).astype(np.float64)  # lines along the last axis
    inside_full = (A[..., :-1] * A[..., 1:]).sum() * h
    sel = keys % 3 == axis
    u = 1 - lam[sel]
    idx = keys[sel] // 3
    Ls = L.reshape(-1)[idx]
    part = np.where(Ls == 1, u, 1 - u) * h
    return h * h * (inside_full + part.sum())


def test_volume_and_area_single_sphere(oracle_mod):
    r = 1.8
    c = np.array([0.013, -0.021, 0.007])
    o = oracle_mod.Oracle(c[None], [r], RHO)
    h = 0.1
    lo = np.array([-2.5, -2.5, -2.5])
    dims = (51, 51, 51)
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(lo, h, dims, keys)
    V = 4 / 3 * math.pi * r ** 3
    for axis in range(3):
        assert abs(line_volume(L, keys, rec["lam"], h, axis) / V - 1) < 2e-3
    area = h * h * np.sum(np.abs(rec["normal"][np.arange(len(keys)), keys % 3]))
    assert abs(area / (4 * math.pi * r * r) - 1) < 1e-2


def test_volume_consistent_across_axes(oracle_mod):
    """The enclosed volume does not depend on the line direction used to
    integrate it (divergence theorem); a reversed lambda or a wrong root
    breaks the agreement."""
    m = _molecule(150, 41, 0.3)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    L = o.labels_grid(m.lo, m.spacing, m.dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(m.lo, m.spacing, m.dims, keys)
    vols = [line_volume(L, keys, rec["lam"], m.spacing, a) for a in range(3)]
    assert max(vols) / min(vols) - 1 < 2e-3
    cnt = L.sum() * m.spacing ** 3
    assert abs(vols[0] / cnt - 1) < 0.05


def test_spindle_axis_crossing_closed_form(oracle_mod):
    """On the axis of a spindle torus (R < rho) every circle point is at the
    same distance, so the label changes where sqrt((xi - a)^2 + R^2) = rho:
    xi = a -+ sqrt(rho^2 - R^2).  There the torus quartic is a perfect square
    and the crossing is a double root."""
    r, d = 1.5, 5.6
    s = r + RHO
    c = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    o = oracle_mod.Oracle(c, [r, r], RHO)
    a = d / 2
    R = math.sqrt(s * s - a * a)
    assert R < RHO
    lo = np.array([-4.0, -4.0, -4.0])
    h = 0.2
    dims = (69, 41, 41)
    nx, ny = dims[0], dims[1]
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    j = k = 20  # y = z = 0
    row = keys[(keys % 3 == 0) & ((keys // 3) // nx == j + ny * k)]
    assert len(row) == 4  # van der Waals exits/entries around the open neck
    rec = o.edges(lo, h, dims, row)
    x = lo[0] + ((row // 3) % nx + 1 - rec["lam"]) * h
    want = sorted([-r, a - math.sqrt(RHO ** 2 - R ** 2), a + math.sqrt(RHO ** 2 - R ** 2), d + r])
    assert np.allclose(np.sort(x), want, atol=1e-9)


def _grid_around(oracle_mod, o, lo, hi, h):
    """Labels, crossing keys and edge records of the box [lo, hi] at spacing h."""
    dims = tuple(int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    return L, keys, o.edges(lo, h, dims, keys), dims


def test_two_atom_pappus_volume_and_area(oracle_mod):
    """Two atoms with an ordinary saddle (R > rho): the SES is a solid of
    revolution whose profile is the two van der Waals arcs joined by the lower
    arc of the probe circle, so Pappus' theorems give its volume and its
    convex (two spherical zones) and saddle areas by 1-D quadrature.  The
    oracle's crossings reproduce them along every axis (lambda, normals and
    patch tags all enter)."""
    from scipy.integrate import quad
    r1, r2, d = 1.7, 1.5, 3.6
    s1, s2 = r1 + RHO, r2 + RHO
    a = (s1 * s1 - s2 * s2 + d * d) / (2 * d)
    R = math.sqrt(s1 * s1 - a * a)
    assert R > RHO
    t1, t2 = a * r1 / s1, d + (a - d) * r2 / s2  # contact points along the axis
    root = lambda x: math.sqrt(RHO * RHO - (x - a) ** 2)
    V = math.pi * (r1 * r1 * (t1 + r1) - (t1 ** 3 + r1 ** 3) / 3
                   + r2 * r2 * (d + r2 - t2) - (r2 ** 3 - (t2 - d) ** 3) / 3)
    V += quad(lambda x: math.pi * (R - root(x)) ** 2, t1, t2, epsabs=1e-13, epsrel=1e-13)[0]
    A_convex = 2 * math.pi * (r1 * (t1 + r1) + r2 * (d + r2 - t2))
    A_saddle = quad(lambda x: 2 * math.pi * (R - root(x)) * RHO / root(x), t1, t2,
                    epsabs=1e-13, epsrel=1e-13)[0]
    q, _ = np.linalg.qr(np.random.default_rng(4).normal(size=(3, 3)))
    c = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]]) @ q.T + np.array([0.0123, -0.0271, 0.0191])
    o = oracle_mod.Oracle(c, [r1, r2], RHO)
    h = 0.1
    lo, hi = c.min(axis=0) - 2.2, c.max(axis=0) + 2.2
    L, keys, rec, dims = _grid_around(oracle_mod, o, lo, hi, h)
    for axis in range(3):
        assert abs(line_volume(L, keys, rec["lam"], h, axis) / V - 1) < 3e-3
    w = h * h * np.abs(rec["normal"][np.arange(len(keys)), keys % 3])
    assert abs(w[rec["type"] == 1].sum() / A_convex - 1) < 4e-3
    assert abs(w[rec["type"] == 2].sum() / A_saddle - 1) < 4e-3
    assert not np.any(rec["type"] == 3)


def test_concave_cap_area_girard(oracle_mod):
    """Three atoms whose two probes do not overlap: each concave patch is the
    spherical triangle on its probe sphere with corners toward the three
    centres, of area rho^2 (alpha + beta + gamma - pi) (Girard); the
    concave-tagged crossings within rho of the probe reproduce it."""
    from tests.parity import crossing_points
    r = np.array([1.7, 1.55, 1.52])
    s = r + RHO
    q, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(3, 3)))
    c = np.array([[0.0, 0.0, 0.0], [3.5, 0.0, 0.0], [1.6, 3.1, 0.0]]) @ q.T + np.array(
        [0.31, -0.17, 0.05])
    o = oracle_mod.Oracle(c, r, RHO)
    P, atoms, sign = o.vertices()
    assert len(sign) == 2 and np.linalg.norm(P[0] - P[1]) > 2 * RHO
    h = 0.04
    for p in P:
        u = (c - p) / s[:, None]
        ang = 0.0
        for i in range(3):
            a, b, e = u[i], u[(i + 1) % 3], u[(i + 2) % 3]
            t1, t2 = b - (a @ b) * a, e - (a @ e) * a
            ang += math.acos(t1 @ t2 / (np.linalg.norm(t1) * np.linalg.norm(t2)))
        A_cap = RHO * RHO * (ang - math.pi)
        lo, hi = p - (RHO + 0.1), p + (RHO + 0.1)
        L, keys, rec, dims = _grid_around(oracle_mod, o, lo, hi, h)
        x = crossing_points({"key": keys, "lam": rec["lam"]}, lo, h, dims)
        sel = (rec["type"] == 3) & (np.linalg.norm(x - p, axis=1) < RHO + 1e-9)
        area = h * h * np.abs(rec["normal"][np.arange(len(keys)), keys % 3])[sel].sum()
        assert abs(area / A_cap - 1) < 1e-2


def test_crossings_lie_on_their_tagged_patch(oracle_mod):
    """Every crossing lies on the surface its tag names (the atom's sphere, the
    pair's torus, the triple's probe sphere) to rounding, and the tags cover
    all three patch types on a molecule."""
    from tests.parity import crossing_points, surface_residual
    m = _molecule(120, 4, 0.5)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    L = o.labels_grid(m.lo, m.spacing, m.dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(m.lo, m.spacing, m.dims, keys)
    x = crossing_points({"key": keys, "lam": rec["lam"]}, m.lo, m.spacing, m.dims)
    resid, _ = surface_residual(o, rec["type"], rec["atoms"], x)
    assert resid.max() < 1e-9, resid.max()
    assert set(np.unique(rec["type"])) == {1, 2, 3}
