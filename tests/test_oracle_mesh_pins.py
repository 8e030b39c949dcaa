"""Pins of the oracle's marching-cubes mesh (oracle/mesh.py) built from its
labels and crossing records: one sphere (closed forms of area and volume, a
closed oriented mesh of Euler characteristic 2), two atoms (the Pappus volume
and area of the solid of revolution, from the profile quadrature of the edge
pins) and the case table's own invariants."""
import math

import numpy as np
import pytest

RHO = 1.4


def run_mesh(oracle_mod, c, r, lo, h, dims, rho=RHO):
    from oracle import mesh as M
    o = oracle_mod.Oracle(c, r, rho)
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(lo, h, dims, keys)
    tri, V = M.mesh(L, lo, h, keys, rec["lam"])
    return L, keys, tri, V


def test_case_table_invariants():
    from oracle import mesh as M
    t = M.case_table()
    assert t[0] == [] and t[255] == []
    for cfg, tris in t.items():
        # complementing the corners keeps the cut edges (orientation reverses)
        cut = {e for tri in tris for e in tri}
        comp = {e for tri in t[255 - cfg] for e in tri}
        ends = [M._edge_ends(e) for e in range(12)]
        want = {e for e, (a, b) in enumerate(ends) if ((cfg >> a) & 1) != ((cfg >> b) & 1)}
        assert cut == want, cfg
        assert comp == want, cfg
    # one corner inside: a single triangle
    assert len(t[1]) == 1


@pytest.mark.parametrize("h", [0.2, 0.1])
def test_sphere_area_volume_closed(oracle_mod, h):
    from oracle import mesh as M
    r = 1.7
    c = np.array([[0.031, -0.017, 0.011]])
    n = int(round(5.0 / h)) + 1
    lo = np.full(3, -2.5)
    L, keys, tri, V = run_mesh(oracle_mod, c, [r], lo, h, (n, n, n))
    assert M.closed_and_oriented(tri)
    nv = len(np.unique(tri))
    ne = len({tuple(sorted(e)) for t in tri for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})
    assert nv - ne + len(tri) == 2  # a sphere
    A, Vol = M.area_volume(tri, V)
    # O(h^2) convergence of the inscribed mesh
    assert abs(A / (4 * math.pi * r * r) - 1) < 1.5 * h * h
    assert abs(Vol / (4 / 3 * math.pi * r ** 3) - 1) < 1.5 * h * h
    assert Vol > 0  # outward orientation


def test_two_atoms_pappus(oracle_mod):
    """Two atoms on the x axis: volume and area of the solid of revolution of
    the profile (van der Waals arcs and the saddle's circular arc), by
    quadrature along the axis."""
    from oracle import mesh as M
    r1, r2, d = 1.7, 1.55, 3.9
    s1, s2 = r1 + RHO, r2 + RHO
    a = (s1 * s1 - s2 * s2 + d * d) / (2 * d)
    R = math.sqrt(s1 * s1 - a * a)
    c = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    h = 0.1
    lo = np.array([-2.3, -2.31, -2.29])
    dims = (int(round((d + 4.6) / h)) + 1, 48, 48)
    L, keys, tri, V = run_mesh(oracle_mod, c, [r1, r2], lo, h, dims)
    assert M.closed_and_oriented(tri)
    A, Vol = M.area_volume(tri, V)
    # profile eta(xi): van der Waals arcs outside the saddle, the probe circle
    # of radius rho around (a, R) between its contact points
    x1 = a * r1 / s1                       # contact with sphere 1 (on segment c1-P)
    x2 = d + (a - d) * r2 / s2            # contact with sphere 2
    xs = np.linspace(-r1, d + r2, 400001)

    def eta(x):
        y = np.zeros_like(x)
        m1 = x <= x1
        y[m1] = np.sqrt(np.maximum(r1 * r1 - x[m1] ** 2, 0))
        m2 = x >= x2
        y[m2] = np.sqrt(np.maximum(r2 * r2 - (x[m2] - d) ** 2, 0))
        mm = ~m1 & ~m2
        y[mm] = R - np.sqrt(np.maximum(RHO * RHO - (x[mm] - a) ** 2, 0))
        return y
    y = eta(xs)
    dx = xs[1] - xs[0]
    vol = math.pi * np.sum(0.5 * (y[1:] ** 2 + y[:-1] ** 2)) * dx
    dy = np.diff(y)
    area = 2 * math.pi * np.sum(0.5 * (y[1:] + y[:-1]) * np.sqrt(dx * dx + dy * dy))
    assert abs(Vol / vol - 1) < 5e-3
    assert abs(A / area - 1) < 5e-3
