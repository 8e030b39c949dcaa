"""Pins of the oracle's certified labels and of their exact re-decision.

The FP64 oracle bounds the rounding error of every comparison; a label that
depends on a comparison within its bound is re-decided in exact rational
arithmetic on the input doubles (oracle/exact.py), so the labels are those of
exact real arithmetic.  Checked here against what fixes them independently:
the closed ball of one atom on a dyadic grid (where squared distances are exact
and points lie exactly on the sphere), the two-atom closed form away from its
decision boundaries, the mirror symmetry of a dyadic configuration (exact
labels cannot break it, whatever the rounding of mirrored points), and the
agreement of the two formulations (FP64 direct membership tests with bounds,
exact reduced half-space forms) on every point of tie-rich lattices.
"""
import decimal
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from tests.test_oracle_pins import two_atom_label, rot

RHO = 1.4


def test_sign_sqrt_sum_against_decimal():
    """sign(a + b sqrt(X)) for random rationals, including exact zeros (a =
    -b sqrt(X) with X a perfect square), against 80-digit decimal arithmetic."""
    from oracle.exact import sign_sqrt_sum
    decimal.getcontext().prec = 80
    rng = np.random.default_rng(5)
    for _ in range(3000):
        a = Fr(int(rng.integers(-50, 50)), int(rng.integers(1, 9)))
        b = Fr(int(rng.integers(-50, 50)), int(rng.integers(1, 9)))
        X = Fr(int(rng.integers(0, 60)), int(rng.integers(1, 9)))
        if rng.random() < 0.3:  # an exact zero
            r = Fr(int(rng.integers(0, 12)), int(rng.integers(1, 5)))
            X = r * r
            a = -b * r
        want = (decimal.Decimal(a.numerator) / a.denominator
                + decimal.Decimal(b.numerator) / b.denominator
                * (decimal.Decimal(X.numerator) / X.denominator).sqrt())
        s = 0 if abs(want) < decimal.Decimal(10) ** -60 else (1 if want > 0 else -1)
        assert sign_sqrt_sum(a, b, X) == s, (a, b, X)


def test_single_atom_exact_ties(oracle_mod):
    """One atom on a dyadic grid: every point exactly on the van der Waals sphere
    is inside (M is closed), every other point follows the closed ball; the
    FP64 comparisons at the ties are left undecided and re-decided exactly."""
    c = np.array([[0.25, -0.5, 0.25]])
    r = np.array([1.25])  # 0.75^2 + 1^2 = 1.25^2: ties on the grid
    o = oracle_mod.Oracle(c, r, RHO)
    lo = np.array([-2.0, -2.5, -2.0])
    h = 0.25
    dims = (19, 17, 18)
    L = o.labels_grid(lo, h, dims)
    assert o.last_undecided > 0
    g = [lo[a] + np.arange(dims[a]) * h for a in range(3)]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    d2 = (X - c[0, 0]) ** 2 + (Y - c[0, 1]) ** 2 + (Z - c[0, 2]) ** 2  # exact (dyadic)
    assert np.array_equal(L, (d2 <= 1.25 ** 2).astype(np.uint8))
    assert np.sum(d2 == 1.25 ** 2) > 10


def test_exact_labeller_two_atoms(oracle_mod):
    """The exact labeller alone (reduced forms in rationals) against the
    two-atom closed form, away from the closed form's own decision
    boundaries."""
    from oracle.exact import ExactLabeller
    for (r1, r2, d) in [(1.7, 1.7, 3.2), (1.5, 1.5, 5.6), (1.2, 1.8, 1.0)]:
        R = rot(int(r1 * 100 + r2 * 10 + d * 7))
        c1 = np.array([0.3, -0.2, 0.1])
        c2 = c1 + R @ np.array([d, 0.0, 0.0])
        E = ExactLabeller(np.stack([c1, c2]), [r1, r2], RHO, np.zeros((0, 3)), np.zeros(0))
        rng = np.random.default_rng(2)
        x = rng.uniform(np.minimum(c1, c2) - 4.0, np.maximum(c1, c2) + 4.0, size=(1500, 3))
        lab, margin = two_atom_label(x, c1, c2, r1, r2, RHO)
        ok = margin > 1e-9
        got = np.array([E.label(p) for p in x[ok]])
        assert np.array_equal(got, lab[ok]), (r1, r2, d)


def dyadic_lattice():
    """A 3 x 3 x 2 block of atoms 2 A apart (dyadic coordinates), radius
    0.75 and probe 0.75 (SAS radius 1.5): probes touch four atoms of each
    square, and many grid points of a 0.25 A grid lie exactly on van der
    Waals and SAS spheres and exactly rho from probe positions."""
    g = np.array([[x, y, z] for z in (0.0, 2.0) for y in (-2.0, 0.0, 2.0) for x in (-2.0, 0.0, 2.0)])
    r = np.full(len(g), 0.75)
    return g, r, 0.75


def decimal_chain():
    """Six atoms 2.6 A apart along x (radius 1.7) on a 0.25 A grid whose
    points sit at decimal offsets from the centres: in real arithmetic on the
    decimal values some points lie on van der Waals spheres (offsets 0.9, 1.2,
    -0.8 from a centre), in doubles they are within rounding of them."""
    c = np.array([[2.6 * q, 0.0, 0.0] for q in range(6)])
    r = np.full(6, 1.7)
    return c, r, 1.4


@pytest.mark.parametrize("case", ["lattice", "chain"])
def test_certified_labels_equal_exact_on_tie_lattices(oracle_mod, case):
    """Every label of a tie-rich input equals the exact labeller's: the
    undecided points (re-decided exactly) and all certified points of a
    sampled set (every point within 1e-6 A of a sphere, plus random ones)."""
    from oracle.exact import ExactLabeller
    c, r, rho = dyadic_lattice() if case == "lattice" else decimal_chain()
    h = 0.25
    lo = (c - r[:, None]).min(axis=0) - 1.0
    hi = (c + r[:, None]).max(axis=0) + 1.0
    if case == "chain":
        lo = np.array([-4.1, -3.0, -3.0])  # offsets 0.9 etc. from the centres
    dims = tuple(int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    o = oracle_mod.Oracle(c, r, rho)
    L = o.labels_grid(lo, h, dims)
    assert o.last_undecided > 0
    p, a, s = o.vertices()
    E = ExactLabeller(c, r, rho, a, s, p)
    Lfp = o.labels_grid(lo, h, dims, certify=False)
    pts = np.stack(np.meshgrid(*[lo[q] + np.arange(dims[q]) * h for q in (2, 1, 0)],
                               indexing="ij"), axis=-1)[..., ::-1].reshape(-1, 3)
    d = np.linalg.norm(pts[:, None, :] - c[None], axis=2)
    near = np.any((np.abs(d - r) < 1e-6) | (np.abs(d - (r + rho)) < 1e-6), axis=1)
    rng = np.random.default_rng(7)
    sample = np.union1d(np.flatnonzero(near),
                        np.union1d(rng.choice(len(pts), 600, replace=False),
                                   np.flatnonzero(L.reshape(-1) != Lfp.reshape(-1))))
    Lf = L.reshape(-1)
    bad = [q for q in sample if E.label(pts[q]) != Lf[q]]
    assert not bad, (len(bad), bad[:5])


def test_mirror_symmetry_exact(oracle_mod):
    """A configuration symmetric under x -> -x on a grid symmetric about 0
    (dyadic: mirrored points are exact mirrors): exact labels are mirror
    symmetric bit for bit, ties included."""
    c, r, rho = dyadic_lattice()
    h = 0.25
    lo = np.array([-4.0, -4.0, -2.0])
    dims = (33, 33, 25)
    o = oracle_mod.Oracle(c, r, rho)
    L = o.labels_grid(lo, h, dims)
    assert o.last_undecided > 0
    assert np.array_equal(L, L[:, :, ::-1])
    assert np.array_equal(L, L[:, ::-1, :])


@pytest.mark.parametrize("n,seed,h", [(120, 4, 0.5), (500, 1, 0.5), (300, 5, 0.25)])
def test_no_undecided_points_on_seeded_globules(oracle_mod, n, seed, h):
    """On the seeded workloads no label depends on a comparison within its
    rounding bound (the bounds are not so wide that FP64 decides nothing)."""
    from eses_inputs import molecule
    m = molecule(n, seed, h)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    o.labels_grid(m.lo, m.spacing, m.dims)
    assert o.last_undecided == 0
