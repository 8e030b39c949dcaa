"""The library's host arbiter of undecided labels (eses_exact_labels: FP64
with a running error bound, dyadic big-integer arithmetic where that bound does
not decide) against the oracle's exact labels, which come from a different
formulation (FP64 direct membership tests with their bounds, rational
re-decision in Python).  Runs on the CPU: the arbiter is host code."""
import math

import numpy as np
import pytest

from tests.test_oracle_exact_pins import dyadic_lattice, decimal_chain


@pytest.fixture(scope="module")
def E():
    from paper_1809_04352_amd import eses
    eses.load()
    return eses


def grid_points(lo, h, dims):
    g = [np.array([float(lo[a]) + float(i) * h for i in range(dims[a])]) for a in range(3)]
    Z, Y, X = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    return np.stack([X, Y, Z], axis=-1).reshape(-1, 3)


@pytest.mark.parametrize("case", ["lattice", "chain", "globule"])
def test_exact_labels_match_oracle(E, oracle_mod, case):
    if case == "globule":
        from eses_inputs import molecule
        m = molecule(60, 3, 0.4)
        c, r, rho, lo, h, dims = m.centres, m.radii, m.probe, m.lo, m.spacing, m.dims
    else:
        c, r, rho = dyadic_lattice() if case == "lattice" else decimal_chain()
        h = 0.25
        lo = (c - r[:, None]).min(axis=0) - 1.0
        hi = (c + r[:, None]).max(axis=0) + 1.0
        if case == "chain":
            lo = np.array([-4.1, -3.0, -3.0])
        dims = tuple(int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    o = oracle_mod.Oracle(c, r, rho)
    ref = o.labels_grid(lo, h, dims).reshape(-1)
    p, a, s = o.vertices()
    x = grid_points(lo, h, dims)
    if case == "globule":
        x, ref = x[::7], ref[::7]
    got = E.exact_labels(c, r, rho, a, s, x)
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, (bad.size, bad[:5])


def test_exact_sign_of_dyadic_ties(E):
    """Points exactly on a sphere, exactly rho from a probe and exactly on an
    admissibility boundary are decided by the big-integer path: one atom at a
    dyadic centre, points on its van der Waals sphere are inside and points
    just off it follow the side."""
    c = np.array([[0.25, -0.5, 0.25]])
    r = np.array([1.25])
    pts = np.array([[0.25 + 0.75, -0.5 + 1.0, 0.25], [0.25 + 0.75 + 2.0 ** -45, -0.5 + 1.0, 0.25],
                    [0.25, -0.5, 0.25 + 1.25], [0.25, -0.5, 0.25 + 1.25 - 2.0 ** -48]])
    got = E.exact_labels(c, r, 1.4, np.zeros((0, 3)), np.zeros(0), pts)
    assert list(got) == [1, 0, 1, 1]
