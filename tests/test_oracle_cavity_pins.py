"""Pins of the cavity-filled variant in the oracle (oracle.fill_cavities:
connected components of outside points that touch no boundary face are
filled): a hollow shell of atoms around a probe-accessible cavity, against the
geometry of the shell and against a breadth-first search written here; a
globule, filled once and twice."""
import math

import numpy as np
import pytest

RHO = 1.4


def shell(n=140, R=8.0, r=1.7):
    """Atoms on a sphere of radius R (Fibonacci points, about 2.6 A apart):
    their SAS balls close the shell to the probe, so the inside of the shell
    holds an enclosed probe-accessible cavity."""
    q = np.arange(n) + 0.5
    z = 1 - 2 * q / n
    phi = math.pi * (1 + 5 ** 0.5) * q
    s = np.sqrt(1 - z * z)
    c = R * np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return c, np.full(n, r)


def bfs_fill(L):
    """Outside points reached from the boundary faces by a queue."""
    from collections import deque
    nz, ny, nx = L.shape
    seen = np.zeros(L.shape, bool)
    dq = deque()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if (i in (0, nx - 1) or j in (0, ny - 1) or k in (0, nz - 1)) and L[k, j, i] == 0:
                    seen[k, j, i] = True
                    dq.append((k, j, i))
    while dq:
        k, j, i = dq.popleft()
        for dk, dj, di in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            a, b, c = k + dk, j + dj, i + di
            if 0 <= a < nz and 0 <= b < ny and 0 <= c < nx and not seen[a, b, c] and L[a, b, c] == 0:
                seen[a, b, c] = True
                dq.append((a, b, c))
    out = L.copy()
    out[(L == 0) & ~seen] = 1
    return out


def test_shell_cavity_filled(oracle_mod):
    c, r = shell()
    h = 0.5
    lo = np.full(3, -12.0)
    dims = (49, 49, 49)
    o = oracle_mod.Oracle(c, r, RHO)
    L = o.labels_grid(lo, h, dims)
    g = lo[0] + np.arange(49) * h
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    rad = np.sqrt(X * X + Y * Y + Z * Z)
    assert np.all(L[rad < 4.0] == 0)  # the cavity is solvent before filling
    F, n = oracle_mod.fill_cavities(L)
    assert n > 0
    assert np.all(F[rad < 8.0] == 1)          # everything within the shell's centres
    assert np.array_equal(F[rad > 8.0 + 1.7 + 0.01], L[rad > 8.0 + 1.7 + 0.01])
    assert np.all(F >= L)
    assert np.array_equal(F, bfs_fill(L))


def test_globule_fill_idempotent(oracle_mod):
    from eses_inputs import molecule
    m = molecule(300, 5, 0.5)
    o = oracle_mod.Oracle(m.centres, m.radii, m.probe)
    L = o.labels_grid(m.lo, m.spacing, m.dims)
    F, n = oracle_mod.fill_cavities(L)
    F2, n2 = oracle_mod.fill_cavities(F)
    assert n2 == 0 and np.array_equal(F, F2)
    assert np.array_equal(F, bfs_fill(L))
    assert np.all(F >= L)
