"""Seeded protein-like globules and the grid box they are sampled on.

The paper measures on protein-ligand complexes whose atoms carry van der Waals
radii (section 4, the appendix table).  Those structures are not available, so
these seeded globules stand in for them with the same kind of geometry: a
bonded random walk at 1.5 A steps, no two non-bonded centres closer than
2.4 A, packed towards 0.1 atoms per cubic angstrom, with radii drawn from the
C/N/O/S/H table below.

Recipe (each step consumes the generator in this order, so a seed fixes the
molecule bit for bit):
  * confinement ball of radius R = (3N / (4 pi 0.1))^(1/3) around the origin;
  * the walk starts at the origin; each step tries up to 64 directions drawn
    uniformly on the sphere, taking the first that stays in the ball and keeps
    2.4 A from every placed atom other than its bonded predecessor;
  * if all 64 fail, the walk restarts from a uniformly drawn placed atom (a
    branch); after 200 consecutive failed restarts R grows by 2 %;
  * radii are drawn i.i.d. after the positions.

The grid box follows the paper's recipe of a tight bounding box of the van der
Waals spheres padded by a margin (section 2.3): lo = min(c - r) - margin,
hi = max(c + r) + margin, dims = ceil((hi - lo) / h) + 1 points per axis and
grid point (i, j, k) at lo + (i, j, k) * h.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# C, N, O, S, H van der Waals radii (angstrom) and their draw probabilities.
RADII_TABLE = np.array([1.70, 1.55, 1.52, 1.80, 1.20], dtype=np.float64)
RADII_PROB = np.array([0.32, 0.09, 0.10, 0.01, 0.48], dtype=np.float64)

PROBE_RADIUS = 1.4
MARGIN = 4.0


def globule(n: int, seed: int, density: float = 0.1, step: float = 1.5,
            min_sep: float = 2.4, tries: int = 64, restarts_before_grow: int = 200,
            grow: float = 1.02):
    """Return (centres [n,3] float64, radii [n] float64) of a seeded globule."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    radius = (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)
    pos = np.zeros((n, 3), dtype=np.float64)
    # Occupancy grid of 2.4 A cells (fixed slots per cell, -1 = empty).  A cell
    # of side min_sep holds few atoms, since non-bonded centres keep min_sep apart.
    cell = min_sep
    reach = int(math.ceil((step + min_sep) / cell))
    slots = 16
    state = {}

    def cell_of(p):
        half = state["half"]
        return (int(math.floor(p[0] / cell)) + half, int(math.floor(p[1] / cell)) + half,
                int(math.floor(p[2] / cell)) + half)

    def insert(idx):
        cx, cy, cz = cell_of(pos[idx])
        f = state["fill"][cx, cy, cz]
        if f >= slots:
            raise RuntimeError("globule: cell slot overflow")
        state["grid"][cx, cy, cz, f] = idx
        state["fill"][cx, cy, cz] = f + 1

    def rebuild(count, rad):
        half = int(math.ceil(1.25 * rad / cell)) + reach + 2
        side = 2 * half
        state["half"] = half
        state["grid"] = np.full((side, side, side, slots), -1, dtype=np.int32)
        state["fill"] = np.zeros((side, side, side), dtype=np.int32)
        for q in range(count):
            insert(q)

    rebuild(0, radius)
    insert(0)
    min_sep2 = min_sep * min_sep
    cur = 0
    failed_restarts = 0
    for m in range(1, n):
        while True:
            d = rng.normal(size=(tries, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            cand = pos[cur] + step * d
            ok = np.einsum("ij,ij->i", cand, cand) <= radius * radius
            cx, cy, cz = cell_of(pos[cur])
            near = state["grid"][cx - reach:cx + reach + 1, cy - reach:cy + reach + 1,
                                 cz - reach:cz + reach + 1].reshape(-1)
            near = near[(near >= 0) & (near != cur)]
            if near.size:
                diff = cand[:, None, :] - pos[near][None, :, :]
                dist2 = np.einsum("ijk,ijk->ij", diff, diff)
                ok &= np.all(dist2 >= min_sep2, axis=1)
            hit = np.flatnonzero(ok)
            if hit.size:
                pos[m] = cand[hit[0]]
                insert(m)
                cur = m
                failed_restarts = 0
                break
            cur = int(rng.integers(m))
            failed_restarts += 1
            if failed_restarts >= restarts_before_grow:
                radius *= grow
                failed_restarts = 0
                if radius / cell + reach + 2 > state["half"]:
                    rebuild(m, radius)
    kinds = rng.choice(len(RADII_TABLE), size=n, p=RADII_PROB)
    radii = RADII_TABLE[kinds].copy()
    return pos, radii


def bbox_from_atoms(centres, radii, margin: float = MARGIN):
    """Tight box of the van der Waals spheres padded by `margin` (section 2.3)."""
    c = np.asarray(centres, dtype=np.float64)
    r = np.asarray(radii, dtype=np.float64)
    lo = (c - r[:, None]).min(axis=0) - margin
    hi = (c + r[:, None]).max(axis=0) + margin
    return lo, hi


def grid_dims(lo, hi, h: float):
    """Points per axis: ceil((hi - lo) / h) + 1."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return tuple(int(math.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))


@dataclass
class Molecule:
    centres: np.ndarray
    radii: np.ndarray
    probe: float
    spacing: float
    lo: np.ndarray
    hi: np.ndarray
    dims: tuple = field(default=())
    seed: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.radii.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


def molecule(n: int, seed: int, spacing: float, probe: float = PROBE_RADIUS,
             margin: float = MARGIN) -> Molecule:
    c, r = globule(n, seed)
    lo, hi = bbox_from_atoms(c, r, margin)
    return Molecule(c, r, probe, spacing, lo, hi, grid_dims(lo, hi, spacing), seed)


# Workloads: (atoms, seed, spacing).  The batch draws its sizes separately.
WORKLOADS = {
    "globule500_h0.5": (500, 1, 0.5),
    "globule5000_h0.25": (5000, 2, 0.25),
    "globule100k_h0.2": (100000, 3, 0.2),
    "globule20k_h0.1": (20000, 4, 0.1),
}


def workload(name: str) -> Molecule:
    n, seed, h = WORKLOADS[name]
    return molecule(n, seed, h)


def batch_sizes(count: int = 256, lo: int = 200, hi: int = 20000, seed: int = 5):
    """Log-uniform molecule sizes for the batched workload; molecule m uses seed 1000 + m."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return [int(round(math.exp(v))) for v in u]
