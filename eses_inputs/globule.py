"""Seeded protein-like globules and the grid box they are sampled on.

The paper measures on protein-ligand complexes whose atoms carry van der Waals
radii (section 4, the appendix table).  Those structures are not available, so
these seeded globules stand in for them with the same kind of geometry: a
bonded random walk at 1.5 A steps, no two non-bonded centres closer than
2.4 A, packed towards 0.1 atoms per cubic angstrom, with radii drawn from the
C/N/O/S/H table below.

Recipe (globule.c; a seed fixes the molecule bit for bit):
  * confinement ball of radius R = (3N / (4 pi 0.1))^(1/3) around the origin;
  * the walk starts at the origin; each step draws up to 64 directions
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

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

# C, N, O, S, H van der Waals radii (angstrom) and their draw probabilities.
RADII_TABLE = np.array([1.70, 1.55, 1.52, 1.80, 1.20], dtype=np.float64)
RADII_PROB = np.array([0.32, 0.09, 0.10, 0.01, 0.48], dtype=np.float64)

PROBE_RADIUS = 1.4
MARGIN = 4.0


_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "globule.c")
_LIB = os.path.join(_HERE, "libglobule.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the generator (plain C, gcc)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.globule_generate.restype = ctypes.c_int
        lib.globule_generate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_int,
                                         dp, dp]
        lib.globule_log_uniform.restype = None
        lib.globule_log_uniform.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                            ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        _lib = lib
    return _lib


def globule(n: int, seed: int, density: float = 0.1, step: float = 1.5,
            min_sep: float = 2.4, tries: int = 64, restarts_before_grow: int = 200,
            grow: float = 1.02):
    """Return (centres [n,3] float64, radii [n] float64) of a seeded globule."""
    if n < 1:
        raise ValueError("n must be >= 1")
    lib = _load()
    pos = np.zeros((n, 3), dtype=np.float64)
    radii = np.zeros(n, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.globule_generate(int(n), int(seed), float(density), float(step), float(min_sep),
                              int(tries), int(restarts_before_grow), float(grow),
                              RADII_TABLE.ctypes.data_as(dp), RADII_PROB.ctypes.data_as(dp),
                              len(RADII_TABLE), pos.ctypes.data_as(dp), radii.ctypes.data_as(dp))
    if rc != 0:
        raise RuntimeError("globule generation failed")
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
    out = (ctypes.c_int * count)()
    _load().globule_log_uniform(int(count), int(seed), float(lo), float(hi), out)
    return [int(v) for v in out]


def batch(count: int = 256, spacing: float = 0.5, seed: int = 5):
    """The batched workload: `count` globules of log-uniform sizes in [200, 20000]."""
    return [molecule(n, 1000 + q, spacing) for q, n in enumerate(batch_sizes(count, seed=seed))]
