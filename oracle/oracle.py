"""ctypes wrapper of the plain FP64 CPU oracle (eses_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.

Labels are certified: the C oracle decides each comparison in FP64 against a
bound on its rounding error, and the points it leaves undecided are re-labelled
in exact rational arithmetic (exact.py), so the labels returned are those of
exact real arithmetic on the input doubles.  `last_undecided` holds the number
of points of the last labelling call that needed the exact re-decision.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eses_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math, no FMA)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double]
    lib.orc_destroy.argtypes = [P]
    lib.orc_num_vertices.restype = ctypes.c_int
    lib.orc_num_vertices.argtypes = [P]
    lib.orc_get_vertices.argtypes = [P, dp, ip, ip]
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_labels_points.argtypes = [P, ctypes.c_long, dp, u8p]
    lib.orc_labels_grid.argtypes = [P, dp, ctypes.c_double, ip, ctypes.c_int, ctypes.c_int, u8p]
    lib.orc_labels_points_cert.argtypes = [P, ctypes.c_long, dp, u8p]
    lib.orc_labels_grid_cert.argtypes = [P, dp, ctypes.c_double, ip, ctypes.c_int, ctypes.c_int,
                                         u8p]
    lib.orc_dist_points.argtypes = [P, ctypes.c_long, dp, ctypes.c_double, dp, ip]
    lib.orc_edges.argtypes = [P, dp, ctypes.c_double, ip, ctypes.c_long, lp, ip, ip, dp, dp, ip,
                              ip]
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def threads() -> int:
    return int(_load().orc_threads())


class Oracle:
    """Oracle for one molecule: atoms (c_i, r_i) and probe radius rho."""

    def __init__(self, centres, radii, probe: float):
        self.lib = _load()
        self.c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        self.r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        if self.c.shape[0] != self.r.shape[0] or self.r.shape[0] < 1:
            raise ValueError("centres [n,3] and radii [n] with n >= 1")
        self.probe = float(probe)
        self.h = self.lib.orc_create(self.r.shape[0], _p(self.c, ctypes.c_double),
                                     _p(self.r, ctypes.c_double), self.probe)
        if not self.h:
            raise ValueError("oracle: invalid input")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def vertices(self):
        """Exposed concave-patch probe positions: (p [m,3], atoms [m,3] ascending, sign [m])."""
        m = int(self.lib.orc_num_vertices(self.h))
        p = np.zeros((m, 3), dtype=np.float64)
        a = np.zeros((m, 3), dtype=np.int32)
        s = np.zeros(m, dtype=np.int32)
        if m:
            self.lib.orc_get_vertices(self.h, _p(p, ctypes.c_double), _p(a, ctypes.c_int),
                                      _p(s, ctypes.c_int))
        return p, a, s

    last_undecided = 0

    def _exact(self):
        ex = getattr(self, "_exact_labeller", None)
        if ex is None:
            from .exact import ExactLabeller
            p, a, sg = self.vertices()
            ex = ExactLabeller(self.c, self.r, self.probe, a, sg, p)
            self._exact_labeller = ex
        return ex

    def labels_points(self, x):
        """Exact labels of points [m,3]."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(x.shape[0], dtype=np.uint8)
        self.lib.orc_labels_points_cert(self.h, x.shape[0], _p(x, ctypes.c_double),
                                        _p(out, ctypes.c_uint8))
        und = np.flatnonzero(out == 2)
        self.last_undecided = int(und.size)
        if und.size:
            ex = self._exact()
            for q in und:
                out[q] = ex.label(x[q])
        return out

    def labels_points_fp64(self, x):
        """Uncertified FP64 labels of points [m,3] (each comparison taken at
        its FP64 value)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(x.shape[0], dtype=np.uint8)
        self.lib.orc_labels_points(self.h, x.shape[0], _p(x, ctypes.c_double),
                                   _p(out, ctypes.c_uint8))
        return out

    def labels_grid(self, lo, h, dims, k0: int = 0, k1: int | None = None, certify: bool = True):
        """Exact labels [k1-k0, ny, nx] (x fastest) of grid points lo + (i,j,k) h
        (certify=False: uncertified FP64 labels)."""
        dims = tuple(int(d) for d in dims)
        k1 = dims[2] if k1 is None else int(k1)
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        d = np.asarray(dims, dtype=np.int32)
        out = np.zeros((k1 - k0, dims[1], dims[0]), dtype=np.uint8)
        fn = self.lib.orc_labels_grid_cert if certify else self.lib.orc_labels_grid
        fn(self.h, _p(lo, ctypes.c_double), float(h), _p(d, ctypes.c_int), int(k0), int(k1),
           _p(out, ctypes.c_uint8))
        if not certify:
            return out
        und = np.argwhere(out == 2)
        self.last_undecided = int(len(und))
        if len(und):
            ex = self._exact()
            for kk, j, i in und:
                x = grid_point(lo, h, (int(i), int(j), int(kk) + k0))
                out[kk, j, i] = ex.label(x)
        return out

    def dist_points(self, x, cap: float):
        """min(cap, dist(x, A)) (0 outside the SAS union) and the owner type of each point."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        out = np.zeros(x.shape[0], dtype=np.float64)
        typ = np.zeros(x.shape[0], dtype=np.int32)
        self.lib.orc_dist_points(self.h, x.shape[0], _p(x, ctypes.c_double), float(cap),
                                 _p(out, ctypes.c_double), _p(typ, ctypes.c_int))
        return out, typ

    def edges(self, lo, h, dims, keys):
        """Records for edge keys 3*(i + nx*(j + ny*k)) + axis.

        Returns dict(status, lam, normal, type, atoms); status 1 = crossing,
        0 = equal labels, -1 = not an edge of the grid.  The two end labels of
        every edge are the exact ones (certified, undecided ones re-decided).
        """
        keys = np.ascontiguousarray(keys, dtype=np.int64).reshape(-1)
        n = keys.shape[0]
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        d = np.asarray([int(v) for v in dims], dtype=np.int32)
        nx, ny, nz = (int(v) for v in dims)
        axis = keys % 3
        idx = keys // 3
        ijk = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1)
        ok = (keys >= 0) & (idx < nx * ny * nz)
        ok &= np.where(ok, ijk[np.arange(n), axis] + 1 < d[axis], False)
        ijk_t = ijk.copy()
        ijk_t[np.arange(n), axis] += 1
        ends = np.zeros((n, 2), dtype=np.int32)
        if ok.any():
            hs = float(h)
            xs = lo[None, :] + ijk[ok].astype(np.float64) * hs  # fl(lo + fl(i h))
            xt = lo[None, :] + ijk_t[ok].astype(np.float64) * hs
            lab = self.labels_points(np.concatenate([xs, xt]))
            m = int(ok.sum())
            ends[ok, 0] = lab[:m]
            ends[ok, 1] = lab[m:]
        st = np.zeros(n, dtype=np.int32)
        lam = np.zeros(n, dtype=np.float64)
        nrm = np.zeros((n, 3), dtype=np.float64)
        typ = np.zeros(n, dtype=np.int32)
        atoms = np.full((n, 3), -1, dtype=np.int32)
        self.lib.orc_edges(self.h, _p(lo, ctypes.c_double), float(h), _p(d, ctypes.c_int), n,
                           _p(keys, ctypes.c_long), _p(ends, ctypes.c_int), _p(st, ctypes.c_int),
                           _p(lam, ctypes.c_double),
                           _p(nrm, ctypes.c_double), _p(typ, ctypes.c_int),
                           _p(atoms, ctypes.c_int))
        return dict(status=st, lam=lam, normal=nrm, type=typ, atoms=atoms)


def grid_point(lo, h, ijk):
    """Grid point (i, j, k): each coordinate fl(lo_a + fl(i_a h)) in FP64."""
    return np.array([float(lo[a]) + float(ijk[a]) * float(h) for a in range(3)])


def crossing_keys(labels):
    """Edge keys (ascending) whose endpoint labels differ; labels [nz, ny, nx]."""
    L = np.asarray(labels, dtype=np.uint8)
    nz, ny, nx = L.shape
    keys = []
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    dx = L[:, :, :-1] != L[:, :, 1:]
    dy = L[:, :-1, :] != L[:, 1:, :]
    dz = L[:-1, :, :] != L[1:, :, :]
    keys.append(3 * idx[:, :, :-1][dx] + 0)
    keys.append(3 * idx[:, :-1, :][dy] + 1)
    keys.append(3 * idx[:-1, :, :][dz] + 2)
    k = np.concatenate(keys)
    k.sort()
    return k


def fill_cavities(labels):
    """Cavity-filled labels [nz, ny, nx]: outside points (0) in 6-connected
    components of outside points that touch no boundary face of the grid
    become inside (1).  Returns (filled labels, number filled)."""
    from scipy import ndimage
    L = np.asarray(labels, dtype=np.uint8)
    out = L.copy()
    comp, n = ndimage.label(L == 0, structure=ndimage.generate_binary_structure(3, 1))
    if n == 0:
        return out, 0
    border = np.zeros(n + 1, dtype=bool)
    for face in (comp[0], comp[-1], comp[:, 0], comp[:, -1], comp[:, :, 0], comp[:, :, -1]):
        border[np.unique(face)] = True
    border[0] = True  # the inside points
    enclosed = ~border[comp]
    out[enclosed] = 1
    return out, int(enclosed.sum())
