"""Python binding of the gfx950 ESES library (include/eses.h).

Argument marshalling only: device memory and streams come from PyTorch, every
step of the computation runs in the HIP library.  Loading fails loudly if the
library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libeses_gfx950.so")

ESES_OK = 0
ESES_EINVAL = -1
ESES_ENOMEM = -2
ESES_ECAPACITY = -3
ESES_EDEVICE = -4
ESES_EINTERNAL = -5

ESES_FP64 = 0
ESES_FP32_RECHECK = 1

EXPORTED = [
    "eses_bbox_from_atoms", "eses_grid_dims", "eses_build_candidates", "eses_candidates_info",
    "eses_copy_vertices", "eses_classify", "eses_edge_intersections", "eses_free_candidates",
    "eses_last_error", "eses_version", "eses_edge_work", "eses_set_timing",
    "eses_get_kernel_times", "eses_trim_cache", "eses_set_allocator", "eses_exact_labels",
    "eses_edge_intersections_noalloc", "eses_fill_cavities", "eses_mesh", "eses_stream_slabs",
]

# C types of the caller-allocator hook (eses_set_allocator).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class EsesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"eses status {status}: {msg}")
        self.status = status


class Molecule(ctypes.Structure):
    _fields_ = [("centers", ctypes.c_void_p), ("radii", ctypes.c_void_p),
                ("n_atoms", ctypes.c_int64), ("probe_radius", ctypes.c_double),
                ("spacing", ctypes.c_double), ("bbox_lo", ctypes.c_double * 3),
                ("bbox_hi", ctypes.c_double * 3)]


class Config(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("force_recheck", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("edge_fallback", ctypes.c_int32),
                ("vertex_pool", ctypes.c_int32), ("tile_pool", ctypes.c_int32),
                ("unc_queue", ctypes.c_int32), ("unit_order", ctypes.c_int32),
                ("edges_per_molecule", ctypes.c_int32)]


class CandidateStats(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("dims", ctypes.c_int32 * 3),
                ("n_points", ctypes.c_int64), ("n_neighbour_pairs", ctypes.c_int64),
                ("n_circles", ctypes.c_int64), ("n_vertices", ctypes.c_int64),
                ("n_exposed_faces", ctypes.c_int64), ("n_exposed_circles", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("tile_list_entries", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["dims"] = tuple(self.dims)
        return d


class ClassifyStats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_inside", ctypes.c_int64),
                ("n_rechecked", ctypes.c_int64), ("n_shell", ctypes.c_int64),
                ("tests_atom", ctypes.c_int64), ("tests_vertex", ctypes.c_int64),
                ("tests_face", ctypes.c_int64), ("tests_face_cut", ctypes.c_int64),
                ("tests_circle", ctypes.c_int64), ("tests_circle_cut", ctypes.c_int64),
                ("n_exact", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class EdgeStats(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("reach_sphere", ctypes.c_int64),
                ("reach_torus", ctypes.c_int64), ("quad_solves", ctypes.c_int64),
                ("quartic_solves", ctypes.c_int64), ("horner_flops", ctypes.c_int64),
                ("cut_tests", ctypes.c_int64), ("label_evals", ctypes.c_int64),
                ("label_tests", ctypes.c_int64 * 6), ("cone_tests", ctypes.c_int64)]

    def as_dict(self):
        d = {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "label_tests"}
        names = ["atom", "vertex", "face", "face_cut", "circle", "circle_cut"]
        for n, v in zip(names, self.label_tests):
            d["label_tests_" + n] = int(v)
        return d


class KernelTimes(ctypes.Structure):
    _fields_ = [("classify_ms", ctypes.c_double), ("edge_detect_ms", ctypes.c_double),
                ("edge_roots_ms", ctypes.c_double)]


class MeshStats(ctypes.Structure):
    _fields_ = [("area", ctypes.c_double), ("volume", ctypes.c_double),
                ("n_triangles", ctypes.c_int64)]


class IsectSoA(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("lambda_", ctypes.c_void_p),
                ("normal", ctypes.c_void_p), ("patch_type", ctypes.c_void_p),
                ("atoms", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


_lib = None


def load():
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"ESES HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    lib.eses_last_error.restype = ctypes.c_char_p
    lib.eses_version.restype = ctypes.c_char_p
    lib.eses_bbox_from_atoms.restype = st
    lib.eses_bbox_from_atoms.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P, P]
    lib.eses_grid_dims.restype = st
    lib.eses_grid_dims.argtypes = [ctypes.POINTER(Molecule), P]
    lib.eses_build_candidates.restype = st
    lib.eses_build_candidates.argtypes = [ctypes.POINTER(Molecule), ctypes.c_int32,
                                          ctypes.POINTER(Config), P, ctypes.POINTER(P)]
    lib.eses_candidates_info.restype = st
    lib.eses_candidates_info.argtypes = [P, ctypes.c_int32, ctypes.POINTER(CandidateStats)]
    lib.eses_copy_vertices.restype = st
    lib.eses_copy_vertices.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), P]
    lib.eses_classify.restype = st
    lib.eses_classify.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(ClassifyStats), P]
    lib.eses_edge_intersections.restype = st
    lib.eses_edge_intersections.argtypes = [P, P, ctypes.POINTER(IsectSoA), P, P]
    lib.eses_edge_intersections_noalloc.restype = st
    lib.eses_edge_intersections_noalloc.argtypes = [P, P, ctypes.POINTER(IsectSoA),
                                                    ctypes.POINTER(ctypes.c_int64), P]
    lib.eses_stream_slabs.restype = st
    lib.eses_stream_slabs.argtypes = [P, ctypes.c_int, ctypes.c_int32, P, ctypes.POINTER(IsectSoA),
                                      ctypes.POINTER(ctypes.c_int64), P]
    lib.eses_mesh.restype = st
    lib.eses_mesh.argtypes = [P, P, ctypes.POINTER(IsectSoA), P, P, P,
                              ctypes.POINTER(MeshStats), P]
    lib.eses_fill_cavities.restype = st
    lib.eses_fill_cavities.argtypes = [P, P, P, P]
    lib.eses_free_candidates.restype = None
    lib.eses_free_candidates.argtypes = [P]
    lib.eses_edge_work.restype = st
    lib.eses_edge_work.argtypes = [P, P, ctypes.POINTER(EdgeStats), P]
    lib.eses_set_allocator.restype = None
    lib.eses_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, P]
    lib.eses_trim_cache.restype = st
    lib.eses_trim_cache.argtypes = []
    lib.eses_set_timing.restype = None
    lib.eses_set_timing.argtypes = [ctypes.c_int]
    lib.eses_exact_labels.restype = st
    lib.eses_exact_labels.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, P, P,
                                      ctypes.c_int64, P, ctypes.c_int64, P]
    lib.eses_get_kernel_times.restype = st
    lib.eses_get_kernel_times.argtypes = [P, ctypes.POINTER(KernelTimes)]
    _lib = lib
    return lib


def _check(status: int):
    if status != ESES_OK:
        raise EsesError(status, load().eses_last_error().decode())


def version() -> str:
    return load().eses_version().decode()


def bbox_from_atoms(centres, radii, margin: float):
    c = np.ascontiguousarray(centres, dtype=np.float64)
    r = np.ascontiguousarray(radii, dtype=np.float64)
    lo = np.zeros(3)
    hi = np.zeros(3)
    _check(load().eses_bbox_from_atoms(c.ctypes.data, r.ctypes.data, r.shape[0], float(margin),
                                       lo.ctypes.data, hi.ctypes.data))
    return lo, hi


def make_molecule(centres_dev, radii_dev, probe: float, spacing: float, lo, hi) -> Molecule:
    """Descriptor over device tensors centres [n,3] and radii [n] (float64)."""
    m = Molecule()
    m.centers = centres_dev.data_ptr()
    m.radii = radii_dev.data_ptr()
    m.n_atoms = int(radii_dev.shape[0])
    m.probe_radius = float(probe)
    m.spacing = float(spacing)
    for a in range(3):
        m.bbox_lo[a] = float(lo[a])
        m.bbox_hi[a] = float(hi[a])
    return m


def grid_dims(mol: Molecule):
    d = (ctypes.c_int32 * 3)()
    _check(load().eses_grid_dims(ctypes.byref(mol), ctypes.addressof(d)))
    return tuple(int(v) for v in d)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream)


class Candidates:
    """Owning wrapper of an eses_candidates handle."""

    def __init__(self, mols, tile: int = 0, stream=None, force_recheck: bool = False,
                 blocks_per_cu: int = 0, edge_fallback: bool = False, vertex_pool: int = 0,
                 tile_pool: int = 0, unc_queue: int = 0, unit_order: int = 0,
                 edges_per_molecule: bool = False):
        lib = load()
        self.mols = list(mols)
        arr = (Molecule * len(self.mols))(*self.mols)
        cfg = Config()
        cfg.tile = int(tile)
        cfg.force_recheck = 1 if force_recheck else 0
        cfg.blocks_per_cu = int(blocks_per_cu)
        cfg.edge_fallback = 1 if edge_fallback else 0
        cfg.vertex_pool = int(vertex_pool)
        cfg.tile_pool = int(tile_pool)
        cfg.unc_queue = int(unc_queue)
        cfg.unit_order = int(unit_order)
        cfg.edges_per_molecule = 1 if edges_per_molecule else 0
        h = ctypes.c_void_p()
        self.stream = _stream_ptr(stream)
        _check(lib.eses_build_candidates(arr, len(self.mols), ctypes.byref(cfg), self.stream,
                                         ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().eses_free_candidates(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, mol: int = 0) -> dict:
        st = CandidateStats()
        _check(load().eses_candidates_info(self.h, int(mol), ctypes.byref(st)))
        return st.as_dict()


def build_candidates(mols, tile: int = 0, stream=None, force_recheck: bool = False,
                     blocks_per_cu: int = 0, edge_fallback: bool = False,
                     vertex_pool: int = 0, tile_pool: int = 0,
                     unc_queue: int = 0, unit_order: int = 0,
                     edges_per_molecule: bool = False) -> Candidates:
    return Candidates(mols, tile, stream, force_recheck, blocks_per_cu, edge_fallback,
                      vertex_pool, tile_pool, unc_queue, unit_order, edges_per_molecule)


def copy_vertices(cand: Candidates, mol: int, p_dev, atoms_dev, sign_dev, stream=None) -> int:
    cnt = ctypes.c_int64()
    cap = int(sign_dev.shape[0])
    st = load().eses_copy_vertices(cand.h, int(mol), p_dev.data_ptr() if cap else None,
                                   atoms_dev.data_ptr() if cap else None,
                                   sign_dev.data_ptr() if cap else None, cap, ctypes.byref(cnt),
                                   _stream_ptr(stream))
    if st not in (ESES_OK, ESES_ECAPACITY):
        _check(st)
    return int(cnt.value)


def classify(cand: Candidates, prec: int, labels_dev, stream=None, stats: bool = False):
    n = len(labels_dev)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in labels_dev])
    out = (ClassifyStats * n)() if stats else None
    _check(load().eses_classify(cand.h, int(prec), ptrs, out, _stream_ptr(stream)))
    if stats:
        return [s.as_dict() for s in out]
    return None


@dataclass
class IsectBuffers:
    key: object
    lam: object
    normal: object
    patch_type: object
    atoms: object

    @property
    def capacity(self) -> int:
        return int(self.key.shape[0])


def alloc_isect(capacity: int, device="cuda"):
    import torch
    cap = max(int(capacity), 1)
    return IsectBuffers(torch.empty(cap, dtype=torch.int64, device=device),
                        torch.empty(cap, dtype=torch.float64, device=device),
                        torch.empty((cap, 3), dtype=torch.float64, device=device),
                        torch.empty(cap, dtype=torch.uint8, device=device),
                        torch.empty((cap, 3), dtype=torch.int32, device=device))


def edge_intersections(cand: Candidates, labels_dev, outs, stream=None):
    """Returns (status, counts).  status is ESES_OK or ESES_ECAPACITY."""
    n = len(labels_dev)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in labels_dev])
    soa = (IsectSoA * n)()
    for q, o in enumerate(outs):
        soa[q].key = o.key.data_ptr()
        soa[q].lambda_ = o.lam.data_ptr()
        soa[q].normal = o.normal.data_ptr()
        soa[q].patch_type = o.patch_type.data_ptr()
        soa[q].atoms = o.atoms.data_ptr()
        soa[q].capacity = o.capacity
    counts = (ctypes.c_int64 * n)()
    st = load().eses_edge_intersections(cand.h, ptrs, soa, counts, _stream_ptr(stream))
    if st not in (ESES_OK, ESES_ECAPACITY):
        _check(st)
    return st, [int(c) for c in counts]


def edge_intersections_noalloc(cand: Candidates, labels_dev, out, stream=None):
    """The allocation-free form of edge_intersections for a one-molecule handle:
    (status, count); status is ESES_OK or ESES_ECAPACITY."""
    soa = IsectSoA()
    soa.key = out.key.data_ptr()
    soa.lambda_ = out.lam.data_ptr()
    soa.normal = out.normal.data_ptr()
    soa.patch_type = out.patch_type.data_ptr()
    soa.atoms = out.atoms.data_ptr()
    soa.capacity = out.capacity
    cnt = ctypes.c_int64()
    st = load().eses_edge_intersections_noalloc(cand.h, labels_dev.data_ptr(), ctypes.byref(soa),
                                                ctypes.byref(cnt), _stream_ptr(stream))
    if st not in (ESES_OK, ESES_ECAPACITY):
        _check(st)
    return st, int(cnt.value)


def stream_slabs(cand: Candidates, prec, slab_planes: int, labels_host, out_host, stream=None):
    """The out-of-core form for a one-molecule handle: labels and records in
    HOST tensors (labels_host uint8 [npoints]; out_host an IsectBuffers of
    host tensors).  Returns (status, count); status is ESES_OK or
    ESES_ECAPACITY."""
    soa = _soa([out_host])
    cnt = ctypes.c_int64()
    st = load().eses_stream_slabs(cand.h, int(prec), int(slab_planes), labels_host.data_ptr(),
                                  soa, ctypes.byref(cnt), _stream_ptr(stream))
    if st not in (ESES_OK, ESES_ECAPACITY):
        _check(st)
    return st, int(cnt.value)


def _soa(outs):
    soa = (IsectSoA * len(outs))()
    for q, o in enumerate(outs):
        soa[q].key = o.key.data_ptr()
        soa[q].lambda_ = o.lam.data_ptr()
        soa[q].normal = o.normal.data_ptr()
        soa[q].patch_type = o.patch_type.data_ptr()
        soa[q].atoms = o.atoms.data_ptr()
        soa[q].capacity = o.capacity
    return soa


def mesh(cand: Candidates, labels_dev, outs, counts, triangles=None, stream=None):
    """Marching-cubes mesh of each molecule from its labels and crossing records:
    returns [dict(area, volume, n_triangles)]; with triangles (a list of device
    int32 tensors [cap, 3]) the triangles' record indices are written too."""
    n = len(labels_dev)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in labels_dev])
    cnt = (ctypes.c_int64 * n)(*[int(k) for k in counts])
    st = (MeshStats * n)()
    tp = tc = None
    if triangles is not None:
        tp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in triangles])
        tc = (ctypes.c_int64 * n)(*[int(t.shape[0]) for t in triangles])
    status = load().eses_mesh(cand.h, ptrs, _soa(outs), cnt, tp, tc, st, _stream_ptr(stream))
    if status not in (ESES_OK, ESES_ECAPACITY):
        _check(status)
    return [dict(area=s.area, volume=s.volume, n_triangles=int(s.n_triangles)) for s in st]


def fill_cavities(cand: Candidates, labels_dev, stream=None):
    """Cavity-filled labels, in place; returns the points filled per molecule."""
    n = len(labels_dev)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in labels_dev])
    out = (ctypes.c_int64 * n)()
    _check(load().eses_fill_cavities(cand.h, ptrs, out, _stream_ptr(stream)))
    return [int(v) for v in out]


def edge_work(cand: Candidates, labels_dev, stream=None):
    n = len(labels_dev)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in labels_dev])
    out = (EdgeStats * n)()
    _check(load().eses_edge_work(cand.h, ptrs, out, _stream_ptr(stream)))
    return [o.as_dict() for o in out]


def exact_labels(centres, radii, probe: float, probe_atoms, probe_sign, points):
    """Exact labels (host arithmetic, no GPU) of points [m,3] for atoms and a
    concave probe list (ascending atom triples [nv,3], sides [nv])."""
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    pa = np.ascontiguousarray(probe_atoms, dtype=np.int32).reshape(-1, 3)
    ps = np.ascontiguousarray(probe_sign, dtype=np.int8).reshape(-1)
    x = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(x.shape[0], dtype=np.uint8)
    _check(load().eses_exact_labels(c.ctypes.data, r.ctypes.data, r.shape[0], float(probe),
                                    pa.ctypes.data if len(pa) else None,
                                    ps.ctypes.data if len(ps) else None, pa.shape[0],
                                    x.ctypes.data if len(x) else None, x.shape[0],
                                    out.ctypes.data if len(x) else None))
    return out


def set_timing(enable: bool):
    load().eses_set_timing(1 if enable else 0)


def trim_cache():
    """Free the library's cached device workspace (synchronises)."""
    _check(load().eses_trim_cache())


_allocator = None  # the callbacks given to the library (kept alive while set)


def set_allocator(alloc=None, release=None):
    """Route the library's device workspace through alloc(bytes, stream) ->
    int pointer (0 for none) and release(ptr, stream); no arguments restore
    the library's own cache.  The callbacks may run on the library's worker
    threads."""
    global _allocator
    lib = load()
    if alloc is None or release is None:
        lib.eses_set_allocator(ALLOC_FN(), RELEASE_FN(), None)
        _allocator = None
        return
    fa = ALLOC_FN(lambda n, st, ctx: alloc(int(n), st or 0) or None)
    fr = RELEASE_FN(lambda p, st, ctx: release(p or 0, st or 0))
    lib.eses_set_allocator(fa, fr, None)
    _allocator = (fa, fr)


def kernel_times(cand: Candidates) -> dict:
    t = KernelTimes()
    _check(load().eses_get_kernel_times(cand.h, ctypes.byref(t)))
    return {"classify_ms": t.classify_ms, "edge_detect_ms": t.edge_detect_ms,
            "edge_roots_ms": t.edge_roots_ms}


def surface(centres, radii, probe: float, spacing: float, lo, hi, prec: int = ESES_FP64,
            tile: int = 0, isect_capacity: int | None = None, device="cuda",
            force_recheck: bool = False, stats: bool = False, edge_fallback: bool = False,
            vertex_pool: int = 0, tile_pool: int = 0, unc_queue: int = 0):
    """Whole hot path for one molecule given host arrays; returns host numpy results."""
    import torch
    c = torch.as_tensor(np.ascontiguousarray(centres, dtype=np.float64), device=device)
    r = torch.as_tensor(np.ascontiguousarray(radii, dtype=np.float64), device=device)
    mol = make_molecule(c, r, probe, spacing, lo, hi)
    dims = grid_dims(mol)
    cand = build_candidates([mol], tile, force_recheck=force_recheck, edge_fallback=edge_fallback,
                            vertex_pool=vertex_pool, tile_pool=tile_pool, unc_queue=unc_queue)
    try:
        info = cand.info(0)
        nv = info["n_vertices"]
        vp = torch.empty((max(nv, 1), 3), dtype=torch.float64, device=device)
        va = torch.empty((max(nv, 1), 3), dtype=torch.int32, device=device)
        vs = torch.empty(max(nv, 1), dtype=torch.int8, device=device)
        copy_vertices(cand, 0, vp, va, vs)
        labels = torch.empty(dims[0] * dims[1] * dims[2], dtype=torch.uint8, device=device)
        cstats = classify(cand, prec, [labels], stats=stats)
        cap = isect_capacity if isect_capacity is not None else 1
        out = alloc_isect(cap, device)
        status, counts = edge_intersections(cand, [labels], [out])
        if status == ESES_ECAPACITY:
            del out
            out = alloc_isect(counts[0], device)
            status, counts = edge_intersections(cand, [labels], [out])
        torch.cuda.synchronize()
        k = counts[0]
        return dict(
            dims=dims,
            info=info,
            vertices=(vp[:nv].cpu().numpy(), va[:nv].cpu().numpy(), vs[:nv].cpu().numpy()),
            labels=labels.cpu().numpy().reshape(dims[2], dims[1], dims[0]),
            key=out.key[:k].cpu().numpy(),
            lam=out.lam[:k].cpu().numpy(),
            normal=out.normal[:k].cpu().numpy(),
            patch_type=out.patch_type[:k].cpu().numpy(),
            atoms=out.atoms[:k].cpu().numpy(),
            classify_stats=cstats[0] if cstats else None,
        )
    finally:
        cand.close()
