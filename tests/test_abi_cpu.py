"""Host-side checks of the C-ABI library: it loads, exports every function the
header declares, and its host helpers and argument checks behave as the
header states.  No device compute is issued here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1809_04352_amd import eses
    if not os.path.exists(eses.LIB_PATH):
        from paper_1809_04352_amd import build
        build.build()
    return eses


def declared_functions():
    text = open(os.path.join(ROOT, "include", "eses.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eses_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 10
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(so, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (eses_\w+)", out))
    assert set(names) <= exported
    assert set(lib.EXPORTED) == set(names)


def test_version_and_error_string(lib):
    assert lib.version().startswith("eses-gfx950")
    assert isinstance(lib.load().eses_last_error(), bytes)


def test_grid_dims_matches_recipe(lib):
    from eses_inputs import molecule, grid_dims
    m = molecule(50, 3, 0.37)
    mol = lib.Molecule()
    mol.spacing = m.spacing
    for a in range(3):
        mol.bbox_lo[a] = m.lo[a]
        mol.bbox_hi[a] = m.hi[a]
    assert lib.grid_dims(mol) == grid_dims(m.lo, m.hi, m.spacing)


def test_bbox_helper(lib):
    from eses_inputs import globule, bbox_from_atoms
    c, r = globule(30, 4)
    lo, hi = lib.bbox_from_atoms(c, r, 4.0)
    lo2, hi2 = bbox_from_atoms(c, r, 4.0)
    assert np.array_equal(lo, lo2) and np.array_equal(hi, hi2)


def test_argument_errors(lib):
    so = lib.load()
    mol = lib.Molecule()
    mol.spacing = 0.0
    d = (ctypes.c_int32 * 3)()
    assert so.eses_grid_dims(ctypes.byref(mol), ctypes.addressof(d)) == lib.ESES_EINVAL
    assert b"spacing" in so.eses_last_error()
    mol.spacing = 0.5
    mol.bbox_lo[0] = float("nan")
    assert so.eses_grid_dims(ctypes.byref(mol), ctypes.addressof(d)) == lib.ESES_EINVAL
    mol.bbox_lo[0] = 1.0
    mol.bbox_hi[0] = 0.5  # empty box
    assert so.eses_grid_dims(ctypes.byref(mol), ctypes.addressof(d)) == lib.ESES_EINVAL
    h = ctypes.c_void_p()
    assert so.eses_build_candidates(None, 1, None, None, ctypes.byref(h)) == lib.ESES_EINVAL
    assert so.eses_build_candidates(ctypes.byref(mol), 0, None, None,
                                    ctypes.byref(h)) == lib.ESES_EINVAL
    assert so.eses_build_candidates(ctypes.byref(mol), 1, None, None, None) == lib.ESES_EINVAL
    cfg = lib.Config()
    cfg.tile = 5
    mol.bbox_hi[0] = 3.0
    assert so.eses_build_candidates(ctypes.byref(mol), 1, ctypes.byref(cfg), None,
                                    ctypes.byref(h)) == lib.ESES_EINVAL
    assert b"tile" in so.eses_last_error()
    assert so.eses_classify(None, 0, None, None, None) == lib.ESES_EINVAL
    assert so.eses_edge_intersections(None, None, None, None, None) == lib.ESES_EINVAL
    so.eses_free_candidates(None)
    bad_c = np.zeros((2, 3))
    bad_r = np.array([1.0, -1.0])
    lo = np.zeros(3)
    hi = np.zeros(3)
    assert so.eses_bbox_from_atoms(bad_c.ctypes.data, bad_r.ctypes.data, 2, 4.0, lo.ctypes.data,
                                   hi.ctypes.data) == lib.ESES_EINVAL


def test_product_path_does_not_touch_the_oracle():
    """The package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1809_04352_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("oracle-free", ""), f
