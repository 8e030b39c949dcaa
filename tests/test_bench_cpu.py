"""Host-side pieces of bench.py: the one-GPU rule and the SES volume and area
it reports from the path's outputs (checked here on the oracle's outputs for
one sphere, whose volume and area are known)."""
import math
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_ses_per_atom_single_sphere(oracle_mod):
    import torch
    sys.path.insert(0, ROOT)
    import bench
    r, h = 1.8, 0.1
    c = np.array([[0.013, -0.021, 0.007]])
    o = oracle_mod.Oracle(c, [r], 1.4)
    lo = np.array([-2.5, -2.5, -2.5])
    dims = (51, 51, 51)
    L = o.labels_grid(lo, h, dims)
    keys = oracle_mod.crossing_keys(L)
    rec = o.edges(lo, h, dims, keys)
    out = SimpleNamespace(key=torch.as_tensor(keys), normal=torch.as_tensor(rec["normal"]))
    mol = SimpleNamespace(spacing=h, n_atoms=1)
    res = bench.ses_per_atom([mol], [{"n_inside": int(L.sum())}], [out], [len(keys)])
    assert abs(res["volume_per_atom_A3"] / (4 / 3 * math.pi * r ** 3) - 1) < 2e-2
    assert abs(res["area_per_atom_A2"] / (4 * math.pi * r * r) - 1) < 1e-2
