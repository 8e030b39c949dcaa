"""Host logic of the autotuner: workload signatures and the result cache
(timing itself needs a GPU and is covered by the GPU batch tests)."""
import json
from types import SimpleNamespace


def mols(*sizes, h=0.5):
    return [SimpleNamespace(n_atoms=n, spacing=h) for n in sizes]


def test_signature_buckets():
    from paper_1809_04352_amd import autotune
    a = autotune.signature(mols(3000, 1200), 1)
    assert a == autotune.signature(mols(2500, 1700), 1)  # same count, log2 bucket, spacing
    assert a != autotune.signature(mols(3000, 1200), 0)  # precision
    assert a != autotune.signature(mols(3000, 1200, 10), 1)  # molecule count
    assert a != autotune.signature(mols(30000, 12000), 1)  # atom bucket
    assert a != autotune.signature(mols(3000, 1200, h=0.25), 1)  # spacing


def test_cached_result_is_returned(tmp_path, monkeypatch):
    from paper_1809_04352_amd import autotune
    path = tmp_path / "tune.json"
    monkeypatch.setenv("ESES_AUTOTUNE_CACHE", str(path))
    ms = mols(4000, 900)
    key = autotune.signature(ms, 1)
    best = {"tile": 4, "blocks_per_cu": 2}
    times = {json.dumps(best, sort_keys=True): 1.5}
    path.write_text(json.dumps({key: {"best": best, "times": times}}))
    got, got_times = autotune.tune(ms, 1)
    assert got == best and got_times == times
