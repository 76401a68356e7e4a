"""Host logic of the schedule autotuner (no GPU): batch signatures and the
JSON cache."""
import os

import synth


def test_signature_depends_on_shape_not_on_object_identity(tmp_path):
    from paper_1610_03918_amd import autotune
    ws = [synth.trench(nx=64, ny=32, width=4, depth=8, ppc=2, seed=31)]
    p1 = [synth.load(w) for w in ws]
    p2 = [synth.load(w) for w in [synth.trench(nx=64, ny=32, width=4, depth=8, ppc=2, seed=31)]]
    assert autotune.signature(ws, p1) == autotune.signature(ws, p2)
    w3 = [synth.trench(nx=64, ny=32, width=6, depth=8, ppc=2, seed=31)]
    assert autotune.signature(w3, [synth.load(w) for w in w3]) != autotune.signature(ws, p1)
    path = os.path.join(tmp_path, "s.json")
    assert autotune.lookup(ws, p1, path) is None
    cache = {autotune.signature(ws, p1): {"schedule": dict(autotune.DEFAULT)}}
    import json
    with open(path, "w") as f:
        json.dump(cache, f)
    assert autotune.lookup(ws, p2, path)["schedule"]["tile"] == [16, 16]


def test_committed_cache_is_well_formed():
    from paper_1610_03918_amd import autotune
    cache = autotune.load_cache()
    for key, e in cache.items():
        s = e["schedule"]
        assert len(key) == 16
        assert s["push_unroll"] in (1, 2, 4) and s["push_merge"] in (0, 2, 4)
        assert all(t in (8, 16, 32, 64) for t in s["tile"])
        assert 0 < s["chunk"] <= 8192
        assert min(x["ms"] for x in e["trials"] if x["converged"]) <= e["ms_per_step"] + 1e-9
